// Adjoint kernels: vector-Jacobian products of deposit, interpolation and
// gradient, used to differentiate the particle-mesh step with respect to the
// particle positions (reverse-mode through the leapfrog of Sect. 3.4).
//
// With u = x n the position in cell units and W(u) the product of the per-axis
// windows of Sect. 3.5, d/dx = n d/du, and per axis (d = u - floor(u) - 1/2):
//   TSC weights (1/2)(1/2 - d)^2, 3/4 - d^2, (1/2)(1/2 + d)^2
//   derivatives  -(1/2 - d),      -2 d,     (1/2 + d)
//   CIC weights 1 - d, d (d = u - 1/2 - floor(u - 1/2)); derivatives -1, 1.
// The TSC window is C^1, so these derivatives are exact.
#include "internal.h"

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ int wrap_index(int i, int n) {
  i += (i < 0) ? n : 0;
  i -= (i >= n) ? n : 0;
  return i;
}

__device__ __forceinline__ int wrap_any(int i, int n) {
  const int r = i % n;
  return r < 0 ? r + n : r;
}

// weights w[] and their derivatives dw[] (per unit of u) along one axis, for
// the in-cell fraction d as defined above; first cell relative to floor
template <int MAS>
__device__ __forceinline__ void axis_wdw(float d, float *w, float *dw) {
  if constexpr (MAS == 3) {
    const float a = 0.5f - d, b = 0.5f + d;
    w[0] = 0.5f * a * a;
    w[1] = 0.75f - d * d;
    w[2] = 0.5f * b * b;
    dw[0] = -a;
    dw[1] = -2.0f * d;
    dw[2] = b;
  } else {
    w[0] = 1.0f - d;
    w[1] = d;
    dw[0] = -1.0f;
    dw[1] = 1.0f;
  }
}

// first (wrapped) cell index and weights/derivatives of particle p on each axis
template <int MAS, int PK>
__device__ __forceinline__ void support_wdw(const float *__restrict__ pos,
                                            const int32_t *__restrict__ cell, int64_t p, int n,
                                            int first[3], float w[3][MAS], float dw[3][MAS]) {
  if constexpr (PK == PM_POS_BOX) {
    // same arithmetic as the forward window evaluation, so that the weights match bit for bit
    const float fn = (float)n;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float u = pos[3 * p + d] * fn;
      if constexpr (MAS == 3) {
        const float fl = floorf(u);
        axis_wdw<3>(u - fl - 0.5f, w[d], dw[d]);
        first[d] = wrap_any((int)fl - 1, n);
      } else {
        const float t = u - 0.5f;
        const float fl = floorf(t);
        axis_wdw<2>(t - fl, w[d], dw[d]);
        first[d] = wrap_any((int)fl, n);
      }
    }
  } else {
    const int q = wrap_any(cell[p], n * n * n);
    int c[3];
    c[0] = q / (n * n);
    c[1] = (q / n) - c[0] * n;
    c[2] = q - (q / n) * n;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float o = pos[3 * p + d];
      if constexpr (MAS == 3) {
        axis_wdw<3>(o - 0.5f, w[d], dw[d]);
        first[d] = wrap_any(c[d] - 1, n);
      } else if (o >= 0.5f) {
        axis_wdw<2>(o - 0.5f, w[d], dw[d]);
        first[d] = wrap_any(c[d], n);
      } else {
        axis_wdw<2>(o + 0.5f, w[d], dw[d]);
        first[d] = wrap_any(c[d] - 1, n);
      }
    }
  }
}

// pos_bar[p] += scale * n * mass * sum_c rho_bar[c] grad_u W(u_p - c - 1/2)
template <int MAS, int PK>
__global__ __launch_bounds__(kThreads) void k_deposit_vjp(const float *__restrict__ pos,
                                                          const int32_t *__restrict__ cell,
                                                          int64_t np, int n,
                                                          const float *__restrict__ rho_bar,
                                                          float scale, float *__restrict__ pos_bar) {
  const int64_t p = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kThreads + threadIdx.x;
  if (p >= np) return;
  int f[3];
  float w[3][MAS], dw[3][MAS];
  support_wdw<MAS, PK>(pos, cell, p, n, f, w, dw);
  float gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
  for (int a = 0; a < MAS; ++a) {
    const size_t ia = (size_t)wrap_index(f[0] + a, n) * n;
#pragma unroll
    for (int b = 0; b < MAS; ++b) {
      const size_t row = (ia + wrap_index(f[1] + b, n)) * n;
#pragma unroll
      for (int c = 0; c < MAS; ++c) {
        const float r = rho_bar[row + wrap_index(f[2] + c, n)];
        gx = fmaf(dw[0][a] * w[1][b] * w[2][c], r, gx);
        gy = fmaf(w[0][a] * dw[1][b] * w[2][c], r, gy);
        gz = fmaf(w[0][a] * w[1][b] * dw[2][c], r, gz);
      }
    }
  }
  pos_bar[3 * p + 0] += scale * gx;
  pos_bar[3 * p + 1] += scale * gy;
  pos_bar[3 * p + 2] += scale * gz;
}

// Transpose of the interpolation, per particle p:
//   pos_bar[p] += scale * n * sum_c grad_u W (g_c . lam_p)   (the position term)
//   g_bar[c]   += W lam_p                                     (the grid term: a 3-component deposit)
// for a chunk of kVChunk consecutive particles per workgroup: the grid term is first
// summed in an LDS box of the chunk's cells (grown by the window's reach) with
// LDS atomics, then added to g_bar with one global atomic per component and touched
// cell (about 11 per particle for particles in lattice or cell order, instead of 81).
// A chunk spread over more than kVTable cells adds every weight with a global atomic.
constexpr int kVThreads = 256;
constexpr int kVPPT = 4;                    // particles per thread
constexpr int kVChunk = kVThreads * kVPPT;  // particles per workgroup
constexpr int kVTable = 4096;               // cells of the chunk box in LDS (3 floats each)

__device__ __forceinline__ int min_image(int d, int n) { return wrap_any(d + n / 2, n) - n / 2; }

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

template <int MAS, int PK>
__global__ __launch_bounds__(kVThreads) void k_interp_vjp_chunk(
    const float *__restrict__ pos, const int32_t *__restrict__ cell, int64_t np, int n,
    const float *__restrict__ g, const float *__restrict__ lam, float pscale, float gscale,
    float *__restrict__ g_bar, float *__restrict__ pos_bar) {
  __shared__ float box[3 * kVTable];
  __shared__ int red[6][kVThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kVChunk;
  int ref[3];
  {
    float w[3][MAS], dw[3][MAS];
    support_wdw<MAS, PK>(pos, cell, base, n, ref, w, dw);
  }
  // window support of each of the thread's particles, relative to the chunk's first
  int rf[kVPPT][3];
  float w[kVPPT][3][MAS], dw[kVPPT][3][MAS];
  bool live[kVPPT];
  int lo[3] = {n, n, n}, hi[3] = {-n, -n, -n};
#pragma unroll
  for (int m = 0; m < kVPPT; ++m) {
    const int64_t p = base + threadIdx.x + (int64_t)m * kVThreads;
    live[m] = p < np;
    int f[3] = {0, 0, 0};
    if (live[m]) support_wdw<MAS, PK>(pos, cell, p, n, f, w[m], dw[m]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      rf[m][a] = min_image(f[a] - ref[a], n);
      if (live[m]) {
        lo[a] = min(lo[a], rf[m][a]);
        hi[a] = max(hi[a], rf[m][a]);
      }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int l = wave_min(lo[a]), h = wave_max(hi[a]);
    if (lane == 0) {
      red[a][wave] = l;
      red[3 + a][wave] = h;
    }
  }
  __syncthreads();
  int ext[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    int l = red[a][0], h = red[3 + a][0];
    for (int q = 1; q < kVThreads / 64; ++q) {
      l = min(l, red[a][q]);
      h = max(h, red[3 + a][q]);
    }
    lo[a] = l;
    ext[a] = h - l + MAS;
  }
  const int vol = ext[0] * ext[1] * ext[2];
  const bool in_lds = vol <= kVTable;
  if (in_lds) {
    for (int i = threadIdx.x; i < 3 * vol; i += kVThreads) box[i] = 0.0f;
    __syncthreads();
  }
#pragma unroll 1
  for (int m = 0; m < kVPPT; ++m) {
    if (!live[m]) continue;
    const int64_t p = base + threadIdx.x + (int64_t)m * kVThreads;
    const float l0 = lam[3 * p + 0], l1 = lam[3 * p + 1], l2 = lam[3 * p + 2];
    float gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
    for (int a = 0; a < MAS; ++a) {
      const size_t ia = (size_t)wrap_any(ref[0] + rf[m][0] + a, n) * n;
#pragma unroll
      for (int b = 0; b < MAS; ++b) {
        const size_t row = (ia + wrap_any(ref[1] + rf[m][1] + b, n)) * n;
        const int lrow = ((rf[m][0] - lo[0] + a) * ext[1] + (rf[m][1] - lo[1] + b)) * ext[2] +
                         (rf[m][2] - lo[2]);
#pragma unroll
        for (int c = 0; c < MAS; ++c) {
          const size_t cc = row + wrap_any(ref[2] + rf[m][2] + c, n);
          if (pos_bar) {
            const float gl = g[3 * cc] * l0 + g[3 * cc + 1] * l1 + g[3 * cc + 2] * l2;
            gx = fmaf(dw[m][0][a] * w[m][1][b] * w[m][2][c], gl, gx);
            gy = fmaf(w[m][0][a] * dw[m][1][b] * w[m][2][c], gl, gy);
            gz = fmaf(w[m][0][a] * w[m][1][b] * dw[m][2][c], gl, gz);
          }
          if (g_bar) {
            const float wt = gscale * w[m][0][a] * w[m][1][b] * w[m][2][c];
            if (in_lds) {
              float *bx = box + 3 * (lrow + c);
              atomicAdd(bx + 0, wt * l0);
              atomicAdd(bx + 1, wt * l1);
              atomicAdd(bx + 2, wt * l2);
            } else {
              unsafeAtomicAdd(&g_bar[3 * cc + 0], wt * l0);
              unsafeAtomicAdd(&g_bar[3 * cc + 1], wt * l1);
              unsafeAtomicAdd(&g_bar[3 * cc + 2], wt * l2);
            }
          }
        }
      }
    }
    if (pos_bar) {
      pos_bar[3 * p + 0] += pscale * gx;
      pos_bar[3 * p + 1] += pscale * gy;
      pos_bar[3 * p + 2] += pscale * gz;
    }
  }
  if (!in_lds || !g_bar) return;
  __syncthreads();
  const int e12 = ext[1] * ext[2];
  for (int t = threadIdx.x; t < vol; t += kVThreads) {
    const float v0 = box[3 * t], v1 = box[3 * t + 1], v2 = box[3 * t + 2];
    if (v0 == 0.0f && v1 == 0.0f && v2 == 0.0f) continue;
    const int x = t / e12, r = t - x * e12;
    const int y = r / ext[2], z = r - y * ext[2];
    const size_t gc = ((size_t)wrap_any(ref[0] + lo[0] + x, n) * n +
                       wrap_any(ref[1] + lo[1] + y, n)) * n + wrap_any(ref[2] + lo[2] + z, n);
    unsafeAtomicAdd(&g_bar[3 * gc + 0], v0);
    unsafeAtomicAdd(&g_bar[3 * gc + 1], v1);
    unsafeAtomicAdd(&g_bar[3 * gc + 2], v2);
  }
}

// Interpolation transpose through the 8^3-tile buckets of a counting sort (the
// deposit's sort): one workgroup per tile stages the force grid of the tile and its
// one-cell halo in LDS (the position term's gathers) and adds the particle cotangents'
// window weights to a 10^3 box of three components in LDS; the box is then added to
// g_bar with one global atomic per touched cell and component (the tiles' boxes
// overlap on their halos). The box holds 64-bit fixed-point sums (integer LDS atomics
// run more than ten times faster than FP32 ones on gfx950): each contribution is
// rounded to 2^-37 of the tile's largest |gscale lambda| (2^38 units; the sum of a
// tile's particles stays far inside 2^63), an absolute error far below the FP32
// rounding of the sums. A particle whose window leaves the box (not possible for a
// bucket that matches its positions), and every particle of a tile with a non-finite
// cotangent, takes the per-weight global path.
constexpr int kVTThreads = 256;
constexpr int kVTT = 8, kVTH = kVTT + 2, kVTHalo = kVTH * kVTH * kVTH;

__device__ __forceinline__ long long fix_contrib(float c, float s) {
  return (long long)(c * s);
}

template <int MAS, int PK>
__global__ __launch_bounds__(kVTThreads) void k_interp_vjp_tile(
    const float *__restrict__ pos, const int32_t *__restrict__ cell,
    const int32_t *__restrict__ end, const int32_t *__restrict__ perm, int n,
    const float *__restrict__ g, const float *__restrict__ lam, float pscale, float gscale,
    float *__restrict__ g_bar, float *__restrict__ pos_bar) {
  __shared__ float4 gs[kVTHalo];
  __shared__ unsigned long long acc[3][kVTHalo];
  __shared__ float wmax[kVTThreads / 64];
  const int nt = n / kVTT;
  const int tile = (int)xcd_block(blockIdx.x, gridDim.x);
  const int p_begin = tile > 0 ? end[tile - 1] : 0, p_end = end[tile];
  if (p_begin >= p_end) return;
  const int t0[3] = {(tile / (nt * nt)) * kVTT, ((tile / nt) % nt) * kVTT, (tile % nt) * kVTT};
  auto box_cell = [&](int h) -> size_t {
    const int hx = h / (kVTH * kVTH), hy = (h / kVTH) % kVTH, hz = h % kVTH;
    return ((size_t)wrap_index(t0[0] + hx - 1, n) * n + wrap_index(t0[1] + hy - 1, n)) * n +
           wrap_index(t0[2] + hz - 1, n);
  };
  // the tile's largest cotangent component (fixed-point unit of the box)
  float mx = 0.0f;
  if (g_bar)
    for (int l = p_begin + (int)threadIdx.x; l < p_end; l += kVTThreads) {
      const size_t q = 3 * (size_t)perm[l];
      mx = fmaxf(mx, fmaxf(fabsf(lam[q]), fmaxf(fabsf(lam[q + 1]), fabsf(lam[q + 2]))));
    }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
  for (int h = threadIdx.x; h < kVTHalo; h += kVTThreads) {
    if (pos_bar) {
      const size_t gc = box_cell(h);
      gs[h] = make_float4(g[3 * gc], g[3 * gc + 1], g[3 * gc + 2], 0.0f);
    }
    acc[0][h] = acc[1][h] = acc[2][h] = 0ull;
  }
  __syncthreads();
  mx = wmax[0];
#pragma unroll
  for (int w = 1; w < kVTThreads / 64; ++w) mx = fmaxf(mx, wmax[w]);
  mx *= fabsf(gscale);
  const bool fixed_ok = mx < 3.0e38f;             // finite (NaN compares false)
  // units per cotangent (a tiny largest value keeps the scale within FP32's range)
  const float fs = mx > 0.0f ? ldexpf(1.0f, min(37 - ilogbf(mx), 126)) : 1.0f;
  for (int l = p_begin + (int)threadIdx.x; l < p_end; l += kVTThreads) {
    const int p = perm[l];
    int first[3];
    float w[3][MAS], dw[3][MAS];
    support_wdw<MAS, PK>(pos, cell, p, n, first, w, dw);
    int b[3];
    bool inbox = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int lf = first[d] - t0[d];
      lf += lf < -n / 2 ? n : 0;
      lf -= lf > n / 2 ? n : 0;
      b[d] = lf + 1;
      inbox = inbox && b[d] >= 0 && b[d] <= kVTH - MAS;
    }
    const float l0 = lam[3 * (size_t)p], l1 = lam[3 * (size_t)p + 1], l2 = lam[3 * (size_t)p + 2];
    float gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
    for (int a = 0; a < MAS; ++a)
#pragma unroll
      for (int bb = 0; bb < MAS; ++bb) {
        const float wab = w[0][a] * w[1][bb];
#pragma unroll
        for (int c = 0; c < MAS; ++c) {
          const int h = ((b[0] + a) * kVTH + (b[1] + bb)) * kVTH + (b[2] + c);
          size_t gc = 0;
          if (!inbox)
            gc = ((size_t)wrap_index(first[0] + a, n) * n + wrap_index(first[1] + bb, n)) * n +
                 wrap_index(first[2] + c, n);
          if (pos_bar) {
            float4 gv;
            if (inbox) gv = gs[h];
            else gv = make_float4(g[3 * gc], g[3 * gc + 1], g[3 * gc + 2], 0.0f);
            const float gl = gv.x * l0 + gv.y * l1 + gv.z * l2;
            gx = fmaf(dw[0][a] * w[1][bb] * w[2][c], gl, gx);
            gy = fmaf(w[0][a] * dw[1][bb] * w[2][c], gl, gy);
            gz = fmaf(w[0][a] * w[1][bb] * dw[2][c], gl, gz);
          }
          if (g_bar) {
            const float wt = gscale * wab * w[2][c];
            if (inbox && fixed_ok) {
              atomicAdd(&acc[0][h], (unsigned long long)fix_contrib(wt * l0, fs));
              atomicAdd(&acc[1][h], (unsigned long long)fix_contrib(wt * l1, fs));
              atomicAdd(&acc[2][h], (unsigned long long)fix_contrib(wt * l2, fs));
            } else {
              if (inbox)
                gc = ((size_t)wrap_index(first[0] + a, n) * n + wrap_index(first[1] + bb, n)) *
                         n + wrap_index(first[2] + c, n);
              unsafeAtomicAdd(&g_bar[3 * gc + 0], wt * l0);
              unsafeAtomicAdd(&g_bar[3 * gc + 1], wt * l1);
              unsafeAtomicAdd(&g_bar[3 * gc + 2], wt * l2);
            }
          }
        }
      }
    if (pos_bar) {
      pos_bar[3 * (size_t)p + 0] += pscale * gx;
      pos_bar[3 * (size_t)p + 1] += pscale * gy;
      pos_bar[3 * (size_t)p + 2] += pscale * gz;
    }
  }
  if (!g_bar || !fixed_ok) return;
  __syncthreads();
  const float inv = 1.0f / fs;
  for (int h = threadIdx.x; h < kVTHalo; h += kVTThreads) {
    const long long v0 = (long long)acc[0][h], v1 = (long long)acc[1][h],
                    v2 = (long long)acc[2][h];
    if (v0 == 0 && v1 == 0 && v2 == 0) continue;
    const size_t gc = box_cell(h);
    unsafeAtomicAdd(&g_bar[3 * gc + 0], (float)((double)v0 * inv));
    unsafeAtomicAdd(&g_bar[3 * gc + 1], (float)((double)v1 * inv));
    unsafeAtomicAdd(&g_bar[3 * gc + 2], (float)((double)v2 * inv));
  }
}

// Transpose of g = -D phi with D the central difference of the gradient table:
// phi_bar += sum_d D_d g_bar_d  (D_d^T = -D_d for the antisymmetric stencil).
template <int P>
__global__ __launch_bounds__(kThreads) void k_divergence(const float *__restrict__ gb, int n,
                                                         float inv_h, int accumulate,
                                                         float *__restrict__ phib) {
  const unsigned lin = xcd_block(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                                 gridDim.x * gridDim.y * gridDim.z);
  const int k = (lin % gridDim.x) * kThreads + threadIdx.x;
  const int j = (lin / gridDim.x) % gridDim.y;
  const int i = lin / (gridDim.x * gridDim.y);
  if (k >= n) return;
  constexpr int R = P / 2;
  const float c3[3] = {P == 3 ? 0.5f : (P == 5 ? 2.0f / 3.0f : 0.75f),
                       P == 3 ? 0.0f : (P == 5 ? -1.0f / 12.0f : -3.0f / 20.0f),
                       P == 7 ? 1.0f / 60.0f : 0.0f};
  const size_t nn = (size_t)n * n;
  const size_t row = ((size_t)i * n + j) * n;
  float s = 0.f;
#pragma unroll
  for (int m = 1; m <= R; ++m) {
    const float cm = c3[m - 1];
    const size_t ip = 3 * ((size_t)wrap_index(i + m, n) * nn + (size_t)j * n + k);
    const size_t im = 3 * ((size_t)wrap_index(i - m, n) * nn + (size_t)j * n + k);
    const size_t jp = 3 * ((size_t)i * nn + (size_t)wrap_index(j + m, n) * n + k);
    const size_t jm = 3 * ((size_t)i * nn + (size_t)wrap_index(j - m, n) * n + k);
    const size_t kp = 3 * (row + wrap_index(k + m, n));
    const size_t km = 3 * (row + wrap_index(k - m, n));
    s = fmaf(cm, gb[ip] - gb[im], s);
    s = fmaf(cm, gb[jp + 1] - gb[jm + 1], s);
    s = fmaf(cm, gb[kp + 2] - gb[km + 2], s);
  }
  phib[row + k] = accumulate ? fmaf(inv_h, s, phib[row + k]) : inv_h * s;
}

__global__ __launch_bounds__(kThreads) void k_fill(float *__restrict__ y, float value,
                                                   int64_t count) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t < count) y[t] = value;
}

// y += alpha x over count floats
__global__ __launch_bounds__(kThreads) void k_axpy(float *__restrict__ y,
                                                   const float *__restrict__ x, float alpha,
                                                   int64_t count) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t < count) y[t] = fmaf(alpha, x[t], y[t]);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

__device__ __forceinline__ double block_sum(double v) {
  __shared__ double part[RED_THREADS / 64];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) part[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < RED_THREADS / 64; ++i) t += part[i];
  return t;
}

// L = sum_c w_c (rho_c - 1)^2 as fixed-order FP64 block partials; rho is replaced by the
// cotangent of the loss, rho_bar = 2 w (rho - 1).
__global__ __launch_bounds__(RED_THREADS) void k_loss_partial(float *__restrict__ rho,
                                                              const float *__restrict__ w,
                                                              int64_t count,
                                                              double *__restrict__ partial) {
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * RED_THREADS;
  for (int64_t i = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; i < count; i += stride) {
    const float delta = rho[i] - 1.0f;
    const float wi = w[i];
    acc += (double)wi * (double)delta * (double)delta;
    rho[i] = 2.0f * wi * delta;
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ __launch_bounds__(RED_THREADS) void k_loss_final(const double *__restrict__ partial,
                                                            int nblocks,
                                                            double *__restrict__ result) {
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += RED_THREADS) acc += partial[b];
  const double t = block_sum(acc);
  if (threadIdx.x == 0) result[0] = t;
}

// Zel'dovich state from a displacement field: x = wrap(q + psi), v = a0^{1/2} psi, one
// thread per particle. With cell != NULL the position is returned in cell-offset form:
// the lattice point q sits at a cell centre (c + 1/2) / n, so u = c + 1/2 + n psi, and
// the in-cell offset keeps the displacement at cell-unit resolution.
template <int PK>
__global__ __launch_bounds__(kThreads) void k_ic_state(const float *__restrict__ q,
                                                       const float *__restrict__ psi,
                                                       int64_t np, int n, float vfac,
                                                       float *__restrict__ pos,
                                                       int32_t *__restrict__ cell,
                                                       float *__restrict__ vel) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= np) return;
  int c[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float dp = psi[3 * p + d];
    vel[3 * p + d] = vfac * dp;
    if constexpr (PK == PM_POS_BOX) {
      float x = q[3 * p + d] + dp;
      x -= floorf(x);
      pos[3 * p + d] = x >= 1.0f ? 0.0f : x;
    } else {
      const float fn = (float)n;
      const int base = (int)floorf(q[3 * p + d] * fn);
      const float s = fmaf(dp, fn, 0.5f);
      float fl = floorf(s);
      float o = s - fl;
      if (o >= 1.0f) {
        o = 0.0f;
        fl += 1.0f;
      }
      c[d] = wrap_any(base + (int)fl, n);
      pos[3 * p + d] = o;
    }
  }
  if constexpr (PK == PM_POS_CELLOFF) cell[p] = (c[0] * n + c[1]) * n + c[2];
}

// Its transpose: psi_bar = x_bar + a0^{1/2} v_bar (the wrap has unit derivative).
__global__ __launch_bounds__(kThreads) void k_ic_vjp(const float *__restrict__ xbar,
                                                     const float *__restrict__ vbar,
                                                     int64_t count, float vfac,
                                                     float *__restrict__ psibar) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t < count) psibar[t] = fmaf(vfac, vbar[t], xbar[t]);
}

inline unsigned blocks_for(int64_t count, int threads) {
  return (unsigned)((count + threads - 1) / threads);
}

}  // namespace

hipError_t launch_deposit_vjp(const float *pos, const int32_t *cell, int64_t np, int poskind,
                              int mas, int n, const float *rho_bar, float scale, float *pos_bar,
                              hipStream_t s) {
  if (np == 0) return hipSuccess;
  const unsigned nb = blocks_for(np, kThreads);
  if (mas == PM_TSC) {
    if (poskind == PM_POS_BOX)
      k_deposit_vjp<3, PM_POS_BOX><<<nb, kThreads, 0, s>>>(pos, cell, np, n, rho_bar, scale, pos_bar);
    else
      k_deposit_vjp<3, PM_POS_CELLOFF><<<nb, kThreads, 0, s>>>(pos, cell, np, n, rho_bar, scale,
                                                               pos_bar);
  } else {
    if (poskind == PM_POS_BOX)
      k_deposit_vjp<2, PM_POS_BOX><<<nb, kThreads, 0, s>>>(pos, cell, np, n, rho_bar, scale, pos_bar);
    else
      k_deposit_vjp<2, PM_POS_CELLOFF><<<nb, kThreads, 0, s>>>(pos, cell, np, n, rho_bar, scale,
                                                               pos_bar);
  }
  return hipGetLastError();
}

hipError_t launch_interp_vjp(const float *pos, const int32_t *cell, int64_t np, int poskind,
                             int mas, int n, const float *g, const float *lam, float pscale,
                             float gscale, float *g_bar, float *pos_bar, hipStream_t s) {
  if (np == 0) return hipSuccess;
  const unsigned nb = blocks_for(np, kVChunk);
#define PM_IV(M, K)                                                                              \
  k_interp_vjp_chunk<M, K><<<nb, kVThreads, 0, s>>>(pos, cell, np, n, g, lam, pscale, gscale,     \
                                                     g_bar, pos_bar)
  if (mas == PM_TSC) {
    if (poskind == PM_POS_BOX) PM_IV(3, PM_POS_BOX);
    else PM_IV(3, PM_POS_CELLOFF);
  } else {
    if (poskind == PM_POS_BOX) PM_IV(2, PM_POS_BOX);
    else PM_IV(2, PM_POS_CELLOFF);
  }
#undef PM_IV
  return hipGetLastError();
}

hipError_t launch_interp_vjp_tile(const float *pos, const int32_t *cell, int64_t np, int poskind,
                                  int mas, int n, const int32_t *end, const int32_t *perm,
                                  const float *g, const float *lam, float pscale, float gscale,
                                  float *g_bar, float *pos_bar, hipStream_t s) {
  if (np == 0) return hipSuccess;
  const unsigned nt = (unsigned)((int64_t)(n / kVTT) * (n / kVTT) * (n / kVTT));
#define PM_IVT(M, K)                                                                         \
  k_interp_vjp_tile<M, K><<<nt, kVTThreads, 0, s>>>(pos, cell, end, perm, n, g, lam, pscale, \
                                                    gscale, g_bar, pos_bar)
  if (mas == PM_TSC) {
    if (poskind == PM_POS_BOX) PM_IVT(3, PM_POS_BOX);
    else PM_IVT(3, PM_POS_CELLOFF);
  } else {
    if (poskind == PM_POS_BOX) PM_IVT(2, PM_POS_BOX);
    else PM_IVT(2, PM_POS_CELLOFF);
  }
#undef PM_IVT
  return hipGetLastError();
}

hipError_t launch_divergence(const float *gb, int n, int points, bool accumulate, float *phib,
                             hipStream_t s) {
  dim3 grid((n + kThreads - 1) / kThreads, n, n);
  const float inv_h = (float)n;
  const int acc = accumulate ? 1 : 0;
  switch (points) {
    case 3: k_divergence<3><<<grid, kThreads, 0, s>>>(gb, n, inv_h, acc, phib); break;
    case 5: k_divergence<5><<<grid, kThreads, 0, s>>>(gb, n, inv_h, acc, phib); break;
    default: k_divergence<7><<<grid, kThreads, 0, s>>>(gb, n, inv_h, acc, phib); break;
  }
  return hipGetLastError();
}

hipError_t launch_fill(float *y, float value, int64_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  k_fill<<<blocks_for(count, kThreads), kThreads, 0, s>>>(y, value, count);
  return hipGetLastError();
}

hipError_t launch_axpy(float *y, const float *x, float alpha, int64_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  k_axpy<<<blocks_for(count, kThreads), kThreads, 0, s>>>(y, x, alpha, count);
  return hipGetLastError();
}

hipError_t launch_density_loss(float *rho, const float *w, int64_t count, double *partial,
                               double *result, hipStream_t s) {
  int nb = (int)std::min<int64_t>(RED_BLOCKS, (count + RED_THREADS - 1) / RED_THREADS);
  if (nb < 1) nb = 1;
  k_loss_partial<<<nb, RED_THREADS, 0, s>>>(rho, w, count, partial);
  k_loss_final<<<1, RED_THREADS, 0, s>>>(partial, nb, result);
  return hipGetLastError();
}

hipError_t launch_ic_state(const float *q, const float *psi, int64_t np, int n, float vfac,
                           float *pos, int32_t *cell, float *vel, hipStream_t s) {
  if (np == 0) return hipSuccess;
  if (cell)
    k_ic_state<PM_POS_CELLOFF><<<blocks_for(np, kThreads), kThreads, 0, s>>>(q, psi, np, n, vfac,
                                                                            pos, cell, vel);
  else
    k_ic_state<PM_POS_BOX><<<blocks_for(np, kThreads), kThreads, 0, s>>>(q, psi, np, n, vfac, pos,
                                                                        nullptr, vel);
  return hipGetLastError();
}

hipError_t launch_ic_vjp(const float *xbar, const float *vbar, int64_t np, float vfac,
                         float *psibar, hipStream_t s) {
  if (np == 0) return hipSuccess;
  k_ic_vjp<<<blocks_for(3 * np, kThreads), kThreads, 0, s>>>(xbar, vbar, 3 * np, vfac, psibar);
  return hipGetLastError();
}
