// Chunked gather deposit (paper Sect. 3.5 windows) shared by the single-box
// atomic mode and the batched ensembles, and the particle helpers it needs.
//
// A workgroup deposits a chunk of up to 2048 particles without per-weight
// global atomics:
//   1. the particles' cells are taken relative to the chunk's first particle
//      (minimum image) and their bounding box is found, grown by one cell per
//      side (the window's reach);
//   2. every particle adds its 27 (8) window weights, as 2^-30 fixed-point
//      integers, to 64-bit accumulators of that box in LDS (integer LDS atomics
//      run at several T ops/s on gfx950, float ones far slower; integer sums are
//      also exact, whatever the order);
//   3. each touched cell of the box is added to the grid with one FP32 global
//      atomic (so the last bits may differ between runs), or, for a 64-bit
//      fixed-point grid, one integer global atomic (exact: the same in every run).
// Chunks whose box exceeds the LDS table fall back to one global atomic per
// weight. Which particles form a chunk is the caller's choice (an Index object
// maps the chunk's slots to particle rows, -1 for an empty slot): runs of
// consecutive rows after a tile-major reorder, or lattice blocks of particles
// that started on a lattice.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hippm.h"

namespace pm_chunk {

// Periodic wrap for indices already within [-n, 2n).
__device__ __forceinline__ int wrap_index(int i, int n) {
  i += (i < 0) ? n : 0;
  i -= (i >= n) ? n : 0;
  return i;
}

// Periodic wrap for any integer (guards every caller-supplied index).
__device__ __forceinline__ int wrap_any(int i, int n) {
  const int r = i % n;
  return r < 0 ? r + n : r;
}

// Grid sides are powers of two in every usual case; then periodic wraps and the
// decoding of row-major cell indices c = (i n + j) n + k are masks and shifts. The test
// is on a kernel argument (wave-uniform), so the divisions of the general case run
// only for other sides.
__device__ __forceinline__ int log2_if_pow2(int n) {
  return (n & (n - 1)) == 0 ? __builtin_ctz((unsigned)n) : -1;
}

__device__ __forceinline__ int wrap_fast(int i, int n, int lg) {
  return lg >= 0 ? (i & (n - 1)) : wrap_any(i, n);
}

// (i, j, k) of any integer cell index (wrapped into [0, n^3))
__device__ __forceinline__ void decode_cell(int q, int n, int lg, int c[3]) {
  if (lg >= 0) {
    const int m = n - 1;
    c[2] = q & m;
    c[1] = (q >> lg) & m;
    c[0] = (q >> (2 * lg)) & m;
  } else {
    q = wrap_any(q, n * n * n);
    c[0] = q / (n * n);
    c[1] = (q / n) - c[0] * n;
    c[2] = q - (q / n) * n;
  }
}

// Per-axis support of the window: first cell index (unwrapped) and MAS weights.
// TSC (MAS = 3): cells floor(u)-1 .. floor(u)+1, d = u - floor(u) - 1/2 in [-1/2, 1/2):
//   W = (1/2)(1/2 - d)^2, 3/4 - d^2, (1/2)(1/2 + d)^2.
// CIC (MAS = 2): cells floor(u - 1/2) and the next, d = u - 1/2 - floor(u - 1/2):
//   W = 1 - d, d.
// NGP (MAS = 1): the cell floor(u), W = 1.
template <int MAS>
__device__ __forceinline__ void weights_from_frac(float d, float *w) {
  if constexpr (MAS == 3) {
    const float a = 0.5f - d, b = 0.5f + d;
    w[0] = 0.5f * a * a;
    w[1] = 0.75f - d * d;
    w[2] = 0.5f * b * b;
  } else if constexpr (MAS == 2) {
    w[0] = 1.0f - d;
    w[1] = d;
  } else {
    (void)d;
    w[0] = 1.0f;
  }
}

// Box-unit coordinate x in [0,1) -> first cell and weights.
template <int MAS>
__device__ __forceinline__ int axis_box(float x, float fn, float *w) {
  const float u = x * fn;
  if constexpr (MAS == 3) {
    const float fl = floorf(u);
    weights_from_frac<3>(u - fl - 0.5f, w);
    return (int)fl - 1;
  } else if constexpr (MAS == 2) {
    const float t = u - 0.5f;
    const float fl = floorf(t);
    weights_from_frac<2>(t - fl, w);
    return (int)fl;
  } else {
    weights_from_frac<1>(0.0f, w);
    return (int)floorf(u);
  }
}

// Cell index c and in-cell offset o in [0,1) -> first cell and weights.
template <int MAS>
__device__ __forceinline__ int axis_off(int c, float o, float *w) {
  if constexpr (MAS == 3) {
    weights_from_frac<3>(o - 0.5f, w);
    return c - 1;
  } else if constexpr (MAS == 1) {
    weights_from_frac<1>(o, w);
    return c;
  } else {
    if (o >= 0.5f) {
      weights_from_frac<2>(o - 0.5f, w);
      return c;
    }
    weights_from_frac<2>(o + 0.5f, w);
    return c - 1;
  }
}

template <int MAS, int PK>
__device__ __forceinline__ void particle_support(const float *__restrict__ pos,
                                                 const int32_t *__restrict__ cell, int64_t p,
                                                 int n, int first[3], float w[3][MAS]) {
  const float x0 = pos[3 * p + 0], x1 = pos[3 * p + 1], x2 = pos[3 * p + 2];
  const int lg = log2_if_pow2(n);
  if constexpr (PK == PM_POS_BOX) {
    const float fn = (float)n;
    first[0] = wrap_fast(axis_box<MAS>(x0, fn, w[0]), n, lg);
    first[1] = wrap_fast(axis_box<MAS>(x1, fn, w[1]), n, lg);
    first[2] = wrap_fast(axis_box<MAS>(x2, fn, w[2]), n, lg);
  } else {
    int c[3];
    decode_cell(cell[p], n, lg, c);
    first[0] = axis_off<MAS>(c[0], x0, w[0]);
    first[1] = axis_off<MAS>(c[1], x1, w[1]);
    first[2] = axis_off<MAS>(c[2], x2, w[2]);
  }
}


constexpr int kGThreads = 256;
constexpr int kGPPT = 8;
constexpr int kGChunk = kGThreads * kGPPT;
constexpr int kGTable = 5120;  // cells of the grown particle box held in LDS (8 B each)

__device__ __forceinline__ int min_image(int d, int n) { return wrap_any(d + n / 2, n) - n / 2; }

__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// Window of the separation s = u - (c + 1/2); NGP takes [-1/2, 1/2) (the cell floor(u)).
template <int MAS>
__device__ __forceinline__ float window_sep_g(float s) {
  const float a = fabsf(s);
  if constexpr (MAS == 3) {
    if (a < 0.5f) return 0.75f - a * a;
    const float b = 1.5f - a;
    return a < 1.5f ? 0.5f * b * b : 0.0f;
  } else if constexpr (MAS == 2) {
    return a < 1.0f ? 1.0f - a : 0.0f;
  } else {
    return (s >= -0.5f && s < 0.5f) ? 1.0f : 0.0f;
  }
}

// Cell (wrapped) and in-cell offset of particle p.
template <int PK>
__device__ __forceinline__ void particle_cell(const float *__restrict__ pos,
                                              const int32_t *__restrict__ cell, int64_t p, int n,
                                              int c[3], float o[3]) {
  const int lg = log2_if_pow2(n);
  if constexpr (PK == PM_POS_BOX) {
    const float fn = (float)n;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float u = pos[3 * p + d] * fn;
      const float fl = floorf(u);
      c[d] = wrap_fast((int)fl, n, lg);
      o[d] = u - fl;
    }
  } else {
    decode_cell(cell[p], n, lg, c);
#pragma unroll
    for (int d = 0; d < 3; ++d) o[d] = pos[3 * p + d];
  }
}

// Slots of a chunk of consecutive rows [base, end).
struct RangeIndex {
  int64_t base, end;
  __device__ int64_t ref() const { return base; }
  __device__ int64_t operator()(int slot) const {
    const int64_t p = base + slot;
    return p < end ? p : -1;
  }
};

// Slots of an 8 x 16 x 16 block of a lattice whose rows are ordered (i, j, k),
// starting at lattice point (i0, j0, k0) of an m^3 lattice at row p0.
struct LatticeIndex {
  int64_t p0;
  int m, i0, j0, k0;
  __device__ int64_t row(int i, int j, int k) const {
    return p0 + ((int64_t)i * m + j) * m + k;
  }
  __device__ int64_t ref() const { return row(i0, j0, k0); }
  __device__ int64_t operator()(int slot) const {
    const int i = i0 + (slot >> 8), j = j0 + ((slot >> 4) & 15), k = k0 + (slot & 15);
    return (i < m && j < m && k < m) ? row(i, j, k) : -1;
  }
};

// FIXED: the sums go to a 64-bit fixed-point grid (2^-30 per unit weight, no mass) with
// integer global atomics instead of FP32 ones, so the grid is exact and the same for
// every order of the particles and chunks (rho and mass are then unused); each
// (particle, cell) weight becomes the same integer on the LDS path and the fallback.
template <int MAS, int PK, class Index, bool FIXED = false>
__device__ void deposit_chunk(const float *__restrict__ pos, const int32_t *__restrict__ cell,
                              const Index idx, int n, float mass, float *__restrict__ rho,
                              unsigned long long *__restrict__ fixg = nullptr) {
  __shared__ unsigned long long acc[kGTable];  // 2^-30 fixed-point sums of the grown box
  __shared__ int red[6][kGThreads / 64];
  int ref[3];
  {
    float o[3];
    particle_cell<PK>(pos, cell, idx.ref(), n, ref, o);
  }
  // 1. cells relative to the reference particle, and their bounding box
  int lc[kGPPT][3];
  float lo_f[kGPPT][3];
  bool ok[kGPPT];
  int lo[3] = {n, n, n}, hi[3] = {-n, -n, -n};
#pragma unroll
  for (int m = 0; m < kGPPT; ++m) {
    const int64_t p = idx(threadIdx.x + m * kGThreads);
    ok[m] = p >= 0;
    int c[3] = {0, 0, 0};
    float o[3] = {0.f, 0.f, 0.f};
    if (ok[m]) particle_cell<PK>(pos, cell, p, n, c, o);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int d = min_image(c[a] - ref[a], n);
      lc[m][a] = d;
      lo_f[m][a] = o[a];
      if (ok[m]) {
        lo[a] = min(lo[a], d);
        hi[a] = max(hi[a], d);
      }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int l = wave_min_i(lo[a]), h = wave_max_i(hi[a]);
    if (lane == 0) {
      red[a][wave] = l;
      red[3 + a][wave] = h;
    }
  }
  __syncthreads();
  int g[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    int l = red[a][0], h = red[3 + a][0];
    for (int w = 1; w < kGThreads / 64; ++w) {
      l = min(l, red[a][w]);
      h = max(h, red[3 + a][w]);
    }
    lo[a] = l;
    g[a] = h - l + 3;  // grown by the window's reach of one cell per side
  }
  const int gvol = g[0] * g[1] * g[2];
  if (gvol > kGTable) {
    // fallback: global atomics per weight
#pragma unroll 1
    for (int m = 0; m < kGPPT; ++m) {
      const int64_t p = idx(threadIdx.x + m * kGThreads);
      if (p < 0) continue;
      int f[3];
      float w[3][MAS];
      particle_support<MAS, PK>(pos, cell, p, n, f, w);
      for (int a = 0; a < MAS; ++a) {
        const size_t ia = (size_t)wrap_index(f[0] + a, n) * n;
        for (int b = 0; b < MAS; ++b) {
          const size_t row = (ia + wrap_index(f[1] + b, n)) * n;
          if constexpr (FIXED) {
            const float wab = w[0][a] * w[1][b] * 1073741824.0f;  // 2^30, as below
            for (int c = 0; c < MAS; ++c)
              atomicAdd(&fixg[row + wrap_index(f[2] + c, n)],
                        (unsigned long long)(unsigned)rintf(wab * w[2][c]));
          } else {
            const float wab = mass * w[0][a] * w[1][b];
            for (int c = 0; c < MAS; ++c)
              unsafeAtomicAdd(&rho[row + wrap_index(f[2] + c, n)], wab * w[2][c]);
          }
        }
      }
    }
    return;
  }
  // 2. scatter the window weights into the LDS box (integer atomics: exact sums)
  for (int i = threadIdx.x; i < gvol; i += kGThreads) acc[i] = 0ull;
  __syncthreads();
  const float kFix = 1073741824.0f;  // 2^30
#pragma unroll 2
  for (int m = 0; m < kGPPT; ++m) {
    if (!ok[m]) continue;
    int f[3];
    float w[3][MAS];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      // local index of the particle's cell is lc - lo + 1; the window's first cell
      // is one below it (TSC), or at or one below it (CIC)
      f[a] = axis_off<MAS>(lc[m][a] - lo[a] + 1, lo_f[m][a], w[a]);
    }
#pragma unroll
    for (int a = 0; a < MAS; ++a) {
#pragma unroll
      for (int b = 0; b < MAS; ++b) {
        const int row = ((f[0] + a) * g[1] + (f[1] + b)) * g[2] + f[2];
        const float wab = w[0][a] * w[1][b] * kFix;
#pragma unroll
        for (int c = 0; c < MAS; ++c)
          atomicAdd(&acc[row + c], (unsigned long long)(unsigned)rintf(wab * w[2][c]));
      }
    }
  }
  __syncthreads();
  // 3. one global atomic per touched cell
  const float scale = mass * (1.0f / kFix);
  const int g12 = g[1] * g[2];
  for (int t = threadIdx.x; t < gvol; t += kGThreads) {
    const unsigned long long v = acc[t];
    if (v == 0ull) continue;
    const int x = t / g12, r = t - x * g12;
    const int y = r / g[2], z = r - y * g[2];
    const int gi = wrap_any(ref[0] + lo[0] - 1 + x, n);
    const int gj = wrap_any(ref[1] + lo[1] - 1 + y, n);
    const int gk = wrap_any(ref[2] + lo[2] - 1 + z, n);
    if constexpr (FIXED)
      atomicAdd(&fixg[((size_t)gi * n + gj) * n + gk], v);
    else
      unsafeAtomicAdd(&rho[((size_t)gi * n + gj) * n + gk], (float)v * scale);
  }
}

}  // namespace pm_chunk
