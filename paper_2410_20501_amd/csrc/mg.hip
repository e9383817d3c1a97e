// Linear multigrid for the periodic seven-point Poisson problem
// (paper Sects. 3.6-3.7.1): red-black Gauss-Seidel smoothing, residual
// restriction to a grid of spacing 2h (full weighting = transpose of the
// prolongation / 8, or the paper's 8-child average), recursive coarse
// correction starting from the Jacobi guess -H^2 d_H / 6, trilinear
// prolongation-correction with the 27/64, 9/64, 3/64, 1/64 weights, and an
// LDS-resident coarsest-level solve.
//
// Every kernel reads the right-hand side as  scale * (f[c] - mean), so the
// finest level uses the density grid directly (scale = (3/2) a Omega_m,
// mean = the density's mean computed on the device) without materialising the
// source term.
#include <algorithm>
#include <cmath>

#include "coarse_solve.h"

// streaming levels at least this large add the prolonged correction inside the first
// post-smoothing pass (measured: 519 us against 434 + 209 us at 512^3; at 256^3 the
// separate prolongation pass is as fast)
#ifndef PM_FUSE_PROLONG_MIN_N
#define PM_FUSE_PROLONG_MIN_N 512
#endif
#include "internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kCoarseThreads = 1024;
constexpr int kCoarseMax = 8000;  // cells held in LDS by the coarsest-level solve (20^3)

__device__ __forceinline__ int wrap_index(int i, int n) {
  i += (i < 0) ? n : 0;
  i -= (i >= n) ? n : 0;
  return i;
}

__device__ __forceinline__ float src_mean(const float *mean) { return mean ? *mean : 0.0f; }

__device__ __forceinline__ float neighbour_sum(const float *__restrict__ u, int i, int j, int k,
                                               int n) {
  const size_t nn = (size_t)n * n;
  const size_t ci = (size_t)i * nn, cj = (size_t)j * n;
  return u[(size_t)wrap_index(i + 1, n) * nn + cj + k] + u[(size_t)wrap_index(i - 1, n) * nn + cj + k] +
         u[ci + (size_t)wrap_index(j + 1, n) * n + k] + u[ci + (size_t)wrap_index(j - 1, n) * n + k] +
         u[ci + cj + wrap_index(k + 1, n)] + u[ci + cj + wrap_index(k - 1, n)];
}

// u = -h^2 f / 6: one Jacobi step from a zero field (paper's first guess).
__global__ __launch_bounds__(kThreads) void k_jacobi_guess(float *__restrict__ u,
                                                           const float *__restrict__ f,
                                                           float scale,
                                                           const float *__restrict__ mean,
                                                           int64_t count, float h2) {
  const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c >= count) return;
  const float m = src_mean(mean);
  u[c] = (-h2 / 6.0f) * (scale * (f[c] - m));
}

// One colour of a red-black Gauss-Seidel sweep: cells with (i + j + k) % 2 == colour.
__global__ __launch_bounds__(kThreads) void k_rbgs_half(float *__restrict__ u,
                                                        const float *__restrict__ f, float scale,
                                                        const float *__restrict__ mean, int n,
                                                        float h2, float omega, int colour) {
  // per-level index math in 32 bits: n^3 <= 2^30
  const unsigned half = (unsigned)n >> 1;
  const unsigned t = blockIdx.x * kThreads + threadIdx.x;
  if (t >= (unsigned)n * n * half) return;
  const unsigned r = t / half;
  const int k2 = (int)(t - r * half);
  const int i = (int)(r / (unsigned)n), j = (int)(r - (unsigned)i * n);
  const int k = 2 * k2 + ((i + j + colour) & 1);
  const size_t c = ((size_t)i * n + j) * n + k;
  const float fv = scale * (f[c] - src_mean(mean));
  const float gs = (neighbour_sum(u, i, j, k, n) - h2 * fv) * (1.0f / 6.0f);
  u[c] = (omega == 1.0f) ? gs : fmaf(omega, gs - u[c], u[c]);
}

__device__ __forceinline__ float residual_at(const float *__restrict__ u,
                                             const float *__restrict__ f, float scale, float m,
                                             int i, int j, int k, int n, float inv_h2) {
  const size_t c = ((size_t)i * n + j) * n + k;
  const float uc = u[c];
  // sum of neighbour differences: exact for nearby values (halves the FP32 floor)
  const size_t nn = (size_t)n * n;
  const size_t ci = (size_t)i * nn, cj = (size_t)j * n;
  const float lap = (u[(size_t)wrap_index(i + 1, n) * nn + cj + k] - uc) +
                    (u[(size_t)wrap_index(i - 1, n) * nn + cj + k] - uc) +
                    (u[ci + (size_t)wrap_index(j + 1, n) * n + k] - uc) +
                    (u[ci + (size_t)wrap_index(j - 1, n) * n + k] - uc) +
                    (u[ci + cj + wrap_index(k + 1, n)] - uc) +
                    (u[ci + cj + wrap_index(k - 1, n)] - uc);
  return scale * (f[c] - m) - lap * inv_h2;
}

// Two-pass restriction for the small levels: r = f - L u once per fine cell, then the
// restriction of r (a coarse cell reads 64 or 8 fine values instead of evaluating 64
// residuals), with the coarse starting guess -H^2 f_H / 6 written alongside.
__global__ __launch_bounds__(kThreads) void k_residual(const float *__restrict__ u,
                                                       const float *__restrict__ f, float scale,
                                                       const float *__restrict__ mean, int n,
                                                       float inv_h2, float *__restrict__ r) {
  const unsigned un = (unsigned)n;
  const unsigned t = blockIdx.x * kThreads + threadIdx.x;
  if (t >= un * un * un) return;
  const unsigned q = t / un;
  const int k = (int)(t - q * un), i = (int)(q / un), j = (int)(q - (unsigned)i * un);
  r[t] = residual_at(u, f, scale, src_mean(mean), i, j, k, n, inv_h2);
}

// Coarse cell (I, J, K) <- restriction of the fine residual r.
// Full weighting: per axis fine cells 2J-1 .. 2J+2 with weights (1, 3, 3, 1) / 8.
// Average: the 8 children 2J, 2J+1 per axis, each with weight 1/8.
template <int KIND>
__global__ __launch_bounds__(kThreads) void k_restrict_r(const float *__restrict__ r, int n,
                                                         float *__restrict__ fc,
                                                         float *__restrict__ uc,
                                                         float gscale) {
  const unsigned nc = (unsigned)n >> 1;
  const unsigned t = blockIdx.x * kThreads + threadIdx.x;
  if (t >= nc * nc * nc) return;
  const unsigned q = t / nc;
  const int K = (int)(t - q * nc), I = (int)(q / nc), J = (int)(q - (unsigned)I * nc);
  const size_t nn = (size_t)n * n;
  float acc = 0.0f;
  if constexpr (KIND == PM_RESTRICT_FW) {
    const float w[4] = {1.0f, 3.0f, 3.0f, 1.0f};
    int kk[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) kk[c] = wrap_index(2 * K - 1 + c, n);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const size_t ri = (size_t)wrap_index(2 * I - 1 + a, n) * nn;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const size_t rj = ri + (size_t)wrap_index(2 * J - 1 + b, n) * n;
        const float row = fmaf(w[0], r[rj + kk[0]],
                               fmaf(w[1], r[rj + kk[1]], fmaf(w[2], r[rj + kk[2]], w[3] * r[rj + kk[3]])));
        acc = fmaf(w[a] * w[b], row, acc);
      }
    }
    acc *= (1.0f / 512.0f);
  } else {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c)
          acc += r[(size_t)(2 * I + a) * nn + (size_t)(2 * J + b) * n + (2 * K + c)];
    acc *= 0.125f;
  }
  fc[t] = acc;
  uc[t] = gscale * acc;
}

// u_fine += P v_coarse: per axis 3/4 from the nearest coarse centre and 1/4 from
// the next one (fine cell 2J has neighbours J, J-1; fine 2J+1 has J, J+1).
// One thread per coarse cell (I, J, K) reads the 27 coarse values around it once
// and updates its 8 fine children (2I+a, 2J+b, 2K+c), writing k-pairs as float2.
__global__ __launch_bounds__(kThreads) void k_prolong_add(float *__restrict__ u, int n,
                                                          const float *__restrict__ v) {
  const unsigned nc = (unsigned)n >> 1;
  const unsigned t = xcd_block(blockIdx.x, gridDim.x) * kThreads + threadIdx.x;
  if (t >= nc * nc * nc) return;
  const unsigned r = t / nc;
  const int K = (int)(t - r * nc), I = (int)(r / nc), J = (int)(r - (unsigned)I * nc);
  const int c = (int)nc;
  const int ix[3] = {wrap_index(I - 1, c), I, wrap_index(I + 1, c)};
  const int jx[3] = {wrap_index(J - 1, c), J, wrap_index(J + 1, c)};
  const int kx[3] = {wrap_index(K - 1, c), K, wrap_index(K + 1, c)};
  const float near = 0.75f, far = 0.25f;
  // along k: even child (2K) takes K-1 and K, odd child (2K+1) takes K and K+1
  float ek[3][3], ok[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const float *row = v + ((size_t)ix[a] * nc + jx[b]) * nc;
      const float vm = row[kx[0]], v0 = row[kx[1]], vp = row[kx[2]];
      ek[a][b] = near * v0 + far * vm;
      ok[a][b] = near * v0 + far * vp;
    }
  const size_t nn = (size_t)n * n;
#pragma unroll
  for (int ai = 0; ai < 2; ++ai) {       // fine plane 2I + ai
    const int an = 1, af = ai ? 2 : 0;   // nearest and far coarse planes
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {     // fine row 2J + bj
      const int bn = 1, bf = bj ? 2 : 0;
      const float se = near * (near * ek[an][bn] + far * ek[an][bf]) +
                       far * (near * ek[af][bn] + far * ek[af][bf]);
      const float so = near * (near * ok[an][bn] + far * ok[an][bf]) +
                       far * (near * ok[af][bn] + far * ok[af][bf]);
      float2 *dst = reinterpret_cast<float2 *>(u + (size_t)(2 * I + ai) * nn +
                                               (size_t)(2 * J + bj) * n + 2 * K);
      float2 cur = *dst;
      cur.x += se;
      cur.y += so;
      *dst = cur;
    }
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Partial sums of the squared residual and squared source.
__global__ __launch_bounds__(RED_THREADS) void k_residual_norm(const float *__restrict__ u,
                                                               const float *__restrict__ f,
                                                               float scale,
                                                               const float *__restrict__ mean,
                                                               int n, float inv_h2,
                                                               double *__restrict__ partial) {
  const int64_t count = (int64_t)n * n * n;
  const float m = src_mean(mean);
  double s1 = 0.0, s2 = 0.0;
  const int64_t stride = (int64_t)gridDim.x * RED_THREADS;
  for (int64_t t = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; t < count; t += stride) {
    const unsigned ut = (unsigned)t, un = (unsigned)n, q = ut / un;
    const int k = (int)(ut - q * un), i = (int)(q / un), j = (int)(q - (unsigned)i * un);
    const double r = residual_at(u, f, scale, m, i, j, k, n, inv_h2);
    const double fv = scale * (f[t] - m);
    s1 += r * r;
    s2 += fv * fv;
  }
  __shared__ double l1[RED_THREADS / 64], l2[RED_THREADS / 64];
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    l1[wave] = s1;
    l2[wave] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < RED_THREADS / 64; ++w) {
      a += l1[w];
      b += l2[w];
    }
    partial[2 * blockIdx.x] = a;
    partial[2 * blockIdx.x + 1] = b;
  }
}

__global__ __launch_bounds__(RED_THREADS) void k_pair_final(const double *__restrict__ partial,
                                                            int nblocks,
                                                            double *__restrict__ result) {
  double s1 = 0.0, s2 = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += RED_THREADS) {
    s1 += partial[2 * b];
    s2 += partial[2 * b + 1];
  }
  __shared__ double l1[RED_THREADS / 64], l2[RED_THREADS / 64];
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    l1[wave] = s1;
    l2[wave] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < RED_THREADS / 64; ++w) {
      a += l1[w];
      b += l2[w];
    }
    result[0] = a;
    result[1] = b;
  }
}

// u *= s (growth rescaling of a warm start).
__global__ __launch_bounds__(kThreads) void k_scale(float *__restrict__ u, int64_t count, float s) {
  const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c >= count) return;
  u[c] *= s;
}

// Subtract the device-resident mean from a grid.
__global__ __launch_bounds__(kThreads) void k_subtract_mean(float *__restrict__ u, int64_t count,
                                                            const float *__restrict__ mean) {
  const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c >= count) return;
  u[c] -= *mean;
}

// Totals of the three per-block sums of the norm-summing smoother pass.
__global__ __launch_bounds__(RED_THREADS) void k_triple_final(const double *__restrict__ partial,
                                                              int nblocks,
                                                              double *__restrict__ result,
                                                              int64_t count,
                                                              float *__restrict__ mean) {
  double v[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += RED_THREADS)
#pragma unroll
    for (int i = 0; i < 3; ++i) v[i] += partial[3 * b + i];
  __shared__ double l[3][RED_THREADS / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    v[i] = wave_sum(v[i]);
    if (lane == 0) l[i][wave] = v[i];
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double a = 0.0;
    for (int w = 0; w < RED_THREADS / 64; ++w) a += l[threadIdx.x][w];
    result[threadIdx.x] = a;
    if (threadIdx.x == 2) *mean = (float)(a / (double)count);  // mean of the input
  }
}

// Truncation-error estimate of the paper's alternative stopping rule (Sect. 3.7.1,
// Eq. multigrid_threshold): tau = L_H(R u) - R(L_h u) on the coarse grid (H = 2h), with
// R the restriction of the cycle. First pass, one thread per coarse cell: R(scale u)
// and R(L_h scale u) over the fine cells the restriction weighs (full weighting: 4^3
// cells with (1,3,3,1)/8 per axis; average: the 8 children).
template <int KIND>
__global__ __launch_bounds__(kThreads) void k_tau_restrict(const float *__restrict__ u, int n,
                                                           float inv_h2, float scale,
                                                           float *__restrict__ ru,
                                                           float *__restrict__ rlu) {
  const int nc = n >> 1;
  const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c >= (int64_t)nc * nc * nc) return;
  const int K = (int)(c % nc), J = (int)((c / nc) % nc), I = (int)(c / ((int64_t)nc * nc));
  constexpr int M = KIND == PM_RESTRICT_FW ? 4 : 2;
  const float w[4] = {1.f, 3.f, 3.f, 1.f};
  const size_t nn = (size_t)n * n;
  float su = 0.f, sl = 0.f;
  for (int a = 0; a < M; ++a)
    for (int b = 0; b < M; ++b)
      for (int e = 0; e < M; ++e) {
        const int off = KIND == PM_RESTRICT_FW ? -1 : 0;
        const int i = wrap_index(2 * I + off + a, n), j = wrap_index(2 * J + off + b, n),
                  k = wrap_index(2 * K + off + e, n);
        const float wt = KIND == PM_RESTRICT_FW ? w[a] * w[b] * w[e] : 1.0f;
        const float uc = u[i * nn + (size_t)j * n + k];
        const float lap = (u[wrap_index(i - 1, n) * nn + (size_t)j * n + k] - uc) +
                          (u[wrap_index(i + 1, n) * nn + (size_t)j * n + k] - uc) +
                          (u[i * nn + (size_t)wrap_index(j - 1, n) * n + k] - uc) +
                          (u[i * nn + (size_t)wrap_index(j + 1, n) * n + k] - uc) +
                          (u[i * nn + (size_t)j * n + wrap_index(k - 1, n)] - uc) +
                          (u[i * nn + (size_t)j * n + wrap_index(k + 1, n)] - uc);
        su = fmaf(wt, uc, su);
        sl = fmaf(wt, lap * inv_h2, sl);
      }
  const float norm = KIND == PM_RESTRICT_FW ? scale / 512.0f : scale / 8.0f;
  ru[c] = norm * su;
  rlu[c] = norm * sl;
}

// Second pass: tau = L_H(R u) - R(L_h u) per coarse cell, block sums of tau^2 (the
// second slot of each pair is zero).
__global__ __launch_bounds__(RED_THREADS) void k_tau_norm(const float *__restrict__ ru,
                                                          const float *__restrict__ rlu, int nc,
                                                          float inv_H2,
                                                          double *__restrict__ partial) {
  const int64_t count = (int64_t)nc * nc * nc;
  const size_t nn = (size_t)nc * nc;
  double s1 = 0.0;
  const int64_t stride = (int64_t)gridDim.x * RED_THREADS;
  for (int64_t t = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; t < count; t += stride) {
    const int k = (int)(t % nc), j = (int)((t / nc) % nc), i = (int)(t / (int64_t)nn);
    const float c = ru[t];
    const float lap = (ru[wrap_index(i - 1, nc) * nn + (size_t)j * nc + k] - c) +
                      (ru[wrap_index(i + 1, nc) * nn + (size_t)j * nc + k] - c) +
                      (ru[i * nn + (size_t)wrap_index(j - 1, nc) * nc + k] - c) +
                      (ru[i * nn + (size_t)wrap_index(j + 1, nc) * nc + k] - c) +
                      (ru[i * nn + (size_t)j * nc + wrap_index(k - 1, nc)] - c) +
                      (ru[i * nn + (size_t)j * nc + wrap_index(k + 1, nc)] - c);
    const double tau = (double)(lap * inv_H2) - (double)rlu[t];
    s1 += tau * tau;
  }
  __shared__ double l1[RED_THREADS / 64];
  s1 = wave_sum(s1);
  if ((threadIdx.x & 63) == 0) l1[threadIdx.x >> 6] = s1;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0;
    for (int q = 0; q < RED_THREADS / 64; ++q) a += l1[q];
    partial[2 * blockIdx.x] = a;
    partial[2 * blockIdx.x + 1] = 0.0;
  }
}

// phi = scale * u - mean, with the device-resident mean of scale * u: the copy of the
// final iterate, its warm-start rescaling (when no cycle ran) and the gauge in one pass.
__global__ __launch_bounds__(kThreads) void k_finish_phi(const float *__restrict__ u,
                                                         float *__restrict__ phi, int64_t count,
                                                         float scale,
                                                         const float *__restrict__ mean) {
  const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c >= count) return;
  phi[c] = fmaf(scale, u[c], -*mean);
}

// The same, four cells per thread (16-byte aligned arrays, count % 4 == 0).
__global__ __launch_bounds__(kThreads) void k_finish_phi4(const float4 *__restrict__ u,
                                                          float4 *__restrict__ phi, int64_t count4,
                                                          float scale,
                                                          const float *__restrict__ mean) {
  const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c >= count4) return;
  const float m = *mean;
  const float4 v = u[c];
  phi[c] = make_float4(fmaf(scale, v.x, -m), fmaf(scale, v.y, -m), fmaf(scale, v.z, -m),
                       fmaf(scale, v.w, -m));
}

// Coarsest level: one workgroup, in LDS (coarse_solve.h).
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_solve(
    float *__restrict__ ug, const float *__restrict__ fg, float scale,
    const float *__restrict__ mean, int n, float h2) {
  __shared__ float re[kCoarseMax];
  __shared__ float im[kCoarseMax];
  __shared__ float tc[pm_coarse::kMaxN], ts[pm_coarse::kMaxN];
  pm_coarse::solve_any(ug, fg, scale, src_mean(mean), n, h2, re, im, tc, ts);
}

inline unsigned blocks_for(int64_t count, int threads) {
  return (unsigned)((count + threads - 1) / threads);
}

// Floor detection of the tolerance loop: below a relative residual of kFloorBelow, a
// cycle that reduced it by less than kFloorGain ends the solve with PM_WARN_FLOOR.
constexpr double kFloorBelow = 1e-4;
constexpr double kFloorGain = 1.5;

struct Src {
  const float *f;
  float scale;
  const float *mean;
};

// Host-side V-cycle driver. Levels with n >= PM_STREAM_MIN_N (and an alt buffer)
// run the streaming kernels with ping-pong buffers: cur[l] holds the current
// iterate, a smoothing pass writes alt and the two are swapped. Every full
// V-cycle swaps twice, so level 0 ends in the caller's phi. Smaller levels run
// one kernel per red-black half-sweep, in place.
struct Solver {
  pm_ctx *ctx;
  hipStream_t s;
  const pm_mg_params *p;
  Src src0;
  float *cur[PM_MAX_LEVELS];
  float *alt[PM_MAX_LEVELS];

  Src src(int l) const { return l == 0 ? src0 : Src{ctx->lev[l].f, 1.0f, nullptr}; }
  float h2(int l) const {
    const double h = 1.0 / ctx->lev[l].n;
    return (float)(h * h);
  }
  bool streaming(int l) const {
    return alt[l] != nullptr && !(ctx->flags & PM_CREATE_REFERENCE_KERNELS);
  }

  hipError_t half_sweeps(int l, int first_colour, int sweeps) {
    const int n = ctx->lev[l].n;
    const int64_t half = (int64_t)n * n * (n / 2);
    const Src sr = src(l);
    for (int sw = 0; sw < sweeps; ++sw)
      for (int c = 0; c < 2; ++c)
        k_rbgs_half<<<blocks_for(half, kThreads), kThreads, 0, s>>>(
            cur[l], sr.f, sr.scale, sr.mean, n, h2(l), p->omega, c ^ first_colour);
    return hipGetLastError();
  }

  // streaming smoothing of `sweeps` full sweeps; the first pass may sum the residual
  // norm of its input.
  hipError_t stream_sweeps(int l, int first_colour, int sweeps, double *partial,
                           float uscale = 1.0f, const float *ec = nullptr) {
    const int n = ctx->lev[l].n;
    const Src sr = src(l);
    hipError_t e = hipSuccess;
    while (sweeps > 0 && e == hipSuccess) {
      const int now = sweeps >= 2 ? 2 : 1;
      if (l == 0) pm_kt_begin(ctx, PM_KERNEL_SMOOTH, s);
      e = launch_smooth_stream(cur[l], alt[l], sr.f, sr.scale, sr.mean, n, h2(l), p->omega,
                               first_colour, 2 * now, partial, uscale, ec, s);
      // algorithmic bytes of one pass: 12 B per cell per red-black sweep (read u and f,
      // write u), the pass fusing `now` sweeps, + the coarse correction (0.5 B per fine
      // cell) when it is prolonged in the pass
      if (l == 0)
        pm_kt_end(ctx, PM_KERNEL_SMOOTH, s, (12.0 * now + (ec ? 0.5 : 0.0)) * (double)n * n * n);
      std::swap(cur[l], alt[l]);
      partial = nullptr;
      uscale = 1.0f;
      ec = nullptr;
      sweeps -= now;
    }
    return e;
  }

  hipError_t pre_smooth(int l) {
    return streaming(l) ? stream_sweeps(l, 0, p->pre, nullptr) : half_sweeps(l, 0, p->pre);
  }

  hipError_t restrict_residual(int l) {
    const int n = ctx->lev[l].n;
    const int nc = n / 2;
    const int64_t ncount = (int64_t)nc * nc * nc;
    const Src sr = src(l);
    const float inv_h2 = 1.0f / h2(l);
    // coarse starting guess: one Jacobi step -H^2 d_H / 6, written with the restriction
    const float gscale = -h2(l + 1) / 6.0f;
    if (streaming(l)) {
      hipError_t e = launch_rr_stream(cur[l], sr.f, sr.scale, sr.mean, n, inv_h2, p->restrict_kind,
                                      ctx->lev[l + 1].f, cur[l + 1], gscale, s);
      if (e != hipSuccess) return e;
    } else {
      float *r = ctx->lev[l].res;
      k_residual<<<blocks_for((int64_t)n * n * n, kThreads), kThreads, 0, s>>>(
          cur[l], sr.f, sr.scale, sr.mean, n, inv_h2, r);
      if (p->restrict_kind == PM_RESTRICT_AVG)
        k_restrict_r<PM_RESTRICT_AVG><<<blocks_for(ncount, kThreads), kThreads, 0, s>>>(
            r, n, ctx->lev[l + 1].f, cur[l + 1], gscale);
      else
        k_restrict_r<PM_RESTRICT_FW><<<blocks_for(ncount, kThreads), kThreads, 0, s>>>(
            r, n, ctx->lev[l + 1].f, cur[l + 1], gscale);
    }
    return hipGetLastError();
  }

  hipError_t correct_and_post_smooth(int l) {
    const int n = ctx->lev[l].n;
    // streaming levels: the first post-smoothing pass adds the prolonged correction as
    // it reads each plane (coarse planes staged in LDS), so u is not read and written
    // an extra time
    if (streaming(l) && p->post > 0 && n >= PM_FUSE_PROLONG_MIN_N)
      return stream_sweeps(l, 1, p->post, nullptr, 1.0f, cur[l + 1]);
    k_prolong_add<<<blocks_for((int64_t)(n / 2) * (n / 2) * (n / 2), kThreads), kThreads, 0, s>>>(
        cur[l], n, cur[l + 1]);
    if (streaming(l)) return stream_sweeps(l, 1, p->post, nullptr);
    return half_sweeps(l, 1, p->post);
  }

  hipError_t coarse(int l) {
    const Src sr = src(l);
    k_coarse_solve<<<1, kCoarseThreads, 0, s>>>(cur[l], sr.f, sr.scale, sr.mean, ctx->lev[l].n,
                                                h2(l));
    return hipGetLastError();
  }

  // One cycle from level l (shape p->cycle unless given); when pre_done, the
  // pre-smoothing of level l has run. The coarse error equation is treated by one V
  // cycle (V), two W cycles in a row (W) or an F cycle and then a V cycle (F); the
  // second recursion continues from the first one's coarse iterate.
  hipError_t vcycle(int l, bool pre_done = false, int shape = -1) {
    if (shape < 0) shape = p->cycle;
    if (l == ctx->nlevels - 1) return coarse(l);
    hipError_t e = pre_done ? hipSuccess : pre_smooth(l);
    if (e == hipSuccess) e = restrict_residual(l);
    if (e == hipSuccess) e = vcycle(l + 1, false, shape == PM_CYCLE_V ? PM_CYCLE_V : shape);
    if (e == hipSuccess && shape != PM_CYCLE_V)
      e = vcycle(l + 1, false, shape == PM_CYCLE_W ? PM_CYCLE_W : PM_CYCLE_V);
    if (e == hipSuccess) e = correct_and_post_smooth(l);
    return e;
  }

  // ||tau||_2 of the iterate scale * u on the level-0 grid, with level 1's arrays as
  // scratch (free between cycles); synchronises the stream
  hipError_t tau_norm(const float *u, float scale, double *out) {
    const int n = ctx->lev[0].n, nc = n / 2;
    const int64_t ncount = (int64_t)nc * nc * nc;
    const float inv_h2 = 1.0f / h2(0);
    float *ru = ctx->lev[1].u, *rlu = ctx->lev[1].f;
    const unsigned gb = (unsigned)((ncount + kThreads - 1) / kThreads);
    if (p->restrict_kind == PM_RESTRICT_AVG)
      k_tau_restrict<PM_RESTRICT_AVG><<<gb, kThreads, 0, s>>>(u, n, inv_h2, scale, ru, rlu);
    else
      k_tau_restrict<PM_RESTRICT_FW><<<gb, kThreads, 0, s>>>(u, n, inv_h2, scale, ru, rlu);
    const int nb = (int)std::min<int64_t>(RED_BLOCKS, (ncount + RED_THREADS - 1) / RED_THREADS);
    k_tau_norm<<<nb, RED_THREADS, 0, s>>>(ru, rlu, nc, 0.25f * inv_h2, ctx->red_partial);
    k_pair_final<<<1, RED_THREADS, 0, s>>>(ctx->red_partial, nb, ctx->red_result);
    hipError_t e = hipMemcpyAsync(ctx->host_result + 2, ctx->red_result, sizeof(double),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    *out = std::sqrt(ctx->host_result[2]);
    return e;
  }

  // ||f - L u||^2 and ||f||^2 at level 0 into ctx->red_result[0..1] (plain kernel)
  void norms() {
    const int n = ctx->lev[0].n;
    const int64_t count = (int64_t)n * n * n;
    const int nb = (int)std::min<int64_t>(RED_BLOCKS, (count + RED_THREADS - 1) / RED_THREADS);
    k_residual_norm<<<nb, RED_THREADS, 0, s>>>(cur[0], src0.f, src0.scale, src0.mean, n,
                                               1.0f / h2(0), ctx->red_partial);
    k_pair_final<<<1, RED_THREADS, 0, s>>>(ctx->red_partial, nb, ctx->red_result);
  }
};

}  // namespace

int pm_mg_setup(pm_ctx *ctx) {
  int n = ctx->n;
  ctx->nlevels = 0;
  ctx->lev[0] = pm_level{n, nullptr, nullptr, nullptr};
  ctx->nlevels = 1;
  while (n > 16 && n % 4 == 0) {
    n /= 2;
    if (ctx->nlevels >= PM_MAX_LEVELS) return PM_ERR_SHAPE;
    pm_level L{n, nullptr, nullptr, nullptr};
    const size_t bytes = sizeof(float) * (size_t)n * n * n;
    if (hipMalloc(&L.u, bytes) != hipSuccess || hipMalloc(&L.f, bytes) != hipSuccess)
      return PM_ERR_NOMEM;
    ctx->lev[ctx->nlevels++] = L;
  }
  if ((int64_t)n * n * n > kCoarseMax) return PM_ERR_SHAPE;
  // residual scratch of the two-pass restriction (levels that do not stream)
  for (int l = 0; l + 1 < ctx->nlevels; ++l) {
    const int m = ctx->lev[l].n;
    const bool streams = m >= PM_STREAM_MIN_N && !(ctx->flags & PM_CREATE_REFERENCE_KERNELS) &&
                         smooth_stream_blocks(m) <= RED_PARTIAL_CAP;
    if (streams) continue;
    if (hipMalloc(&ctx->lev[l].res, sizeof(float) * (size_t)m * m * m) != hipSuccess)
      return PM_ERR_NOMEM;
  }
  // ping-pong buffers for the streaming levels (not the coarsest)
  for (int l = 0; l + 1 < ctx->nlevels; ++l) {
    const int m = ctx->lev[l].n;
    if (m < PM_STREAM_MIN_N || (ctx->flags & PM_CREATE_REFERENCE_KERNELS)) continue;
    if (smooth_stream_blocks(m) > RED_PARTIAL_CAP) continue;
    if (hipMalloc(&ctx->lev[l].alt, sizeof(float) * (size_t)m * m * m) != hipSuccess)
      return PM_ERR_NOMEM;
  }
  return PM_OK;
}

int pm_mg_solve(pm_ctx *ctx, const float *rho, float coef, float *phi, const pm_mg_params *p,
                pm_mg_stats *stats, hipStream_t s, float warm_scale, bool rho_mean_ready) {
  const int n = ctx->n;
  const int64_t count = (int64_t)n * n * n;
  // mean of the density, kept on the device
  if (!rho_mean_ready)
    PM_HIP(ctx, launch_sum_moments(rho, count, ctx->red_partial, ctx->red_result, ctx->mean_f, s));
  Solver sv{ctx, s, p, Src{rho, coef, ctx->mean_f}, {}, {}};
  for (int l = 0; l < ctx->nlevels; ++l) {
    sv.cur[l] = l == 0 ? phi : ctx->lev[l].u;
    sv.alt[l] = ctx->lev[l].alt;
  }
  const bool fused_norm = sv.streaming(0) && p->pre > 0 && ctx->nlevels > 1;
  if (p->alpha > 0.0f && p->fixed_cycles <= 0 && ctx->nlevels < 2)
    return pm_fail(ctx, PM_ERR_ARG, "alpha needs a coarser multigrid level (n > 16)");
  // with the fused norm, the tolerance loop's first pass reads the warm start rescaled
  float uscale = 1.0f;
  if (p->guess == PM_GUESS_JACOBI)
    k_jacobi_guess<<<blocks_for(count, kThreads), kThreads, 0, s>>>(phi, rho, coef, ctx->mean_f,
                                                                     count, sv.h2(0));
  else if (warm_scale != 1.0f && fused_norm && p->fixed_cycles <= 0)
    uscale = warm_scale;
  else if (warm_scale != 1.0f)
    k_scale<<<blocks_for(count, kThreads), kThreads, 0, s>>>(phi, count, warm_scale);
  // the final iterate's sum, when a norm pass has taken it (ctx->red_result[2])
  bool have_sum = false;
  int status = PM_OK;
  int cycles = 0;
  if (p->fixed_cycles > 0) {
    for (int c = 0; c < p->fixed_cycles; ++c) PM_HIP(ctx, sv.vcycle(0));
    cycles = p->fixed_cycles;
  } else {
    double rel[64];
    double fnorm = 0.0;
    status = PM_WARN_NOT_CONVERGED;
    for (;;) {
      // residual norm of the current iterate: fused into the next pre-smoothing
      // pass when streaming (its output is used only if another cycle is needed)
      if (fused_norm) {
        const int64_t nb = smooth_stream_blocks(n);
        PM_HIP(ctx, sv.stream_sweeps(0, 0, std::min(p->pre, 2), ctx->red_partial,
                                     cycles == 0 ? uscale : 1.0f));
        k_triple_final<<<1, RED_THREADS, 0, s>>>(ctx->red_partial, (int)nb, ctx->red_result,
                                                  count, ctx->mean_f + 1);
      } else {
        sv.norms();
      }
      PM_HIP(ctx, hipMemcpyAsync(ctx->host_result, ctx->red_result, 2 * sizeof(double),
                                 hipMemcpyDeviceToHost, s));
      PM_HIP(ctx, hipStreamSynchronize(s));
      if (cycles == 0) fnorm = sqrt(ctx->host_result[1]);
      if (fnorm == 0.0) {
        if (fused_norm) std::swap(sv.cur[0], sv.alt[0]);  // drop the speculative pass
        PM_HIP(ctx, launch_fill(phi, 0.0f, count, s));
        if (stats) {
          stats->cycles = 0;
          stats->status = PM_OK;
          stats->relres[0] = 0.0;
        }
        return PM_OK;
      }
      rel[cycles] = sqrt(ctx->host_result[0]) / fnorm;
      bool converged = rel[cycles] < p->tol;
      if (p->alpha > 0.0f) {
        // the paper's rule: residual below alpha times the truncation-error estimate of
        // the same iterate (the input of the norm pass, read rescaled in the first one)
        const double dnorm = sqrt(ctx->host_result[0]);
        double tnorm = 0.0;
        PM_HIP(ctx, sv.tau_norm(fused_norm ? sv.alt[0] : sv.cur[0],
                                fused_norm && cycles == 0 ? uscale : 1.0f, &tnorm));
        converged = dnorm < (double)p->alpha * tnorm;
      }
      if (converged) {
        status = PM_OK;
      } else if (cycles > 0 && rel[cycles] < kFloorBelow &&
                 rel[cycles - 1] < kFloorGain * rel[cycles]) {
        // a V-cycle removes most of the algebraic residual (about 6 to 10 times, App. C);
        // a cycle that gained less than kFloorGain met the FP32 rounding floor
        status = PM_WARN_FLOOR;
      }
      if (status != PM_WARN_NOT_CONVERGED || cycles == p->max_cycles) {
        if (fused_norm) {
          // the speculative pass smoothed the tested iterate twice more: keep its output
          // (smoothing does not raise the error); its mean is taken as the tested
          // iterate's (the pass changes it by far less than the solve's error)
          have_sum = true;
        }
        break;
      }
      if (fused_norm) {
        // finish the cycle whose pre-smoothing already ran (remaining pre sweeps first)
        if (p->pre > 2) PM_HIP(ctx, sv.stream_sweeps(0, 0, p->pre - 2, nullptr));
        PM_HIP(ctx, sv.vcycle(0, true));
      } else {
        PM_HIP(ctx, sv.vcycle(0));
      }
      ++cycles;
    }
    if (stats)
      for (int c = 0; c <= cycles; ++c) stats->relres[c] = rel[c];
  }
  if (have_sum) {
    // copy (when the iterate is in the other buffer) and remove the mean (gauge) in one
    // pass
    const bool vec = count % 4 == 0 && reinterpret_cast<uintptr_t>(sv.cur[0]) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(phi) % 16 == 0;
    if (vec)
      k_finish_phi4<<<blocks_for(count / 4, kThreads), kThreads, 0, s>>>(
          reinterpret_cast<const float4 *>(sv.cur[0]), reinterpret_cast<float4 *>(phi), count / 4,
          1.0f, ctx->mean_f + 1);
    else
      k_finish_phi<<<blocks_for(count, kThreads), kThreads, 0, s>>>(sv.cur[0], phi, count,
                                                                     1.0f, ctx->mean_f + 1);
  } else {
    if (sv.cur[0] != phi)
      PM_HIP(ctx, hipMemcpyAsync(phi, sv.cur[0], sizeof(float) * count, hipMemcpyDeviceToDevice, s));
    // remove the mean of phi (gauge)
    PM_HIP(ctx, launch_sum_moments(phi, count, ctx->red_partial, ctx->red_result, ctx->mean_f + 1, s));
    k_subtract_mean<<<blocks_for(count, kThreads), kThreads, 0, s>>>(phi, count, ctx->mean_f + 1);
  }
  PM_HIP(ctx, hipGetLastError());
  if (stats) {
    stats->cycles = cycles;
    stats->status = status;
  }
  if (status == PM_WARN_NOT_CONVERGED) pm_fail(ctx, status, "multigrid: max_cycles reached above tol");
  if (status == PM_WARN_FLOOR) pm_fail(ctx, status, "multigrid: stagnated at the FP32 floor above tol");
  return status;
}
