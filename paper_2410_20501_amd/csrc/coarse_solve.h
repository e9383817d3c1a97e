// Coarsest multigrid level (at most 20^3 cells), solved exactly by one 1024-thread
// workgroup in LDS (the recursion's last level, paper Sect. 3.7.1). On a periodic
// grid the seven-point operator is diagonal in the discrete Fourier basis:
//   L e^{i 2 pi (a i + b j + c k)/n} = lambda e^{...},
//   lambda = (2 cos(2 pi a/n) + 2 cos(2 pi b/n) + 2 cos(2 pi c/n) - 6) / h^2,
// so u = DFT^-1[ DFT[f] / lambda ] with the zero mode set to zero (the periodic
// problem's mean: the right-hand side's mean is dropped, the solution has mean zero).
// The transforms are direct DFTs along each axis (n <= 20, any n), in FP32.
#pragma once

#include <hip/hip_runtime.h>

namespace pm_coarse {

constexpr int kThreads = 1024;
constexpr int kMaxCells = 8000;
constexpr int kMaxN = 20;
constexpr int kItems = (kMaxCells + kThreads - 1) / kThreads;  // outputs per thread and pass

// One DFT pass along `axis` (0: i, stride n^2; 1: j, stride n; 2: k, stride 1) over the
// planar complex grid (re, im), in place: every thread forms its outputs from the
// line in LDS, then all write after a barrier. sgn = -1 forward, +1 inverse.
__device__ __forceinline__ void dft_pass(float *re, float *im, const float *tc, const float *ts,
                                         int n, int axis, float sgn) {
  const int count = n * n * n;
  const int st = axis == 0 ? n * n : (axis == 1 ? n : 1);
  float orr[kItems], oii[kItems];
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const int c = threadIdx.x + it * kThreads;
    orr[it] = oii[it] = 0.f;
    if (c < count) {
      const int i = c / (n * n), j = (c / n) % n, k = c % n;
      const int p = axis == 0 ? i : (axis == 1 ? j : k);
      const int base = c - p * st;
      float sr = 0.f, si = 0.f;
      int idx = 0;  // (m p) mod n
      for (int m = 0; m < n; ++m) {
        const float wr = tc[idx], wi = sgn * ts[idx];
        const float xr = re[base + m * st], xi = im[base + m * st];
        sr = fmaf(xr, wr, fmaf(-xi, wi, sr));
        si = fmaf(xr, wi, fmaf(xi, wr, si));
        idx += p;
        if (idx >= n) idx -= n;
      }
      orr[it] = sr;
      oii[it] = si;
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const int c = threadIdx.x + it * kThreads;
    if (c < count) {
      re[c] = orr[it];
      im[c] = oii[it];
    }
  }
  __syncthreads();
}

// ug = L^-1 (scale (fg - mean)) with zero mean. re, im: LDS arrays of kMaxCells floats;
// tc, ts: LDS arrays of kMaxN floats (cosine and sine table).
__device__ void solve_any(float *__restrict__ ug, const float *__restrict__ fg, float scale,
                          float mean, int n, float h2, float *re, float *im, float *tc,
                          float *ts) {
  const int count = n * n * n;
  for (int c = threadIdx.x; c < count; c += kThreads) {
    re[c] = scale * (fg[c] - mean);
    im[c] = 0.f;
  }
  for (int m = threadIdx.x; m < n; m += kThreads) {
    double s, co;
    sincospi(2.0 * m / n, &s, &co);  // table in FP64, then rounded
    tc[m] = (float)co;
    ts[m] = (float)s;
  }
  __syncthreads();
  for (int axis = 0; axis < 3; ++axis) dft_pass(re, im, tc, ts, n, axis, -1.0f);
  const float inv_h2 = 1.0f / h2;
  for (int c = threadIdx.x; c < count; c += kThreads) {
    const int a = c / (n * n), b = (c / n) % n, k = c % n;
    const float lam = (2.0f * (tc[a] + tc[b] + tc[k]) - 6.0f) * inv_h2;
    const float r = c == 0 ? 0.f : 1.0f / lam;
    re[c] *= r;
    im[c] *= r;
  }
  __syncthreads();
  for (int axis = 0; axis < 3; ++axis) dft_pass(re, im, tc, ts, n, axis, 1.0f);
  const float inv_count = 1.0f / (float)count;
  for (int c = threadIdx.x; c < count; c += kThreads) ug[c] = re[c] * inv_count;
}

}  // namespace pm_coarse
