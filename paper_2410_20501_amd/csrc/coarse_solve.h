// Coarsest multigrid level (at most 20^3 cells) solved by one 1024-thread
// workgroup in LDS: red-black Gauss-Seidel sweeps until the residual has
// dropped by `reduction` (checked every 4 sweeps), stagnates, or max_sweeps
// (paper Sect. 3.7.1, the recursion's last level). The mean of the right-hand
// side is removed first and the mean of the solution last (periodic problem).
//
// Every thread owns at most SLOTS cells of each colour; their LDS index and
// the six neighbour indices are computed once, so a sweep is loads, one fma
// chain and a store per cell, with no index arithmetic.
#pragma once

#include <hip/hip_runtime.h>

namespace pm_coarse {

constexpr int kThreads = 1024;
constexpr int kMaxCells = 8000;

__device__ __forceinline__ int wrapc(int i, int n) {
  i += (i < 0) ? n : 0;
  i -= (i >= n) ? n : 0;
  return i;
}

__device__ __forceinline__ double block_sum(double v, double *red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) s += red[w];
  return s;
}

// su, sf: LDS arrays of kMaxCells floats; red: LDS array of kThreads / 64 doubles.
template <int SLOTS>
__device__ void solve(float *__restrict__ ug, const float *__restrict__ fg, float scale,
                      float mean, int n, float h2, float reduction, int max_sweeps, float *su,
                      float *sf, double *red) {
  const int count = n * n * n;
  const int half = n >> 1;
  const int hcount = count >> 1;  // cells of one colour (n even)
  double fs = 0.0;
  for (int c = threadIdx.x; c < count; c += kThreads) {
    su[c] = ug[c];
    const float fv = scale * (fg[c] - mean);
    sf[c] = fv;
    fs += fv;
  }
  const float fmean = (float)(block_sum(fs, red) / count);
  for (int c = threadIdx.x; c < count; c += kThreads) sf[c] -= fmean;
  // this thread's cells: half-cell t -> (i, j, k2), k = 2 k2 + ((i + j + colour) & 1)
  int cc[2][SLOTS];
  int nb[2][SLOTS][6];
#pragma unroll
  for (int col = 0; col < 2; ++col) {
#pragma unroll
    for (int m = 0; m < SLOTS; ++m) {
      const int t = threadIdx.x + m * kThreads;
      cc[col][m] = -1;
      if (t < hcount) {
        const int k2 = t % half, r = t / half;
        const int j = r % n, i = r / n;
        const int k = 2 * k2 + ((i + j + col) & 1);
        cc[col][m] = (i * n + j) * n + k;
        nb[col][m][0] = (wrapc(i + 1, n) * n + j) * n + k;
        nb[col][m][1] = (wrapc(i - 1, n) * n + j) * n + k;
        nb[col][m][2] = (i * n + wrapc(j + 1, n)) * n + k;
        nb[col][m][3] = (i * n + wrapc(j - 1, n)) * n + k;
        nb[col][m][4] = (i * n + j) * n + wrapc(k + 1, n);
        nb[col][m][5] = (i * n + j) * n + wrapc(k - 1, n);
      }
    }
  }
  __syncthreads();
  const float inv_h2 = 1.0f / h2;
  auto resid_norm = [&]() {
    double s = 0.0;
#pragma unroll
    for (int col = 0; col < 2; ++col)
#pragma unroll
      for (int m = 0; m < SLOTS; ++m) {
        const int c = cc[col][m];
        if (c < 0) continue;
        const float uc = su[c];
        // difference form: exact for close values
        const float lap = (su[nb[col][m][0]] - uc) + (su[nb[col][m][1]] - uc) +
                          (su[nb[col][m][2]] - uc) + (su[nb[col][m][3]] - uc) +
                          (su[nb[col][m][4]] - uc) + (su[nb[col][m][5]] - uc);
        const double r = sf[c] - lap * inv_h2;
        s += r * r;
      }
    return sqrt(block_sum(s, red));
  };
  const double r0 = resid_norm();
  double prev = r0;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
#pragma unroll
    for (int col = 0; col < 2; ++col) {
#pragma unroll
      for (int m = 0; m < SLOTS; ++m) {
        const int c = cc[col][m];
        if (c < 0) continue;
        const float s = su[nb[col][m][0]] + su[nb[col][m][1]] + su[nb[col][m][2]] +
                        su[nb[col][m][3]] + su[nb[col][m][4]] + su[nb[col][m][5]];
        su[c] = (s - h2 * sf[c]) * (1.0f / 6.0f);
      }
      __syncthreads();
    }
    if ((sweep & 3) == 3) {
      const double r = resid_norm();
      if (r <= reduction * r0 || r > 0.98 * prev) break;
      prev = r;
    }
  }
  double us = 0.0;
  for (int c = threadIdx.x; c < count; c += kThreads) us += su[c];
  const float umean = (float)(block_sum(us, red) / count);
  for (int c = threadIdx.x; c < count; c += kThreads) ug[c] = su[c] - umean;
}

// Dispatch on the number of cells per colour and thread.
__device__ __forceinline__ void solve_any(float *ug, const float *fg, float scale, float mean,
                                          int n, float h2, float reduction, int max_sweeps,
                                          float *su, float *sf, double *red) {
  const int hcount = (n * n * n) >> 1;
  if (hcount <= kThreads)
    solve<1>(ug, fg, scale, mean, n, h2, reduction, max_sweeps, su, sf, red);
  else if (hcount <= 2 * kThreads)
    solve<2>(ug, fg, scale, mean, n, h2, reduction, max_sweeps, su, sf, red);
  else
    solve<4>(ug, fg, scale, mean, n, h2, reduction, max_sweeps, su, sf, red);
}

}  // namespace pm_coarse
