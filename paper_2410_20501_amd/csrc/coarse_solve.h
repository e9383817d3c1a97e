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

// 16^3 (the coarsest level of every power-of-two grid): each of 256 threads transforms
// one whole line in registers with a radix-2 FFT, so a pass reads and writes every value
// of the grid once (the direct DFT reads each line n times). LDS index c + c / 16 (one
// padding word per line along k) keeps the stride-1 lines of the k pass off a single
// bank.
constexpr int kFftN = 16;
__device__ __forceinline__ int pad16(int c) { return c + (c >> 4); }

// cos and sin of 2 pi k / 16, k = 0 .. 7
__device__ constexpr float kC16[8] = {1.0f, 0.92387953251128674f, 0.70710678118654752f,
                                      0.38268343236508977f, 0.0f, -0.38268343236508977f,
                                      -0.70710678118654752f, -0.92387953251128674f};
__device__ constexpr float kS16[8] = {0.0f, 0.38268343236508977f, 0.70710678118654752f,
                                      0.92387953251128674f, 1.0f, 0.92387953251128674f,
                                      0.70710678118654752f, 0.38268343236508977f};

// in-place 16-point FFT of (xr, xi): bit-reversed order, then four radix-2 stages with
// twiddles e^{sgn 2 pi i j / len}; sgn = -1 forward, +1 inverse (unnormalised)
__device__ __forceinline__ void fft16(float (&xr)[kFftN], float (&xi)[kFftN], float sgn) {
#pragma unroll
  for (int i = 0; i < kFftN; ++i) {
    const int r = ((i & 1) << 3) | ((i & 2) << 1) | ((i & 4) >> 1) | ((i & 8) >> 3);
    if (r > i) {
      const float tr = xr[i], ti = xi[i];
      xr[i] = xr[r];
      xi[i] = xi[r];
      xr[r] = tr;
      xi[r] = ti;
    }
  }
#pragma unroll
  for (int len = 2; len <= kFftN; len <<= 1) {
#pragma unroll
    for (int i = 0; i < kFftN; i += len) {
#pragma unroll
      for (int j = 0; j < len / 2; ++j) {
        const int t = j * (kFftN / len);  // twiddle index in sixteenths
        const float wr = kC16[t], wi = sgn * kS16[t];
        const int a = i + j, b = a + len / 2;
        const float vr = xr[b] * wr - xi[b] * wi, vi = xr[b] * wi + xi[b] * wr;
        xr[b] = xr[a] - vr;
        xi[b] = xi[a] - vi;
        xr[a] += vr;
        xi[a] += vi;
      }
    }
  }
}

__device__ void fft16_pass(float *re, float *im, int axis, float sgn) {
  const int t = threadIdx.x;
  if (t < kFftN * kFftN) {
    const int st = axis == 0 ? kFftN * kFftN : (axis == 1 ? kFftN : 1);
    const int u = t / kFftN, v = t % kFftN;  // the line's two other coordinates
    const int base = axis == 0 ? u * kFftN + v : (axis == 1 ? u * kFftN * kFftN + v
                                                            : (u * kFftN + v) * kFftN);
    float xr[kFftN], xi[kFftN];
#pragma unroll
    for (int m = 0; m < kFftN; ++m) {
      const int c = pad16(base + m * st);
      xr[m] = re[c];
      xi[m] = im[c];
    }
    fft16(xr, xi, sgn);
#pragma unroll
    for (int m = 0; m < kFftN; ++m) {
      const int c = pad16(base + m * st);
      re[c] = xr[m];
      im[c] = xi[m];
    }
  }
  __syncthreads();
}

__device__ void solve16(float *__restrict__ ug, const float *__restrict__ fg, float scale,
                        float mean, float h2, float *re, float *im) {
  constexpr int count = kFftN * kFftN * kFftN;
  for (int c = threadIdx.x; c < count; c += kThreads) {
    re[pad16(c)] = scale * (fg[c] - mean);
    im[pad16(c)] = 0.f;
  }
  __syncthreads();
  for (int axis = 0; axis < 3; ++axis) fft16_pass(re, im, axis, -1.0f);
  const float inv_h2 = 1.0f / h2;
  for (int c = threadIdx.x; c < count; c += kThreads) {
    const int a = c >> 8, b = (c >> 4) & 15, k = c & 15;
    auto cs = [](int m) { return m < 8 ? kC16[m] : -kC16[m - 8]; };  // cos(2 pi m / 16)
    const float lam = (2.0f * (cs(a) + cs(b) + cs(k)) - 6.0f) * inv_h2;
    const float r = c == 0 ? 0.f : 1.0f / lam;
    re[pad16(c)] *= r;
    im[pad16(c)] *= r;
  }
  __syncthreads();
  for (int axis = 0; axis < 3; ++axis) fft16_pass(re, im, axis, 1.0f);
  const float inv_count = 1.0f / (float)count;
  for (int c = threadIdx.x; c < count; c += kThreads) ug[c] = re[pad16(c)] * inv_count;
}

// ug = L^-1 (scale (fg - mean)) with zero mean. re, im: LDS arrays of kMaxCells floats;
// tc, ts: LDS arrays of kMaxN floats (cosine and sine table).
__device__ void solve_any(float *__restrict__ ug, const float *__restrict__ fg, float scale,
                          float mean, int n, float h2, float *re, float *im, float *tc,
                          float *ts) {
  if (n == kFftN) {
    solve16(ug, fg, scale, mean, h2, re, im);
    return;
  }
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
