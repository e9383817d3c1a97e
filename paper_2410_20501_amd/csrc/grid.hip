// Grid kernels: central finite-difference gradient (paper gradient table,
// g = -grad phi) and deterministic FP64 moment reductions.
#include "internal.h"

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ int wrap_index(int i, int n) {
  i += (i < 0) ? n : 0;
  i -= (i >= n) ? n : 0;
  return i;
}

// Central-difference coefficients c_1..c_3 of the paper's table; c_{-m} = -c_m.
template <int P>
struct Stencil;
template <>
struct Stencil<3> {
  static constexpr int R = 1;
  __device__ static float c(int m) { return 0.5f; }
};
template <>
struct Stencil<5> {
  static constexpr int R = 2;
  __device__ static float c(int m) { return m == 1 ? (2.0f / 3.0f) : (-1.0f / 12.0f); }
};
template <>
struct Stencil<7> {
  static constexpr int R = 3;
  __device__ static float c(int m) {
    return m == 1 ? 0.75f : (m == 2 ? (-3.0f / 20.0f) : (1.0f / 60.0f));
  }
};

// One thread per cell along k; a block covers a run of one (i, j) row.
// g_d = -(1/h) sum_m c_m (phi_{+m} - phi_{-m}) along axis d.
template <int P>
__global__ __launch_bounds__(kThreads) void k_gradient(const float *__restrict__ phi, int n,
                                                       float inv_h, float *__restrict__ g) {
  constexpr int R = Stencil<P>::R;
  const unsigned lin = xcd_block(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                                 gridDim.x * gridDim.y * gridDim.z);
  const int k = (lin % gridDim.x) * kThreads + threadIdx.x;
  const int j = (lin / gridDim.x) % gridDim.y;
  const int i = lin / (gridDim.x * gridDim.y);
  if (k >= n) return;
  const size_t nn = (size_t)n * n;
  const size_t row = ((size_t)i * n + j) * n;
  float gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
  for (int m = 1; m <= R; ++m) {
    const float cm = Stencil<P>::c(m);
    const size_t ip = (size_t)wrap_index(i + m, n) * nn + (size_t)j * n + k;
    const size_t im = (size_t)wrap_index(i - m, n) * nn + (size_t)j * n + k;
    const size_t jp = (size_t)i * nn + (size_t)wrap_index(j + m, n) * n + k;
    const size_t jm = (size_t)i * nn + (size_t)wrap_index(j - m, n) * n + k;
    gx = fmaf(cm, phi[ip] - phi[im], gx);
    gy = fmaf(cm, phi[jp] - phi[jm], gy);
    gz = fmaf(cm, phi[row + wrap_index(k + m, n)] - phi[row + wrap_index(k - m, n)], gz);
  }
  float *out = g + 3 * (row + k);
  out[0] = -inv_h * gx;
  out[1] = -inv_h * gy;
  out[2] = -inv_h * gz;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Block partials of sum x and sum x^2 over a fixed grid (deterministic order). VEC: x
// 16-byte aligned, read as float4 two at a time (the loads of a thread in flight
// together); the count % 4 trailing values go to the first threads.
template <bool VEC>
__global__ __launch_bounds__(RED_THREADS) void k_moments_partial(const float *__restrict__ x,
                                                                 int64_t count,
                                                                 double *__restrict__ partial) {
  double s1 = 0.0, s2 = 0.0;
  const int64_t stride = (int64_t)gridDim.x * RED_THREADS;
  const int64_t t = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x;
  if constexpr (VEC) {
    const float4 *x4 = reinterpret_cast<const float4 *>(x);
    const int64_t c4 = count / 4;
    int64_t i = t;
    for (; i + stride < c4; i += 2 * stride) {
      const float4 a = x4[i], b = x4[i + stride];
      for (const float v : {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w}) {
        const double d = v;
        s1 += d;
        s2 += d * d;
      }
    }
    if (i < c4) {
      const float4 a = x4[i];
      for (const float v : {a.x, a.y, a.z, a.w}) {
        const double d = v;
        s1 += d;
        s2 += d * d;
      }
    }
    if (t < count % 4) {
      const double d = x[4 * c4 + t];
      s1 += d;
      s2 += d * d;
    }
  } else {
    for (int64_t i = t; i < count; i += stride) {
      const double v = x[i];
      s1 += v;
      s2 += v * v;
    }
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

__global__ __launch_bounds__(RED_THREADS) void k_moments_final(const double *__restrict__ partial,
                                                               int nblocks, int64_t count,
                                                               double *__restrict__ result,
                                                               float *__restrict__ mean_out) {
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
    result[2] = count > 0 ? a / (double)count : 0.0;
    if (mean_out) mean_out[0] = (float)result[2];
  }
}

// extrapolated warm start: phi = c1 phi + c2 prev, prev = the old phi (float4 per thread)
__global__ __launch_bounds__(RED_THREADS) void k_extrapolate(float4 *__restrict__ phi,
                                                             float4 *__restrict__ prev,
                                                             int64_t count4, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x;
  if (i >= count4) return;
  const float4 u = phi[i], v = prev[i];
  phi[i] = make_float4(fmaf(c1, u.x, c2 * v.x), fmaf(c1, u.y, c2 * v.y), fmaf(c1, u.z, c2 * v.z),
                       fmaf(c1, u.w, c2 * v.w));
  prev[i] = u;
}

__global__ __launch_bounds__(RED_THREADS) void k_extrapolate1(float *__restrict__ phi,
                                                              float *__restrict__ prev,
                                                              int64_t count, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x;
  if (i >= count) return;
  const float u = phi[i];
  phi[i] = fmaf(c1, u, c2 * prev[i]);
  prev[i] = u;
}

// count of non-finite values (grid-stride; one atomic per wave into *out)
__global__ __launch_bounds__(RED_THREADS) void k_count_nonfinite(const float *__restrict__ x,
                                                                 int64_t count,
                                                                 unsigned long long *out) {
  unsigned long long c = 0;
  const int64_t stride = (int64_t)gridDim.x * RED_THREADS;
  for (int64_t i = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; i < count; i += stride)
    c += isfinite(x[i]) ? 0ull : 1ull;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

}  // namespace

hipError_t launch_extrapolate(float *phi, float *prev, int64_t count, float c1, float c2,
                              hipStream_t s) {
  if (count <= 0) return hipSuccess;
  // float4 accesses when both arrays are 16-byte aligned and count is a multiple of 4
  // (n^3 cells with n even)
  if (count % 4 != 0 || (((uintptr_t)phi | (uintptr_t)prev) & 15u) != 0) {
    k_extrapolate1<<<(unsigned)((count + RED_THREADS - 1) / RED_THREADS), RED_THREADS, 0, s>>>(
        phi, prev, count, c1, c2);
    return hipGetLastError();
  }
  const int64_t c4 = count / 4;
  k_extrapolate<<<(unsigned)((c4 + RED_THREADS - 1) / RED_THREADS), RED_THREADS, 0, s>>>(
      reinterpret_cast<float4 *>(phi), reinterpret_cast<float4 *>(prev), c4, c1, c2);
  return hipGetLastError();
}

hipError_t launch_count_nonfinite(const float *x, int64_t count, unsigned long long *out,
                                  hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int nb = (int)std::min<int64_t>(RED_BLOCKS, (count + RED_THREADS - 1) / RED_THREADS);
  k_count_nonfinite<<<nb, RED_THREADS, 0, s>>>(x, count, out);
  return hipGetLastError();
}

hipError_t launch_gradient(const float *phi, int n, int points, float *g, hipStream_t s) {
  dim3 grid((n + kThreads - 1) / kThreads, n, n);
  const float inv_h = (float)n;
  switch (points) {
    case 3: k_gradient<3><<<grid, kThreads, 0, s>>>(phi, n, inv_h, g); break;
    case 5: k_gradient<5><<<grid, kThreads, 0, s>>>(phi, n, inv_h, g); break;
    default: k_gradient<7><<<grid, kThreads, 0, s>>>(phi, n, inv_h, g); break;
  }
  return hipGetLastError();
}

hipError_t launch_sum_moments(const float *x, int64_t count, double *partial, double *result,
                              float *mean_out, hipStream_t s) {
  int nb = (int)std::min<int64_t>(RED_BLOCKS, (count + RED_THREADS - 1) / RED_THREADS);
  if (nb < 1) nb = 1;
  if ((reinterpret_cast<uintptr_t>(x) & 15) == 0)
    k_moments_partial<true><<<nb, RED_THREADS, 0, s>>>(x, count, partial);
  else
    k_moments_partial<false><<<nb, RED_THREADS, 0, s>>>(x, count, partial);
  k_moments_final<<<1, RED_THREADS, 0, s>>>(partial, nb, count, result, mean_out);
  return hipGetLastError();
}
