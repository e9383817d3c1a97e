// Particle-side kernels: mass assignment (atomic scatter and cell-sorted gather),
// interpolation with an optional fused kick, kick + drift, and the counting sort
// that buckets particles by cell. Paper Sect. 3.5 (windows), Sect. 3.4 (leapfrog),
// App. E (particle ordering for locality).
#include "internal.h"

namespace {

constexpr int kThreads = 256;

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

// Per-axis support of the window: first cell index (unwrapped) and MAS weights.
// TSC (MAS = 3): cells floor(u)-1 .. floor(u)+1, d = u - floor(u) - 1/2 in [-1/2, 1/2):
//   W = (1/2)(1/2 - d)^2, 3/4 - d^2, (1/2)(1/2 + d)^2.
// CIC (MAS = 2): cells floor(u - 1/2) and the next, d = u - 1/2 - floor(u - 1/2):
//   W = 1 - d, d.
template <int MAS>
__device__ __forceinline__ void weights_from_frac(float d, float *w) {
  if constexpr (MAS == 3) {
    const float a = 0.5f - d, b = 0.5f + d;
    w[0] = 0.5f * a * a;
    w[1] = 0.75f - d * d;
    w[2] = 0.5f * b * b;
  } else {
    w[0] = 1.0f - d;
    w[1] = d;
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
  } else {
    const float t = u - 0.5f;
    const float fl = floorf(t);
    weights_from_frac<2>(t - fl, w);
    return (int)fl;
  }
}

// Cell index c and in-cell offset o in [0,1) -> first cell and weights.
template <int MAS>
__device__ __forceinline__ int axis_off(int c, float o, float *w) {
  if constexpr (MAS == 3) {
    weights_from_frac<3>(o - 0.5f, w);
    return c - 1;
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
  if constexpr (PK == PM_POS_BOX) {
    const float fn = (float)n;
    first[0] = wrap_any(axis_box<MAS>(x0, fn, w[0]), n);
    first[1] = wrap_any(axis_box<MAS>(x1, fn, w[1]), n);
    first[2] = wrap_any(axis_box<MAS>(x2, fn, w[2]), n);
  } else {
    const int c = wrap_any(cell[p], n * n * n);
    const int nn = n * n;
    const int ci = c / nn, cj = (c / n) - ci * n, ck = c - (c / n) * n;
    first[0] = axis_off<MAS>(ci, x0, w[0]);
    first[1] = axis_off<MAS>(cj, x1, w[1]);
    first[2] = axis_off<MAS>(ck, x2, w[2]);
  }
}

template <int MAS, int PK>
__global__ __launch_bounds__(kThreads) void k_deposit_atomic(const float *__restrict__ pos,
                                                             const int32_t *__restrict__ cell,
                                                             int64_t np, int n, float mass,
                                                             float *__restrict__ rho) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= np) return;
  int first[3];
  float w[3][MAS];
  particle_support<MAS, PK>(pos, cell, p, n, first, w);
  int iy[MAS], iz[MAS];
#pragma unroll
  for (int b = 0; b < MAS; ++b) {
    iy[b] = wrap_index(first[1] + b, n);
    iz[b] = wrap_index(first[2] + b, n);
  }
#pragma unroll
  for (int a = 0; a < MAS; ++a) {
    const size_t ia = (size_t)wrap_index(first[0] + a, n) * n;
    const float wa = mass * w[0][a];
#pragma unroll
    for (int b = 0; b < MAS; ++b) {
      const size_t row = (ia + iy[b]) * n;
      const float wab = wa * w[1][b];
#pragma unroll
      for (int c = 0; c < MAS; ++c) unsafeAtomicAdd(&rho[row + iz[c]], wab * w[2][c]);
    }
  }
}

template <int MAS, int PK>
__global__ __launch_bounds__(kThreads) void k_interp(const float *__restrict__ pos,
                                                     const int32_t *__restrict__ cell,
                                                     int64_t np, int n,
                                                     const float *__restrict__ g,
                                                     float *__restrict__ acc,
                                                     float *__restrict__ vel, float kick) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= np) return;
  int first[3];
  float w[3][MAS];
  particle_support<MAS, PK>(pos, cell, p, n, first, w);
  int iy[MAS], iz[MAS];
#pragma unroll
  for (int b = 0; b < MAS; ++b) {
    iy[b] = wrap_index(first[1] + b, n);
    iz[b] = wrap_index(first[2] + b, n);
  }
  float ax = 0.f, ay = 0.f, az = 0.f;
#pragma unroll
  for (int a = 0; a < MAS; ++a) {
    const size_t ia = (size_t)wrap_index(first[0] + a, n) * n;
#pragma unroll
    for (int b = 0; b < MAS; ++b) {
      const size_t row = (ia + iy[b]) * n;
      const float wab = w[0][a] * w[1][b];
#pragma unroll
      for (int c = 0; c < MAS; ++c) {
        const float *gc = g + 3 * (row + iz[c]);
        const float wc = wab * w[2][c];
        ax = fmaf(wc, gc[0], ax);
        ay = fmaf(wc, gc[1], ay);
        az = fmaf(wc, gc[2], az);
      }
    }
  }
  if (acc) {
    acc[3 * p + 0] = ax;
    acc[3 * p + 1] = ay;
    acc[3 * p + 2] = az;
  }
  if (vel) {
    vel[3 * p + 0] = fmaf(kick, ax, vel[3 * p + 0]);
    vel[3 * p + 1] = fmaf(kick, ay, vel[3 * p + 1]);
    vel[3 * p + 2] = fmaf(kick, az, vel[3 * p + 2]);
  }
}

// Wrap a box-unit coordinate into [0, 1); -0.0 and values that round to 1.0 map to 0.
__device__ __forceinline__ float wrap_unit(float x) {
  x = x - floorf(x);
  return (x >= 1.0f) ? 0.0f : x;
}

// v += kick * acc (when acc != NULL); x += dt * v, wrapped (box) or carried (cell offset).
template <int PK>
__global__ __launch_bounds__(kThreads) void k_kick_drift(float *__restrict__ pos,
                                                         int32_t *__restrict__ cell,
                                                         float *__restrict__ vel,
                                                         const float *__restrict__ acc,
                                                         int64_t np, int n, float kick,
                                                         float dt) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= np) return;
  float v[3], x[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    v[d] = vel[3 * p + d];
    if (acc) v[d] = fmaf(kick, acc[3 * p + d], v[d]);
    x[d] = pos[3 * p + d];
  }
  if constexpr (PK == PM_POS_BOX) {
#pragma unroll
    for (int d = 0; d < 3; ++d) x[d] = wrap_unit(fmaf(dt, v[d], x[d]));
  } else {
    const float scale = dt * (float)n;
    const int c = wrap_any(cell[p], n * n * n);
    const int nn = n * n;
    int ci[3] = {c / nn, (c / n) - (c / nn) * n, c - (c / n) * n};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      float o = fmaf(scale, v[d], x[d]);
      float fl = floorf(o);
      o -= fl;
      if (o >= 1.0f) {
        o = 0.0f;
        fl += 1.0f;
      }
      int q = (ci[d] + (int)fl) % n;
      ci[d] = q < 0 ? q + n : q;
      x[d] = o;
    }
    cell[p] = (ci[0] * n + ci[1]) * n + ci[2];
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    vel[3 * p + d] = v[d];
    pos[3 * p + d] = x[d];
  }
}

// ------------------------------------------------------------------ counting sort

// Cell containing each particle; histogram of cells.
template <int PK>
__global__ __launch_bounds__(kThreads) void k_cell_hist(const float *__restrict__ pos,
                                                        const int32_t *__restrict__ cell,
                                                        int64_t np, int n,
                                                        int32_t *__restrict__ pcell,
                                                        int32_t *__restrict__ count) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= np) return;
  int c;
  if constexpr (PK == PM_POS_BOX) {
    const float fn = (float)n;
    int q[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int i = (int)floorf(pos[3 * p + d] * fn);
      q[d] = wrap_any(i, n);
    }
    c = (q[0] * n + q[1]) * n + q[2];
  } else {
    c = wrap_any(cell[p], n * n * n);
  }
  pcell[p] = c;
  atomicAdd(&count[c], 1);
}

__global__ __launch_bounds__(kThreads) void k_scatter_perm(const int32_t *__restrict__ pcell,
                                                           int64_t np,
                                                           int32_t *__restrict__ cursor,
                                                           int32_t *__restrict__ perm) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= np) return;
  const int slot = atomicAdd(&cursor[pcell[p]], 1);
  perm[slot] = (int32_t)p;
}

// Exclusive scan of `count` (len entries) into `start`, in three passes.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ int block_exclusive_scan(int v, int *lds, int &total) {
  // inclusive scan within the wave, then across waves through LDS
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds[wave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int i = 0; i < kScanThreads / 64; ++i) {
      int t = lds[i];
      lds[i] = acc;
      acc += t;
    }
    lds[kScanThreads / 64] = acc;
  }
  __syncthreads();
  total = lds[kScanThreads / 64];
  const int r = x - v + lds[wave];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int32_t *__restrict__ in,
                                                              int64_t len,
                                                              int32_t *__restrict__ partial) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int s = 0;
  for (int i = threadIdx.x; i < kScanTile; i += kScanThreads) {
    int64_t idx = base + i;
    if (idx < len) s += in[idx];
  }
  __shared__ int lds[kScanThreads / 64 + 1];
  int total;
  block_exclusive_scan(s, lds, total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_partials(int32_t *__restrict__ partial,
                                                                int nblocks) {
  __shared__ int lds[kScanThreads / 64 + 1];
  int carry = 0;
  for (int base = 0; base < nblocks; base += kScanThreads) {
    const int i = base + threadIdx.x;
    const int v = (i < nblocks) ? partial[i] : 0;
    int total;
    const int ex = block_exclusive_scan(v, lds, total);
    if (i < nblocks) partial[i] = ex + carry;
    carry += total;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const int32_t *__restrict__ in,
                                                             int64_t len,
                                                             const int32_t *__restrict__ partial,
                                                             int32_t *__restrict__ out,
                                                             int32_t *__restrict__ out2) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int v[kScanItems];
  int s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < len) ? in[base + i] : 0;
    s += v[i];
  }
  __shared__ int lds[kScanThreads / 64 + 1];
  int total;
  int ex = block_exclusive_scan(s, lds, total) + partial[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < len) {
      out[base + i] = ex;
      if (out2) out2[base + i] = ex;
    }
    ex += v[i];
  }
}

// ------------------------------------------------------------------ gathered deposit

// Fixed point used to sum window values: 2^40 units per particle weight.
constexpr double kFixScale = 1099511627776.0;  // 2^40

template <int MAS>
__device__ __forceinline__ float window_sep(float s) {
  const float a = fabsf(s);
  if constexpr (MAS == 3) {
    if (a < 0.5f) return 0.75f - a * a;
    const float b = 1.5f - a;
    return a < 1.5f ? 0.5f * b * b : 0.0f;
  } else {
    return a < 1.0f ? 1.0f - a : 0.0f;
  }
}

// One thread per cell: sums the window values of the particles bucketed in the
// 27 neighbouring cells. The separation along an axis is (q - c) + o - 1/2, where
// q - c in {-1, 0, 1} is the periodic cell difference and o the particle's in-cell
// offset. Sums are exact in 64-bit fixed point, hence independent of order.
template <int MAS, int PK>
__global__ __launch_bounds__(kThreads) void k_deposit_pull(const float *__restrict__ pos,
                                                           const int32_t *__restrict__ start,
                                                           const int32_t *__restrict__ perm,
                                                           int n, float mass,
                                                           float *__restrict__ rho) {
  const int64_t ncell = (int64_t)n * n * n;
  const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c >= ncell) return;
  const int ci = (int)(c / ((int64_t)n * n)), cj = (int)((c / n) % n), ck = (int)(c % n);
  const float fn = (float)n;
  long long acc = 0;
  for (int di = -1; di <= 1; ++di) {
    const int qi = wrap_index(ci + di, n);
    for (int dj = -1; dj <= 1; ++dj) {
      const int qj = wrap_index(cj + dj, n);
      for (int dk = -1; dk <= 1; ++dk) {
        const int qk = wrap_index(ck + dk, n);
        const int q = (qi * n + qj) * n + qk;
        const int s0 = start[q], s1 = start[q + 1];
        for (int s = s0; s < s1; ++s) {
          const int p = perm[s];
          float o[3];
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const float x = pos[3 * (int64_t)p + d];
            if constexpr (PK == PM_POS_BOX) {
              const float u = x * fn;
              o[d] = u - floorf(u);
            } else {
              o[d] = x;
            }
          }
          const float w = window_sep<MAS>((float)di + o[0] - 0.5f) *
                          window_sep<MAS>((float)dj + o[1] - 0.5f) *
                          window_sep<MAS>((float)dk + o[2] - 0.5f);
          acc += (long long)__double2ll_rn((double)w * kFixScale);
        }
      }
    }
  }
  rho[c] = (float)((double)acc * (1.0 / kFixScale) * (double)mass);
}

inline unsigned blocks_for(int64_t count, int threads) {
  return (unsigned)((count + threads - 1) / threads);
}

}  // namespace

hipError_t launch_deposit_atomic(const float *pos, const int32_t *cell, int64_t np, int poskind,
                                 int mas, int n, float mass, float *rho, hipStream_t s) {
  if (np == 0) return hipSuccess;
  const unsigned nb = blocks_for(np, kThreads);
  if (mas == PM_TSC) {
    if (poskind == PM_POS_BOX)
      k_deposit_atomic<3, PM_POS_BOX><<<nb, kThreads, 0, s>>>(pos, cell, np, n, mass, rho);
    else
      k_deposit_atomic<3, PM_POS_CELLOFF><<<nb, kThreads, 0, s>>>(pos, cell, np, n, mass, rho);
  } else {
    if (poskind == PM_POS_BOX)
      k_deposit_atomic<2, PM_POS_BOX><<<nb, kThreads, 0, s>>>(pos, cell, np, n, mass, rho);
    else
      k_deposit_atomic<2, PM_POS_CELLOFF><<<nb, kThreads, 0, s>>>(pos, cell, np, n, mass, rho);
  }
  return hipGetLastError();
}

hipError_t launch_interp(const float *pos, const int32_t *cell, int64_t np, int poskind, int mas,
                         int n, const float *g, float *acc, float *vel, float kick,
                         hipStream_t s) {
  if (np == 0) return hipSuccess;
  const unsigned nb = blocks_for(np, kThreads);
  if (mas == PM_TSC) {
    if (poskind == PM_POS_BOX)
      k_interp<3, PM_POS_BOX><<<nb, kThreads, 0, s>>>(pos, cell, np, n, g, acc, vel, kick);
    else
      k_interp<3, PM_POS_CELLOFF><<<nb, kThreads, 0, s>>>(pos, cell, np, n, g, acc, vel, kick);
  } else {
    if (poskind == PM_POS_BOX)
      k_interp<2, PM_POS_BOX><<<nb, kThreads, 0, s>>>(pos, cell, np, n, g, acc, vel, kick);
    else
      k_interp<2, PM_POS_CELLOFF><<<nb, kThreads, 0, s>>>(pos, cell, np, n, g, acc, vel, kick);
  }
  return hipGetLastError();
}

hipError_t launch_kick_drift(float *pos, int32_t *cell, float *vel, const float *acc, int64_t np,
                             int poskind, int n, float kick, float dt, hipStream_t s) {
  if (np == 0) return hipSuccess;
  const unsigned nb = blocks_for(np, kThreads);
  if (poskind == PM_POS_BOX)
    k_kick_drift<PM_POS_BOX><<<nb, kThreads, 0, s>>>(pos, cell, vel, acc, np, n, kick, dt);
  else
    k_kick_drift<PM_POS_CELLOFF><<<nb, kThreads, 0, s>>>(pos, cell, vel, acc, np, n, kick, dt);
  return hipGetLastError();
}

hipError_t launch_sort_by_cell(pm_ctx *ctx, const float *pos, const int32_t *cell, int64_t np,
                               int poskind, hipStream_t s) {
  const int n = ctx->n;
  const int64_t ncell = (int64_t)n * n * n;
  const int64_t len = ncell + 1;
  hipError_t e = hipMemsetAsync(ctx->cell_count, 0, sizeof(int32_t) * len, s);
  if (e != hipSuccess) return e;
  if (np > 0) {
    const unsigned nb = blocks_for(np, kThreads);
    if (poskind == PM_POS_BOX)
      k_cell_hist<PM_POS_BOX><<<nb, kThreads, 0, s>>>(pos, cell, np, n, ctx->pcell,
                                                        ctx->cell_count);
    else
      k_cell_hist<PM_POS_CELLOFF><<<nb, kThreads, 0, s>>>(pos, cell, np, n, ctx->pcell,
                                                            ctx->cell_count);
  }
  const unsigned nblk = blocks_for(len, kScanTile);
  k_scan_reduce<<<nblk, kScanThreads, 0, s>>>(ctx->cell_count, len, ctx->scan_partial);
  k_scan_partials<<<1, kScanThreads, 0, s>>>(ctx->scan_partial, (int)nblk);
  // start = exclusive scan; count becomes the scatter cursor (a copy of start)
  k_scan_apply<<<nblk, kScanThreads, 0, s>>>(ctx->cell_count, len, ctx->scan_partial,
                                             ctx->cell_start, ctx->cell_count);
  if (np > 0)
    k_scatter_perm<<<blocks_for(np, kThreads), kThreads, 0, s>>>(ctx->pcell, np,
                                                                  ctx->cell_count, ctx->perm);
  return hipGetLastError();
}

int64_t scan_blocks_needed(int64_t len) { return (len + kScanTile - 1) / kScanTile; }

hipError_t launch_deposit_pull(pm_ctx *ctx, const float *pos, int64_t np, int poskind, int mas,
                               float mass, float *rho, hipStream_t s) {
  (void)np;
  const int n = ctx->n;
  const int64_t ncell = (int64_t)n * n * n;
  const unsigned nb = blocks_for(ncell, kThreads);
  if (mas == PM_TSC) {
    if (poskind == PM_POS_BOX)
      k_deposit_pull<3, PM_POS_BOX><<<nb, kThreads, 0, s>>>(pos, ctx->cell_start, ctx->perm, n,
                                                              mass, rho);
    else
      k_deposit_pull<3, PM_POS_CELLOFF><<<nb, kThreads, 0, s>>>(pos, ctx->cell_start, ctx->perm,
                                                                  n, mass, rho);
  } else {
    if (poskind == PM_POS_BOX)
      k_deposit_pull<2, PM_POS_BOX><<<nb, kThreads, 0, s>>>(pos, ctx->cell_start, ctx->perm, n,
                                                              mass, rho);
    else
      k_deposit_pull<2, PM_POS_CELLOFF><<<nb, kThreads, 0, s>>>(pos, ctx->cell_start, ctx->perm,
                                                                  n, mass, rho);
  }
  return hipGetLastError();
}
