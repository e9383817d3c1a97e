// Batched ensembles: many independent periodic boxes of different grid sizes
// advanced together (the paper's stated purpose is producing large suites of
// simulations). Every stage of the kick-drift-kick step is ONE launch for the
// whole batch: particle arrays and grids of all boxes are packed into arenas,
// and each launch walks a work list of (box, block) items with a persistent
// grid (each workgroup strides through the list), so small boxes do not pay a
// launch each and the GPU stays full. Per-step scalars (time step, source
// coefficient, warm-start factor) are read from a device table indexed by a
// device step counter, so one captured step graph can be replayed for every
// step. Positions are box units; window, solver and gradient follow the same
// definitions as the single-box kernels (Sects. 3.4-3.7).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "coarse_solve.h"
#include "deposit_chunk.h"
#include "internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kCoarseThreads = 1024;
constexpr int kCoarseMax = 8000;
constexpr int kPersistCap = 4096;  // workgroups of a persistent launch (>> 256 CUs)
constexpr int kGraphSteps = 1024;  // step-table entries reserved when a step is captured

struct BoxDev {
  int n;                          // cells per side of the finest level
  int nlev;                       // multigrid levels; level nlev-1 is solved in LDS
  int lattice;                    // deposit chunks are lattice blocks (np = n^3, 16 | n)
  int pad;
  int64_t p0, np;                 // rows of the packed particle arrays
  int64_t c0;                     // offset of the box in the level-0 arenas (rho, phi, g)
  int64_t lo[PM_MAX_LEVELS];      // offset of level l >= 1 in the level arenas (u, f)
};

struct StepDev {
  float half;   // tau / 2
  float dt;     // tau
  float coef;   // (3/2) Omega_m a1 mu(a1) (source coefficient at the end of the step)
  float warm;   // warm-start factor (a1 / a0)^2, or 1
};

__device__ __forceinline__ int wrap_index(int i, int n) {
  i += (i < 0) ? n : 0;
  i -= (i >= n) ? n : 0;
  return i;
}

__device__ __forceinline__ int wrap_any(int i, int n) {
  const int r = i % n;
  return r < 0 ? r + n : r;
}

__device__ __forceinline__ float wrap_unit(float x) {
  x = x - floorf(x);
  return (x >= 1.0f) ? 0.0f : x;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

template <int T>
__device__ __forceinline__ double block_sum(double v, double *lds) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < T / 64; ++w) s += lds[w];
  return s;
}

template <int MAS>
__device__ __forceinline__ int axis_box(float x, float fn, float *w) {
  const float u = x * fn;
  if constexpr (MAS == 3) {
    const float fl = floorf(u);
    const float d = u - fl - 0.5f;
    const float a = 0.5f - d, b = 0.5f + d;
    w[0] = 0.5f * a * a;
    w[1] = 0.75f - d * d;
    w[2] = 0.5f * b * b;
    return (int)fl - 1;
  } else {
    const float t = u - 0.5f;
    const float fl = floorf(t);
    const float d = t - fl;
    w[0] = 1.0f - d;
    w[1] = d;
    return (int)fl;
  }
}

// ------------------------------------------------------------------ particle stages

// v += (tau/2) acc;  x = wrap(x + tau v)   (all particles of all boxes)
__global__ __launch_bounds__(kThreads) void kb_kick_drift(float *__restrict__ pos,
                                                          float *__restrict__ vel,
                                                          const float *__restrict__ acc,
                                                          int64_t count3,
                                                          const StepDev *__restrict__ steps,
                                                          const int *__restrict__ ctr) {
  const StepDev st = steps[*ctr];
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < count3; t += stride) {
    const float v = fmaf(st.half, acc[t], vel[t]);
    vel[t] = v;
    pos[t] = wrap_unit(fmaf(st.dt, v, pos[t]));
  }
}

// Slots of one deposit chunk of a box: an 8 x 16 x 16 block of its particle lattice
// (particles that started on the lattice stay spatially coherent for many steps), or
// 2048 consecutive rows.
struct BatchIndex {
  int64_t p0, end;
  int m, i0, j0, k0, lattice;
  __device__ int64_t ref() const {
    return lattice ? p0 + ((int64_t)i0 * m + j0) * m + k0 : p0;
  }
  __device__ int64_t operator()(int slot) const {
    if (lattice) {
      const int i = i0 + (slot >> 8), j = j0 + ((slot >> 4) & 15), k = k0 + (slot & 15);
      return p0 + ((int64_t)i * m + j) * m + k;
    }
    const int64_t p = p0 + slot;
    return p < end ? p : -1;
  }
};

// rho_box += w W(u_p - c - 1/2), w = n^3 / np of the box: the chunked LDS deposit
// (deposit_chunk.h) for every (box, chunk) item
template <int MAS>
__global__ __launch_bounds__(pm_chunk::kGThreads) void kb_deposit(
    const float *__restrict__ pos, const int2 *__restrict__ items, int nitems,
    const BoxDev *__restrict__ boxes, unsigned long long *__restrict__ fix) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    __syncthreads();  // the previous item's LDS tables are no longer read
    const int2 item = items[it];
    const BoxDev &bx = boxes[item.x];
    BatchIndex idx;
    idx.m = bx.n;
    idx.lattice = bx.lattice;
    idx.p0 = bx.p0;
    idx.end = bx.p0 + bx.np;
    if (bx.lattice) {
      const int cj = bx.n >> 4;  // chunks along j and k
      idx.i0 = 8 * (item.y / (cj * cj));
      idx.j0 = 16 * ((item.y / cj) % cj);
      idx.k0 = 16 * (item.y % cj);
    } else {
      idx.i0 = idx.j0 = idx.k0 = 0;
      idx.p0 = bx.p0 + (int64_t)item.y * pm_chunk::kGChunk;
    }
    pm_chunk::deposit_chunk<MAS, PM_POS_BOX, BatchIndex, true>(pos, nullptr, idx, bx.n, 0.0f,
                                                               nullptr, fix + bx.c0);
  }
}

// rho = w 2^-30 fix (w = n^3 / np of the box), fix = 0 for the next deposit, and the
// per-item FP64 partial sums of rho (fixed order), one item of cells at a time
__global__ __launch_bounds__(kThreads) void kb_fix_to_rho(unsigned long long *__restrict__ fix,
                                                          float *__restrict__ rho,
                                                          const int2 *__restrict__ items,
                                                          int nitems,
                                                          const BoxDev *__restrict__ boxes,
                                                          double *__restrict__ partial) {
  __shared__ double lds[kThreads / 64];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 item = items[it];
    const BoxDev &bx = boxes[item.x];
    const int64_t count = (int64_t)bx.n * bx.n * bx.n;
    const double scale = (double)count / (double)bx.np * (1.0 / 1073741824.0);
    const int64_t c = (int64_t)item.y * kThreads + threadIdx.x;
    double v = 0.0;
    if (c < count) {
      const unsigned long long q = fix[bx.c0 + c];
      fix[bx.c0 + c] = 0ull;
      const float r = (float)((double)q * scale);
      rho[bx.c0 + c] = r;
      v = (double)r;
    }
    const double sum = block_sum<kThreads>(v, lds);
    if (threadIdx.x == 0) partial[it] = sum;
  }
}

// acc = interp(g); v += (tau/2) acc (when kick)
template <int MAS>
__global__ __launch_bounds__(kThreads) void kb_interp(const float *__restrict__ pos,
                                                      const int2 *__restrict__ items, int nitems,
                                                      const BoxDev *__restrict__ boxes,
                                                      const float *__restrict__ g,
                                                      float *__restrict__ acc,
                                                      float *__restrict__ vel,
                                                      const StepDev *__restrict__ steps,
                                                      const int *__restrict__ ctr) {
  const float half = vel ? steps[*ctr].half : 0.0f;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 item = items[it];
    const BoxDev &bx = boxes[item.x];
    const int64_t lp = (int64_t)item.y * kThreads + threadIdx.x;
    if (lp >= bx.np) continue;
    const int64_t p = bx.p0 + lp;
    const int n = bx.n;
    const float fn = (float)n;
    float w[3][MAS];
    int f[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) f[d] = wrap_any(axis_box<MAS>(pos[3 * p + d], fn, w[d]), n);
    const float *gb = g + 3 * bx.c0;
    float ax = 0.f, ay = 0.f, az = 0.f;
#pragma unroll
    for (int a = 0; a < MAS; ++a) {
      const size_t ia = (size_t)wrap_index(f[0] + a, n) * n;
#pragma unroll
      for (int b = 0; b < MAS; ++b) {
        const size_t row = (ia + wrap_index(f[1] + b, n)) * n;
        const float wab = w[0][a] * w[1][b];
#pragma unroll
        for (int c = 0; c < MAS; ++c) {
          const float *gc = gb + 3 * (row + wrap_index(f[2] + c, n));
          const float wc = wab * w[2][c];
          ax = fmaf(wc, gc[0], ax);
          ay = fmaf(wc, gc[1], ay);
          az = fmaf(wc, gc[2], az);
        }
      }
    }
    acc[3 * p + 0] = ax;
    acc[3 * p + 1] = ay;
    acc[3 * p + 2] = az;
    if (vel) {
      vel[3 * p + 0] = fmaf(half, ax, vel[3 * p + 0]);
      vel[3 * p + 1] = fmaf(half, ay, vel[3 * p + 1]);
      vel[3 * p + 2] = fmaf(half, az, vel[3 * p + 2]);
    }
  }
}

// ------------------------------------------------------------------ grid stages

__global__ __launch_bounds__(kThreads) void kb_fill(float *__restrict__ x, int64_t count, float v) {
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < count; t += stride) x[t] = v;
}

// u *= warm factor of the step (growth rescaling of the previous potential)
__global__ __launch_bounds__(kThreads) void kb_scale(float *__restrict__ x, int64_t count,
                                                     const StepDev *__restrict__ steps,
                                                     const int *__restrict__ ctr) {
  const float s = steps[*ctr].warm;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < count; t += stride) x[t] *= s;
}

// Per-item FP64 partial sums of a level-0 field (fixed order: deterministic).
__global__ __launch_bounds__(kThreads) void kb_sum_partial(const float *__restrict__ x,
                                                           const int2 *__restrict__ items,
                                                           int nitems,
                                                           const BoxDev *__restrict__ boxes,
                                                           double *__restrict__ partial) {
  __shared__ double lds[kThreads / 64];
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 item = items[it];
    const BoxDev &bx = boxes[item.x];
    const int64_t count = (int64_t)bx.n * bx.n * bx.n;
    const int64_t c = (int64_t)item.y * kThreads + threadIdx.x;
    const double v = c < count ? (double)x[bx.c0 + c] : 0.0;
    const double s = block_sum<kThreads>(v, lds);
    if (threadIdx.x == 0) partial[it] = s;
  }
}

// mean[b] = sum of the box's partials / n^3 (one workgroup per box)
__global__ __launch_bounds__(kThreads) void kb_sum_final(const double *__restrict__ partial,
                                                         const int *__restrict__ range,
                                                         const BoxDev *__restrict__ boxes,
                                                         float *__restrict__ mean) {
  __shared__ double lds[kThreads / 64];
  const int b = blockIdx.x;
  double s = 0.0;
  for (int i = range[b] + threadIdx.x; i < range[b + 1]; i += kThreads) s += partial[i];
  s = block_sum<kThreads>(s, lds);
  if (threadIdx.x == 0) {
    const double n = boxes[b].n;
    mean[b] = (float)(s / (n * n * n));
  }
}

__global__ __launch_bounds__(kThreads) void kb_subtract_mean(float *__restrict__ x,
                                                             const int2 *__restrict__ items,
                                                             int nitems,
                                                             const BoxDev *__restrict__ boxes,
                                                             const float *__restrict__ mean) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 item = items[it];
    const BoxDev &bx = boxes[item.x];
    const int64_t c = (int64_t)item.y * kThreads + threadIdx.x;
    if (c < (int64_t)bx.n * bx.n * bx.n) x[bx.c0 + c] -= mean[item.x];
  }
}

// View of one box's level: u, f (right-hand side read as scale * (f - mean)).
struct LevelView {
  float *u;
  const float *f;
  float scale, mean;
  int n;
};

__device__ __forceinline__ LevelView level_view(const BoxDev &bx, int l, float *phi,
                                                const float *rho, float *lu, const float *lf,
                                                float coef, const float *rmean, int b) {
  LevelView v;
  if (l == 0) {
    v.u = phi + bx.c0;
    v.f = rho + bx.c0;
    v.scale = coef;
    v.mean = rmean[b];
    v.n = bx.n;
  } else {
    v.u = lu + bx.lo[l];
    v.f = lf + bx.lo[l];
    v.scale = 1.0f;
    v.mean = 0.0f;
    v.n = bx.n >> l;
  }
  return v;
}

struct Arenas {
  float *phi;
  const float *rho;
  float *lu, *lf;
  const float *rmean;
  const StepDev *steps;
  const int *ctr;
};

// u = -h^2 scale (f - mean) / 6 on level 0 (first solve of a run)
__global__ __launch_bounds__(kThreads) void kb_jacobi0(Arenas A, const int2 *__restrict__ items,
                                                       int nitems,
                                                       const BoxDev *__restrict__ boxes) {
  const float coef = A.steps[*A.ctr].coef;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 item = items[it];
    const BoxDev &bx = boxes[item.x];
    const LevelView v = level_view(bx, 0, A.phi, A.rho, A.lu, A.lf, coef, A.rmean, item.x);
    const int64_t c = (int64_t)item.y * kThreads + threadIdx.x;
    if (c >= (int64_t)v.n * v.n * v.n) continue;
    const float h = 1.0f / (float)v.n;
    v.u[c] = (-(h * h) / 6.0f) * (v.scale * (v.f[c] - v.mean));
  }
}

// One colour of a red-black Gauss-Seidel sweep on level l of every listed box.
// Tile shape (chosen by the tuner): a thread owns one k-position of its colour in CPT
// consecutive rows j of one plane i (CPT divides n), so a wavefront still reads
// contiguous runs along k.
template <int CPT>
__global__ __launch_bounds__(kThreads) void kb_rbgs_half(Arenas A, const int2 *__restrict__ items,
                                                         int nitems,
                                                         const BoxDev *__restrict__ boxes, int l,
                                                         float omega, int colour) {
  const float coef = A.steps[*A.ctr].coef;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 item = items[it];
    const BoxDev &bx = boxes[item.x];
    const LevelView v = level_view(bx, l, A.phi, A.rho, A.lu, A.lf, coef, A.rmean, item.x);
    const int n = v.n, half = n >> 1;
    const float h = 1.0f / (float)n, h2 = h * h;
    const size_t nn = (size_t)n * n;
    const unsigned tid = (unsigned)item.y * kThreads + threadIdx.x;
    const unsigned rg = tid / (unsigned)half;  // row group: CPT rows j of plane i
    const int k2 = (int)(tid - rg * (unsigned)half);
    const unsigned groups = (unsigned)(n / CPT);
    if (rg >= (unsigned)n * groups) continue;
    const int i = (int)(rg / groups), j0 = (int)(rg - (unsigned)i * groups) * CPT;
    const size_t ci = (size_t)i * nn;
    const size_t cip = (size_t)wrap_index(i + 1, n) * nn, cim = (size_t)wrap_index(i - 1, n) * nn;
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int j = j0 + q;
      const int k = 2 * k2 + ((i + j + colour) & 1);
      const size_t cj = (size_t)j * n;
      const size_t c = ci + cj + k;
      const float fv = v.scale * (v.f[c] - v.mean);
      const float nb = v.u[cip + cj + k] + v.u[cim + cj + k] +
                       v.u[ci + (size_t)wrap_index(j + 1, n) * n + k] +
                       v.u[ci + (size_t)wrap_index(j - 1, n) * n + k] +
                       v.u[ci + cj + wrap_index(k + 1, n)] + v.u[ci + cj + wrap_index(k - 1, n)];
      const float gs = (nb - h2 * fv) * (1.0f / 6.0f);
      v.u[c] = (omega == 1.0f) ? gs : fmaf(omega, gs - v.u[c], v.u[c]);
    }
  }
}

__device__ __forceinline__ float residual_at(const LevelView &v, int i, int j, int k,
                                             float inv_h2) {
  const int n = v.n;
  const size_t nn = (size_t)n * n;
  const size_t ci = (size_t)i * nn, cj = (size_t)j * n;
  const size_t c = ci + cj + k;
  const float uc = v.u[c];
  const float lap = (v.u[(size_t)wrap_index(i + 1, n) * nn + cj + k] - uc) +
                    (v.u[(size_t)wrap_index(i - 1, n) * nn + cj + k] - uc) +
                    (v.u[ci + (size_t)wrap_index(j + 1, n) * n + k] - uc) +
                    (v.u[ci + (size_t)wrap_index(j - 1, n) * n + k] - uc) +
                    (v.u[ci + cj + wrap_index(k + 1, n)] - uc) +
                    (v.u[ci + cj + wrap_index(k - 1, n)] - uc);
  return v.scale * (v.f[c] - v.mean) - lap * inv_h2;
}

__device__ __forceinline__ void decode3(unsigned t, unsigned n, int &i, int &j, int &k) {
  const unsigned r = t / n;
  k = (int)(t - r * n);
  i = (int)(r / n);
  j = (int)(r - (unsigned)i * n);
}

// r = f - L u on level l of every box that has a level l+1, into a scratch arena (the
// force-grid arena, idle during the solve) at the box's level-0 offset.
__global__ __launch_bounds__(kThreads) void kb_residual(Arenas A, const int2 *__restrict__ items,
                                                        int nitems,
                                                        const BoxDev *__restrict__ boxes, int l,
                                                        float *__restrict__ rbuf) {
  const float coef = A.steps[*A.ctr].coef;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 item = items[it];
    const BoxDev &bx = boxes[item.x];
    const LevelView v = level_view(bx, l, A.phi, A.rho, A.lu, A.lf, coef, A.rmean, item.x);
    const unsigned n = (unsigned)v.n;
    const unsigned t = (unsigned)item.y * kThreads + threadIdx.x;
    if (t >= n * n * n) continue;
    int i, j, k;
    decode3(t, n, i, j, k);
    rbuf[bx.c0 + t] = residual_at(v, i, j, k, (float)n * (float)n);
  }
}

// Restriction of the level-l residual to level l+1 (full weighting (1,3,3,1)/8 per
// axis, or the 8-child average), with the coarse starting guess -H^2 f_H / 6.
template <int KIND>
__global__ __launch_bounds__(kThreads) void kb_restrict(Arenas A, const int2 *__restrict__ items,
                                                        int nitems,
                                                        const BoxDev *__restrict__ boxes, int l,
                                                        const float *__restrict__ rbuf) {
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 item = items[it];
    const BoxDev &bx = boxes[item.x];
    const int n = bx.n >> l;
    const unsigned nc = (unsigned)n >> 1;
    const unsigned t = (unsigned)item.y * kThreads + threadIdx.x;
    if (t >= nc * nc * nc) continue;
    int I, J, K;
    decode3(t, nc, I, J, K);
    const float *r = rbuf + bx.c0;
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
          const float wab = w[a] * w[b];
          const float row = fmaf(w[0], r[rj + kk[0]], fmaf(w[1], r[rj + kk[1]],
                                 fmaf(w[2], r[rj + kk[2]], w[3] * r[rj + kk[3]])));
          acc = fmaf(wab, row, acc);
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
    const float H = 1.0f / (float)nc;
    A.lf[bx.lo[l + 1] + t] = acc;
    A.lu[bx.lo[l + 1] + t] = (-(H * H) / 6.0f) * acc;
  }
}

// u_l += P u_{l+1} (trilinear: 3/4 nearest coarse centre, 1/4 the next, per axis);
// one thread per coarse cell reads its 27 coarse neighbours once and updates its 8
// fine children (k-pairs as float2)
__global__ __launch_bounds__(kThreads) void kb_prolong_add(Arenas A, const int2 *__restrict__ items,
                                                           int nitems,
                                                           const BoxDev *__restrict__ boxes,
                                                           int l) {
  const float near = 0.75f, far = 0.25f;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 item = items[it];
    const BoxDev &bx = boxes[item.x];
    const int n = bx.n >> l, c = n >> 1;
    const unsigned t = (unsigned)item.y * kThreads + threadIdx.x;
    if (t >= (unsigned)c * c * c) continue;
    float *u = l == 0 ? A.phi + bx.c0 : A.lu + bx.lo[l];
    const float *vc = A.lu + bx.lo[l + 1];
    int I, J, K;
    decode3(t, (unsigned)c, I, J, K);
    const int ix[3] = {wrap_index(I - 1, c), I, wrap_index(I + 1, c)};
    const int jx[3] = {wrap_index(J - 1, c), J, wrap_index(J + 1, c)};
    const int kx[3] = {wrap_index(K - 1, c), K, wrap_index(K + 1, c)};
    float ek[3][3], ok[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const float *row = vc + ((size_t)ix[a] * c + jx[b]) * c;
        const float vm = row[kx[0]], v0 = row[kx[1]], vp = row[kx[2]];
        ek[a][b] = near * v0 + far * vm;
        ok[a][b] = near * v0 + far * vp;
      }
    const size_t nn = (size_t)n * n;
#pragma unroll
    for (int ai = 0; ai < 2; ++ai) {
      const int af = ai ? 2 : 0;
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        const int bf = bj ? 2 : 0;
        const float se = near * (near * ek[1][1] + far * ek[1][bf]) +
                         far * (near * ek[af][1] + far * ek[af][bf]);
        const float so = near * (near * ok[1][1] + far * ok[1][bf]) +
                         far * (near * ok[af][1] + far * ok[af][bf]);
        float2 *dst = reinterpret_cast<float2 *>(u + (size_t)(2 * I + ai) * nn +
                                                 (size_t)(2 * J + bj) * n + 2 * K);
        float2 cur = *dst;
        cur.x += se;
        cur.y += so;
        *dst = cur;
      }
    }
  }
}

// Coarsest level of every box, one workgroup per box, in LDS (coarse_solve.h).
__global__ __launch_bounds__(kCoarseThreads) void kb_coarse_solve(Arenas A,
                                                                  const BoxDev *__restrict__ boxes) {
  __shared__ float re[kCoarseMax];
  __shared__ float im[kCoarseMax];
  __shared__ float tc[pm_coarse::kMaxN], ts[pm_coarse::kMaxN];
  const int b = blockIdx.x;
  const BoxDev &bx = boxes[b];
  const float coef = A.steps[*A.ctr].coef;
  const LevelView v = level_view(bx, bx.nlev - 1, A.phi, A.rho, A.lu, A.lf, coef, A.rmean, b);
  const float h = 1.0f / (float)v.n;
  pm_coarse::solve_any(v.u, v.f, v.scale, v.mean, v.n, h * h, re, im, tc, ts);
}

// Per-item partial sums of |f - L u|^2 and |f|^2 on level 0 (convergence records).
__global__ __launch_bounds__(kThreads) void kb_residual_partial(Arenas A,
                                                                const int2 *__restrict__ items,
                                                                int nitems,
                                                                const BoxDev *__restrict__ boxes,
                                                                double *__restrict__ partial) {
  __shared__ double lds[kThreads / 64];
  const float coef = A.steps[*A.ctr].coef;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 item = items[it];
    const BoxDev &bx = boxes[item.x];
    const LevelView v = level_view(bx, 0, A.phi, A.rho, A.lu, A.lf, coef, A.rmean, item.x);
    const int n = v.n;
    const unsigned t = (unsigned)item.y * kThreads + threadIdx.x;
    double r2 = 0.0, f2 = 0.0;
    if (t < (unsigned)n * n * n) {
      int i, j, k;
      decode3(t, (unsigned)n, i, j, k);
      const double r = residual_at(v, i, j, k, (float)n * (float)n);
      const double fv = v.scale * (v.f[t] - v.mean);
      r2 = r * r;
      f2 = fv * fv;
    }
    r2 = block_sum<kThreads>(r2, lds);
    f2 = block_sum<kThreads>(f2, lds);
    if (threadIdx.x == 0) {
      partial[2 * it] = r2;
      partial[2 * it + 1] = f2;
    }
  }
}

__global__ __launch_bounds__(kThreads) void kb_residual_final(const double *__restrict__ partial,
                                                              const int *__restrict__ range,
                                                              double *__restrict__ out) {
  __shared__ double lds[kThreads / 64];
  const int b = blockIdx.x;
  double r = 0.0, f = 0.0;
  for (int i = range[b] + threadIdx.x; i < range[b + 1]; i += kThreads) {
    r += partial[2 * i];
    f += partial[2 * i + 1];
  }
  r = block_sum<kThreads>(r, lds);
  f = block_sum<kThreads>(f, lds);
  if (threadIdx.x == 0) out[b] = f > 0.0 ? sqrt(r / f) : 0.0;
}

// g = -grad phi, 5-point central difference. Tile shape: a thread owns one k-position in
// CPT consecutive rows j of one plane i and slides a window of CPT + 4 values along j.
template <int CPT>
__global__ __launch_bounds__(kThreads) void kb_gradient(const float *__restrict__ phi,
                                                        const int2 *__restrict__ items,
                                                        int nitems,
                                                        const BoxDev *__restrict__ boxes,
                                                        float *__restrict__ g) {
  const float c1 = 2.0f / 3.0f, c2 = -1.0f / 12.0f;
  for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 item = items[it];
    const BoxDev &bx = boxes[item.x];
    const int n = bx.n;
    const float inv_h = (float)n;
    const float *u = phi + bx.c0;
    float *gb = g + 3 * bx.c0;
    const size_t nn = (size_t)n * n;
    const unsigned tid = (unsigned)item.y * kThreads + threadIdx.x;
    const unsigned rg = tid / (unsigned)n;
    const int k = (int)(tid - rg * (unsigned)n);
    const unsigned groups = (unsigned)(n / CPT);
    if (rg >= (unsigned)n * groups) continue;
    const int i = (int)(rg / groups), j0 = (int)(rg - (unsigned)i * groups) * CPT;
    const size_t ci = (size_t)i * nn;
    const size_t cp1 = (size_t)wrap_index(i + 1, n) * nn, cm1 = (size_t)wrap_index(i - 1, n) * nn;
    const size_t cp2 = (size_t)wrap_index(i + 2, n) * nn, cm2 = (size_t)wrap_index(i - 2, n) * nn;
    float col[CPT + 4];
#pragma unroll
    for (int q = 0; q < CPT + 4; ++q) col[q] = u[ci + (size_t)wrap_any(j0 - 2 + q, n) * n + k];
    const int kp1 = wrap_index(k + 1, n), km1 = wrap_index(k - 1, n);
    const int kp2 = wrap_index(k + 2, n), km2 = wrap_index(k - 2, n);
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int j = j0 + q;
      const size_t cj = (size_t)j * n;
      const size_t row = ci + cj;
      const float gx = fmaf(c1, u[cp1 + cj + k] - u[cm1 + cj + k], c2 * (u[cp2 + cj + k] - u[cm2 + cj + k]));
      const float gy = fmaf(c1, col[q + 3] - col[q + 1], c2 * (col[q + 4] - col[q]));
      const float gz = fmaf(c1, u[row + kp1] - u[row + km1], c2 * (u[row + kp2] - u[row + km2]));
      float *o = gb + 3 * (row + k);
      o[0] = -inv_h * gx;
      o[1] = -inv_h * gy;
      o[2] = -inv_h * gz;
    }
  }
}

__global__ void kb_set_counter(int *ctr, int v) { *ctr = v; }
__global__ void kb_advance_counter(int *ctr) { *ctr += 1; }

inline unsigned persist_grid(int64_t nitems) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(nitems, kPersistCap));
}

inline unsigned flat_grid(int64_t count) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((count + kThreads - 1) / kThreads,
                                                          kPersistCap));
}

}  // namespace

// ------------------------------------------------------------------ host side

struct pm_batch {
  int nboxes = 0;
  int device = 0;
  std::string err;
  std::vector<int> n;
  std::vector<int64_t> np, p_off, c_off;
  int64_t np_total = 0, ncell_total = 0, lev_total = 0;
  int maxlev = 0;
  std::vector<BoxDev> boxes_h;
  BoxDev *boxes = nullptr;
  // work lists packed into one device array
  struct List {
    int64_t off = 0;
    int count = 0;
  };
  std::vector<int2> items_h;
  int2 *items = nullptr;
  List part;                        // particle blocks
  List chunks;                      // deposit chunks (lattice blocks or runs of 2048 rows)
  List cells[PM_MAX_LEVELS];        // cell blocks of level l (boxes with nlev > l)
  List halfc[PM_MAX_LEVELS][3];     // red-black half-sweep blocks of level l, per tile shape
  List finer[PM_MAX_LEVELS];        // cell blocks of level l for boxes with a level l+1
  List coarser[PM_MAX_LEVELS];      // cell blocks of level l+1 (restriction targets)
  List grad[3];                     // gradient blocks per tile shape
  int *range = nullptr;             // [nboxes + 1] item range of each box in cells[0]
  // arenas
  float *rho = nullptr, *g = nullptr, *lu = nullptr, *lf = nullptr;
  unsigned long long *fix = nullptr;  // [ncell_total] fixed-point deposit, zero between steps
  float *rmean = nullptr, *pmean = nullptr;
  double *partial = nullptr;        // 2 per item of cells[0]
  double *relres = nullptr;         // [nboxes]
  StepDev *steps = nullptr;
  StepDev *steps_host = nullptr;    // pinned staging
  int steps_cap = 0;
  hipEvent_t steps_copied = nullptr;  // recorded after the last copy out of steps_host
  bool steps_pending = false;
  int *ctr = nullptr;
  // tuned tile shapes (rows per thread of the stencil kernels); a shape is usable only
  // when it divides the side of every level it would run on
  int cpt_smooth = 1, cpt_grad = 1;
  bool ok_smooth[3] = {true, true, true}, ok_grad[3] = {true, true, true};
  // captured step graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void *g_pos = nullptr, *g_vel = nullptr, *g_acc = nullptr, *g_phi = nullptr;
  pm_step_params g_params{};
};

namespace {

int bfail(pm_batch *b, int code, const std::string &m) {
  if (b) b->err = m;
  return code;
}

#define BHIP(b, call)                                                                     \
  do {                                                                                    \
    hipError_t _e = (call);                                                               \
    if (_e != hipSuccess)                                                                 \
      return bfail(b, _e == hipErrorOutOfMemory ? PM_ERR_NOMEM : PM_ERR_HIP,              \
                   std::string(#call) + ": " + hipGetErrorString(_e));                    \
  } while (0)

int cpt_index(int cpt) { return cpt == 1 ? 0 : (cpt == 2 ? 1 : 2); }

int levels_of(int n) {
  int l = 1;
  while (n > 16 && n % 4 == 0) {
    n /= 2;
    ++l;
  }
  return l;
}

// all stencil launches of one step, on stream s; first = true for the Jacobi-guess solve
int enqueue_accel(pm_batch *B, const float *pos, float *acc, float *vel, float *phi,
                  const pm_step_params *p, bool first, bool with_residual, hipStream_t s) {
  const Arenas A{phi, B->rho, B->lu, B->lf, B->rmean, B->steps, B->ctr};
  // deposit
  // (exact fixed-point sums: the density is the same for every run and every order)
  if (p->mas == PM_TSC)
    kb_deposit<3><<<persist_grid(B->chunks.count), pm_chunk::kGThreads, 0, s>>>(
        pos, B->items + B->chunks.off, B->chunks.count, B->boxes, B->fix);
  else
    kb_deposit<2><<<persist_grid(B->chunks.count), pm_chunk::kGThreads, 0, s>>>(
        pos, B->items + B->chunks.off, B->chunks.count, B->boxes, B->fix);
  const pm_batch::List &c0 = B->cells[0];
  kb_fix_to_rho<<<persist_grid(c0.count), kThreads, 0, s>>>(B->fix, B->rho, B->items + c0.off,
                                                            c0.count, B->boxes, B->partial);
  kb_sum_final<<<B->nboxes, kThreads, 0, s>>>(B->partial, B->range, B->boxes, B->rmean);
  // multigrid: starting guess, then a fixed number of V-cycles
  if (first)
    kb_jacobi0<<<persist_grid(c0.count), kThreads, 0, s>>>(A, B->items + c0.off, c0.count,
                                                           B->boxes);
  else
    kb_scale<<<flat_grid(B->ncell_total), kThreads, 0, s>>>(phi, B->ncell_total, B->steps, B->ctr);
  const int ci = cpt_index(B->cpt_smooth);
  auto sweeps = [&](int l, int count, int first_colour) {
    const pm_batch::List &L = B->halfc[l][ci];
    for (int sw = 0; sw < count; ++sw)
      for (int c = 0; c < 2; ++c) {
        const int colour = c ^ first_colour;
        if (B->cpt_smooth == 1)
          kb_rbgs_half<1><<<persist_grid(L.count), kThreads, 0, s>>>(
              A, B->items + L.off, L.count, B->boxes, l, p->mg.omega, colour);
        else if (B->cpt_smooth == 2)
          kb_rbgs_half<2><<<persist_grid(L.count), kThreads, 0, s>>>(
              A, B->items + L.off, L.count, B->boxes, l, p->mg.omega, colour);
        else
          kb_rbgs_half<4><<<persist_grid(L.count), kThreads, 0, s>>>(
              A, B->items + L.off, L.count, B->boxes, l, p->mg.omega, colour);
      }
  };
  const int cycles = p->mg.fixed_cycles;
  for (int cyc = 0; cyc < cycles; ++cyc) {
    for (int l = 0; l + 1 < B->maxlev; ++l) {
      if (B->finer[l].count == 0) break;
      sweeps(l, p->mg.pre, 0);
      const pm_batch::List &F = B->finer[l];
      kb_residual<<<persist_grid(F.count), kThreads, 0, s>>>(A, B->items + F.off, F.count,
                                                             B->boxes, l, B->g);
      const pm_batch::List &R = B->coarser[l];
      if (p->mg.restrict_kind == PM_RESTRICT_AVG)
        kb_restrict<PM_RESTRICT_AVG><<<persist_grid(R.count), kThreads, 0, s>>>(
            A, B->items + R.off, R.count, B->boxes, l, B->g);
      else
        kb_restrict<PM_RESTRICT_FW><<<persist_grid(R.count), kThreads, 0, s>>>(
            A, B->items + R.off, R.count, B->boxes, l, B->g);
    }
    kb_coarse_solve<<<B->nboxes, kCoarseThreads, 0, s>>>(A, B->boxes);
    for (int l = B->maxlev - 2; l >= 0; --l) {
      const pm_batch::List &F = B->finer[l];
      if (F.count == 0) continue;
      const pm_batch::List &Cl = B->coarser[l];  // one thread per coarse cell
      kb_prolong_add<<<persist_grid(Cl.count), kThreads, 0, s>>>(A, B->items + Cl.off, Cl.count,
                                                                 B->boxes, l);
      sweeps(l, p->mg.post, 1);
    }
  }
  if (with_residual) {
    kb_residual_partial<<<persist_grid(c0.count), kThreads, 0, s>>>(A, B->items + c0.off, c0.count,
                                                                    B->boxes, B->partial);
    kb_residual_final<<<B->nboxes, kThreads, 0, s>>>(B->partial, B->range, B->relres);
  }
  // zero-mean potential (gauge), gradient, interpolation (+ kick)
  kb_sum_partial<<<persist_grid(c0.count), kThreads, 0, s>>>(phi, B->items + c0.off, c0.count,
                                                             B->boxes, B->partial);
  kb_sum_final<<<B->nboxes, kThreads, 0, s>>>(B->partial, B->range, B->boxes, B->pmean);
  kb_subtract_mean<<<persist_grid(c0.count), kThreads, 0, s>>>(phi, B->items + c0.off, c0.count,
                                                               B->boxes, B->pmean);
  const pm_batch::List &G = B->grad[cpt_index(B->cpt_grad)];
  if (B->cpt_grad == 1)
    kb_gradient<1><<<persist_grid(G.count), kThreads, 0, s>>>(phi, B->items + G.off, G.count,
                                                              B->boxes, B->g);
  else if (B->cpt_grad == 2)
    kb_gradient<2><<<persist_grid(G.count), kThreads, 0, s>>>(phi, B->items + G.off, G.count,
                                                              B->boxes, B->g);
  else
    kb_gradient<4><<<persist_grid(G.count), kThreads, 0, s>>>(phi, B->items + G.off, G.count,
                                                              B->boxes, B->g);
  if (p->mas == PM_TSC)
    kb_interp<3><<<persist_grid(B->part.count), kThreads, 0, s>>>(
        pos, B->items + B->part.off, B->part.count, B->boxes, B->g, acc, vel, B->steps, B->ctr);
  else
    kb_interp<2><<<persist_grid(B->part.count), kThreads, 0, s>>>(
        pos, B->items + B->part.off, B->part.count, B->boxes, B->g, acc, vel, B->steps, B->ctr);
  BHIP(B, hipGetLastError());
  return PM_OK;
}

int enqueue_step(pm_batch *B, float *pos, float *vel, float *acc, float *phi,
                 const pm_step_params *p, hipStream_t s) {
  kb_kick_drift<<<flat_grid(3 * B->np_total), kThreads, 0, s>>>(pos, vel, acc, 3 * B->np_total,
                                                                B->steps, B->ctr);
  int st = enqueue_accel(B, pos, acc, vel, phi, p, false, false, s);
  if (st != PM_OK) return st;
  kb_advance_counter<<<1, 1, 0, s>>>(B->ctr);
  BHIP(B, hipGetLastError());
  return PM_OK;
}

int check_batch_params(pm_batch *B, const pm_step_params *p) {
  if (!p) return bfail(B, PM_ERR_ARG, "null step params");
  if (p->mas != PM_TSC && p->mas != PM_CIC) return bfail(B, PM_ERR_ARG, "bad mas");
  if (p->solver != PM_SOLVER_MG) return bfail(B, PM_ERR_ARG, "batched runs use the multigrid solver");
  if (p->gravity != PM_GRAVITY_NEWTON && p->gravity != PM_GRAVITY_MU)
    return bfail(B, PM_ERR_ARG, "batched runs take Newtonian or parametrised gravity");
  if (!(p->omega_m > 0.0) || !std::isfinite(p->omega_l) ||
      (p->gravity == PM_GRAVITY_MU && !(p->omega_l > 0.0)))
    return bfail(B, PM_ERR_ARG, "bad background or gravity parameters");
  if (p->mg.fixed_cycles < 1 || p->mg.fixed_cycles > 64)
    return bfail(B, PM_ERR_ARG, "batched runs need mg.fixed_cycles in [1, 64]");
  if (p->mg.pre < 0 || p->mg.post < 0 || p->mg.pre > 16 || p->mg.post > 16)
    return bfail(B, PM_ERR_ARG, "sweep counts must be in [0, 16]");
  if (!(p->mg.omega > 0.0f && p->mg.omega < 2.0f)) return bfail(B, PM_ERR_ARG, "bad omega");
  if (p->mg.restrict_kind != PM_RESTRICT_FW && p->mg.restrict_kind != PM_RESTRICT_AVG)
    return bfail(B, PM_ERR_ARG, "bad restrict_kind");
  return PM_OK;
}

void drop_graph(pm_batch *B) {
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->exec = nullptr;
  B->graph = nullptr;
}

int ensure_steps(pm_batch *B, int count) {
  if (count <= B->steps_cap) return PM_OK;
  drop_graph(B);  // a captured step holds the address of the old table
  if (B->steps) (void)hipFree(B->steps);
  if (B->steps_host) (void)hipHostFree(B->steps_host);
  B->steps = nullptr;
  B->steps_host = nullptr;
  B->steps_cap = 0;
  BHIP(B, hipMalloc(&B->steps, sizeof(StepDev) * count));
  BHIP(B, hipHostMalloc(&B->steps_host, sizeof(StepDev) * count, hipHostMallocDefault));
  B->steps_cap = count;
  return PM_OK;
}

// step table for a[0..nsteps]: entry i drives the step a[i] -> a[i+1]
int upload_steps(pm_batch *B, const double *a, int nsteps, const pm_step_params *p, bool rescale,
                 hipStream_t s) {
  for (int i = 0; i < nsteps; ++i) {
    const double a0 = a[i], a1 = a[i + 1];
    if (!(a0 > 0.0) || !(a1 > 0.0) || !std::isfinite(a0) || !std::isfinite(a1))
      return bfail(B, PM_ERR_ARG, "scale factors must be > 0");
  }
  // the pinned staging table is reused: the previous call's copy out of it (queued on
  // whichever stream that call used) must have finished before it is overwritten
  if (B->steps_pending) {
    BHIP(B, hipEventSynchronize(B->steps_copied));
    B->steps_pending = false;
  }
  int st = ensure_steps(B, nsteps);
  if (st != PM_OK) return st;
  for (int i = 0; i < nsteps; ++i) {
    const double a0 = a[i], a1 = a[i + 1];
    const double tau = pm_bg_tau(p->omega_m, p->omega_l, a0, a1);
    B->steps_host[i] = StepDev{(float)(0.5 * tau), (float)tau, (float)pm_bg_coef(p, a1),
                               rescale ? (float)pm_bg_warm_scale(p, a0, a1) : 1.0f};
  }
  BHIP(B, hipMemcpyAsync(B->steps, B->steps_host, sizeof(StepDev) * nsteps, hipMemcpyHostToDevice,
                         s));
  BHIP(B, hipEventRecord(B->steps_copied, s));
  B->steps_pending = true;
  kb_set_counter<<<1, 1, 0, s>>>(B->ctr, 0);
  BHIP(B, hipGetLastError());
  return PM_OK;
}

void append_blocks(pm_batch *B, pm_batch::List &L, int b, int64_t threads_needed) {
  const int64_t nb = (threads_needed + kThreads - 1) / kThreads;
  for (int64_t k = 0; k < nb; ++k) B->items_h.push_back(int2{b, (int)k});
  L.count += (int)nb;
}

}  // namespace

extern "C" {

int pm_batch_create(pm_batch **out, int nboxes, const int *n, const int64_t *np, int flags) {
  (void)flags;
  if (!out) return PM_ERR_ARG;
  *out = nullptr;
  if (nboxes < 1 || nboxes > (1 << 20) || !n || !np) return PM_ERR_ARG;
  for (int b = 0; b < nboxes; ++b) {
    if (n[b] < 8 || n[b] > 1024 || (n[b] & 1)) return PM_ERR_SHAPE;
    int m = n[b];
    while (m > 16 && m % 4 == 0) m /= 2;
    if ((int64_t)m * m * m > kCoarseMax) return PM_ERR_SHAPE;
    if (np[b] < 1 || np[b] > INT32_MAX / 2) return PM_ERR_SHAPE;
  }
  pm_batch *B = new pm_batch();
  B->nboxes = nboxes;
  (void)hipGetDevice(&B->device);
  B->n.assign(n, n + nboxes);
  B->np.assign(np, np + nboxes);
  B->p_off.resize(nboxes + 1);
  B->c_off.resize(nboxes + 1);
  B->boxes_h.resize(nboxes);
  int64_t lev = 0;
  for (int b = 0; b < nboxes; ++b) {
    B->p_off[b + 1] = B->p_off[b] + np[b];
    B->c_off[b + 1] = B->c_off[b] + (int64_t)n[b] * n[b] * n[b];
    BoxDev &d = B->boxes_h[b];
    std::memset(&d, 0, sizeof(d));
    d.n = n[b];
    d.nlev = levels_of(n[b]);
    d.p0 = B->p_off[b];
    d.np = np[b];
    d.c0 = B->c_off[b];
    for (int l = 1; l < d.nlev; ++l) {
      const int64_t m = n[b] >> l;
      d.lo[l] = lev;
      lev += m * m * m;
    }
    B->maxlev = std::max(B->maxlev, d.nlev);
  }
  B->np_total = B->p_off[nboxes];
  B->ncell_total = B->c_off[nboxes];
  B->lev_total = std::max<int64_t>(lev, 1);
  // work lists
  B->part.off = (int64_t)B->items_h.size();
  for (int b = 0; b < nboxes; ++b) append_blocks(B, B->part, b, np[b]);
  B->chunks.off = (int64_t)B->items_h.size();
  for (int b = 0; b < nboxes; ++b) {
    BoxDev &d = B->boxes_h[b];
    d.lattice = (np[b] == (int64_t)n[b] * n[b] * n[b] && n[b] % 16 == 0) ? 1 : 0;
    const int64_t nc = d.lattice ? (int64_t)(n[b] / 8) * (n[b] / 16) * (n[b] / 16)
                                 : (np[b] + pm_chunk::kGChunk - 1) / pm_chunk::kGChunk;
    for (int64_t k = 0; k < nc; ++k) B->items_h.push_back(int2{b, (int)k});
    B->chunks.count += (int)nc;
  }
  std::vector<int> range(nboxes + 1, 0);
  for (int l = 0; l < B->maxlev; ++l) {
    B->cells[l].off = (int64_t)B->items_h.size();
    for (int b = 0; b < nboxes; ++b) {
      if (l == 0) range[b] = B->cells[0].count;
      if (B->boxes_h[b].nlev <= l) continue;
      const int64_t m = n[b] >> l;
      append_blocks(B, B->cells[l], b, m * m * m);
    }
    if (l == 0) range[nboxes] = B->cells[0].count;
  }
  for (int l = 0; l + 1 < B->maxlev; ++l) {
    const int cpts[3] = {1, 2, 4};
    for (int ci = 0; ci < 3; ++ci) {
      B->halfc[l][ci].off = (int64_t)B->items_h.size();
      for (int b = 0; b < nboxes; ++b) {
        if (B->boxes_h[b].nlev <= l + 1) continue;
        const int64_t m = n[b] >> l;
        if (m % cpts[ci]) {
          B->ok_smooth[ci] = false;  // shape not usable for this batch (tuner skips it)
          continue;
        }
        append_blocks(B, B->halfc[l][ci], b, m * (m / cpts[ci]) * (m / 2));
      }
    }
    B->finer[l].off = (int64_t)B->items_h.size();
    B->coarser[l].off = 0;
    for (int b = 0; b < nboxes; ++b) {
      if (B->boxes_h[b].nlev <= l + 1) continue;
      const int64_t m = n[b] >> l;
      append_blocks(B, B->finer[l], b, m * m * m);
    }
    B->coarser[l].off = (int64_t)B->items_h.size();
    for (int b = 0; b < nboxes; ++b) {
      if (B->boxes_h[b].nlev <= l + 1) continue;
      const int64_t m = n[b] >> (l + 1);
      append_blocks(B, B->coarser[l], b, m * m * m);
    }
  }
  {
    const int cpts[3] = {1, 2, 4};
    for (int ci = 0; ci < 3; ++ci) {
      B->grad[ci].off = (int64_t)B->items_h.size();
      for (int b = 0; b < nboxes; ++b) {
        const int64_t m = n[b];
        if (m % cpts[ci]) {
          B->ok_grad[ci] = false;
          continue;
        }
        append_blocks(B, B->grad[ci], b, m * (m / cpts[ci]) * m);
      }
    }
  }
  int st = PM_OK;
  auto alloc = [&](void **p, size_t bytes) {
    if (st == PM_OK && hipMalloc(p, std::max<size_t>(bytes, 16)) != hipSuccess) st = PM_ERR_NOMEM;
  };
  alloc((void **)&B->boxes, sizeof(BoxDev) * nboxes);
  alloc((void **)&B->items, sizeof(int2) * B->items_h.size());
  alloc((void **)&B->range, sizeof(int) * (nboxes + 1));
  alloc((void **)&B->rho, sizeof(float) * B->ncell_total);
  alloc((void **)&B->fix, sizeof(unsigned long long) * B->ncell_total);
  alloc((void **)&B->g, 3 * sizeof(float) * B->ncell_total);
  alloc((void **)&B->lu, sizeof(float) * B->lev_total);
  alloc((void **)&B->lf, sizeof(float) * B->lev_total);
  alloc((void **)&B->rmean, sizeof(float) * nboxes);
  alloc((void **)&B->pmean, sizeof(float) * nboxes);
  alloc((void **)&B->partial, 2 * sizeof(double) * B->cells[0].count);
  alloc((void **)&B->relres, sizeof(double) * nboxes);
  alloc((void **)&B->ctr, sizeof(int));
  if (st == PM_OK &&
      (hipMemcpy(B->boxes, B->boxes_h.data(), sizeof(BoxDev) * nboxes, hipMemcpyHostToDevice) !=
           hipSuccess ||
       hipMemcpy(B->items, B->items_h.data(), sizeof(int2) * B->items_h.size(),
                 hipMemcpyHostToDevice) != hipSuccess ||
       hipMemcpy(B->range, range.data(), sizeof(int) * (nboxes + 1), hipMemcpyHostToDevice) !=
           hipSuccess ||
       hipMemset(B->fix, 0, sizeof(unsigned long long) * B->ncell_total) != hipSuccess ||
       hipEventCreateWithFlags(&B->steps_copied, hipEventDisableTiming) != hipSuccess))
    st = PM_ERR_HIP;
  if (st != PM_OK) {
    pm_batch_destroy(B);
    return st;
  }
  *out = B;
  return PM_OK;
}

void pm_batch_destroy(pm_batch *B) {
  if (!B) return;
  (void)hipDeviceSynchronize();
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  void *ptrs[] = {B->boxes, B->items, B->range, B->rho, B->fix, B->g, B->lu, B->lf, B->rmean,
                  B->pmean, B->partial, B->relres, B->steps, B->ctr};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  if (B->steps_host) (void)hipHostFree(B->steps_host);
  if (B->steps_copied) (void)hipEventDestroy(B->steps_copied);
  delete B;
}

const char *pm_batch_last_error(const pm_batch *B) { return B ? B->err.c_str() : "null batch"; }

int pm_batch_layout(const pm_batch *B, int64_t *p_off, int64_t *c_off) {
  if (!B || !p_off || !c_off) return PM_ERR_ARG;
  for (int b = 0; b <= B->nboxes; ++b) {
    p_off[b] = B->p_off[b];
    c_off[b] = B->c_off[b];
  }
  return PM_OK;
}

int pm_batch_accel(pm_batch *B, const float *pos, float *acc, float *phi, double a,
                   const pm_step_params *params, double *relres, pm_stream stream) {
  if (!B) return PM_ERR_ARG;
  int st = check_batch_params(B, params);
  if (st != PM_OK) return st;
  if (!pos || !acc || !phi) return bfail(B, PM_ERR_ARG, "null pointer");
  hipStream_t s = (hipStream_t)stream;
  const double aa[2] = {a, a};
  st = upload_steps(B, aa, 1, params, false, s);
  if (st != PM_OK) return st;
  st = enqueue_accel(B, pos, acc, nullptr, phi, params, params->mg.guess == PM_GUESS_JACOBI,
                     relres != nullptr, s);
  if (st != PM_OK) return st;
  if (relres) {
    BHIP(B, hipMemcpyAsync(relres, B->relres, sizeof(double) * B->nboxes, hipMemcpyDeviceToHost, s));
    BHIP(B, hipStreamSynchronize(s));
  }
  return PM_OK;
}

int pm_batch_kdk(pm_batch *B, float *pos, float *vel, float *acc, float *phi, int nsteps,
                 const double *a, const pm_step_params *params, int use_graph, pm_stream stream) {
  if (!B) return PM_ERR_ARG;
  int st = check_batch_params(B, params);
  if (st != PM_OK) return st;
  if (!pos || !vel || !acc || !phi || !a) return bfail(B, PM_ERR_ARG, "null pointer");
  if (nsteps < 0) return bfail(B, PM_ERR_ARG, "negative step count");
  if (nsteps == 0) return PM_OK;
  hipStream_t s = (hipStream_t)stream;
  if (use_graph) {
    if (!B->exec) return bfail(B, PM_ERR_ARG, "no captured step: call pm_graph_capture_step");
    if (nsteps > B->steps_cap)
      return bfail(B, PM_ERR_ARG, "more steps than the captured step table holds");
    if (B->g_pos != pos || B->g_vel != vel || B->g_acc != acc || B->g_phi != phi)
      return bfail(B, PM_ERR_ARG, "buffers differ from the captured step");
    if (std::memcmp(&B->g_params, params, sizeof(pm_step_params)) != 0)
      return bfail(B, PM_ERR_ARG, "step parameters differ from the captured step");
  }
  st = upload_steps(B, a, nsteps, params,
                    params->mg.guess == PM_GUESS_WARM_RESCALED ||
                        params->mg.guess == PM_GUESS_EXTRAPOLATED,
                    s);
  if (st != PM_OK) return st;
  for (int i = 0; i < nsteps; ++i) {
    if (use_graph) {
      BHIP(B, hipGraphLaunch(B->exec, s));
    } else {
      st = enqueue_step(B, pos, vel, acc, phi, params, s);
      if (st != PM_OK) return st;
    }
  }
  return PM_OK;
}

int pm_graph_capture_step(pm_batch *B, float *pos, float *vel, float *acc, float *phi,
                          const pm_step_params *params, pm_stream stream) {
  if (!B) return PM_ERR_ARG;
  int st = check_batch_params(B, params);
  if (st != PM_OK) return st;
  if (!pos || !vel || !acc || !phi) return bfail(B, PM_ERR_ARG, "null pointer");
  hipStream_t s = (hipStream_t)stream;
  if (!s) return bfail(B, PM_ERR_ARG, "graph capture needs a non-null stream");
  // the step table must exist before capture (its address is baked into the graph)
  st = ensure_steps(B, std::max(B->steps_cap, kGraphSteps));
  if (st != PM_OK) return st;
  BHIP(B, hipStreamSynchronize(s));
  drop_graph(B);
  BHIP(B, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  st = enqueue_step(B, pos, vel, acc, phi, params, s);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &graph);
  if (st != PM_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  BHIP(B, e);
  B->graph = graph;
  BHIP(B, hipGraphInstantiate(&B->exec, graph, nullptr, nullptr, 0));
  B->g_pos = pos;
  B->g_vel = vel;
  B->g_acc = acc;
  B->g_phi = phi;
  B->g_params = *params;
  return PM_OK;
}

int pm_tune(pm_batch *B, float *pos, float *phi, const pm_step_params *params, int *choice,
            pm_stream stream) {
  if (!B) return PM_ERR_ARG;
  int st = check_batch_params(B, params);
  if (st != PM_OK) return st;
  if (!pos || !phi) return bfail(B, PM_ERR_ARG, "null pointer");
  hipStream_t s = (hipStream_t)stream;
  const double aa[2] = {1.0, 1.0};
  st = upload_steps(B, aa, 1, params, false, s);
  if (st != PM_OK) return st;
  hipEvent_t e0, e1;
  BHIP(B, hipEventCreate(&e0));
  BHIP(B, hipEventCreate(&e1));
  const Arenas A{phi, B->rho, B->lu, B->lf, B->rmean, B->steps, B->ctr};
  // a valid source: deposit the current particles and their means
  kb_deposit<3><<<persist_grid(B->chunks.count), pm_chunk::kGThreads, 0, s>>>(
      pos, B->items + B->chunks.off, B->chunks.count, B->boxes, B->fix);
  const pm_batch::List &c0 = B->cells[0];
  kb_fix_to_rho<<<persist_grid(c0.count), kThreads, 0, s>>>(B->fix, B->rho, B->items + c0.off,
                                                            c0.count, B->boxes, B->partial);
  kb_sum_final<<<B->nboxes, kThreads, 0, s>>>(B->partial, B->range, B->boxes, B->rmean);
  const int cpts[3] = {1, 2, 4};
  float best_s = 1e30f, best_g = 1e30f;
  int pick_s = 1, pick_g = 1;
  for (int ci = 0; ci < 3; ++ci) {
    if (!B->ok_smooth[ci] || !B->ok_grad[ci]) continue;
    const pm_batch::List &L = B->halfc[0][ci];
    const pm_batch::List &G = B->grad[ci];
    for (int rep = 0; rep < 2; ++rep) {  // first repetition warms caches and code
      BHIP(B, hipEventRecord(e0, s));
      for (int c = 0; c < 4; ++c) {
        if (cpts[ci] == 1)
          kb_rbgs_half<1><<<persist_grid(L.count), kThreads, 0, s>>>(A, B->items + L.off, L.count,
                                                                     B->boxes, 0, 1.0f, c & 1);
        else if (cpts[ci] == 2)
          kb_rbgs_half<2><<<persist_grid(L.count), kThreads, 0, s>>>(A, B->items + L.off, L.count,
                                                                     B->boxes, 0, 1.0f, c & 1);
        else
          kb_rbgs_half<4><<<persist_grid(L.count), kThreads, 0, s>>>(A, B->items + L.off, L.count,
                                                                     B->boxes, 0, 1.0f, c & 1);
      }
      BHIP(B, hipEventRecord(e1, s));
      BHIP(B, hipEventSynchronize(e1));
      float ms = 0.f;
      BHIP(B, hipEventElapsedTime(&ms, e0, e1));
      if (rep == 1 && ms < best_s) {
        best_s = ms;
        pick_s = cpts[ci];
      }
      BHIP(B, hipEventRecord(e0, s));
      for (int c = 0; c < 2; ++c) {
        if (cpts[ci] == 1)
          kb_gradient<1><<<persist_grid(G.count), kThreads, 0, s>>>(phi, B->items + G.off, G.count,
                                                                    B->boxes, B->g);
        else if (cpts[ci] == 2)
          kb_gradient<2><<<persist_grid(G.count), kThreads, 0, s>>>(phi, B->items + G.off, G.count,
                                                                    B->boxes, B->g);
        else
          kb_gradient<4><<<persist_grid(G.count), kThreads, 0, s>>>(phi, B->items + G.off, G.count,
                                                                    B->boxes, B->g);
      }
      BHIP(B, hipEventRecord(e1, s));
      BHIP(B, hipEventSynchronize(e1));
      BHIP(B, hipEventElapsedTime(&ms, e0, e1));
      if (rep == 1 && ms < best_g) {
        best_g = ms;
        pick_g = cpts[ci];
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  B->cpt_smooth = pick_s;
  B->cpt_grad = pick_g;
  if (choice) {
    choice[0] = pick_s;
    choice[1] = pick_g;
  }
  drop_graph(B);  // a captured step holds the previous tile shapes
  return PM_OK;
}

}  // extern "C"
