// Particle-side kernels: mass assignment (atomic scatter and cell-sorted gather),
// interpolation with an optional fused kick, kick + drift, and the counting sort
// that buckets particles by cell. Paper Sect. 3.5 (windows), Sect. 3.4 (leapfrog),
// App. E (particle ordering for locality).
#include "deposit_chunk.h"
#include "tile_box.h"
#include "internal.h"

namespace {

using pm_chunk::axis_box;
using pm_chunk::axis_off;
using pm_chunk::kGChunk;
using pm_chunk::kGPPT;
using pm_chunk::kGThreads;
using pm_chunk::min_image;
using pm_chunk::particle_cell;
using pm_chunk::particle_support;
using pm_chunk::wave_max_i;
using pm_chunk::wave_min_i;
using pm_chunk::weights_from_frac;
using pm_chunk::window_sep_g;
using pm_chunk::decode_cell;
using pm_chunk::log2_if_pow2;
using pm_chunk::wrap_any;
using pm_chunk::wrap_fast;
using pm_chunk::wrap_index;

constexpr int kThreads = 256;

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
  const int64_t p = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kThreads + threadIdx.x;
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

// Runs of equal keys among the lanes of a wave (particles that are neighbours in
// memory often share a cell): head lanes start a run; run length and head lane
// of every lane come from the ballot of heads.
struct WaveRun {
  bool head;
  int len;       // run length (valid on head lanes)
  int headlane;  // lane that starts this lane's run
};

__device__ __forceinline__ WaveRun wave_runs(int key) {
  const int lane = threadIdx.x & 63;
  const int prev = __shfl_up(key, 1, 64);
  WaveRun r;
  r.head = (lane == 0) || (prev != key);
  const unsigned long long heads = __ballot(r.head);
  const unsigned long long above = lane == 63 ? 0ull : (heads & ~((2ull << lane) - 1ull));
  const int next = above ? (__ffsll((long long)above) - 1) : 64;
  r.len = next - lane;
  const unsigned long long upto = heads & ((lane == 63) ? ~0ull : ((2ull << lane) - 1ull));
  r.headlane = 63 - __clzll((long long)upto);
  return r;
}

// v += kick * acc (when acc != NULL); x += dt * v, wrapped (box) or carried (cell offset).
// With count != NULL the kernel also does the first pass of the deposit's tile sort
// for the new positions: the particle's 8^3-tile key goes to pcell and the tile
// histogram gets one atomic per run of equal keys in a wave (same key rule as
// k_cell_hist), which saves that kernel's re-read of the particles.
// x += dt * v for particle p, wrapped (box) or carried into the cell index (cell
// offset); writes pos (and cell) and returns the particle's 8^3-tile key.
template <int PK>
__device__ __forceinline__ int drift_from(float *__restrict__ pos, int32_t *__restrict__ cell,
                                          int64_t p, int n, float dt, const float v[3],
                                          const float xin[3], int cin) {
  float x[3] = {xin[0], xin[1], xin[2]};
  int ci[3];
  const int lg = log2_if_pow2(n);
  if constexpr (PK == PM_POS_BOX) {
    const float fn = (float)n;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      x[d] = wrap_unit(fmaf(dt, v[d], x[d]));
      ci[d] = wrap_fast((int)floorf(x[d] * fn), n, lg);
    }
  } else {
    const float scale = dt * (float)n;
    decode_cell(cin, n, lg, ci);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      float o = fmaf(scale, v[d], x[d]);
      float fl = floorf(o);
      o -= fl;
      if (o >= 1.0f) {
        o = 0.0f;
        fl += 1.0f;
      }
      ci[d] = wrap_fast(ci[d] + (int)fl, n, lg);
      x[d] = o;
    }
    cell[p] = (ci[0] * n + ci[1]) * n + ci[2];
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) pos[3 * p + d] = x[d];
  const int nt = n >> 3;
  return ((ci[0] >> 3) * nt + (ci[1] >> 3)) * nt + (ci[2] >> 3);
}

template <int PK>
__device__ __forceinline__ int drift_one(float *__restrict__ pos, int32_t *__restrict__ cell,
                                         int64_t p, int n, float dt, const float v[3]) {
  const float x[3] = {pos[3 * p + 0], pos[3 * p + 1], pos[3 * p + 2]};
  return drift_from<PK>(pos, cell, p, n, dt, v, x, PK == PM_POS_BOX ? 0 : cell[p]);
}

template <int PK>
__global__ __launch_bounds__(kThreads) void k_kick_drift(float *__restrict__ pos,
                                                         int32_t *__restrict__ cell,
                                                         float *__restrict__ vel,
                                                         const float *__restrict__ acc,
                                                         int64_t np, int n, float kick,
                                                         float dt, int32_t *__restrict__ pcell,
                                                         int32_t *__restrict__ count) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const bool live = p < np;
  int key = -1;
  if (live) {
    float v[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      v[d] = vel[3 * p + d];
      if (acc) v[d] = fmaf(kick, acc[3 * p + d], v[d]);
      vel[3 * p + d] = v[d];
    }
    const int k = drift_one<PK>(pos, cell, p, n, dt, v);
    if (count) {
      key = k;
      pcell[p] = key;
    }
  }
  if (count) {  // uniform: the whole wave takes part in the run detection
    const WaveRun r = wave_runs(key);
    if (r.head && key >= 0) atomicAdd(&count[key], r.len);
  }
}

// ------------------------------------------------------------------ counting sort

// Sort keys: 0 = row-major cell, 2 = 8^3-cell tile (tiles row-major). The tile-major
// cell order of pm_reorder is the tile sort followed by k_tile_cell_sort.
constexpr int kKeyCell = 0, kKeyTile = 2;
// Every wave of the histogram and scatter kernels handles kSortRounds runs of 64
// consecutive particles; the scatter issues the cursor atomics of all rounds before it
// needs their results, so their latencies overlap.
constexpr int kSortRounds = 4;
constexpr int kScatterHash = 2048;  // LDS hash slots of the scatter (block's distinct keys)

// Key of each particle's cell; histogram with one atomic per run of equal keys in a
// wave (particles that are neighbours in memory mostly share keys).
template <int PK, int KEY>
__global__ __launch_bounds__(kThreads) void k_cell_hist(const float *__restrict__ pos,
                                                        const int32_t *__restrict__ cell,
                                                        int64_t np, int n,
                                                        int32_t *__restrict__ pcell,
                                                        int32_t *__restrict__ count) {
  const int lane = threadIdx.x & 63;
  const int64_t wbase =
      ((int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6)) * 64 * kSortRounds;
#pragma unroll
  for (int m = 0; m < kSortRounds; ++m) {
    const int64_t p = wbase + m * 64 + lane;
    int c = -1;
    if (p < np) {
      int q[3];
      const int lg = log2_if_pow2(n);
      if constexpr (PK == PM_POS_BOX) {
        const float fn = (float)n;
#pragma unroll
        for (int d = 0; d < 3; ++d) q[d] = wrap_fast((int)floorf(pos[3 * p + d] * fn), n, lg);
      } else {
        decode_cell(cell[p], n, lg, q);
      }
      if constexpr (KEY == kKeyTile) {
        const int nt = n >> 3;
        c = ((q[0] >> 3) * nt + (q[1] >> 3)) * nt + (q[2] >> 3);
      } else {
        c = (q[0] * n + q[1]) * n + q[2];
      }
      pcell[p] = c;
    }
    const WaveRun r = wave_runs(c);
    if (r.head && c >= 0) atomicAdd(&count[c], r.len);
  }
}

// dst[p] = src[perm[p]] for W elements of type T per particle.
template <typename T, int W>
__global__ __launch_bounds__(kThreads) void k_gather_perm(const T *__restrict__ src,
                                                          const int32_t *__restrict__ perm,
                                                          int64_t np, T *__restrict__ dst) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= np) return;
  const int64_t q = perm[p];
#pragma unroll
  for (int w = 0; w < W; ++w) dst[W * p + w] = src[W * q + w];
}

// ------------------------------------------------------------------ chunked gather deposit

template <int MAS, int PK>
__global__ __launch_bounds__(kGThreads) void k_deposit_chunk(const float *__restrict__ pos,
                                                             const int32_t *__restrict__ cell,
                                                             int64_t np, int n, float mass,
                                                             float *__restrict__ rho) {
  const int64_t base = (int64_t)blockIdx.x * kGChunk;
  pm_chunk::deposit_chunk<MAS, PK>(pos, cell, pm_chunk::RangeIndex{base, np}, n, mass, rho);
}

// Scatter of the counting sort: every particle takes the next place of its key's
// bucket (cursor[key] runs from the bucket's start to its end) and writes its index
// there; the order within a bucket is not fixed.
__global__ __launch_bounds__(kThreads) void k_scatter_perm(const int32_t *__restrict__ pcell,
                                                           int64_t np,
                                                           int32_t *__restrict__ cursor,
                                                           int32_t *__restrict__ perm) {
  // the block's distinct keys in an LDS hash table (open addressing; at most
  // kThreads * kSortRounds keys in twice as many slots, so every probe sequence ends);
  // each run of equal keys in a wave adds its length to its key's count and takes its
  // place from it, then one global cursor atomic per distinct key serves the block
  constexpr int H = kScatterHash;
  static_assert(H >= 2 * kThreads * kSortRounds && (H & (H - 1)) == 0, "scatter hash size");
  __shared__ int s_key[H];
  __shared__ int s_cnt[H];
  __shared__ int s_base[H];
  for (int i = threadIdx.x; i < H; i += kThreads) {
    s_key[i] = -1;
    s_cnt[i] = 0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t wbase =
      ((int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6)) * 64 * kSortRounds;
  int c[kSortRounds], slot[kSortRounds], rank[kSortRounds];
#pragma unroll
  for (int m = 0; m < kSortRounds; ++m) {
    const int64_t p = wbase + m * 64 + lane;
    c[m] = p < np ? pcell[p] : -1;
  }
#pragma unroll
  for (int m = 0; m < kSortRounds; ++m) {
    const WaveRun r = wave_runs(c[m]);
    int sl = 0, rb = 0;
    if (r.head && c[m] >= 0) {
      // slot = key mod H: neighbouring keys take neighbouring slots, so the cursor
      // atomics below (thread i serves slots i, i + kThreads, ...) stay coalesced
      unsigned h = (unsigned)c[m] & (unsigned)(H - 1);
      for (int probe = 0; probe < H; ++probe) {
        const int old = atomicCAS(&s_key[h], -1, c[m]);
        if (old == -1 || old == c[m]) break;
        h = (h + 1u) & (unsigned)(H - 1);
      }
      sl = (int)h;
      rb = atomicAdd(&s_cnt[h], r.len);
    }
    slot[m] = __shfl(sl, r.headlane, 64);
    rank[m] = __shfl(rb, r.headlane, 64) + (lane - r.headlane);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < H; i += kThreads)
    if (s_key[i] >= 0) s_base[i] = atomicAdd(&cursor[s_key[i]], s_cnt[i]);
  __syncthreads();
#pragma unroll
  for (int m = 0; m < kSortRounds; ++m)
    if (c[m] >= 0) perm[s_base[slot[m]] + rank[m]] = (int32_t)(wbase + m * 64 + lane);
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
    const int64_t idx = base + i;
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

// In-place exclusive scan of one tile: coalesced loads into LDS, per-thread scan of
// kScanItems consecutive entries, block scan of the thread totals.
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(int32_t *__restrict__ data,
                                                             int64_t len,
                                                             const int32_t *__restrict__ partial) {
  __shared__ int tile[kScanTile + kScanTile / 32];  // padded against bank conflicts
  __shared__ int lds[kScanThreads / 64 + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  auto pad = [](int i) { return i + (i >> 5); };
  for (int i = threadIdx.x; i < kScanTile; i += kScanThreads)
    tile[pad(i)] = (base + i < len) ? data[base + i] : 0;
  __syncthreads();
  int v[kScanItems];
  int sum = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = tile[pad(threadIdx.x * kScanItems + i)];
    sum += v[i];
  }
  int total;
  int ex = block_exclusive_scan(sum, lds, total) + partial[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    tile[pad(threadIdx.x * kScanItems + i)] = ex;
    ex += v[i];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kScanTile; i += kScanThreads)
    if (base + i < len) data[base + i] = tile[pad(i)];
}

// ------------------------------------------------------------------ gathered deposit

// Fixed point used to sum window values: 2^40 units per particle weight.
constexpr double kFixScale = 1099511627776.0;  // 2^40

template <int MAS>
__device__ __forceinline__ float window_sep(float s) {
  return window_sep_g<MAS>(s);
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
        const int s0 = q > 0 ? start[q - 1] : 0, s1 = start[q];  // `start` holds cell ends
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

// ------------------------------------------------------------------ fixed-point helpers

constexpr int kTT = 8;                        // tile edge
constexpr int kTThreads = kTT * kTT * kTT;    // cells per tile (512)
constexpr int kTH = kTT + 2;                  // tile + one-cell halo
constexpr int kTHalo = kTH * kTH * kTH;       // 1000
constexpr float kFix30 = 1073741824.0f;       // 2^30 units per unit weight

// Fixed-point unit of a weight: w 2^30, with 0 <= w <= 27/64 < 2, so it fits an
// int32. The kernels scale one axis's weights by 2^30 (exact: a power of two) and
// truncate the product: every bit of the FP32 weight above 2^-30 is kept, and each
// (particle, cell) pair gives the same integer on every path, so the integer sums do
// not depend on the order of the particles.
__device__ __forceinline__ unsigned long long fix_scaled(float w_scaled) {
  return (unsigned long long)(unsigned int)w_scaled;
}

__device__ __forceinline__ unsigned long long wave_sum_ull(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// wave sum in a fixed order (the shuffle tree is the same in every run)
__device__ __forceinline__ double wave_sum_double(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

inline unsigned blocks_for(int64_t count, int threads) {
  return (unsigned)((count + threads - 1) / threads);
}

// ------------------------------------------------------------------ particle-owned tile deposit

// Deterministic deposit from particles bucketed by 8^3-cell tile: one workgroup per
// tile reads only the particles of its own tile (each particle once), adds their 27
// (8) window weights as 2^-30 fixed-point integers to an LDS box of the tile plus a
// one-cell halo, and stores the whole box (10^3 values, each exact sum times the
// particle weight rounded once to FP32) with plain coalesced stores to the tile's slot
// of a box array; an empty tile stores nothing. A gather pass then forms each cell's
// density from the one to eight boxes that cover it (a cell on a tile face, edge or
// corner is also in the halo of one, three or seven neighbours), summed in FP64 in a
// fixed order, skipping empty tiles. The LDS sums are integer sums and the gather's
// order is fixed, so the result is bitwise the same for any particle order, any
// interleaving of the LDS atomics and any run; no global atomics, and nothing to clear
// between deposits.
// A wave whose 64 particles share one cell (dense cells: particles kept in
// tile-major cell order by pm_reorder stay together) first reduces its 27 window
// moments across lanes.
constexpr int kOThreads = 256;
#ifndef PM_DEPOSIT_THREADS
#define PM_DEPOSIT_THREADS 256
#endif
#ifndef PM_INTERP_THREADS
#define PM_INTERP_THREADS 256
#endif
constexpr int kDThreads = PM_DEPOSIT_THREADS;  // tile deposit block
constexpr int kIThreads = PM_INTERP_THREADS;   // tile interpolation block

// One particle of a tile bucket, loaded ahead of its use.
struct TileParticle {
  bool live;
  int p, c;    // particle index, cell index (cell-offset positions)
  float x[3];  // box-unit position or in-cell offset
  float v[3];  // velocity (when the kernel kicks)
};

// Index of this thread's particle in the pass of the bucket starting at l0 (-1 past
// its end). The tile kernels load indices two passes ahead of use and particle data
// one pass ahead, so that every wait is on loads issued a whole pass earlier.
__device__ __forceinline__ int tile_index(const int32_t *__restrict__ perm, int l0, int p_end) {
  const int l = l0 + (int)threadIdx.x;
  return l < p_end ? perm[l] : -1;
}

template <int PK>
__device__ __forceinline__ TileParticle load_particle(const float *__restrict__ pos,
                                                      const int32_t *__restrict__ cell,
                                                      const float *__restrict__ vel, int p) {
  TileParticle t{};
  t.live = p >= 0;
  if (t.live) {
    t.p = p;
    const size_t q = 3 * (size_t)p;
    t.x[0] = pos[q];
    t.x[1] = pos[q + 1];
    t.x[2] = pos[q + 2];
    t.c = PK == PM_POS_BOX ? 0 : cell[p];
    if (vel) {
      t.v[0] = vel[q];
      t.v[1] = vel[q + 1];
      t.v[2] = vel[q + 2];
    }
  }
  return t;
}

// cell and in-cell offset of a loaded particle (the particle_cell rule)
template <int PK>
__device__ __forceinline__ void cell_offset_of(const float x[3], int cin, int n, int c[3],
                                               float o[3]) {
  const int lg = log2_if_pow2(n);
  if constexpr (PK == PM_POS_BOX) {
    const float fn = (float)n;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float u = x[d] * fn;
      const float fl = floorf(u);
      c[d] = wrap_fast((int)fl, n, lg);
      o[d] = u - fl;
    }
  } else {
    decode_cell(cin, n, lg, c);
#pragma unroll
    for (int d = 0; d < 3; ++d) o[d] = x[d];
  }
}

template <int MAS, int PK>
__global__ __launch_bounds__(kDThreads) void k_deposit_own(const float *__restrict__ pos,
                                                           const int32_t *__restrict__ cell,
                                                           const int32_t *__restrict__ end,
                                                           const int32_t *__restrict__ perm,
                                                           int n, double scale,
                                                           float *__restrict__ tbox) {
  __shared__ unsigned long long box[kTHalo];
  // per-wave particle count of each cell of the tile in the current pass (kept zero
  // between passes): a lane's rank among the wave's lanes in its cell
  __shared__ unsigned int s_cnt[kDThreads / 64][kTThreads];
  const int nt = n / kTT;
  const int tile = (int)xcd_block(blockIdx.x, gridDim.x);
  const int tk = tile % nt, tj = (tile / nt) % nt, ti = tile / (nt * nt);
  // particles bucketed by tile: end[t] is the end of tile t's bucket; the first pass's
  // particles (and the second's indices) are loaded before the box is cleared, each
  // later pass's particles during the pass before it, their indices two passes before
  const int p_begin = tile > 0 ? end[tile - 1] : 0;
  const int p_end = end[tile];
  if (p_begin >= p_end) return;  // empty tile: the gather pass skips its box
  TileParticle cur = load_particle<PK>(pos, cell, nullptr, tile_index(perm, p_begin, p_end));
  int pnext = tile_index(perm, p_begin + kDThreads, p_end);
  for (int i = threadIdx.x; i < kTHalo; i += kDThreads) box[i] = 0ull;
  for (int i = threadIdx.x; i < (kDThreads / 64) * kTThreads; i += kDThreads)
    (&s_cnt[0][0])[i] = 0u;
  __syncthreads();
  unsigned int *cnt = s_cnt[threadIdx.x >> 6];
  for (int l0 = p_begin; l0 < p_end; l0 += kDThreads) {
    const TileParticle nxt = load_particle<PK>(pos, cell, nullptr, pnext);
    pnext = tile_index(perm, l0 + 2 * kDThreads, p_end);
    bool act = cur.live;
    int c[3] = {0, 0, 0};
    float o[3] = {0.f, 0.f, 0.f};
    if (act) cell_offset_of<PK>(cur.x, cur.c, n, c, o);
    cur = nxt;
    const int lx = c[0] - ti * kTT, ly = c[1] - tj * kTT, lz = c[2] - tk * kTT;
    // every particle of the bucket lies in this tile (same cell rule as the sort)
    act = act && (unsigned)lx < (unsigned)kTT && (unsigned)ly < (unsigned)kTT &&
          (unsigned)lz < (unsigned)kTT;
    const int key = act ? (lx * kTT + ly) * kTT + lz : -1;
    const int rank = act ? (int)atomicAdd(&cnt[key], 1u) : 0;
    float wx[MAS], wy[MAS], wz[MAS];
    // box coordinates are tile coordinates + 1; the window's first cell follows
    const int fx = axis_off<MAS>(lx + 1, o[0], wx);
    const int fy = axis_off<MAS>(ly + 1, o[1], wy);
    const int fz = axis_off<MAS>(lz + 1, o[2], wz);
#pragma unroll
    for (int t = 0; t < MAS; ++t) wz[t] *= kFix30;
    const int key_first = __shfl(key, 0, 64);
    const bool uniform = __ballot(act && key == key_first) == __ballot(l0 + (int)threadIdx.x < p_end) &&
                         key_first >= 0;
    if (uniform) {
      // one cell for the whole wave: every lane's window lies in the 3^3 cells around
      // it (box coordinates lx .. lx + 2); reduce the 27 moments, one lane adds them
      float ex[3], ey[3], ez[3];
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const int ax = t - (fx - lx), ay = t - (fy - ly), az = t - (fz - lz);
        ex[t] = (ax >= 0 && ax < MAS) ? wx[ax] : 0.0f;
        ey[t] = (ay >= 0 && ay < MAS) ? wy[ay] : 0.0f;
        ez[t] = (az >= 0 && az < MAS) ? wz[az] : 0.0f;
      }
      const int bx = __shfl(lx, 0, 64), by = __shfl(ly, 0, 64), bz = __shfl(lz, 0, 64);
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          const float eab = ex[a] * ey[b];
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) {
            unsigned long long v = act ? fix_scaled(eab * ez[cc]) : 0ull;
            v = wave_sum_ull(v);
            if ((threadIdx.x & 63) == 0)
              atomicAdd(&box[((bx + a) * kTH + (by + b)) * kTH + (bz + cc)], v);
          }
        }
    } else if (__ballot(rank >= MAS) == 0ull) {
      // at most MAS lanes of the wave share a cell: the lane of rank r walks the window's
      // k cells rotated by r, so lanes of one cell add to different LDS words in each
      // instruction; the rotation only changes the register part of the address (the
      // (a, b) row is the instruction's constant offset)
      if (act) {
        const int base = (fx * kTH + fy) * kTH + fz;
        float pz[MAS];
        int oz[MAS];
#pragma unroll
        for (int t = 0; t < MAS; ++t) {
          const int sc = t + rank >= MAS ? t + rank - MAS : t + rank;
          pz[t] = sc == 0 ? wz[0] : (sc == 1 ? wz[MAS > 1 ? 1 : 0] : wz[MAS - 1]);
          oz[t] = base + sc;
        }
#pragma unroll
        for (int a = 0; a < MAS; ++a)
#pragma unroll
          for (int b = 0; b < MAS; ++b) {
            const float wab = wx[a] * wy[b];
            const int row = (a * kTH + b) * kTH;
#pragma unroll
            for (int cc = 0; cc < MAS; ++cc)
              atomicAdd(&box[oz[cc] + row], fix_scaled(wab * pz[cc]));
          }
      }
    } else if (act) {
      // more lanes share a cell: the window's cells in an order rotated per axis by the
      // base-MAS digits of the lane's rank among the wave's lanes in its cell, so that
      // lanes of one cell (up to MAS^3 of them) add to different LDS words in each
      // instruction instead of serialising on one. The rotation is applied once per
      // particle to the three weights and offsets of each axis.
      const int r = rank % (MAS * MAS * MAS);
      const int ra = r / (MAS * MAS), rb = (r / MAS) % MAS, rc = r % MAS;
      float px[MAS], py[MAS], pz[MAS];
      int ox[MAS], oy[MAS], oz[MAS];
#pragma unroll
      for (int t = 0; t < MAS; ++t) {
        const int sa = t + ra - (t + ra >= MAS ? MAS : 0);
        const int sb = t + rb - (t + rb >= MAS ? MAS : 0);
        const int sc = t + rc - (t + rc >= MAS ? MAS : 0);
        px[t] = sa == 0 ? wx[0] : (sa == 1 ? wx[MAS > 1 ? 1 : 0] : wx[MAS - 1]);
        py[t] = sb == 0 ? wy[0] : (sb == 1 ? wy[MAS > 1 ? 1 : 0] : wy[MAS - 1]);
        pz[t] = sc == 0 ? wz[0] : (sc == 1 ? wz[MAS > 1 ? 1 : 0] : wz[MAS - 1]);
        ox[t] = sa * (kTH * kTH);
        oy[t] = sb * kTH;
        oz[t] = sc;
      }
      const int base = (fx * kTH + fy) * kTH + fz;
#pragma unroll
      for (int a = 0; a < MAS; ++a)
#pragma unroll
        for (int b = 0; b < MAS; ++b) {
          const float wab = px[a] * py[b];
          const int row = base + ox[a] + oy[b];
#pragma unroll
          for (int cc = 0; cc < MAS; ++cc)
            atomicAdd(&box[row + oz[cc]], fix_scaled(wab * pz[cc]));
        }
    }
    if (act) cnt[key] = 0u;  // counts start from zero in the next pass (same wave)
  }
  __syncthreads();
  // the box belongs to this tile alone: stored whole (zeros included) in the slot order
  // of its consumers, with coalesced stores, each exact integer sum rounded once to FP32
  // (times the particle weight: scale = w 2^-30)
  static_assert(kTHalo == pm_tilebox::kSlots, "tile box shape");
  float *dst = tbox + (size_t)tile * kTHalo;
  for (int o = threadIdx.x; o < kTHalo; o += kDThreads) {
    int hx, hy, hz;
    pm_tilebox::box_of(o, hx, hy, hz);
    dst[o] = (float)((double)box[(hx * kTH + hy) * kTH + hz] * scale);
  }
}

// Second level of the tile-major cell sort (pm_reorder): particles already bucketed by
// 8^3 tile (perm, end) are ordered by cell within their tile, one workgroup per tile
// with a counting sort over the tile's 512 cells in LDS (the tile-major key of a cell
// is tile * 512 + its local index); out[i] is the particle at place i. The order within
// a cell is not fixed.
template <int PK>
__device__ __forceinline__ int local_cell_of(const float *__restrict__ pos,
                                             const int32_t *__restrict__ cell, int p, int n,
                                             int ti, int tj, int tk) {
  float x[3] = {0.f, 0.f, 0.f};
  if constexpr (PK == PM_POS_BOX) {
    x[0] = pos[3 * (size_t)p];
    x[1] = pos[3 * (size_t)p + 1];
    x[2] = pos[3 * (size_t)p + 2];
  }
  int c[3];
  float o[3];
  cell_offset_of<PK>(x, PK == PM_POS_BOX ? 0 : cell[p], n, c, o);
  const int lx = c[0] - ti * 8, ly = c[1] - tj * 8, lz = c[2] - tk * 8;
  // the bucket's particles lie in this tile (same cell rule as its key); the clamp only
  // keeps every index in the table
  const int l = (lx * 8 + ly) * 8 + lz;
  return l < 0 ? 0 : (l > 511 ? 511 : l);
}

template <int PK>
__global__ __launch_bounds__(kThreads) void k_tile_cell_sort(const float *__restrict__ pos,
                                                             const int32_t *__restrict__ cell,
                                                             const int32_t *__restrict__ end,
                                                             const int32_t *__restrict__ perm,
                                                             int n, int32_t *__restrict__ out) {
  static_assert(2 * kThreads == 512, "two cells per thread");
  __shared__ int s_cnt[512];
  __shared__ int s_wave[kThreads / 64];
  const int nt = n / 8;
  const int tile = blockIdx.x;
  const int tk = tile % nt, tj = (tile / nt) % nt, ti = tile / (nt * nt);
  const int b = tile > 0 ? end[tile - 1] : 0, e = end[tile];
  if (b >= e) return;
  s_cnt[2 * threadIdx.x] = 0;
  s_cnt[2 * threadIdx.x + 1] = 0;
  __syncthreads();
  for (int l = b + (int)threadIdx.x; l < e; l += kThreads)
    atomicAdd(&s_cnt[local_cell_of<PK>(pos, cell, perm[l], n, ti, tj, tk)], 1);
  __syncthreads();
  // exclusive scan of the 512 counts (two per thread) into per-cell cursors
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c0 = s_cnt[2 * threadIdx.x], c1 = s_cnt[2 * threadIdx.x + 1];
  int v = c0 + c1;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(v, o, 64);
    if (lane >= o) v += u;
  }
  if (lane == 63) s_wave[wave] = v;
  __syncthreads();
  int off = 0;
  for (int w = 0; w < wave; ++w) off += s_wave[w];
  const int excl = off + v - (c0 + c1);
  s_cnt[2 * threadIdx.x] = excl;
  s_cnt[2 * threadIdx.x + 1] = excl + c0;
  __syncthreads();
  for (int l = b + (int)threadIdx.x; l < e; l += kThreads) {
    const int p = perm[l];
    const int slot = atomicAdd(&s_cnt[local_cell_of<PK>(pos, cell, p, n, ti, tj, tk)], 1);
    out[b + slot] = p;
  }
}

// Gather pass of the tile deposit: one workgroup per row of up to kGRow tiles along k
// (8 x 8 x 8 kGRow cells); a wave step covers one x, one y and the row's 64 cells
// along k. Cell c of tile t sums the interior value of t's box and, on a tile face,
// edge or corner, the halo values that the one, three or seven neighbours t + d stored
// for it (tile_box.h). Interior, x and y faces and the edges along k are read by the
// wave steps (64 lanes, 8 runs of 64 bytes); the pieces only the cells at k = 0 or 7
// of a tile need (k faces, the edges along i and j, corners) are first staged in LDS
// with whole-group loads. Empty tiles (no particles in their bucket) stored no box and
// add nothing. With partial != NULL each block also adds up its fixed-point sums
// (exact), for the mean of rho.
constexpr int kGRow = 8;             // tiles per gather row
constexpr int kGatherThreads = 256;  // four waves, 16 steps of 64 cells each
constexpr int kGatherBlocks = 65536; // grid-stride above this many rows
static_assert(kGatherThreads == 4 * 64 && kGRow * kTT == 64, "gather row shape");

__global__ __launch_bounds__(kGatherThreads) void k_tile_gather(
    const float *__restrict__ tbox, const int32_t *__restrict__ end, int n, int64_t rows,
    float *__restrict__ rho, double *__restrict__ partial) {
  using pm_tilebox::gather_slot;
  using pm_tilebox::kCornerBase;
  using pm_tilebox::kEdgeBase;
  using pm_tilebox::kFaceBase;
  constexpr int S = pm_tilebox::kSlots;
  // neighbour tiles of the row: [dx + 1][dy + 1][1 + tile in row + dz], -1 when empty
  __shared__ int s_tile[3][3][kGRow + 2];
  // staged halo: k faces [dz > 0][tile][x * 8 + y], edges along j [dx > 0][dz > 0][tile][y],
  // edges along i [dy > 0][dz > 0][tile][x], corners [dx > 0][dy > 0][dz > 0][tile]
  __shared__ float s_zf[2][kGRow][64];
  __shared__ float s_exz[2][2][kGRow][8];
  __shared__ float s_eyz[2][2][kGRow][8];
  __shared__ float s_cr[2][2][2][kGRow];
  __shared__ double ws[kGatherThreads / 64];
  constexpr int kStage = 2 * kGRow * 64 + 2 * 2 * 2 * kGRow * 8 + 8 * kGRow;  // 1600
  constexpr int kStageIt = (kStage + kGatherThreads - 1) / kGatherThreads;
  const int nt = n / kTT;
  const int nkb = (nt + kGRow - 1) / kGRow;
  const int z = threadIdx.x & 63;     // cell along k within the row
  const int m = z >> 3, zl = z & 7;   // tile within the row, k within the tile
  const int w = threadIdx.x >> 6;     // wave: y = w (even steps) or 4 + w (odd steps)
  double sum = 0.0;
  for (int64_t row = xcd_block(blockIdx.x, gridDim.x); row < rows; row += gridDim.x) {
    const int tkb = (int)(row % nkb);
    const int tj = (int)((row / nkb) % nt);
    const int ti = (int)(row / ((int64_t)nkb * nt));
    const int tk0 = tkb * kGRow;
    __syncthreads();  // the previous row's table and staged halo are no longer read
    if (threadIdx.x < 9 * (kGRow + 2)) {
      const int q = threadIdx.x / (kGRow + 2), mm = threadIdx.x % (kGRow + 2);
      const int tt = (wrap_any(ti + q / 3 - 1, nt) * nt + wrap_any(tj + q % 3 - 1, nt)) * nt +
                     wrap_any(tk0 - 1 + mm, nt);
      const int cnt = end[tt] - (tt > 0 ? end[tt - 1] : 0);
      (&s_tile[0][0][0])[threadIdx.x] = cnt > 0 ? tt : -1;
    }
    __syncthreads();
    // halo pieces for the cells at k = 0, 7 of each tile: loaded whole (zero when empty)
    float st[kStageIt];
#pragma unroll
    for (int u = 0; u < kStageIt; ++u) {
      const int q = (int)threadIdx.x + u * kGatherThreads;
      int t = -1, slot = 0;
      if (q < 1024) {  // k faces: side 0 from tile mm - 1 (its high k face), 1 from mm + 1
        const int sd = q >> 9, mm = (q >> 6) & 7, in = q & 63;
        t = s_tile[1][1][mm + 2 * sd];
        slot = kFaceBase + 64 * (5 - sd) + in;
      } else if (q < 1280) {  // edges along j: neighbour (dx, 0, dz)
        const int o = q - 1024, sx = o >> 7, sz = (o >> 6) & 1, mm = (o >> 3) & 7, yy = o & 7;
        t = s_tile[2 * sx][1][mm + 2 * sz];
        slot = kEdgeBase + 8 * (4 + 2 * (1 - sx) + (1 - sz)) + yy;
      } else if (q < 1536) {  // edges along i: neighbour (0, dy, dz)
        const int o = q - 1280, sy = o >> 7, sz = (o >> 6) & 1, mm = (o >> 3) & 7, xx = o & 7;
        t = s_tile[1][2 * sy][mm + 2 * sz];
        slot = kEdgeBase + 8 * (0 + 2 * (1 - sy) + (1 - sz)) + xx;
      } else if (q < kStage) {  // corners: neighbour (dx, dy, dz)
        const int o = q - 1536, sx = o >> 5, sy = (o >> 4) & 1, sz = (o >> 3) & 1, mm = o & 7;
        t = s_tile[2 * sx][2 * sy][mm + 2 * sz];
        slot = kCornerBase + 4 * (1 - sx) + 2 * (1 - sy) + (1 - sz);
      }
      // loaded unconditionally (an empty tile or a surplus item reads tile 0's box and
      // is dropped), so that all of a thread's loads are in flight together
      const float val = tbox[(size_t)(t >= 0 ? t : 0) * S + slot];
      st[u] = t >= 0 ? val : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kStageIt; ++u) {
      const int q = (int)threadIdx.x + u * kGatherThreads;
      if (q < 1024) (&s_zf[0][0][0])[q] = st[u];
      else if (q < 1280) (&s_exz[0][0][0][0])[q - 1024] = st[u];
      else if (q < 1536) (&s_eyz[0][0][0][0])[q - 1280] = st[u];
      else if (q < kStage) (&s_cr[0][0][0][0])[q - 1536] = st[u];
    }
    __syncthreads();
    // per wave step: interior, x and y faces, edges along k from the boxes, the rest
    // from LDS; cells of tiles past the end of a short row are not written
    const bool live = tk0 + m < nt;
    const int tc = s_tile[1][1][m + 1];
    const int txm = s_tile[0][1][m + 1], txp = s_tile[2][1][m + 1];
    const int tym = s_tile[1][0][m + 1], typ = s_tile[1][2][m + 1];
    const size_t own = (size_t)(tc >= 0 ? tc : 0) * S;  // an empty tile's box is not used
    const size_t kg = (size_t)tk0 * kTT + z;
    const int sz = zl == kTT - 1;
    const bool kedge = zl == 0 || zl == kTT - 1;
    // every load of a half row (x = 4 h .. 4 h + 3) is issued unconditionally and
    // without branches between them (a piece a cell does not take reads the cell's own
    // interior value instead and is dropped), so that they are in flight together; the
    // LDS pieces and the stores follow
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
      double v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int x = 4 * h + (j >> 1), y = 4 * (j & 1) + w;
        const size_t self = own + gather_slot(0, 0, 0, x, y, zl);
        const float q = tbox[self];
        double a = tc >= 0 ? (double)q : 0.0;
        const bool xe = x == 0 || x == kTT - 1;
        const int tx = x == 0 ? txm : txp;
        const bool tkx = xe && tx >= 0;
        const float vx =
            tbox[tkx ? (size_t)tx * S + gather_slot(x == 0 ? -1 : 1, 0, 0, x, y, zl) : self];
        a += tkx ? (double)vx : 0.0;
        const bool ye = y == 0 || y == kTT - 1;  // wave-uniform
        const int ty = y == 0 ? tym : typ;
        const bool tky = ye && ty >= 0;
        const float vy =
            tbox[tky ? (size_t)ty * S + gather_slot(0, y == 0 ? -1 : 1, 0, x, y, zl) : self];
        a += tky ? (double)vy : 0.0;
        if (j < 2 || j >= 6) {  // x = 0 or 3 (h = 0), x = 4 or 7 (h = 1): the edges along k
          const int dx = j < 2 ? -1 : 1, dy = y == 0 ? -1 : 1;
          const int t = s_tile[dx + 1][dy + 1][m + 1];
          const bool te = xe && ye && t >= 0;
          const float ve = tbox[te ? (size_t)t * S + gather_slot(dx, dy, 0, x, y, zl) : self];
          a += te ? (double)ve : 0.0;
        }
        v[j] = a;
      }
      if (kedge) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int x = 4 * h + (j >> 1), y = 4 * (j & 1) + w;
          double a = (double)s_zf[sz][m][x * 8 + y];
          if (x == 0 || x == kTT - 1) a += (double)s_exz[x != 0][sz][m][y];
          if (y == 0 || y == kTT - 1) a += (double)s_eyz[y != 0][sz][m][x];
          if ((x == 0 || x == kTT - 1) && (y == 0 || y == kTT - 1))
            a += (double)s_cr[x != 0][y != 0][sz][m];
          v[j] += a;
        }
      }
      if (live) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int x = 4 * h + (j >> 1), y = 4 * (j & 1) + w;
          const float r = (float)v[j];
          rho[((size_t)(ti * kTT + x) * n + (tj * kTT + y)) * n + kg] = r;
          sum += (double)r;
        }
      }
    }
  }
  if (partial) {
    sum = wave_sum_double(sum);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
      double b = 0.0;
      for (int q = 0; q < kGatherThreads / 64; ++q) b += ws[q];
      partial[blockIdx.x] = b;
    }
  }
}

// mean = (sum of the block sums of rho) / count, in FP64 in a fixed order
__global__ __launch_bounds__(kThreads) void k_fix_mean(const double *__restrict__ partial,
                                                       int nblocks, int64_t count,
                                                       float *__restrict__ mean) {
  double sum = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kThreads) sum += partial[b];
  __shared__ double ws[kThreads / 64];
  sum = wave_sum_double(sum);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) t += ws[w];
    *mean = (float)(t / (double)count);
  }
}

// Interpolation + kick from particles bucketed by tile (the deposit's sort of the same
// positions): one workgroup per 8^3 tile stages the force grid of the tile plus a
// one-cell halo in LDS, then each particle of the tile gathers its 27 (8) window
// values from LDS instead of from the cache hierarchy.
template <int MAS, int PK>
__global__ __launch_bounds__(kOThreads) void k_interp_tile(const float *__restrict__ pos,
                                                           const int32_t *__restrict__ cell,
                                                           const int32_t *__restrict__ end,
                                                           const int32_t *__restrict__ perm,
                                                           int n, const float *__restrict__ g,
                                                           float *__restrict__ acc,
                                                           float *__restrict__ vel, float kick) {
  __shared__ float gs[3][kTHalo];
  const int nt = n / kTT;
  const int tile = (int)xcd_block(blockIdx.x, gridDim.x);
  const int tk = tile % nt, tj = (tile / nt) % nt, ti = tile / (nt * nt);
  const int i0 = ti * kTT - 1, j0 = tj * kTT - 1, k0 = tk * kTT - 1;
  // all of a thread's loads in flight before the first LDS write
  constexpr int kGS = 3 * kTHalo, kGSIt = (kGS + kOThreads - 1) / kOThreads;
  float gv[kGSIt];
#pragma unroll
  for (int u = 0; u < kGSIt; ++u) {
    const int e = (int)threadIdx.x + u * kOThreads;
    if (e < kGS) {
      const int h = e / 3, d = e - 3 * h;
      const int hx = h / (kTH * kTH), hy = (h / kTH) % kTH, hz = h % kTH;
      const size_t gc = ((size_t)wrap_index(i0 + hx, n) * n + wrap_index(j0 + hy, n)) * n +
                        wrap_index(k0 + hz, n);
      gv[u] = g[3 * gc + d];
    }
  }
#pragma unroll
  for (int u = 0; u < kGSIt; ++u) {
    const int e = (int)threadIdx.x + u * kOThreads;
    if (e < kGS) gs[e % 3][e / 3] = gv[u];
  }
  __syncthreads();
  const int p_begin = tile > 0 ? end[tile - 1] : 0;
  const int p_end = end[tile];
  for (int l = p_begin + (int)threadIdx.x; l < p_end; l += kOThreads) {
    const int p = perm[l];
    int c[3];
    float o[3];
    particle_cell<PK>(pos, cell, p, n, c, o);
    const int lx = c[0] - ti * kTT, ly = c[1] - tj * kTT, lz = c[2] - tk * kTT;
    if ((unsigned)lx >= (unsigned)kTT || (unsigned)ly >= (unsigned)kTT ||
        (unsigned)lz >= (unsigned)kTT)
      continue;  // not this tile's particle (cannot happen with the same cell rule)
    float wx[MAS], wy[MAS], wz[MAS];
    const int fx = axis_off<MAS>(lx + 1, o[0], wx);
    const int fy = axis_off<MAS>(ly + 1, o[1], wy);
    const int fz = axis_off<MAS>(lz + 1, o[2], wz);
    float ax = 0.f, ay = 0.f, az = 0.f;
#pragma unroll
    for (int a = 0; a < MAS; ++a)
#pragma unroll
      for (int b = 0; b < MAS; ++b) {
        const float wab = wx[a] * wy[b];
        const int row = ((fx + a) * kTH + (fy + b)) * kTH + fz;
#pragma unroll
        for (int cc = 0; cc < MAS; ++cc) {
          const float wc = wab * wz[cc];
          ax = fmaf(wc, gs[0][row + cc], ax);
          ay = fmaf(wc, gs[1][row + cc], ay);
          az = fmaf(wc, gs[2][row + cc], az);
        }
      }
    if (acc) {
      acc[3 * (size_t)p + 0] = ax;
      acc[3 * (size_t)p + 1] = ay;
      acc[3 * (size_t)p + 2] = az;
    }
    if (vel) {
      vel[3 * (size_t)p + 0] = fmaf(kick, ax, vel[3 * (size_t)p + 0]);
      vel[3 * (size_t)p + 1] = fmaf(kick, ay, vel[3 * (size_t)p + 1]);
      vel[3 * (size_t)p + 2] = fmaf(kick, az, vel[3 * (size_t)p + 2]);
    }
  }
}

// Gradient and interpolation in one pass: the tile's potential plus a three-cell halo
// is staged in LDS, g = -grad phi (5-point central difference, same arithmetic as the
// gradient kernel) is formed for the tile plus a one-cell halo, and the particles
// gather from it; the force grid never goes to memory.
//
// DRIFT: after the kick the particle also drifts by dt (the opening kick of the next
// leapfrog step is folded into `kick`), and the new 8^3-tile key and histogram of the
// next deposit's sort go to pcell and count, as in the kick-drift kernel. Each particle
// is read and written by the one thread that owns it in its tile bucket.
template <int MAS, int PK, bool DRIFT, bool VEC>
__global__ __launch_bounds__(kIThreads) void k_interp_tile_phi(float *__restrict__ pos,
                                                               int32_t *__restrict__ cell,
                                                               const int32_t *__restrict__ end,
                                                               const int32_t *__restrict__ perm,
                                                               int n,
                                                               const float *__restrict__ phi,
                                                               float *__restrict__ acc,
                                                               float *__restrict__ vel,
                                                               float kick, float dt,
                                                               int32_t *__restrict__ pcell,
                                                               int32_t *__restrict__ count) {
  // potential of the tile plus 3 cells per side along i and j; along k 16 cells from 4
  // below the tile (rows of four aligned float4, one of them unused per side)
  constexpr int PH = kTT + 6, PZ = kTT + 8;
  __shared__ __align__(16) float ps[PH * PH * PZ + 4];  // + a slot for surplus staging items
  __shared__ float gs[3][kTHalo];
  const int nt = n / kTT;
  const int tile = (int)xcd_block(blockIdx.x, gridDim.x);
  const int tk = tile % nt, tj = (tile / nt) % nt, ti = tile / (nt * nt);
  const int i0 = ti * kTT - 3, j0 = tj * kTT - 3, k0 = tk * kTT - 4;
  const int p_begin = tile > 0 ? end[tile - 1] : 0;
  const int p_end = end[tile];
  if (p_begin >= p_end) return;  // no particles: nothing to stage (the histogram gets none)
  TileParticle cur = load_particle<PK>(pos, cell, vel, tile_index(perm, p_begin, p_end));
  int pnext = tile_index(perm, p_begin + kIThreads, p_end);
  // all of a thread's loads in flight before the first LDS write
  if constexpr (VEC) {
    // n % 8 == 0 and phi 16-byte aligned: every float4 of a row (k0 + 4 q, q = 0..3,
    // wrapped) lies in one row of the grid at a multiple of four
    constexpr int kItems = PH * PH * 4, kIt = (kItems + kIThreads - 1) / kIThreads;
    float4 pv[kIt];
#pragma unroll
    for (int u = 0; u < kIt; ++u) {
      // past the last item: a repeated load of it (every element written, so the array
      // stays in registers and all loads are in flight together)
      const int e = min((int)threadIdx.x + u * kIThreads, kItems - 1);
      const int r = e >> 2, q = e & 3, hx = r / PH, hy = r % PH;
      pv[u] = *reinterpret_cast<const float4 *>(
          phi + ((size_t)wrap_index(i0 + hx, n) * n + wrap_index(j0 + hy, n)) * n +
          wrap_index(k0 + 4 * q, n));
    }
#pragma unroll
    for (int u = 0; u < kIt; ++u) {
      const int e = (int)threadIdx.x + u * kIThreads;
      const int at = e < kItems ? (e >> 2) * PZ + 4 * (e & 3) : PH * PH * PZ;
      *reinterpret_cast<float4 *>(ps + at) = pv[u];
    }
  } else {
    constexpr int kPS = PH * PH * PZ, kPSIt = (kPS + kIThreads - 1) / kIThreads;
    float pv[kPSIt];
#pragma unroll
    for (int u = 0; u < kPSIt; ++u) {
      const int e = min((int)threadIdx.x + u * kIThreads, kPS - 1);
      const int hx = e / (PH * PZ), hy = (e / PZ) % PH, hz = e % PZ;
      pv[u] = phi[((size_t)wrap_index(i0 + hx, n) * n + wrap_index(j0 + hy, n)) * n +
                  wrap_index(k0 + hz, n)];
    }
#pragma unroll
    for (int u = 0; u < kPSIt; ++u) {
      const int e = (int)threadIdx.x + u * kIThreads;
      ps[e < kPS ? e : kPS] = pv[u];
    }
  }
  __syncthreads();
  const float c1 = 2.0f / 3.0f, c2 = -1.0f / 12.0f, inv_h = (float)n;
  for (int h = threadIdx.x; h < kTHalo; h += kIThreads) {
    const int cx = h / (kTH * kTH) + 2, cy = (h / kTH) % kTH + 2, cz = h % kTH + 3;
    const int c = (cx * PH + cy) * PZ + cz;
    float gx = c1 * (ps[c + PH * PZ] - ps[c - PH * PZ]);
    gx = fmaf(c2, ps[c + 2 * PH * PZ] - ps[c - 2 * PH * PZ], gx);
    float gy = c1 * (ps[c + PZ] - ps[c - PZ]);
    gy = fmaf(c2, ps[c + 2 * PZ] - ps[c - 2 * PZ], gy);
    float gz = c1 * (ps[c + 1] - ps[c - 1]);
    gz = fmaf(c2, ps[c + 2] - ps[c - 2], gz);
    gs[0][h] = -inv_h * gx;
    gs[1][h] = -inv_h * gy;
    gs[2][h] = -inv_h * gz;
  }
  __syncthreads();
  // uniform trip count: with DRIFT the whole wave takes part in the histogram's run
  // detection. Each pass loads the particles of the next pass and the indices of the
  // one after before it works on its own; the first pass's particles and the second's
  // indices are loaded before the potential is staged.
  for (int l0 = p_begin; l0 < p_end; l0 += kIThreads) {
    const TileParticle nxt = load_particle<PK>(pos, cell, vel, pnext);
    pnext = tile_index(perm, l0 + 2 * kIThreads, p_end);
    int key = -1;
    if (cur.live) {
      const int p = cur.p;
      int c[3];
      float o[3];
      cell_offset_of<PK>(cur.x, cur.c, n, c, o);
      const int lx = c[0] - ti * kTT, ly = c[1] - tj * kTT, lz = c[2] - tk * kTT;
      // every particle of the bucket lies in this tile (same cell rule as the sort)
      if ((unsigned)lx < (unsigned)kTT && (unsigned)ly < (unsigned)kTT &&
          (unsigned)lz < (unsigned)kTT) {
        float wx[MAS], wy[MAS], wz[MAS];
        const int fx = axis_off<MAS>(lx + 1, o[0], wx);
        const int fy = axis_off<MAS>(ly + 1, o[1], wy);
        const int fz = axis_off<MAS>(lz + 1, o[2], wz);
        float ax = 0.f, ay = 0.f, az = 0.f;
#pragma unroll
        for (int a = 0; a < MAS; ++a)
#pragma unroll
          for (int b = 0; b < MAS; ++b) {
            const float wab = wx[a] * wy[b];
            const int row = ((fx + a) * kTH + (fy + b)) * kTH + fz;
#pragma unroll
            for (int cc = 0; cc < MAS; ++cc) {
              const float wc = wab * wz[cc];
              ax = fmaf(wc, gs[0][row + cc], ax);
              ay = fmaf(wc, gs[1][row + cc], ay);
              az = fmaf(wc, gs[2][row + cc], az);
            }
          }
        if (acc) {
          acc[3 * (size_t)p + 0] = ax;
          acc[3 * (size_t)p + 1] = ay;
          acc[3 * (size_t)p + 2] = az;
        }
        if (vel) {
          float v[3];
          v[0] = fmaf(kick, ax, cur.v[0]);
          v[1] = fmaf(kick, ay, cur.v[1]);
          v[2] = fmaf(kick, az, cur.v[2]);
#pragma unroll
          for (int d = 0; d < 3; ++d) vel[3 * (size_t)p + d] = v[d];
          if constexpr (DRIFT) {
            key = drift_from<PK>(pos, cell, p, n, dt, v, cur.x, cur.c);
            pcell[p] = key;
          }
        }
      }
    }
    if constexpr (DRIFT) {
      const WaveRun r = wave_runs(key);
      if (r.head && key >= 0) atomicAdd(&count[key], r.len);
    }
    cur = nxt;
  }
}


}  // namespace

hipError_t launch_deposit_atomic(const float *pos, const int32_t *cell, int64_t np, int poskind,
                                 int mas, int n, float mass, float *rho, hipStream_t s) {
  if (np == 0) return hipSuccess;
  const unsigned nb = blocks_for(np, kGChunk);
  if (mas == PM_TSC) {
    if (poskind == PM_POS_BOX)
      k_deposit_chunk<3, PM_POS_BOX><<<nb, kGThreads, 0, s>>>(pos, cell, np, n, mass, rho);
    else
      k_deposit_chunk<3, PM_POS_CELLOFF><<<nb, kGThreads, 0, s>>>(pos, cell, np, n, mass, rho);
  } else if (mas == PM_NGP) {
    if (poskind == PM_POS_BOX)
      k_deposit_chunk<1, PM_POS_BOX><<<nb, kGThreads, 0, s>>>(pos, cell, np, n, mass, rho);
    else
      k_deposit_chunk<1, PM_POS_CELLOFF><<<nb, kGThreads, 0, s>>>(pos, cell, np, n, mass, rho);
  } else {
    if (poskind == PM_POS_BOX)
      k_deposit_chunk<2, PM_POS_BOX><<<nb, kGThreads, 0, s>>>(pos, cell, np, n, mass, rho);
    else
      k_deposit_chunk<2, PM_POS_CELLOFF><<<nb, kGThreads, 0, s>>>(pos, cell, np, n, mass, rho);
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
  } else if (mas == PM_NGP) {
    if (poskind == PM_POS_BOX)
      k_interp<1, PM_POS_BOX><<<nb, kThreads, 0, s>>>(pos, cell, np, n, g, acc, vel, kick);
    else
      k_interp<1, PM_POS_CELLOFF><<<nb, kThreads, 0, s>>>(pos, cell, np, n, g, acc, vel, kick);
  } else {
    if (poskind == PM_POS_BOX)
      k_interp<2, PM_POS_BOX><<<nb, kThreads, 0, s>>>(pos, cell, np, n, g, acc, vel, kick);
    else
      k_interp<2, PM_POS_CELLOFF><<<nb, kThreads, 0, s>>>(pos, cell, np, n, g, acc, vel, kick);
  }
  return hipGetLastError();
}

hipError_t launch_kick_drift(float *pos, int32_t *cell, float *vel, const float *acc, int64_t np,
                             int poskind, int n, float kick, float dt, hipStream_t s,
                             int32_t *pcell, int32_t *count) {
  if (np == 0) return hipSuccess;
  const unsigned nb = blocks_for(np, kThreads);
  if (poskind == PM_POS_BOX)
    k_kick_drift<PM_POS_BOX><<<nb, kThreads, 0, s>>>(pos, cell, vel, acc, np, n, kick, dt, pcell,
                                                      count);
  else
    k_kick_drift<PM_POS_CELLOFF><<<nb, kThreads, 0, s>>>(pos, cell, vel, acc, np, n, kick, dt,
                                                          pcell, count);
  return hipGetLastError();
}

hipError_t launch_sort_by_cell(pm_ctx *ctx, const float *pos, const int32_t *cell, int64_t np,
                               int poskind, hipStream_t s, int keymode, bool hist_done) {
  const int n = ctx->n;
  const int64_t nkeys = keymode == kKeyTile ? (int64_t)(n / 8) * (n / 8) * (n / 8)
                                            : (int64_t)n * n * n;
  const int64_t len = nkeys + 1;
  if (!hist_done) {
    hipError_t e = hipMemsetAsync(ctx->cell_count, 0, sizeof(int32_t) * len, s);
    if (e != hipSuccess) return e;
  }
  if (np > 0 && !hist_done) {
    const unsigned nbr = blocks_for(np, kThreads * kSortRounds);
#define PM_HIST(PKV, KEYV)                                                                   \
  k_cell_hist<PKV, KEYV><<<nbr, kThreads, 0, s>>>(pos, cell, np, n, ctx->pcell, ctx->cell_count)
    if (poskind == PM_POS_BOX) {
      if (keymode == kKeyTile) PM_HIST(PM_POS_BOX, kKeyTile);
      else PM_HIST(PM_POS_BOX, kKeyCell);
    } else {
      if (keymode == kKeyTile) PM_HIST(PM_POS_CELLOFF, kKeyTile);
      else PM_HIST(PM_POS_CELLOFF, kKeyCell);
    }
#undef PM_HIST
  }
  const unsigned nblk = blocks_for(len, kScanTile);
  k_scan_reduce<<<nblk, kScanThreads, 0, s>>>(ctx->cell_count, len, ctx->scan_partial);
  k_scan_partials<<<1, kScanThreads, 0, s>>>(ctx->scan_partial, (int)nblk);
  // in-place exclusive scan: cell_count[c] = start of cell c; the scatter then
  // advances it to the end of cell c (= start of c + 1), the layout the gathers read
  k_scan_apply<<<nblk, kScanThreads, 0, s>>>(ctx->cell_count, len, ctx->scan_partial);
  if (np > 0)
    k_scatter_perm<<<blocks_for(np, kThreads * kSortRounds), kThreads, 0, s>>>(ctx->pcell, np,
                                                                  ctx->cell_count, ctx->perm);
  return hipGetLastError();
}

int64_t scan_blocks_needed(int64_t len) { return (len + kScanTile - 1) / kScanTile; }

hipError_t launch_deposit_own(pm_ctx *ctx, const float *pos, const int32_t *cell, int poskind,
                              int mas, float mass, float *rho, float *mean, hipStream_t s) {
  const int n = ctx->n;
  const int64_t ncell = (int64_t)n * n * n;
  const unsigned nt = (unsigned)(ncell / kTThreads);
  float *tbox = ctx->tile_box;
  // fixed-point unit 2^-30 times the particle weight
  const double scale = (double)mass / 1073741824.0;
#define PM_DO(M, K)                                                                             \
  k_deposit_own<M, K><<<nt, kDThreads, 0, s>>>(pos, cell, ctx->cell_count, ctx->perm, n, scale, \
                                               tbox)
  if (mas == PM_TSC) {
    if (poskind == PM_POS_BOX) PM_DO(3, PM_POS_BOX);
    else PM_DO(3, PM_POS_CELLOFF);
  } else if (mas == PM_NGP) {
    if (poskind == PM_POS_BOX) PM_DO(1, PM_POS_BOX);
    else PM_DO(1, PM_POS_CELLOFF);
  } else {
    if (poskind == PM_POS_BOX) PM_DO(2, PM_POS_BOX);
    else PM_DO(2, PM_POS_CELLOFF);
  }
#undef PM_DO
  // block sums go to the reduction scratch (free until the solve that follows)
  double *partial = ctx->red_partial;
  const int ntile = n / kTT;
  const int64_t rows = (int64_t)ntile * ntile * ((ntile + kGRow - 1) / kGRow);
  const int nb = (int)std::min<int64_t>(rows, kGatherBlocks);
  k_tile_gather<<<nb, kGatherThreads, 0, s>>>(tbox, ctx->cell_count, n, rows, rho,
                                              mean ? partial : nullptr);
  if (mean) k_fix_mean<<<1, kThreads, 0, s>>>(partial, nb, ncell, mean);
  return hipGetLastError();
}

hipError_t launch_interp_tile(pm_ctx *ctx, const float *pos, const int32_t *cell, int poskind,
                              int mas, const float *g, float *acc, float *vel, float kick,
                              hipStream_t s) {
  const int n = ctx->n;
  const unsigned nt = (unsigned)((int64_t)n * n * n / kTThreads);
#define PM_IT(M, K)                                                                           \
  k_interp_tile<M, K><<<nt, kOThreads, 0, s>>>(pos, cell, ctx->cell_count, ctx->perm, n, g, acc, \
                                               vel, kick)
  if (mas == PM_TSC) {
    if (poskind == PM_POS_BOX) PM_IT(3, PM_POS_BOX);
    else PM_IT(3, PM_POS_CELLOFF);
  } else if (mas == PM_NGP) {
    if (poskind == PM_POS_BOX) PM_IT(1, PM_POS_BOX);
    else PM_IT(1, PM_POS_CELLOFF);
  } else {
    if (poskind == PM_POS_BOX) PM_IT(2, PM_POS_BOX);
    else PM_IT(2, PM_POS_CELLOFF);
  }
#undef PM_IT
  return hipGetLastError();
}

hipError_t launch_interp_tile_phi(pm_ctx *ctx, float *pos, int32_t *cell, int poskind, int mas,
                                  const float *phi, float *acc, float *vel, float kick, float dt,
                                  int32_t *pcell, int32_t *count, hipStream_t s) {
  const int n = ctx->n;
  const unsigned nt = (unsigned)((int64_t)n * n * n / kTThreads);
  const bool drift = count != nullptr;
  if (drift && (!vel || !pcell)) return hipErrorInvalidValue;
  // the potential is staged with float4 loads when its rows are 16-byte aligned
  const bool vec = reinterpret_cast<uintptr_t>(phi) % 16 == 0;
#define PM_ITP2(M, K, V)                                                                         \
  do {                                                                                           \
    if (drift)                                                                                   \
      k_interp_tile_phi<M, K, true, V><<<nt, kIThreads, 0, s>>>(                                 \
          pos, cell, ctx->cell_count, ctx->perm, n, phi, acc, vel, kick, dt, pcell, count);      \
    else                                                                                         \
      k_interp_tile_phi<M, K, false, V><<<nt, kIThreads, 0, s>>>(                                \
          pos, cell, ctx->cell_count, ctx->perm, n, phi, acc, vel, kick, dt, nullptr, nullptr);  \
  } while (0)
#define PM_ITP(M, K)                                                                             \
  do {                                                                                           \
    if (vec) PM_ITP2(M, K, true);                                                                \
    else PM_ITP2(M, K, false);                                                                   \
  } while (0)
  if (mas == PM_TSC) {
    if (poskind == PM_POS_BOX) PM_ITP(3, PM_POS_BOX);
    else PM_ITP(3, PM_POS_CELLOFF);
  } else if (mas == PM_NGP) {
    if (poskind == PM_POS_BOX) PM_ITP(1, PM_POS_BOX);
    else PM_ITP(1, PM_POS_CELLOFF);
  } else {
    if (poskind == PM_POS_BOX) PM_ITP(2, PM_POS_BOX);
    else PM_ITP(2, PM_POS_CELLOFF);
  }
#undef PM_ITP
#undef PM_ITP2
  return hipGetLastError();
}

hipError_t launch_deposit_pull(pm_ctx *ctx, const float *pos, int64_t np, int poskind, int mas,
                               float mass, float *rho, hipStream_t s) {
  (void)np;
  const int n = ctx->n;
  const int64_t ncell = (int64_t)n * n * n;
  const unsigned nb = blocks_for(ncell, kThreads);
  if (mas == PM_TSC) {
    if (poskind == PM_POS_BOX)
      k_deposit_pull<3, PM_POS_BOX><<<nb, kThreads, 0, s>>>(pos, ctx->cell_count, ctx->perm, n,
                                                              mass, rho);
    else
      k_deposit_pull<3, PM_POS_CELLOFF><<<nb, kThreads, 0, s>>>(pos, ctx->cell_count, ctx->perm,
                                                                  n, mass, rho);
  } else if (mas == PM_NGP) {
    if (poskind == PM_POS_BOX)
      k_deposit_pull<1, PM_POS_BOX><<<nb, kThreads, 0, s>>>(pos, ctx->cell_count, ctx->perm, n,
                                                              mass, rho);
    else
      k_deposit_pull<1, PM_POS_CELLOFF><<<nb, kThreads, 0, s>>>(pos, ctx->cell_count, ctx->perm,
                                                                  n, mass, rho);
  } else {
    if (poskind == PM_POS_BOX)
      k_deposit_pull<2, PM_POS_BOX><<<nb, kThreads, 0, s>>>(pos, ctx->cell_count, ctx->perm, n,
                                                              mass, rho);
    else
      k_deposit_pull<2, PM_POS_CELLOFF><<<nb, kThreads, 0, s>>>(pos, ctx->cell_count, ctx->perm,
                                                                  n, mass, rho);
  }
  return hipGetLastError();
}

// Permute particle arrays in place through ctx->perm (the sorted order), via scratch.
hipError_t launch_tile_cell_sort(pm_ctx *ctx, const float *pos, const int32_t *cell,
                                 int poskind, int32_t *out, hipStream_t s) {
  const int n = ctx->n;
  const unsigned nt = (unsigned)((int64_t)n * n * n / 512);
  if (poskind == PM_POS_BOX)
    k_tile_cell_sort<PM_POS_BOX><<<nt, kThreads, 0, s>>>(pos, cell, ctx->cell_count, ctx->perm, n,
                                                         out);
  else
    k_tile_cell_sort<PM_POS_CELLOFF><<<nt, kThreads, 0, s>>>(pos, cell, ctx->cell_count,
                                                             ctx->perm, n, out);
  return hipGetLastError();
}

hipError_t launch_apply_perm(pm_ctx *ctx, const int32_t *order, float *pos, int32_t *cell,
                             float *vel, float *acc, int64_t *ids, int64_t np, hipStream_t s) {
  if (np == 0) return hipSuccess;
  const unsigned nb = blocks_for(np, kThreads);
  float *tmp = (float *)ctx->reorder_tmp;
  hipError_t e = hipSuccess;
  float *f3[3] = {pos, vel, acc};
  for (int a = 0; a < 3 && e == hipSuccess; ++a) {
    if (!f3[a]) continue;
    k_gather_perm<float, 3><<<nb, kThreads, 0, s>>>(f3[a], order, np, tmp);
    e = hipMemcpyAsync(f3[a], tmp, sizeof(float) * 3 * (size_t)np, hipMemcpyDeviceToDevice, s);
  }
  if (e == hipSuccess && cell) {
    k_gather_perm<int32_t, 1><<<nb, kThreads, 0, s>>>(cell, order, np, (int32_t *)tmp);
    e = hipMemcpyAsync(cell, tmp, sizeof(int32_t) * (size_t)np, hipMemcpyDeviceToDevice, s);
  }
  if (e == hipSuccess && ids) {
    k_gather_perm<int64_t, 1><<<nb, kThreads, 0, s>>>(ids, order, np, (int64_t *)tmp);
    e = hipMemcpyAsync(ids, tmp, sizeof(int64_t) * (size_t)np, hipMemcpyDeviceToDevice, s);
  }
  if (e != hipSuccess) return e;
  return hipGetLastError();
}
