// Particle-side kernels: mass assignment (atomic scatter and cell-sorted gather),
// interpolation with an optional fused kick, kick + drift, and the counting sort
// that buckets particles by cell. Paper Sect. 3.5 (windows), Sect. 3.4 (leapfrog),
// App. E (particle ordering for locality).
#include "deposit_chunk.h"
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
using pm_chunk::wrap_any;
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

// Tile-major cell key: 8^3-cell tiles in row-major order, cells row-major inside
// a tile (a bijection of [0, n^3) when n is a multiple of 8).
__device__ __forceinline__ int tile_key(int ci, int cj, int ck, int n) {
  const int nt = n >> 3;
  return ((((ci >> 3) * nt + (cj >> 3)) * nt + (ck >> 3)) << 9) +
         ((((ci & 7) << 3) + (cj & 7)) << 3) + (ck & 7);
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

// Cell containing each particle (as a row-major or tile-major key); histogram with
// one atomic per run of equal keys in a wave.
template <int PK, bool TILE>
__global__ __launch_bounds__(kThreads) void k_cell_hist(const float *__restrict__ pos,
                                                        const int32_t *__restrict__ cell,
                                                        int64_t np, int n,
                                                        int32_t *__restrict__ pcell,
                                                        int32_t *__restrict__ count) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  int c = -1;
  if (p < np) {
    int q[3];
    if constexpr (PK == PM_POS_BOX) {
      const float fn = (float)n;
#pragma unroll
      for (int d = 0; d < 3; ++d) q[d] = wrap_any((int)floorf(pos[3 * p + d] * fn), n);
    } else {
      const int cc = wrap_any(cell[p], n * n * n);
      q[0] = cc / (n * n);
      q[1] = (cc / n) - q[0] * n;
      q[2] = cc - (cc / n) * n;
    }
    c = TILE ? tile_key(q[0], q[1], q[2], n) : (q[0] * n + q[1]) * n + q[2];
    pcell[p] = c;
  }
  const WaveRun r = wave_runs(c);
  if (r.head && c >= 0) atomicAdd(&count[c], r.len);
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


__global__ __launch_bounds__(kThreads) void k_scatter_perm(const int32_t *__restrict__ pcell,
                                                           int64_t np,
                                                           int32_t *__restrict__ cursor,
                                                           int32_t *__restrict__ perm) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int c = p < np ? pcell[p] : -1;
  const WaveRun r = wave_runs(c);
  int base = 0;
  if (r.head && c >= 0) base = atomicAdd(&cursor[c], r.len);
  base = __shfl(base, r.headlane, 64);
  if (c >= 0) perm[base + ((int)(threadIdx.x & 63) - r.headlane)] = (int32_t)p;
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

// ------------------------------------------------------------------ tile-owned deposit

// One block owns an 8^3 tile of output cells and reads the particles of the
// tile's 10^3 halo cells through the per-cell ranges of the counting sort. A
// particle in cell q adds to output cell t = q - D (D in {-1,0,1}^3) the weight
// prod_d W(D_d + o_d - 1/2), o its in-cell offset. Weights are rounded to
// multiples of 2^-30 and summed in 64-bit integers held in LDS (integer LDS
// atomics are an order of magnitude faster than FP32 ones on this GPU, and the
// integer sum is exact, so the grid is bitwise reproducible):
//   * particles of sparse halo cells (<= kDense) add their in-tile weights with
//     one LDS atomic each;
//   * the particles of a dense halo cell are first reduced by one wave to the
//     cell's 27 window moments M_q[D] = sum_p prod_d W(D_d + o_pd - 1/2), which
//     are then added to the tile (avoiding 64 lanes updating the same words).
// Every output cell is written once: no atomics on the grid.
constexpr int kTT = 8;                        // tile edge
constexpr int kTThreads = kTT * kTT * kTT;    // 512
constexpr int kTH = kTT + 2;                  // halo edge
constexpr int kTHalo = kTH * kTH * kTH;       // 1000
constexpr int kDense = 32;                    // particles above which a cell is dense
constexpr float kFix30 = 1073741824.0f;       // 2^30 units per unit weight

__device__ __forceinline__ unsigned long long fix30(float w) {
  // 0 <= w <= 27/64 < 2: w 2^30 fits an int32; rounding to 2^-30 keeps every bit
  // of the FP32 weight above 2^-30
  return (unsigned long long)(unsigned int)rintf(w * kFix30);
}

__device__ __forceinline__ unsigned long long wave_sum_ull(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

template <int PK>
__device__ __forceinline__ void load_offset(const float *__restrict__ pos, int64_t p, int n,
                                            float o[3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    float x = pos[3 * p + d];
    if constexpr (PK == PM_POS_BOX) {
      const float u = x * (float)n;
      x = u - floorf(u);
    }
    o[d] = x;
  }
}

template <int MAS, int PK>
__global__ __launch_bounds__(kTThreads) void k_deposit_tile(const float *__restrict__ pos,
                                                            const int32_t *__restrict__ start,
                                                            const int32_t *__restrict__ perm,
                                                            int n, float mass,
                                                            float *__restrict__ rho) {
  __shared__ unsigned long long accum[kTThreads];
  __shared__ int lstart[kTHalo + 1];     // local starts of the sparse halo cells
  __shared__ int gstart[kTHalo];         // global starts (in the sorted order)
  __shared__ int gcount[kTHalo];         // particle counts
  __shared__ short dlist[kTHalo];        // dense halo cells
  __shared__ int wsum[kTThreads / 64];
  __shared__ int wdense[kTThreads / 64];
  const int nt = n / kTT;
  const int tile = (int)xcd_block(blockIdx.x, gridDim.x);
  const int tk = tile % nt, tj = (tile / nt) % nt, ti = tile / (nt * nt);
  const int i0 = ti * kTT - 1, j0 = tj * kTT - 1, k0 = tk * kTT - 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  accum[threadIdx.x] = 0ull;

  // 1. halo cell ranges (two per thread); sparse counts are scanned, dense cells listed
  int cnt[2], gs[2];
  bool dn[2];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int h = threadIdx.x * 2 + r;
    cnt[r] = 0;
    gs[r] = 0;
    if (h < kTHalo) {
      const int hx = h / (kTH * kTH), hy = (h / kTH) % kTH, hz = h % kTH;
      const int g = (wrap_index(i0 + hx, n) * n + wrap_index(j0 + hy, n)) * n + wrap_index(k0 + hz, n);
      gs[r] = g > 0 ? start[g - 1] : 0;   // `start` holds cell ends: end[g] = start of g + 1
      cnt[r] = start[g] - gs[r];
      gstart[h] = gs[r];
      gcount[h] = cnt[r];
    }
    dn[r] = cnt[r] > kDense;
  }
  const int sp0 = dn[0] ? 0 : cnt[0], sp1 = dn[1] ? 0 : cnt[1];
  const int tot = sp0 + sp1, dtot = (int)dn[0] + (int)dn[1];
  int x = tot, y = dtot;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int xs = __shfl_up(x, o, 64), ys = __shfl_up(y, o, 64);
    if (lane >= o) {
      x += xs;
      y += ys;
    }
  }
  if (lane == 63) {
    wsum[wave] = x;
    wdense[wave] = y;
  }
  __syncthreads();
  int woff = 0, all = 0, doff = 0, ndense = 0;
  for (int w = 0; w < kTThreads / 64; ++w) {
    if (w < wave) {
      woff += wsum[w];
      doff += wdense[w];
    }
    all += wsum[w];
    ndense += wdense[w];
  }
  {
    const int h = threadIdx.x * 2;
    int ex = x - tot + woff, dx = y - dtot + doff;
    if (h < kTHalo) {
      lstart[h] = ex;
      if (dn[0]) dlist[dx++] = (short)h;
    }
    if (h + 1 < kTHalo) {
      lstart[h + 1] = ex + sp0;
      if (dn[1]) dlist[dx] = (short)(h + 1);
    }
    if (threadIdx.x == 0) lstart[kTHalo] = all;
  }
  __syncthreads();

  // 2. sparse particles: one per thread at a time, in-tile weights added to LDS;
  //    the slot's halo cell comes from a binary search in the local starts
  for (int l = threadIdx.x; l < all; l += kTThreads) {
    int lo_h = 0, hi_h = kTHalo;  // h with lstart[h] <= l < lstart[h + 1]
    while (hi_h - lo_h > 1) {
      const int mid = (lo_h + hi_h) >> 1;
      if (lstart[mid] <= l) lo_h = mid; else hi_h = mid;
    }
    const int h = lo_h;
    float o[3];
    load_offset<PK>(pos, perm[gstart[h] + (l - lstart[h])], n, o);
    const int hx = h / (kTH * kTH), hy = (h / kTH) % kTH, hz = h % kTH;
    float wx[3], wy[3], wz[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      wx[t] = window_sep<MAS>((float)(t - 1) + o[0] - 0.5f);
      wy[t] = window_sep<MAS>((float)(t - 1) + o[1] - 0.5f);
      wz[t] = window_sep<MAS>((float)(t - 1) + o[2] - 0.5f);
    }
    // target t = q - D in tile coordinates: (hx - 1) - (a - 1) = hx - a
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int tx = hx - a;
      if (tx < 0 || tx >= kTT) continue;
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const int ty = hy - b;
        if (ty < 0 || ty >= kTT) continue;
        const float wab = wx[a] * wy[b];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const int tz = hz - c;
          if (tz < 0 || tz >= kTT) continue;
          const unsigned long long v = fix30(wab * wz[c]);
          if (v) atomicAdd(&accum[(tx * kTT + ty) * kTT + tz], v);
        }
      }
    }
  }

  // 3. dense cells: one wave reduces a cell's particles to 27 moments, then lanes
  //    0..26 add them to the in-tile targets
  for (int di = wave; di < ndense; di += kTThreads / 64) {
    const int h = dlist[di];
    const int g0 = gstart[h], c = gcount[h];
    unsigned long long m[27];
#pragma unroll
    for (int q = 0; q < 27; ++q) m[q] = 0ull;
    for (int l = lane; l < c; l += 64) {
      float o[3];
      load_offset<PK>(pos, perm[g0 + l], n, o);
      float wx[3], wy[3], wz[3];
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        wx[t] = window_sep<MAS>((float)(t - 1) + o[0] - 0.5f);
        wy[t] = window_sep<MAS>((float)(t - 1) + o[1] - 0.5f);
        wz[t] = window_sep<MAS>((float)(t - 1) + o[2] - 0.5f);
      }
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          const float wab = wx[a] * wy[b];
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) m[(a * 3 + b) * 3 + cc] += fix30(wab * wz[cc]);
        }
    }
    const int hx = h / (kTH * kTH), hy = (h / kTH) % kTH, hz = h % kTH;
#pragma unroll
    for (int q = 0; q < 27; ++q) {
      const unsigned long long v = wave_sum_ull(m[q]);
      const int a = q / 9, b = (q / 3) % 3, cc = q % 3;
      const int tx = hx - a, ty = hy - b, tz = hz - cc;
      if (lane == 0 && tx >= 0 && tx < kTT && ty >= 0 && ty < kTT && tz >= 0 && tz < kTT)
        atomicAdd(&accum[(tx * kTT + ty) * kTT + tz], v);
    }
  }
  __syncthreads();
  const int cx = threadIdx.x / (kTT * kTT), cy = (threadIdx.x / kTT) % kTT, cz = threadIdx.x % kTT;
  const int gi = ti * kTT + cx, gj = tj * kTT + cy, gk = tk * kTT + cz;
  rho[((size_t)gi * n + gj) * n + gk] =
      (float)((double)accum[threadIdx.x] * (1.0 / 1073741824.0) * (double)mass);
}

inline unsigned blocks_for(int64_t count, int threads) {
  return (unsigned)((count + threads - 1) / threads);
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
                               int poskind, hipStream_t s, bool tile_major) {
  const int n = ctx->n;
  const int64_t ncell = (int64_t)n * n * n;
  const int64_t len = ncell + 1;
  hipError_t e = hipMemsetAsync(ctx->cell_count, 0, sizeof(int32_t) * len, s);
  if (e != hipSuccess) return e;
  if (np > 0) {
    const unsigned nb = blocks_for(np, kThreads);
    if (tile_major) {
      if (poskind == PM_POS_BOX)
        k_cell_hist<PM_POS_BOX, true><<<nb, kThreads, 0, s>>>(pos, cell, np, n, ctx->pcell,
                                                               ctx->cell_count);
      else
        k_cell_hist<PM_POS_CELLOFF, true><<<nb, kThreads, 0, s>>>(pos, cell, np, n, ctx->pcell,
                                                                   ctx->cell_count);
    } else {
      if (poskind == PM_POS_BOX)
        k_cell_hist<PM_POS_BOX, false><<<nb, kThreads, 0, s>>>(pos, cell, np, n, ctx->pcell,
                                                                ctx->cell_count);
      else
        k_cell_hist<PM_POS_CELLOFF, false><<<nb, kThreads, 0, s>>>(pos, cell, np, n, ctx->pcell,
                                                                    ctx->cell_count);
    }
  }
  const unsigned nblk = blocks_for(len, kScanTile);
  k_scan_reduce<<<nblk, kScanThreads, 0, s>>>(ctx->cell_count, len, ctx->scan_partial);
  k_scan_partials<<<1, kScanThreads, 0, s>>>(ctx->scan_partial, (int)nblk);
  // in-place exclusive scan: cell_count[c] = start of cell c; the scatter then
  // advances it to the end of cell c (= start of c + 1), the layout the gathers read
  k_scan_apply<<<nblk, kScanThreads, 0, s>>>(ctx->cell_count, len, ctx->scan_partial);
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
  if (n % kTT == 0) {
    const unsigned nt = (unsigned)(ncell / kTThreads);
    if (mas == PM_TSC) {
      if (poskind == PM_POS_BOX)
        k_deposit_tile<3, PM_POS_BOX><<<nt, kTThreads, 0, s>>>(pos, ctx->cell_count, ctx->perm, n,
                                                                mass, rho);
      else
        k_deposit_tile<3, PM_POS_CELLOFF><<<nt, kTThreads, 0, s>>>(pos, ctx->cell_count, ctx->perm,
                                                                    n, mass, rho);
    } else {
      if (poskind == PM_POS_BOX)
        k_deposit_tile<2, PM_POS_BOX><<<nt, kTThreads, 0, s>>>(pos, ctx->cell_count, ctx->perm, n,
                                                                mass, rho);
      else
        k_deposit_tile<2, PM_POS_CELLOFF><<<nt, kTThreads, 0, s>>>(pos, ctx->cell_count, ctx->perm,
                                                                    n, mass, rho);
    }
    return hipGetLastError();
  }
  const unsigned nb = blocks_for(ncell, kThreads);
  if (mas == PM_TSC) {
    if (poskind == PM_POS_BOX)
      k_deposit_pull<3, PM_POS_BOX><<<nb, kThreads, 0, s>>>(pos, ctx->cell_count, ctx->perm, n,
                                                              mass, rho);
    else
      k_deposit_pull<3, PM_POS_CELLOFF><<<nb, kThreads, 0, s>>>(pos, ctx->cell_count, ctx->perm,
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
hipError_t launch_apply_perm(pm_ctx *ctx, float *pos, int32_t *cell, float *vel, float *acc,
                             int64_t *ids, int64_t np, hipStream_t s) {
  if (np == 0) return hipSuccess;
  const unsigned nb = blocks_for(np, kThreads);
  float *tmp = (float *)ctx->reorder_tmp;
  hipError_t e = hipSuccess;
  float *f3[3] = {pos, vel, acc};
  for (int a = 0; a < 3 && e == hipSuccess; ++a) {
    if (!f3[a]) continue;
    k_gather_perm<float, 3><<<nb, kThreads, 0, s>>>(f3[a], ctx->perm, np, tmp);
    e = hipMemcpyAsync(f3[a], tmp, sizeof(float) * 3 * (size_t)np, hipMemcpyDeviceToDevice, s);
  }
  if (e == hipSuccess && cell) {
    k_gather_perm<int32_t, 1><<<nb, kThreads, 0, s>>>(cell, ctx->perm, np, (int32_t *)tmp);
    e = hipMemcpyAsync(cell, tmp, sizeof(int32_t) * (size_t)np, hipMemcpyDeviceToDevice, s);
  }
  if (e == hipSuccess && ids) {
    k_gather_perm<int64_t, 1><<<nb, kThreads, 0, s>>>(ids, ctx->perm, np, (int64_t *)tmp);
    e = hipMemcpyAsync(ids, tmp, sizeof(int64_t) * (size_t)np, hipMemcpyDeviceToDevice, s);
  }
  if (e != hipSuccess) return e;
  return hipGetLastError();
}
