// Chunked gather deposit (paper Sect. 3.5 windows) shared by the single-box
// atomic mode and the batched ensembles, and the particle helpers it needs.
//
// A workgroup deposits a chunk of up to 2048 particles without per-weight
// atomics:
//   1. the particles' cells are taken relative to the chunk's first particle
//      (minimum image) and their bounding box P is found;
//   2. the particles are counting-sorted by cell of P inside LDS (two integer
//      LDS atomics per particle), keeping only their in-cell offsets;
//   3. every cell of P grown by one cell per side (the window's reach) sums,
//      in registers, the window values of the particles in its 27 neighbour
//      cells of P; the separation along an axis is (q - c) + o - 1/2 with
//      q - c in {-1, 0, 1} and o the in-cell offset;
//   4. non-zero sums are added to the grid with one global atomic per cell.
// Chunks whose cell box exceeds the LDS table fall back to one global atomic
// per weight. Which particles form a chunk is the caller's choice (an Index
// object maps the chunk's slots to particle rows, -1 for an empty slot): runs
// of consecutive rows after a tile-major reorder, or lattice blocks of
// particles that started on a lattice.
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


constexpr int kGThreads = 256;
constexpr int kGPPT = 8;
constexpr int kGChunk = kGThreads * kGPPT;
constexpr int kGCells = 4096;  // max cells of the particle box P

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

template <int MAS>
__device__ __forceinline__ float window_sep_g(float s) {
  const float a = fabsf(s);
  if constexpr (MAS == 3) {
    if (a < 0.5f) return 0.75f - a * a;
    const float b = 1.5f - a;
    return a < 1.5f ? 0.5f * b * b : 0.0f;
  } else {
    return a < 1.0f ? 1.0f - a : 0.0f;
  }
}

// Cell (wrapped) and in-cell offset of particle p.
template <int PK>
__device__ __forceinline__ void particle_cell(const float *__restrict__ pos,
                                              const int32_t *__restrict__ cell, int64_t p, int n,
                                              int c[3], float o[3]) {
  if constexpr (PK == PM_POS_BOX) {
    const float fn = (float)n;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float u = pos[3 * p + d] * fn;
      const float fl = floorf(u);
      c[d] = wrap_any((int)fl, n);
      o[d] = u - fl;
    }
  } else {
    const int q = wrap_any(cell[p], n * n * n);
    c[0] = q / (n * n);
    c[1] = (q / n) - c[0] * n;
    c[2] = q - (q / n) * n;
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

template <int MAS, int PK, class Index>
__device__ void deposit_chunk(const float *__restrict__ pos, const int32_t *__restrict__ cell,
                              const Index idx, int n, float mass, float *__restrict__ rho) {
  __shared__ float so[3][kGChunk];        // sorted in-cell offsets
  __shared__ int cstart[kGCells + 1];     // cell counts, then starts, then cursors
  __shared__ int red[6][kGThreads / 64];
  __shared__ int wsum[kGThreads / 64];
  int ref[3];
  {
    float o[3];
    particle_cell<PK>(pos, cell, idx.ref(), n, ref, o);
  }
  int lc[kGPPT][3];
  float lo_f[kGPPT][3];
  int lo[3] = {n, n, n}, hi[3] = {-n, -n, -n};
#pragma unroll
  for (int m = 0; m < kGPPT; ++m) {
    const int64_t p = idx(threadIdx.x + m * kGThreads);
    int c[3] = {0, 0, 0};
    float o[3] = {0.f, 0.f, 0.f};
    if (p >= 0) particle_cell<PK>(pos, cell, p, n, c, o);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int d = min_image(c[a] - ref[a], n);
      lc[m][a] = d;
      lo_f[m][a] = o[a];
      if (p >= 0) {
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
  int e[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    int l = red[a][0], h = red[3 + a][0];
    for (int w = 1; w < kGThreads / 64; ++w) {
      l = min(l, red[a][w]);
      h = max(h, red[3 + a][w]);
    }
    lo[a] = l;
    e[a] = h - l + 1;
  }
  const int vol = e[0] * e[1] * e[2];
  if (vol > kGCells) {
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
          const float wab = mass * w[0][a] * w[1][b];
          for (int c = 0; c < MAS; ++c)
            unsafeAtomicAdd(&rho[row + wrap_index(f[2] + c, n)], wab * w[2][c]);
        }
      }
    }
    return;
  }
  // 2. counting sort by local cell
  for (int i = threadIdx.x; i <= vol; i += kGThreads) cstart[i] = 0;
  __syncthreads();
  int key[kGPPT];
#pragma unroll
  for (int m = 0; m < kGPPT; ++m) {
    const int64_t p = idx(threadIdx.x + m * kGThreads);
    key[m] = -1;
    if (p >= 0) {
      key[m] = ((lc[m][0] - lo[0]) * e[1] + (lc[m][1] - lo[1])) * e[2] + (lc[m][2] - lo[2]);
      atomicAdd(&cstart[key[m]], 1);
    }
  }
  __syncthreads();
  // exclusive scan of cstart[0 .. vol) (kGCells / kGThreads = 16 entries per thread)
  {
    constexpr int PER = kGCells / kGThreads;
    const int b0 = threadIdx.x * PER;
    int v[PER];
    int tot = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      v[i] = (b0 + i < vol) ? cstart[b0 + i] : 0;
      tot += v[i];
    }
    int x = tot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    int woff = 0;
    for (int w = 0; w < wave; ++w) woff += wsum[w];
    int run = x - tot + woff;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      if (b0 + i < vol) cstart[b0 + i] = run;
      run += v[i];
    }
    __syncthreads();
  }
  // scatter offsets: the cursor of a cell is its start, advanced atomically
#pragma unroll
  for (int m = 0; m < kGPPT; ++m) {
    if (key[m] < 0) continue;
    const int slot = atomicAdd(&cstart[key[m]], 1);
    so[0][slot] = lo_f[m][0];
    so[1][slot] = lo_f[m][1];
    so[2][slot] = lo_f[m][2];
  }
  __syncthreads();
  // after the scatter cstart[c] is the end of cell c, i.e. the start of cell c+1;
  // the start of cell c is cstart[c-1] (0 for c = 0)
  // 3. gather into the grown box, 4. flush
  const int g0 = e[0] + 2, g1 = e[1] + 2, g2 = e[2] + 2;
  const int gvol = g0 * g1 * g2;
  for (int t = threadIdx.x; t < gvol; t += kGThreads) {
    const int x = t / (g1 * g2), r = t - x * (g1 * g2);
    const int y = r / g2, z = r - y * g2;
    // target cell in P coordinates: (x-1, y-1, z-1)
    float acc = 0.0f;
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) {
      const int qx = x - 1 + dx;
      if (qx < 0 || qx >= e[0]) continue;
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
        const int qy = y - 1 + dy;
        if (qy < 0 || qy >= e[1]) continue;
        const int row = (qx * e[1] + qy) * e[2];
        const float wxy_dx = (float)dx - 0.5f, wxy_dy = (float)dy - 0.5f;
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz) {
          const int qz = z - 1 + dz;
          if (qz < 0 || qz >= e[2]) continue;
          const int q = row + qz;
          const int s0 = q > 0 ? cstart[q - 1] : 0, s1 = cstart[q];
          for (int sidx = s0; sidx < s1; ++sidx) {
            acc += window_sep_g<MAS>(wxy_dx + so[0][sidx]) * window_sep_g<MAS>(wxy_dy + so[1][sidx]) *
                   window_sep_g<MAS>((float)dz - 0.5f + so[2][sidx]);
          }
        }
      }
    }
    if (acc != 0.0f) {
      const int gi = wrap_any(ref[0] + lo[0] + x - 1, n);
      const int gj = wrap_any(ref[1] + lo[1] + y - 1, n);
      const int gk = wrap_any(ref[2] + lo[2] + z - 1, n);
      unsafeAtomicAdd(&rho[((size_t)gi * n + gj) * n + gk], mass * acc);
    }
  }
}

}  // namespace pm_chunk
