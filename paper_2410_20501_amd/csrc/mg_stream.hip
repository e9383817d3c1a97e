// Streaming multigrid kernels for the large levels (n >= 256).
//
// A block owns an SJ x SK tile of (j, k) columns and a chunk of CI consecutive
// i-planes, and walks through the planes once. Each thread keeps a fixed set of
// (j, k) points of the tile plus halo, and holds in registers the values of its
// points for the planes in flight, so the i-1 / i+1 neighbours never leave
// registers; in-plane neighbours are exchanged through LDS.
//
// k_smooth_stream<H>: H red-black half-sweeps (H/2 Gauss-Seidel sweeps) in one
// pass over HBM. Half-sweep s is applied to plane q - s while plane q is
// loaded, on a region that shrinks by one cell per half-sweep from the loaded
// halo of H cells, so every value it reads is already at the right stage. The
// result goes to a different buffer (out of place), because neighbouring blocks
// still read the old values of the shared halo. Options:
//   NORM     sums ||f - L u||^2 and ||f||^2 of the *input* field on the block's
//            interior (the convergence test of the previous cycle, for free);
// k_rr_stream: residual f - L u on the fine grid, restricted to the coarse grid
// (full weighting (1,3,3,1)/8 per axis, or the 8-child average), in one pass.
#include "internal.h"

namespace {

constexpr int SJ = 32, SK = 64;  // interior tile of the smoother
constexpr int ST = 1024;         // threads per smoother block

__device__ __forceinline__ int wrap_any(int i, int n) {
  const int r = i % n;
  return r < 0 ? r + n : r;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

template <int NT>
__device__ void block_pair_to_partial(double s1, double s2, double *partial) {
  __shared__ double l1[NT / 64], l2[NT / 64];
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
    for (int w = 0; w < NT / 64; ++w) {
      a += l1[w];
      b += l2[w];
    }
    const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    partial[2 * bid] = a;
    partial[2 * bid + 1] = b;
  }
}

template <int H, bool NORM>
__global__ __launch_bounds__(ST) void k_smooth_stream(
    const float *__restrict__ uin, float *__restrict__ uout, const float *__restrict__ f,
    float fscale, const float *__restrict__ fmean, int n, int ci, float h2, float omega,
    int first_colour, double *__restrict__ partial) {
  constexpr int RJ = SJ + 2 * H, RK = SK + 2 * H, NP = RJ * RK;
  constexpr int PPT = (NP + ST - 1) / ST;
  __shared__ float lds[H][NP];

  // XCD-aware order: consecutive logical blocks are k-, then j-neighbours
  const unsigned lin = xcd_block(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                                 gridDim.x * gridDim.y * gridDim.z);
  const int bx = lin % gridDim.x, by = (lin / gridDim.x) % gridDim.y, bz = lin / (gridDim.x * gridDim.y);
  const int k0 = bx * SK, j0 = by * SJ, i0 = bz * ci;
  const float m = fmean ? *fmean : 0.0f;
  const float inv_h2 = 1.0f / h2;
  const size_t nn = (size_t)n * n;

  int rjv[PPT], rkv[PPT];
  uint32_t colv[PPT];
  bool inside[PPT];
#pragma unroll
  for (int t = 0; t < PPT; ++t) {
    const int e = threadIdx.x + t * ST;
    const int rj = (e < NP) ? e / RK : -100, rk = (e < NP) ? e % RK : -100;
    rjv[t] = rj;
    rkv[t] = rk;
    const int gj = j0 - H + rj, gk = k0 - H + rk;
    colv[t] = (e < NP) ? (uint32_t)(wrap_any(gj, n) * n + wrap_any(gk, n)) : 0u;
    inside[t] = (e < NP) && rj >= H && rj < H + SJ && rk >= H && rk < H + SK && gj < n && gk < n;
  }

  float ur[H + 2][PPT];   // ur[t] = plane q - (H + 1) + t
  float fr[H + 1][PPT];   // fr[t] = plane q - H + t, already scaled: fscale (f - mean)
  float uo_prev[PPT];     // original values of plane q - 2 (NORM)
  // two prefetch slots: planes q + 1 and q + 2 are in flight while plane q is worked on
  float pa_u[PPT], pa_f[PPT], pb_u[PPT], pb_f[PPT];
#pragma unroll
  for (int a = 0; a < H + 2; ++a)
#pragma unroll
    for (int t = 0; t < PPT; ++t) ur[a][t] = 0.f;
#pragma unroll
  for (int a = 0; a < H + 1; ++a)
#pragma unroll
    for (int t = 0; t < PPT; ++t) fr[a][t] = 0.f;
#pragma unroll
  for (int t = 0; t < PPT; ++t) uo_prev[t] = pa_u[t] = pa_f[t] = pb_u[t] = pb_f[t] = 0.f;

  auto load = [&](int q, float (&pu)[PPT], float (&pf)[PPT]) {
    const size_t plane = (size_t)wrap_any(q, n) * nn;
#pragma unroll
    for (int t = 0; t < PPT; ++t) {
      if (rjv[t] >= 0) {
        pu[t] = uin[plane + colv[t]];
        pf[t] = f[plane + colv[t]];
      }
    }
  };

  double s_r = 0.0, s_f = 0.0;
  const int qbeg = i0 - H, qend = i0 + ci + H;

  // one plane: take plane q from its slot, refill the slot with plane q + 2, then run
  // the H half-sweeps of the pipeline and retire plane q - H
  auto step = [&](int q, float (&pu)[PPT], float (&pf)[PPT]) {
#pragma unroll
    for (int a = 0; a < H + 1; ++a)
#pragma unroll
      for (int t = 0; t < PPT; ++t) ur[a][t] = ur[a + 1][t];
#pragma unroll
    for (int a = 0; a < H; ++a)
#pragma unroll
      for (int t = 0; t < PPT; ++t) fr[a][t] = fr[a + 1][t];
#pragma unroll
    for (int t = 0; t < PPT; ++t) {
      ur[H + 1][t] = pu[t];
      fr[H][t] = fscale * (pf[t] - m);
    }
    if (q + 2 < qend) load(q + 2, pu, pf);
    // Half-sweep s = 1 .. H runs on plane q - s. Its in-plane neighbours (the other
    // colour, which half-sweep s does not change) come from LDS slot s - 1 and its
    // i-neighbours from this thread's registers, so all H planes are published
    // before one barrier and the stages then run back to back.
#pragma unroll
    for (int s = 1; s <= H; ++s) {
      const int p = q - s;
      if (p < i0 - H + s || p >= i0 + ci + H - s) continue;  // uniform across the block
      float *L = lds[s - 1];
#pragma unroll
      for (int t = 0; t < PPT; ++t)
        if (rjv[t] >= 0) L[rjv[t] * RK + rkv[t]] = ur[H + 1 - s][t];
    }
    __syncthreads();
#pragma unroll
    for (int s = 1; s <= H; ++s) {
      const int p = q - s;
      if (p < i0 - H + s || p >= i0 + ci + H - s) continue;  // uniform across the block
      const float *L = lds[s - 1];
      const int colour = (first_colour + s - 1) & 1;
#pragma unroll
      for (int t = 0; t < PPT; ++t) {
        const int rj = rjv[t], rk = rkv[t];
        if (rj < s || rj >= RJ - s || rk < s || rk >= RK - s) continue;
        const int e = rj * RK + rk;
        const float uc = ur[H + 1 - s][t];
        const float inpl = L[e - RK] + L[e + RK] + L[e - 1] + L[e + 1];
        if constexpr (NORM) {
          // residual of the input field at plane q-1 (before its first update)
          if (s == 1 && inside[t] && p >= i0 && p < i0 + ci) {
            const float lap = (L[e - RK] - uc) + (L[e + RK] - uc) + (L[e - 1] - uc) +
                              (L[e + 1] - uc) + (uo_prev[t] - uc) + (ur[H + 1][t] - uc);
            const double r = fr[H - 1][t] - lap * inv_h2;
            s_r += r * r;
            s_f += (double)fr[H - 1][t] * fr[H - 1][t];
          }
        }
        const int gj = j0 - H + rj, gk = k0 - H + rk;
        if (((p + gj + gk) & 1) != colour) continue;
        const float nb = inpl + ur[H - s][t] + ur[H + 2 - s][t];
        const float gs = (nb - h2 * fr[H - s][t]) * (1.0f / 6.0f);
        ur[H + 1 - s][t] = (omega == 1.0f) ? gs : fmaf(omega, gs - uc, uc);
      }
      if constexpr (NORM) {
        if (s == 1) {
#pragma unroll
          for (int t = 0; t < PPT; ++t) uo_prev[t] = L[rjv[t] >= 0 ? rjv[t] * RK + rkv[t] : 0];
        }
      }
    }
    // plane q - H is final
    const int pout = q - H;
    if (pout >= i0 && pout < i0 + ci) {
      const size_t op = (size_t)wrap_any(pout, n) * nn;
#pragma unroll
      for (int t = 0; t < PPT; ++t)
        if (inside[t]) uout[op + colv[t]] = ur[1][t];
    }
    // the LDS slots are rewritten by the next plane
    __syncthreads();
  };

  load(qbeg, pa_u, pa_f);
  if (qbeg + 1 < qend) load(qbeg + 1, pb_u, pb_f);
  for (int q = qbeg; q < qend; q += 2) {
    step(q, pa_u, pa_f);
    if (q + 1 < qend) step(q + 1, pb_u, pb_f);
  }
  if constexpr (NORM) block_pair_to_partial<ST>(s_r, s_f, partial);
}

// ---------------------------------------------------------------- residual + restrict

constexpr int CJ = 16, CK = 32;        // coarse tile
constexpr int RT = 512;                // threads
constexpr int UJ = 2 * CJ + 4, UK = 2 * CK + 4, UNP = UJ * UK;  // fine u region (+2 halo)
constexpr int UPPT = (UNP + RT - 1) / RT;
constexpr int CPPT = CJ * CK / RT;     // coarse points per thread

template <int KIND>
__global__ __launch_bounds__(RT) void k_rr_stream(const float *__restrict__ u,
                                                  const float *__restrict__ f, float fscale,
                                                  const float *__restrict__ fmean, int n,
                                                  int cic, float inv_h2,
                                                  float *__restrict__ fc,
                                                  float *__restrict__ ucg, float gscale) {
  __shared__ float Lu[UNP];
  __shared__ float Lr[UNP];
  const int nc = n >> 1;
  const unsigned lin = xcd_block(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                                 gridDim.x * gridDim.y * gridDim.z);
  const int bx = lin % gridDim.x, by = (lin / gridDim.x) % gridDim.y, bz = lin / (gridDim.x * gridDim.y);
  const int K0 = bx * CK, J0 = by * CJ, I0 = bz * cic;
  // fine region origin: fine (2 J0 - 2, 2 K0 - 2)
  const int fj0 = 2 * J0 - 2, fk0 = 2 * K0 - 2;
  const float m = fmean ? *fmean : 0.0f;
  const size_t nn = (size_t)n * n;

  int rjv[UPPT], rkv[UPPT];
  uint32_t colv[UPPT];
#pragma unroll
  for (int t = 0; t < UPPT; ++t) {
    const int e = threadIdx.x + t * RT;
    rjv[t] = e < UNP ? e / UK : -100;
    rkv[t] = e < UNP ? e % UK : -100;
    colv[t] = e < UNP ? (uint32_t)(wrap_any(fj0 + rjv[t], n) * n + wrap_any(fk0 + rkv[t], n)) : 0u;
  }
  float um[UPPT], uc[UPPT], up[UPPT];  // planes p-1, p, p+1
  float fcur[UPPT], fnext[UPPT];       // f of planes p and p+1
  float nu[UPPT];                      // prefetched u of the next plane
  float acc[3][CPPT];                  // coarse accumulators indexed by coarse plane mod 3
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < CPPT; ++c) acc[a][c] = 0.f;
#pragma unroll
  for (int t = 0; t < UPPT; ++t) um[t] = uc[t] = up[t] = fcur[t] = fnext[t] = nu[t] = 0.f;

  // fine planes whose residual is needed: FW 2 I0 - 1 .. 2 (I0 + cic); AVG 2 I0 .. 2 (I0 + cic) - 1
  const int pbeg = (KIND == PM_RESTRICT_FW) ? 2 * I0 - 1 : 2 * I0;
  const int pend = (KIND == PM_RESTRICT_FW) ? 2 * (I0 + cic) + 1 : 2 * (I0 + cic);
  auto prefetch = [&](int q) {
    const size_t plane = (size_t)wrap_any(q, n) * nn;
    const size_t fplane = (size_t)wrap_any(q - 1, n) * nn;
#pragma unroll
    for (int t = 0; t < UPPT; ++t)
      if (rjv[t] >= 0) {
        nu[t] = u[plane + colv[t]];
        fnext[t] = f[fplane + colv[t]];
      }
  };
  prefetch(pbeg - 1);
  for (int q = pbeg - 1; q <= pend; ++q) {
#pragma unroll
    for (int t = 0; t < UPPT; ++t) {
      um[t] = uc[t];
      uc[t] = up[t];
      up[t] = nu[t];
      fcur[t] = fnext[t];  // f of plane q - 1
    }
    if (q < pend) prefetch(q + 1);
    const int p = q - 1;  // residual plane
    if (p < pbeg) continue;
#pragma unroll
    for (int t = 0; t < UPPT; ++t)
      if (rjv[t] >= 0) Lu[rjv[t] * UK + rkv[t]] = uc[t];
    __syncthreads();
#pragma unroll
    for (int t = 0; t < UPPT; ++t) {
      const int rj = rjv[t], rk = rkv[t];
      if (rj < 1 || rj >= UJ - 1 || rk < 1 || rk >= UK - 1) continue;
      const int e = rj * UK + rk;
      const float c = uc[t];
      const float lap = (Lu[e - UK] - c) + (Lu[e + UK] - c) + (Lu[e - 1] - c) + (Lu[e + 1] - c) +
                        (um[t] - c) + (up[t] - c);
      Lr[e] = fscale * (fcur[t] - m) - lap * inv_h2;
    }
    __syncthreads();
    // restrict within the plane, then accumulate into the coarse planes
#pragma unroll
    for (int c = 0; c < CPPT; ++c) {
      const int cidx = threadIdx.x + c * RT;
      const int cj = cidx / CK, ck = cidx % CK;
      float s = 0.f;
      if constexpr (KIND == PM_RESTRICT_FW) {
        // fine (2J-1 .. 2J+2) relative to the region: rj = 2 cj + 1 + b
        const float w[4] = {1.f, 3.f, 3.f, 1.f};
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const float *row = Lr + (2 * cj + 1 + b) * UK + 2 * ck + 1;
          s = fmaf(w[b], row[0] + 3.f * (row[1] + row[2]) + row[3], s);
        }
        // only coarse planes owned by this block accumulate (slots are shared mod 3)
        const int Ip = (p >= 0) ? p / 2 : -((1 - p) / 2);
        const bool odd = (p & 1) != 0;
        const int Io = odd ? Ip + 1 : Ip - 1;
        if (Ip >= I0 && Ip < I0 + cic) acc[Ip % 3][c] += 3.f * s;
        if (Io >= I0 && Io < I0 + cic) acc[Io % 3][c] += s;
      } else {
        const float *row0 = Lr + (2 * cj + 2) * UK + 2 * ck + 2;
        s = row0[0] + row0[1] + row0[UK] + row0[UK + 1];
        acc[(p >> 1) % 3][c] += s;
      }
    }
    // coarse plane complete: FW after fine 2 I + 2 (p even, I = p/2 - 1); AVG after 2 I + 1
    int Idone;
    bool done;
    if constexpr (KIND == PM_RESTRICT_FW) {
      done = ((p & 1) == 0) && p >= 2 * I0 + 2;
      Idone = p / 2 - 1;
    } else {
      done = (p & 1) == 1;
      Idone = p >> 1;
    }
    if (done) {
      const int slot = Idone % 3;
      const float scale = (KIND == PM_RESTRICT_FW) ? (1.0f / 512.0f) : 0.125f;
#pragma unroll
      for (int c = 0; c < CPPT; ++c) {
        const int cidx = threadIdx.x + c * RT;
        const int J = J0 + cidx / CK, K = K0 + cidx % CK;
        if (J < nc && K < nc) {
          const size_t ci = ((size_t)Idone * nc + J) * nc + K;
          const float v = acc[slot][c] * scale;
          fc[ci] = v;
          if (ucg) ucg[ci] = gscale * v;  // coarse starting guess -H^2 f_H / 6
        }
        acc[slot][c] = 0.f;
      }
    }
    __syncthreads();
  }
}

// Planes per block: halve while the grid has fewer than want_blocks blocks and
// the chunk stays >= min_ci (the i-halo is recomputed per chunk).
inline int chunk_for(int n, int tiles, int want_blocks, int min_ci) {
  int ci = n;
  while (ci / 2 >= min_ci && (int64_t)tiles * (n / ci) < want_blocks && n % (ci / 2) == 0) ci /= 2;
  return ci;
}

}  // namespace

int64_t smooth_stream_blocks(int n) {
  const int tj = (n + SJ - 1) / SJ, tk = (n + SK - 1) / SK;
  const int ci = chunk_for(n, tj * tk, 1024, 16);
  return (int64_t)tj * tk * (n / ci);
}

hipError_t launch_smooth_stream(const float *uin, float *uout, const float *f, float fscale,
                                const float *fmean, int n, float h2, float omega,
                                int first_colour, int half_sweeps, double *partial,
                                hipStream_t s) {
  const int tj = (n + SJ - 1) / SJ, tk = (n + SK - 1) / SK;
  const int ci = chunk_for(n, tj * tk, 1024, 16);
  dim3 grid(tk, tj, n / ci);
  const bool norm = partial != nullptr;
  if (half_sweeps == 4) {
    if (norm)
      k_smooth_stream<4, true><<<grid, ST, 0, s>>>(uin, uout, f, fscale, fmean, n, ci, h2, omega,
                                                   first_colour, partial);
    else
      k_smooth_stream<4, false><<<grid, ST, 0, s>>>(uin, uout, f, fscale, fmean, n, ci, h2, omega,
                                                    first_colour, partial);
  } else if (half_sweeps == 2) {
    if (norm)
      k_smooth_stream<2, true><<<grid, ST, 0, s>>>(uin, uout, f, fscale, fmean, n, ci, h2, omega,
                                                   first_colour, partial);
    else
      k_smooth_stream<2, false><<<grid, ST, 0, s>>>(uin, uout, f, fscale, fmean, n, ci, h2, omega,
                                                    first_colour, partial);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_rr_stream(const float *u, const float *f, float fscale, const float *fmean,
                            int n, float inv_h2, int kind, float *fc, float *ucg, float gscale,
                            hipStream_t s) {
  const int nc = n / 2;
  const int tj = (nc + CJ - 1) / CJ, tk = (nc + CK - 1) / CK;
  const int cic = chunk_for(nc, tj * tk, 1024, 8);
  dim3 grid(tk, tj, nc / cic);
  if (kind == PM_RESTRICT_AVG)
    k_rr_stream<PM_RESTRICT_AVG><<<grid, RT, 0, s>>>(u, f, fscale, fmean, n, cic, inv_h2, fc, ucg,
                                                     gscale);
  else
    k_rr_stream<PM_RESTRICT_FW><<<grid, RT, 0, s>>>(u, f, fscale, fmean, n, cic, inv_h2, fc, ucg,
                                                    gscale);
  return hipGetLastError();
}
