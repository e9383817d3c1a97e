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

#ifndef PM_SMOOTH_SJ
#define PM_SMOOTH_SJ 16
#endif
#ifndef PM_SMOOTH_THREADS
#define PM_SMOOTH_THREADS 512
#endif
constexpr int SJ = PM_SMOOTH_SJ, SK = 64;  // interior tile of the smoother (SJ, SK even)
constexpr int ST = PM_SMOOTH_THREADS;      // threads per smoother block
#ifndef PM_SMOOTH_BLOCKS
#define PM_SMOOTH_BLOCKS 512
#endif
#ifndef PM_RR_BLOCKS
#define PM_RR_BLOCKS 2048
#endif
#ifndef PM_SMOOTH_WAVES
#define PM_SMOOTH_WAVES 4  // waves per SIMD the smoother is compiled for (VGPR budget 512 / it)
#endif
constexpr int kSmoothBlocks = PM_SMOOTH_BLOCKS;  // blocks wanted per pass (i-chunks shrink to reach it)

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
__device__ void block_triple_to_partial(double s1, double s2, double s3, double *partial) {
  __shared__ double l1[NT / 64], l2[NT / 64], l3[NT / 64];
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  s3 = wave_sum(s3);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    l1[wave] = s1;
    l2[wave] = s2;
    l3[wave] = s3;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0, c = 0.0;
    for (int w = 0; w < NT / 64; ++w) {
      a += l1[w];
      b += l2[w];
      c += l3[w];
    }
    const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    partial[3 * bid] = a;
    partial[3 * bid + 1] = b;
    partial[3 * bid + 2] = c;
  }
}

// Colour-split pairs: a thread owns pairs of k-neighbouring points (k even, k + 1)
// of the tile plus halo; the two points of a pair have opposite colours. Plane q of
// the pipeline receives half-sweep s on plane q - s, whose colour alternates with s
// exactly as the plane parity does, so one plane step updates the same point of every
// pair in all its half-sweeps: point E in steps with q even, point O with q odd (E is
// the point with j + k + first_colour odd). Every lane does one update per pair and
// half-sweep, with no per-lane colour test and no masked lanes; the ring of planes is
// unrolled, so which point a step updates is known at compile time. The halo is not
// masked either: points near the tile edge read padding or wrapped-row values and come
// out wrong, but a wrong value moves inward by one cell per half-sweep and the halo is
// H cells wide, so the interior is exact.
// The norm-accumulating and the prolongating passes run twice the threads with half the
// pairs each: at two pairs per thread their extra live values spill, and a spill reload
// waits for the plane prefetches.
template <int H, bool NORM, bool PRO = false>
struct SmoothShape {
  static constexpr int NT = (NORM || PRO) ? 2 * ST : ST;  // threads per block
  static constexpr int RJ = SJ + 2 * H, RK = SK + 2 * H, RK2 = RK / 2, NPAIR = RJ * RK2;
  static constexpr int PP = (NPAIR + NT - 1) / NT;  // pairs per thread
  // LDS: per published plane one array of E values and one of O values, each indexed
  // by pair (consecutive lanes, consecutive banks) with padding rows around it
  static constexpr int PAD = RK2 + 2;                // floats before and after a colour array
  static constexpr int ARR = NPAIR + 2 * PAD;        // floats per colour array
  static constexpr int SLOT = 2 * ARR;               // floats per published plane (E, then O)
  static constexpr int RING = H + 2;                 // planes held in registers
  // PRO: the coarse correction's region (tile plus halo, halved, plus one coarse cell
  // per side) staged raw in LDS, then interpolated along k to the tile's fine columns
  // into a ring of three planes (CJR rows of RK values)
  static constexpr int CJR = RJ / 2 + 2, CKR = RK / 2 + 2, CPLANE = CJR * CKR;
  static constexpr int CPT = (CPLANE + NT - 1) / NT;  // coarse values loaded per thread
  static constexpr int KPLANE = CJR * RK;             // k-interpolated plane
};

// planes in flight from HBM (a third one measured no faster and costs registers)
template <int H, bool NORM, bool PRO = false>
constexpr int smooth_prefetch() {
  return 2;
}

template <int H, bool NORM, bool OMEGA1, bool PRO>
struct SmoothState {
  using S = SmoothShape<H, NORM, PRO>;
  // per-thread constants
  // LDS index of the pair in a colour array (padding included); the first of the two
  // k-neighbours of E (in the O array) is li - 1 + offe, of O (in the E array) li - offe,
  // with offe = swp the k offset of E in its pair
  int li[S::PP];
  uint32_t col[S::PP];        // in-plane offset of the pair's even-k point
  bool swp[S::PP];            // E is the odd-k point of its pair
  bool inside[S::PP];
  // pipeline registers: ring slot (q - d) mod RING holds plane q - d
  float uE[S::RING][S::PP], uO[S::RING][S::PP];
  float fE[S::RING][S::PP], fO[S::RING][S::PP];  // fscale (f - mean)
  static constexpr int PF = smooth_prefetch<H, NORM, PRO>();
  float2 pu[PF][S::PP], pf[PF][S::PP];            // planes in flight from HBM
  double s_r, s_f, s_u;  // NORM: ||f - L u||^2, ||f||^2 and sum u of the input
  // PRO: u += P e as each plane enters (trilinear prolongation of the coarse correction)
  const float *ec;          // coarse grid, nc^3
  float *craw;              // LDS: one raw coarse plane
  float *ck;                // LDS: ring of three k-interpolated coarse planes
  int nc, k0h, cjb, ckb;    // coarse size; first fine column of the tile; coarse origin
  int cr[S::PP], cr2[S::PP];  // offset of the pair's values in a k-interpolated plane:
                              // row J and row J' (its other coarse row)
  float cpre[S::CPT];       // a coarse plane in flight
  // uniform
  const float *uin, *f;
  float *uout, *lds;
  float fscale, m, h2, omega, inv_h2, uscale;
  int n, i0, ci, qend;
  size_t nn;

  // planes of a chunk lie within one period of the grid on either side
  __device__ __forceinline__ int wrap_plane(int q) const { return q < 0 ? q + n : (q >= n ? q - n : q); }

  __device__ __forceinline__ void load(int q, float2 (&u)[S::PP], float2 (&fv)[S::PP]) {
    const size_t plane = (size_t)wrap_plane(q) * nn;
#pragma unroll
    for (int t = 0; t < S::PP; ++t) {
      u[t] = *reinterpret_cast<const float2 *>(uin + plane + col[t]);
      fv[t] = *reinterpret_cast<const float2 *>(f + plane + col[t]);
    }
  }

  static __device__ __forceinline__ int cslot(int I) { return ((I % 3) + 3) % 3; }
  // coarse indices of a tile lie within one period of the coarse grid on either side
  __device__ __forceinline__ int cwrap(int i) const { return i < 0 ? i + nc : (i >= nc ? i - nc : i); }
  __device__ __forceinline__ void cload(int I) {
    const float *plane = ec + (size_t)cwrap(I) * nc * nc;
#pragma unroll
    for (int m = 0; m < S::CPT; ++m) {
      // (offsets recomputed here rather than held: registers are the smoother's limit;
      // the empty asm keeps the compiler from hoisting them out of the plane loop)
      int e = threadIdx.x + m * S::NT;
      asm volatile("" : "+v"(e));
      const int jj = e / S::CKR, kk = e - jj * S::CKR;
      if (e < S::CPLANE) cpre[m] = plane[cwrap(cjb + jj) * nc + cwrap(ckb + kk)];
    }
  }
  __device__ __forceinline__ void cstore_raw() {
#pragma unroll
    for (int m = 0; m < S::CPT; ++m) {
      const int e = threadIdx.x + m * S::NT;
      if (e < S::CPLANE) craw[e] = cpre[m];
    }
  }
  // fine column k of the tile: 3/4 of coarse column k >> 1 and 1/4 of its neighbour
  // on k's side (after a barrier that follows cstore_raw)
  __device__ __forceinline__ void cinterp_k(int I) {
    float *dst = ck + cslot(I) * S::KPLANE;
    for (int e = threadIdx.x; e < S::KPLANE; e += S::NT) {
      const int jj = e / S::RK, kf = e - jj * S::RK;
      const int gk = k0h + kf;
      const int K = (gk >> 1) - ckb, K2 = K + ((gk & 1) ? 1 : -1);
      dst[e] = fmaf(0.75f, craw[jj * S::CKR + K], 0.25f * craw[jj * S::CKR + K2]);
    }
  }
};

// Gauss-Seidel update of one point per pair on the plane in ring slot c (neighbour
// planes in slots cm and cp), in-plane neighbours from L.
// L is the colour array of the other points: k-neighbours at kn, kn + 1, j-neighbours
// one row (RK2 pairs) up and down.
template <int c, int cm, int cp, int RING, int PP, int RK2, bool OMEGA1, bool E>
__device__ __forceinline__ void smooth_relax(float (&u)[RING][PP], const float (&fv)[RING][PP],
                                             const int (&li)[PP], const bool (&swp)[PP],
                                             const float *L, float h2, float omega) {
#pragma unroll
  for (int t = 0; t < PP; ++t) {
    const int e = li[t], k = E ? (swp[t] ? e : e - 1) : (swp[t] ? e - 1 : e);
    const float nb = (L[k] + L[k + 1]) + (L[e - RK2] + L[e + RK2]) + (u[cm][t] + u[cp][t]);
    const float gs = (nb - h2 * fv[c][t]) * (1.0f / 6.0f);
    const float uc = u[c][t];
    u[c][t] = OMEGA1 ? gs : fmaf(omega, gs - uc, uc);
  }
}

#ifndef PM_SMOOTH_LDS_SETS
#define PM_SMOOTH_LDS_SETS 1
#endif
// LDS slot sets. With one set every plane step ends with a barrier before the next step
// overwrites the slots. With rotating sets (step q publishes into set q mod sets) the
// barrier that starts a step also guarantees that every wave has finished reading the
// set the step after next overwrites, so a step needs one barrier. The residual of the
// norm pass also reads the previous step's set, hence three sets; they rotate with the
// ring of planes, whose length must then be a multiple of three.
template <int H, bool NORM>
constexpr int lds_sets() {
  return PM_SMOOTH_LDS_SETS == 0 ? 1 : (NORM ? ((H + 2) % 3 == 0 ? 3 : 1) : 2);
}

// LDS slot of half-sweep s in a step with q = R mod RING. With one set and NORM the slot
// of s = 1 alternates between slot 0 and slot H, so the input values of plane q - 2
// published by the previous step are still there for the residual of plane q - 1.
template <int R, int H, bool NORM>
constexpr int lds_slot(int s) {
  constexpr int sets = lds_sets<H, NORM>();
  if constexpr (sets > 1) return (R % sets) * H + s - 1;
  return (NORM && s == 1 && (R & 1)) ? H : s - 1;
}

// slot of the previous step's s = 1 values (the norm pass's plane q - 2 inputs)
template <int R, int H>
constexpr int lds_prev_slot1() {
  constexpr int sets = lds_sets<H, true>();
  if constexpr (sets > 1) return ((R + sets - 1) % sets) * H;
  return lds_slot<R + 1, H, true>(1);
}

template <int H, bool NORM>
constexpr int lds_slots() {
  return lds_sets<H, NORM>() > 1 ? lds_sets<H, NORM>() * H : H + (NORM ? 1 : 0);
}

// ring slot of plane q - d in a step with q = R mod RING
template <int R, int RING>
constexpr int ring_slot(int d) {
  return ((R - d) % RING + RING) % RING;
}

// Half-sweep S of a plane step: plane q - S.
template <int R, int S, int H, bool NORM, bool OMEGA1, bool PRO>
__device__ __forceinline__ void smooth_half(SmoothState<H, NORM, OMEGA1, PRO> &c, int q) {
  using Sh = SmoothShape<H, NORM, PRO>;
  constexpr int RING = Sh::RING, PP = Sh::PP, RK2 = Sh::RK2;
  constexpr int c0 = ring_slot<R, RING>(0), c1 = ring_slot<R, RING>(1);
  constexpr int cs = ring_slot<R, RING>(S), cm = ring_slot<R, RING>(S + 1),
                cp = ring_slot<R, RING>(S - 1);
  const int p = q - S;
  const float *LE = c.lds + lds_slot<R, H, NORM>(S) * Sh::SLOT, *LO = LE + Sh::ARR;
  if constexpr ((R & 1) == 0)
    smooth_relax<cs, cm, cp, RING, PP, RK2, OMEGA1, true>(c.uE, c.fE, c.li, c.swp, LO, c.h2,
                                                          c.omega);
  else
    smooth_relax<cs, cm, cp, RING, PP, RK2, OMEGA1, false>(c.uO, c.fO, c.li, c.swp, LE, c.h2,
                                                           c.omega);
}

// NORM: residual of the input field at plane q - 1, from the values published before
// its first update (LDS slot of s = 1), the input values of plane q - 2 (the previous
// step's slot) and plane q (registers, not yet updated). Run after the relaxations, so
// its live values do not add to theirs.
template <int R, int H, bool OMEGA1, bool PRO>
__device__ __forceinline__ void smooth_norm(SmoothState<H, true, OMEGA1, PRO> &c, int q) {
  using Sh = SmoothShape<H, true>;
  constexpr int RING = Sh::RING, PP = Sh::PP, RK2 = Sh::RK2;
  constexpr int c0 = ring_slot<R, RING>(0), c1 = ring_slot<R, RING>(1);
  const int p = q - 1;
  if (p < c.i0 || p >= c.i0 + c.ci) return;  // uniform
  const float *LE = c.lds + lds_slot<R, H, true>(1) * Sh::SLOT, *LO = LE + Sh::ARR;
  const float *PE = c.lds + lds_prev_slot1<R, H>() * Sh::SLOT, *PO = PE + Sh::ARR;
  float sr = 0.f, sf = 0.f, su = 0.f;  // this plane's few terms in FP32, the sums in FP64
#pragma unroll
  for (int t = 0; t < PP; ++t) {
    if (!c.inside[t]) continue;
    const int e = c.li[t], ka = c.swp[t] ? e : e - 1, kb = c.swp[t] ? e - 1 : e;
    const float a = LE[e], b = LO[e];
    const float lapa = (LO[ka] - a) + (LO[ka + 1] - a) + (LO[e - RK2] - a) + (LO[e + RK2] - a) +
                       (PE[e] - a) + (c.uE[c0][t] - a);
    const float lapb = (LE[kb] - b) + (LE[kb + 1] - b) + (LE[e - RK2] - b) + (LE[e + RK2] - b) +
                       (PO[e] - b) + (c.uO[c0][t] - b);
    const float fa = c.fE[c1][t], fb = c.fO[c1][t];
    const float ra = fa - lapa * c.inv_h2, rb = fb - lapb * c.inv_h2;
    sr = fmaf(ra, ra, fmaf(rb, rb, sr));
    sf = fmaf(fa, fa, fmaf(fb, fb, sf));
    su += a + b;
  }
  c.s_r += sr;
  c.s_f += sf;
  c.s_u += su;
}

template <int R, int S, int H, bool NORM, bool OMEGA1, bool PRO>
__device__ __forceinline__ void smooth_halves(SmoothState<H, NORM, OMEGA1, PRO> &c, int q) {
  if constexpr (S <= H) {
    smooth_half<R, S, H, NORM, OMEGA1, PRO>(c, q);
    smooth_halves<R, S + 1, H, NORM, OMEGA1, PRO>(c, q);
  }
}

// One plane of the pipeline, for ring position R = q mod RING (q has the parity of R).
template <int R, int H, bool NORM, bool OMEGA1, bool PRO>
__device__ __forceinline__ void smooth_step(SmoothState<H, NORM, OMEGA1, PRO> &c, int q) {
  using Sh = SmoothShape<H, NORM, PRO>;
  constexpr int RING = Sh::RING, PP = Sh::PP, SLOT = Sh::SLOT;
  constexpr int PF = smooth_prefetch<H, NORM, PRO>();
  constexpr int P = R % PF;  // prefetch slot of plane q
  constexpr int c0 = ring_slot<R, RING>(0), cH = ring_slot<R, RING>(H);
  // plane q enters the ring; its slot is refilled with plane q + PF
#pragma unroll
  for (int t = 0; t < PP; ++t) {
    const float2 u = c.pu[P][t], fv = c.pf[P][t];
    const float fx = c.fscale * (fv.x - c.m), fy = c.fscale * (fv.y - c.m);
    // (uscale: growth rescaling of a warm start, applied as the input is read)
    c.uE[c0][t] = c.uscale * (c.swp[t] ? u.y : u.x);
    c.uO[c0][t] = c.uscale * (c.swp[t] ? u.x : u.y);
    c.fE[c0][t] = c.swp[t] ? fy : fx;
    c.fO[c0][t] = c.swp[t] ? fx : fy;
  }
  c.load(min(q + PF, c.qend - 1), c.pu[P], c.pf[P]);  // past the end: a harmless reload
  // Half-sweep s runs on plane q - s. Its in-plane neighbours (the points it does not
  // change: O when it updates E and the reverse) come from LDS slot s - 1, its
  // i-neighbours from registers, so all H planes are published before one barrier.
  // The residual of the input (NORM, s = 1) needs both points.
#pragma unroll
  for (int s = 1; s <= H; ++s) {
    float *LE = c.lds + lds_slot<R, H, NORM>(s) * SLOT, *LO = LE + Sh::ARR;
    const int cs = ((R - s) % RING + RING) % RING;
    const bool both = NORM && s == 1;
#pragma unroll
    for (int t = 0; t < PP; ++t) {
      if (both || (R & 1) == 1) LE[c.li[t]] = c.uE[cs][t];
      if (both || (R & 1) == 0) LO[c.li[t]] = c.uO[cs][t];
    }
  }
  if constexpr (PRO) {
    if constexpr ((R & 1) == 1) {
      // q = 2I + 1: coarse plane I + 2 (loaded two steps ago) is staged raw; plane
      // I + 3 goes in flight
      c.cstore_raw();
      c.cload((q >> 1) + 3);
    }
  }
  __syncthreads();
  if constexpr (PRO) {
    // (scheduling fences around this block keep its LDS reads from being hoisted into
    // the relaxations, whose live values they would add to)
    __builtin_amdgcn_sched_barrier(0);
    // q = 2I + 1: the staged plane I + 2 goes into the ring, in place of plane I - 1
    // (last read at step 2I); it is first read at step 2I + 3
    if constexpr ((R & 1) == 1) {
      c.cinterp_k((q >> 1) + 2);
      __builtin_amdgcn_sched_barrier(0);
    }
    // plane q enters with the coarse correction: per axis 3/4 from the nearest coarse
    // cell and 1/4 from the next one (planes A, B; rows J, J'; columns K, K -+ 1)
    constexpr int KP = Sh::KPLANE;
    const int A = q >> 1, B = (R & 1) ? A + 1 : A - 1;
    const float *CA = c.ck + c.cslot(A) * KP, *CB = c.ck + c.cslot(B) * KP;
#pragma unroll
    for (int t = 0; t < PP; ++t) {
      // (k-interpolated values of the pair's even and odd column, one float2)
      const float2 a1 = *reinterpret_cast<const float2 *>(CA + c.cr[t]);
      const float2 a2 = *reinterpret_cast<const float2 *>(CA + c.cr2[t]);
      const float2 b1 = *reinterpret_cast<const float2 *>(CB + c.cr[t]);
      const float2 b2 = *reinterpret_cast<const float2 *>(CB + c.cr2[t]);
      const float ev = fmaf(0.5625f, a1.x, fmaf(0.1875f, a2.x + b1.x, 0.0625f * b2.x));
      const float od = fmaf(0.5625f, a1.y, fmaf(0.1875f, a2.y + b1.y, 0.0625f * b2.y));
      c.uE[c0][t] += c.swp[t] ? od : ev;  // E is the odd-k point when swp
      c.uO[c0][t] += c.swp[t] ? ev : od;
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  smooth_halves<R, 1, H, NORM, OMEGA1, PRO>(c, q);
  if constexpr (NORM) {
    __builtin_amdgcn_sched_barrier(0);
    smooth_norm<R, H, OMEGA1, PRO>(c, q);
  }
  // plane q - H is final
  const int pout = q - H;
  if (pout >= c.i0 && pout < c.i0 + c.ci) {
    const size_t op = (size_t)pout * c.nn;  // output planes lie in [0, n)
#pragma unroll
    for (int t = 0; t < PP; ++t)
      if (c.inside[t]) {
        const float a = c.uE[cH][t], b = c.uO[cH][t];
        *reinterpret_cast<float2 *>(c.uout + op + c.col[t]) =
            c.swp[t] ? make_float2(b, a) : make_float2(a, b);
      }
  }
  // the LDS slots are rewritten by the next plane (rotating sets: by the one after it,
  // behind the next step's barrier)
  if constexpr (lds_sets<H, NORM>() == 1) __syncthreads();
}

template <int R, bool GUARD, int H, bool NORM, bool OMEGA1, bool PRO>
__device__ __forceinline__ void smooth_steps(SmoothState<H, NORM, OMEGA1, PRO> &c, int q) {
  if constexpr (R < SmoothShape<H, NORM, PRO>::RING) {
    if (!GUARD || q + R < c.qend) smooth_step<R, H, NORM, OMEGA1, PRO>(c, q + R);
    smooth_steps<R + 1, GUARD, H, NORM, OMEGA1, PRO>(c, q);
  }
}

template <int H, bool NORM, bool OMEGA1, bool PRO>
// at least 4 waves per SIMD: two 512-thread blocks (or one of 1024) per CU; with rotating
// LDS sets (60 to 90 KB per block) that is also what the LDS holds
__global__ __launch_bounds__((SmoothShape<H, NORM, PRO>::NT)) __attribute__((amdgpu_waves_per_eu(PM_SMOOTH_WAVES))) void k_smooth_stream(
    const float *__restrict__ uin, float *__restrict__ uout, const float *__restrict__ f,
    float fscale, const float *__restrict__ fmean, int n, int ci, float h2, float omega,
    int first_colour, double *__restrict__ partial, float uscale, const float *__restrict__ ec) {
  using S = SmoothShape<H, NORM, PRO>;
  constexpr int PF = smooth_prefetch<H, NORM, PRO>();
  static_assert(S::RING % 2 == 0 && S::RING % PF == 0,
                "plane parity and prefetch slots repeat within one ring period");
  static_assert(lds_sets<H, NORM>() == 1 || S::RING % lds_sets<H, NORM>() == 0,
                "LDS slot sets rotate with the ring of planes");
  constexpr int NSLOT = lds_slots<H, NORM>();
  __shared__ float lds[NSLOT * S::SLOT];
  __shared__ float craw[PRO ? S::CPLANE : 1];
  __shared__ float __align__(8) ckl[PRO ? 3 * S::KPLANE : 2];

  // XCD-aware order: consecutive logical blocks are k-, then j-neighbours
  const unsigned lin = xcd_block(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                                 gridDim.x * gridDim.y * gridDim.z);
  const int bx = lin % gridDim.x, by = (lin / gridDim.x) % gridDim.y, bz = lin / (gridDim.x * gridDim.y);
  const int k0 = bx * SK, j0 = by * SJ;

  SmoothState<H, NORM, OMEGA1, PRO> c;
  c.uin = uin;
  c.f = f;
  c.uout = uout;
  c.lds = lds;
  c.fscale = fscale;
  c.uscale = uscale;
  c.m = fmean ? *fmean : 0.0f;
  c.h2 = h2;
  c.omega = omega;
  c.inv_h2 = 1.0f / h2;
  c.n = n;
  c.i0 = bz * ci;
  c.ci = ci;
  c.qend = c.i0 + ci + H;
  c.nn = (size_t)n * n;
  c.s_r = c.s_f = c.s_u = 0.0;

  // padding is read by edge points (and written only by slots without a pair)
  for (int e = threadIdx.x; e < S::PAD; e += S::NT)
#pragma unroll
    for (int a = 0; a < 2 * NSLOT; ++a) {
      lds[a * S::ARR + e] = 0.0f;
      lds[a * S::ARR + S::PAD + S::NPAIR + e] = 0.0f;
    }
#pragma unroll
  for (int t = 0; t < S::PP; ++t) {
    const int e = threadIdx.x + t * S::NT;
    const bool v = e < S::NPAIR;
    const int rj = v ? e / S::RK2 : 0, r2 = v ? e % S::RK2 : 0;
    const int gj = j0 - H + rj, gk = k0 - H + 2 * r2;  // gk even (k0, H even)
    c.swp[t] = ((gj + first_colour) & 1) == 0;  // E = the point with j + k + first_colour odd
    // a slot without a pair loads column 0 and works on the trailing padding, whose
    // values only reach halo points, so every lane runs the same code unmasked
    const int li = v ? S::PAD + e : S::PAD + S::NPAIR + 1;
    // E at k = 2 r2 + offe has O neighbours in pairs r2 - 1 + offe and r2 + offe; O at
    // k = 2 r2 + 1 - offe has E neighbours in pairs r2 - offe and r2 + 1 - offe
    c.li[t] = li;
    c.col[t] = v ? (uint32_t)(wrap_any(gj, n) * n + wrap_any(gk, n)) : 0u;
    c.inside[t] = v && rj >= H && rj < H + SJ && 2 * r2 >= H && 2 * r2 < H + SK && gj < n &&
                  gk < n;
#pragma unroll
    for (int a = 0; a < S::RING; ++a) c.uE[a][t] = c.uO[a][t] = c.fE[a][t] = c.fO[a][t] = 0.f;
#pragma unroll
    for (int a = 0; a < PF; ++a) c.pu[a][t] = c.pf[a][t] = make_float2(0.f, 0.f);
  }
  const int qbeg = c.i0 - H;  // even (ci even, H even): step R of a ring period has q = R mod 2
  if constexpr (PRO) {
    c.ec = ec;
    c.craw = craw;
    c.ck = ckl;
    c.nc = n >> 1;
    const int cjb = ((j0 - H) >> 1) - 1, ckb = ((k0 - H) >> 1) - 1;  // coarse tile origin
    c.k0h = k0 - H;
    c.cjb = cjb;
    c.ckb = ckb;
#pragma unroll
    for (int t = 0; t < S::PP; ++t) {
      const int e = threadIdx.x + t * S::NT;
      const bool v = e < S::NPAIR;
      const int rj = v ? e / S::RK2 : 0, r2 = v ? e % S::RK2 : 0;
      const int gj = j0 - H + rj, gk = k0 - H + 2 * r2;
      // fine j -> coarse J = j >> 1 (3/4) and J' = J -+ 1 (1/4) for j even / odd;
      // fine k = 2K, 2K + 1 -> coarse K and K - 1 / K + 1
      const int jr = (gj >> 1) - cjb, jr2 = jr + ((gj & 1) ? 1 : -1);
      c.cr[t] = jr * S::RK + 2 * r2;
      c.cr2[t] = jr2 * S::RK + 2 * r2;
      (void)gk;
    }
    // coarse planes of the first two steps (q even needs q/2 - 1 and q/2, q + 1 needs
    // q/2 and q/2 + 1), and the next one in flight
    const int I0 = qbeg >> 1;
    for (int I = I0 - 1; I <= I0 + 1; ++I) {
      c.cload(I);
      c.cstore_raw();
      __syncthreads();
      c.cinterp_k(I);
      __syncthreads();
    }
    c.cload(I0 + 2);
  }
#pragma unroll
  for (int a = 0; a < PF; ++a) c.load(qbeg + a, c.pu[a], c.pf[a]);
  int q = qbeg;
  for (; q + S::RING <= c.qend; q += S::RING) smooth_steps<0, false, H, NORM, OMEGA1, PRO>(c, q);
  smooth_steps<0, true, H, NORM, OMEGA1, PRO>(c, q);
  if constexpr (NORM) block_triple_to_partial<S::NT>(c.s_r, c.s_f, c.s_u, partial);
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
  __shared__ float Lu[2 * UNP];  // u of the last two published planes
  __shared__ float Lr[2 * UNP];  // residual of the last two planes
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
  float um[UPPT], uc[UPPT], up[UPPT];  // u of planes t - 2, t - 1, t
  float fcur[UPPT], fnext[UPPT];       // f of planes t - 1 and t
  float nu[UPPT];                      // prefetched u of plane t + 1
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
  // One barrier per fine plane: iteration t publishes u of plane t (Lu), forms the
  // residual of plane t - 1 from the previous iteration's Lu (Lr), and restricts the
  // residual of plane t - 2 from the previous iteration's Lr. Lu and Lr alternate between
  // two buffers by plane parity, so a buffer is rewritten two iterations after it was
  // written, behind the barrier that ended every read of it.
  prefetch(pbeg - 1);
  for (int t = pbeg - 1; t <= pend + 1; ++t) {
#pragma unroll
    for (int v = 0; v < UPPT; ++v) {
      um[v] = uc[v];
      uc[v] = up[v];
      up[v] = nu[v];       // u of plane t
      fcur[v] = fnext[v];  // f of plane t - 1
    }
    if (t < pend) prefetch(t + 1);
    if (t >= pbeg && t < pend) {
      float *lu = Lu + (t & 1) * UNP;
#pragma unroll
      for (int v = 0; v < UPPT; ++v)
        if (rjv[v] >= 0) lu[rjv[v] * UK + rkv[v]] = up[v];
    }
    if (t - 1 >= pbeg && t - 1 < pend) {
      // residual of plane t - 1 (centre uc, i-neighbours um and up)
      const float *lu = Lu + ((t - 1) & 1) * UNP;
      float *lr = Lr + ((t - 1) & 1) * UNP;
#pragma unroll
      for (int v = 0; v < UPPT; ++v) {
        const int rj = rjv[v], rk = rkv[v];
        if (rj < 1 || rj >= UJ - 1 || rk < 1 || rk >= UK - 1) continue;
        const int e = rj * UK + rk;
        const float c = uc[v];
        const float lap = (lu[e - UK] - c) + (lu[e + UK] - c) + (lu[e - 1] - c) +
                          (lu[e + 1] - c) + (um[v] - c) + (up[v] - c);
        lr[e] = fscale * (fcur[v] - m) - lap * inv_h2;
      }
    }
    const int p = t - 2;  // plane restricted in this iteration
    if (p >= pbeg && p < pend) {
      const float *Lrp = Lr + (p & 1) * UNP;
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
            const float *row = Lrp + (2 * cj + 1 + b) * UK + 2 * ck + 1;
            s = fmaf(w[b], row[0] + 3.f * (row[1] + row[2]) + row[3], s);
          }
          // only coarse planes owned by this block accumulate (slots are shared mod 3)
          const int Ip = (p >= 0) ? p / 2 : -((1 - p) / 2);
          const bool odd = (p & 1) != 0;
          const int Io = odd ? Ip + 1 : Ip - 1;
          if (Ip >= I0 && Ip < I0 + cic) acc[Ip % 3][c] += 3.f * s;
          if (Io >= I0 && Io < I0 + cic) acc[Io % 3][c] += s;
        } else {
          const float *row0 = Lrp + (2 * cj + 2) * UK + 2 * ck + 2;
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
  const int ci = chunk_for(n, tj * tk, kSmoothBlocks, 16);
  return (int64_t)tj * tk * (n / ci);
}

hipError_t launch_smooth_stream(const float *uin, float *uout, const float *f, float fscale,
                                const float *fmean, int n, float h2, float omega,
                                int first_colour, int half_sweeps, double *partial,
                                float uscale, const float *ec, hipStream_t s) {
  const int tj = (n + SJ - 1) / SJ, tk = (n + SK - 1) / SK;
  const int ci = chunk_for(n, tj * tk, kSmoothBlocks, 16);
  dim3 grid(tk, tj, n / ci);
  const bool norm = partial != nullptr;
  const bool om1 = omega == 1.0f;
  const bool pro = ec != nullptr;
  if (norm && pro) return hipErrorInvalidValue;  // the norm pass is a pre-smoothing pass
#define PM_SMOOTH_LAUNCH(H_, N_, O_, P_)                                                 \
  k_smooth_stream<H_, N_, O_, P_><<<grid, (SmoothShape<H_, N_, P_>::NT), 0, s>>>(       \
      uin, uout, f, fscale, fmean, n, ci, h2, omega, first_colour, partial, uscale, ec)
#define PM_SMOOTH_PLAIN(H_)                                                              \
  do {                                                                                   \
    if (pro) {                                                                           \
      if (om1) PM_SMOOTH_LAUNCH(H_, false, true, true);                                  \
      else PM_SMOOTH_LAUNCH(H_, false, false, true);                                     \
    } else {                                                                             \
      if (om1) PM_SMOOTH_LAUNCH(H_, false, true, false);                                 \
      else PM_SMOOTH_LAUNCH(H_, false, false, false);                                    \
    }                                                                                    \
  } while (0)
  if (half_sweeps == 4) {
    if (norm) {
      if (om1) PM_SMOOTH_LAUNCH(4, true, true, false); else PM_SMOOTH_LAUNCH(4, true, false, false);
    } else {
      PM_SMOOTH_PLAIN(4);
    }
  } else if (half_sweeps == 2) {
    if (norm) {
      if (om1) PM_SMOOTH_LAUNCH(2, true, true, false); else PM_SMOOTH_LAUNCH(2, true, false, false);
    } else {
      PM_SMOOTH_PLAIN(2);
    }
  } else {
    return hipErrorInvalidValue;
  }
#undef PM_SMOOTH_PLAIN
#undef PM_SMOOTH_LAUNCH
  return hipGetLastError();
}

hipError_t launch_rr_stream(const float *u, const float *f, float fscale, const float *fmean,
                            int n, float inv_h2, int kind, float *fc, float *ucg, float gscale,
                            hipStream_t s) {
  const int nc = n / 2;
  const int tj = (nc + CJ - 1) / CJ, tk = (nc + CK - 1) / CK;
  const int cic = chunk_for(nc, tj * tk, PM_RR_BLOCKS, 8);
  dim3 grid(tk, tj, nc / cic);
  if (kind == PM_RESTRICT_AVG)
    k_rr_stream<PM_RESTRICT_AVG><<<grid, RT, 0, s>>>(u, f, fscale, fmean, n, cic, inv_h2, fc, ucg,
                                                     gscale);
  else
    k_rr_stream<PM_RESTRICT_FW><<<grid, RT, 0, s>>>(u, f, fscale, fmean, n, cic, inv_h2, fc, ucg,
                                                    gscale);
  return hipGetLastError();
}
