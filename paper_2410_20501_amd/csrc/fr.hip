// f(R) gravity (Hu-Sawicki): the scalaron by non-linear multigrid (paper Sects. 2.5,
// 3.7.2, 3.11).
//
// The unknown is u = (f~ / f~_bar)^(1/(n+1)), 1 in the background. Per cell the seven-
// point form of the field equation is
//   N_h(u) = (f~_bar / h^2) [sum_nb u_nb^(n+1) - 6 u^(n+1)] - K / u = s,
// and with the neighbours fixed it is u^(n+2) + p u + q = 0,
//   p = -(1/6) sum_nb u_nb^(n+1) + h^2 s / (6 f~_bar),   q = h^2 K / (6 f~_bar) < 0,
// a depressed cubic (n = 1) or quartic (n = 2) whose positive root has the closed forms
// of Sect. 3.11. Everything here is FP64, as the paper prescribes for the root branches.
//
// Full approximation storage (Sect. 3.7.2): after pre-smoothing, the residual
// d = s - N_h(u) and u are restricted (full weighting), the coarse right-hand side is
// N_H(R u) + R d, the coarse problem starts from R u, and u += P(u_H - R u) (trilinear).
// The coarsest grid gets a fixed number of sweeps (one workgroup in LDS when it is
// small).
#include <cmath>

#include "internal.h"

namespace {

constexpr int kFrThreads = 256;
constexpr int kFrCoarseThreads = 512;
constexpr int kFrCoarseMax = 2048;   // coarsest cells held in LDS (two FP64 arrays)

__host__ __device__ inline int wrapn(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ __forceinline__ double pow_n1(double u, int ne) { return ne == 1 ? u * u : u * u * u; }

// the finest grid's right-hand side from the density, s = -cA (rho - mean) - K, in one
// fused multiply-add: k_fr_source and the finest grid's streaming kernels, which read rho
// in place of s, get the same bits
__device__ __forceinline__ double fr_source(float rho, double mean, double cA, double K) {
  return fma(-cA, (double)rho - mean, -K);
}

// (i, j, k) of cell c = (i n + j) n + k in 32-bit arithmetic (n^3 <= 2^30): masks and
// shifts for a power-of-two side (the usual case; n is uniform over the launch),
// 32-bit divisions otherwise. (64-bit divisions, a long software sequence per cell,
// would dominate these memory-bound kernels.)
__device__ __forceinline__ void cell_ijk(unsigned c, int n, int &i, int &j, int &k) {
  if ((n & (n - 1)) == 0) {
    const int lg = __builtin_ctz((unsigned)n);
    k = (int)(c & (unsigned)(n - 1));
    j = (int)((c >> lg) & (unsigned)(n - 1));
    i = (int)(c >> (2 * lg));
  } else {
    const unsigned un = (unsigned)n, q = c / un;
    k = (int)(c - q * un);
    i = (int)(q / un);
    j = (int)(q - (unsigned)i * un);
  }
}

__device__ __forceinline__ unsigned fr_thread() {
  return xcd_block(blockIdx.x, gridDim.x) * kFrThreads + threadIdx.x;
}

// For Delta0 < 0, with B = (-Delta0)^(3/2), sqrt(disc) = sqrt(Delta1^2 + 4 B^2) and
// A = (|Delta1| + sqrt(disc)) / 2: Q = A^(1/3) and diff = Q^2 - (-Delta0), the latter as
// (A - B)(A + B) / (Q^4 + Q^2 (-Delta0) + Delta0^2) with A - B = |Delta1| / 2 +
// Delta1^2 / (2 (sqrt(disc) + 2 B)), which involves no subtraction of close numbers
__device__ __forceinline__ void stable_root_difference(double d0, double d1, double &Q,
                                                       double &diff) {
  const double B = -d0 * sqrt(-d0);
  const double sq = sqrt(d1 * d1 + 4.0 * B * B);
  const double ad1 = fabs(d1);
  const double A = 0.5 * (ad1 + sq);
  Q = cbrt(A);
  const double amb = 0.5 * ad1 + 0.5 * d1 * d1 / (sq + 2.0 * B);
  const double Q2 = Q * Q;
  diff = amb * (A + B) / (Q2 * Q2 - d0 * Q2 + d0 * d0);
}

// Two Newton steps on f(u) = u^3 + p u + q from an FP32 estimate u of the positive root r
// (q < 0). In every case of root3, f'(r) = 3 r^2 + p >= 1.5 r^2 and f'' = 6u, so a step
// takes a relative error e to at most 2 e^2: an estimate good to about 1e-6 reaches FP64
// rounding in two steps. The reciprocal of f' is the hardware estimate, refined by one
// Newton-Raphson step in the first step only: the second step's correction is of order
// 1e-12 u, so an estimate good to 1e-4 leaves an error far below rounding.
__device__ __forceinline__ double newton3(double u, double p, double q) {
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double f = fma(fma(u, u, p), u, q);
    const double fp = fma(3.0 * u, u, p);
    double rc = __builtin_amdgcn_rcp(fp);
    if (it == 0) rc = fma(rc, fma(-fp, rc, 1.0), rc);
    u = fma(-f, rc, u);
  }
  return u;
}

// positive root of u^3 + p u + q = 0 (q < 0), the closed forms of Sect. 3.11. Where p and
// q are in a range whose FP32 intermediates neither overflow nor underflow, the form of
// the case is evaluated in FP32 (the cancellation-free arrangements below, the
// discriminant in FP64) and polished by newton3: the same root to FP64 rounding at a
// fraction of the cost of FP64 cube roots, arccosines and cosines, which would dominate
// the sweep's arithmetic. Outside that range the forms are evaluated in FP64.
__device__ double root3(double p, double q) {
  if (p == 0.0) return cbrt(-q);
  const double d0 = -3.0 * p, d1 = 27.0 * q;
  const double ap = fabs(p), aq = -q;
  const bool f32 = ap > 1e-10 && ap < 1e10 && aq > 1e-15 && aq < 1e10;
  if (p > 0.0) {
    // one real root -(C + Delta0 / C) / 3 = (|C|^2 + Delta0) / (3 |C|), formed without
    // cancellation (the root is small where p is large). f' >= 3 r^2 here.
    if (f32) {
      const float d0f = (float)d0, d1f = (float)d1, tp = -d0f;
      const float B = tp * sqrtf(tp);
      const float sq = sqrtf(d1f * d1f + 4.0f * B * B);
      const float ad1 = fabsf(d1f);
      const float A = 0.5f * (ad1 + sq);
      const float Q = cbrtf(A), Q2 = Q * Q;
      const float amb = 0.5f * ad1 + __fdividef(0.5f * d1f * d1f, sq + 2.0f * B);
      const float diff = __fdividef(amb * (A + B), Q2 * Q2 - d0f * Q2 + d0f * d0f);
      return newton3((double)__fdividef(diff, 3.0f * Q), p, q);
    }
    double C, diff;
    stable_root_difference(d0, d1, C, diff);
    return diff / (3.0 * C);
  }
  const double disc = d1 * d1 - 4.0 * d0 * d0 * d0;
  if (disc > 0.0) {
    // one real root; C^3 = (Delta1 - sqrt(disc)) / 2 (the other sign gives Delta0 / C
    // and the same root); C and Delta0 / C have one sign here. The root exceeds
    // sqrt(-p) (f(sqrt(-p)) = q < 0), so f' >= 2 r^2.
    if (f32) {
      const float c = cbrtf(0.5f * ((float)d1 - sqrtf((float)disc)));
      return newton3((double)(-(c + __fdividef((float)d0, c)) * (1.0f / 3.0f)), p, q);
    }
    const double c = cbrt(0.5 * (d1 - sqrt(disc)));
    return -(c + d0 / c) / 3.0;
  }
  // three real roots: the largest, by the trigonometric form. With q < 0 it lies in
  // [sqrt(-p), 2 sqrt(-p/3)], where f' >= 1.5 r^2. With cos(theta) = Delta1 /
  // (2 Delta0^(3/2)) = -s (s in [0, 1]) the form -(2/3) sqrt(Delta0) cos(theta/3 + 2pi/3)
  // is (2/3) sqrt(Delta0) g(s), g(s) = cos(arccos(s) / 3), a smooth function from
  // cos(pi/6) to 1; the estimate takes g from a degree-5 least-squares polynomial
  // (fitted on Chebyshev nodes of [0, 1], relative error 7e-7).
  if (f32) {
    const float pf = (float)ap;
    const float sd0f = __builtin_amdgcn_sqrtf(3.0f * pf);
    const float sf = fminf(1.0f, fmaxf(0.0f, __fdividef(-(float)d1, 6.0f * pf * sd0f)));
    float g = 0.00198191f;
    g = fmaf(g, sf, -0.00905417f);
    g = fmaf(g, sf, 0.02197779f);
    g = fmaf(g, sf, -0.04755363f);
    g = fmaf(g, sf, 0.16662256f);
    g = fmaf(g, sf, 0.86602598f);
    return newton3((double)(0.6666667f * sd0f * g), p, q);
  }
  const double sd0 = sqrt(d0);
  const double ct = fmin(1.0, fmax(-1.0, d1 / (2.0 * d0 * sd0)));
  return -2.0 * sd0 * cos(acos(ct) / 3.0 + 2.0 * M_PI / 3.0) / 3.0;
}

// positive root of u^4 + p u + q = 0 (q < 0), the closed forms of Sect. 3.11 with
// Q + Delta0 / Q formed without cancellation (p near 0); (-q)^(1/4) where no real S
// remains
__device__ double root4(double p, double q) {
  const double fb = sqrt(sqrt(-q));
  if (p == 0.0) return fb;
  const double d0 = 12.0 * q, d1 = 27.0 * p * p;
  const double disc = d1 * d1 - 4.0 * d0 * d0 * d0;
  if (disc < 0.0) return fb;
  double Q, diff;
  stable_root_difference(d0, d1, Q, diff);
  const double w = diff / Q;
  if (!(w > 0.0)) return fb;
  const double S = 0.5 * sqrt(w / 3.0);
  const double arg = p > 0.0 ? -4.0 * S * S + p / S : -4.0 * S * S - p / S;
  return (p > 0.0 ? -S : S) + 0.5 * sqrt(fmax(arg, 0.0));
}

struct FrLevel {
  int n;
  double h2;      // h^2
  double q;       // h^2 K / (6 f~_bar)
  double ps;      // h^2 / (6 f~_bar), the factor of s in p
  double a_op;    // f~_bar / h^2
};

__device__ __forceinline__ double nb_sum(const double *__restrict__ u, int n, int i, int j, int k,
                                         int ne) {
  const size_t nn = (size_t)n * n;
  const size_t ri = (size_t)i * nn, rj = (size_t)j * n;
  const size_t im = (size_t)wrapn(i - 1, n) * nn, ip = (size_t)wrapn(i + 1, n) * nn;
  const size_t jm = (size_t)wrapn(j - 1, n) * n, jp = (size_t)wrapn(j + 1, n) * n;
  const int km = wrapn(k - 1, n), kp = wrapn(k + 1, n);
  return pow_n1(u[im + rj + k], ne) + pow_n1(u[ip + rj + k], ne) + pow_n1(u[ri + jm + k], ne) +
         pow_n1(u[ri + jp + k], ne) + pow_n1(u[ri + rj + km], ne) + pow_n1(u[ri + rj + kp], ne);
}

// the sum of u^(n+1) over the six neighbours (i-1, i+1, j-1, j+1, k-1, k+1, in this
// order) with its multiplies and adds fused explicitly, so the compiler has no choice
// left: every sweep kernel that calls it gets the same bits
template <int NE>
__device__ __forceinline__ double nb6(double a, double b, double c, double d, double e,
                                      double f) {
  double t = NE == 1 ? a * a : (a * a) * a;
  t = fma(NE == 1 ? b : b * b, b, t);
  t = fma(NE == 1 ? c : c * c, c, t);
  t = fma(NE == 1 ? d : d * d, d, t);
  t = fma(NE == 1 ? e : e * e, e, t);
  return fma(NE == 1 ? f : f * f, f, t);
}

// one colour of the non-linear red-black Gauss-Seidel: the cells with (i+j+k) % 2 ==
// colour take the root of their polynomial (n even)
template <int NE>
__global__ __launch_bounds__(kFrThreads) void k_fr_sweep(double *__restrict__ u,
                                                         const double *__restrict__ s, FrLevel L,
                                                         int colour) {
  const int n = L.n, hn = n >> 1;
  const unsigned t = fr_thread();
  if (t >= (unsigned)n * n * hn) return;
  // t = (i n + j) (n/2) + k/2: the same decoding as a grid of side n with n/2 columns
  int i, j, k2;
  if ((n & (n - 1)) == 0) {
    const int lg = __builtin_ctz((unsigned)n);
    k2 = (int)(t & (unsigned)(hn - 1));
    j = (int)((t >> (lg - 1)) & (unsigned)(n - 1));
    i = (int)(t >> (2 * lg - 1));
  } else {
    const unsigned q = t / (unsigned)hn;
    k2 = (int)(t - q * (unsigned)hn);
    i = (int)(q / (unsigned)n);
    j = (int)(q - (unsigned)i * n);
  }
  const int k = 2 * k2 + ((i + j + colour) & 1);
  const size_t nn = (size_t)n * n, ri = (size_t)i * nn, rj = (size_t)j * n;
  const size_t c = ri + rj + k;
  const size_t im = (size_t)wrapn(i - 1, n) * nn, ip = (size_t)wrapn(i + 1, n) * nn;
  const size_t jm = (size_t)wrapn(j - 1, n) * n, jp = (size_t)wrapn(j + 1, n) * n;
  const double nb = nb6<NE>(u[im + rj + k], u[ip + rj + k], u[ri + jm + k], u[ri + jp + k],
                            u[ri + rj + wrapn(k - 1, n)], u[ri + rj + wrapn(k + 1, n)]);
  const double p = fma(nb, -1.0 / 6.0, L.ps * s[c]);
  u[c] = NE == 1 ? root3(p, L.q) : root4(p, L.q);
}

// One full non-linear red-black sweep per pass over HBM (grids of at least 256 cells per
// side, n % 64 == 0): the 2.5D streaming scheme of the linear smoother, in FP64. A block
// owns a 16 x 64 (j, k) tile plus a 2-cell halo and a chunk of i-planes; each thread holds
// one pair of k-neighbouring points (opposite colours) of the tile plus halo in a ring of
// four planes in registers. Step q loads plane q, applies the first colour to plane q - 1
// and the second to plane q - 2, and writes plane q - 2; in-plane neighbours come through
// LDS, published before one barrier (two sets of slots, used by alternate steps). With the
// colour of a point (i + j + k) mod 2, a step updates the same point of every pair in both
// of its half-sweeps (E, the point with j + k + first_colour odd, in steps with q even; O
// with q odd). Halo points are computed unmasked (a wrong value moves one cell per
// half-sweep and never reaches the tile). Out of place: neighbouring blocks still read the
// input's halo. The root and the neighbour sum (nb6) are those of k_fr_sweep, so both
// kernels give the same bits.
constexpr int kFsSJ = 16, kFsSK = 64, kFsH = 2;
constexpr int kFsRJ = kFsSJ + 2 * kFsH, kFsRK = kFsSK + 2 * kFsH, kFsRK2 = kFsRK / 2;
constexpr int kFsNPAIR = kFsRJ * kFsRK2;              // 680
constexpr int kFsNT = (kFsNPAIR + 63) / 64 * 64;      // 704 threads, one pair each
constexpr int kFsPAD = kFsRK2 + 2;
constexpr int kFsARR = kFsNPAIR + 2 * kFsPAD;         // doubles per colour array
constexpr int kFsSLOT = 2 * kFsARR;                   // E then O
constexpr int kFsRING = kFsH + 2;                     // planes in registers
constexpr int kFsPF = 2;                              // planes in flight

struct FrStream {
  int li, col;
  bool swp, inside;
  double uE[kFsRING], uO[kFsRING], sE[kFsRING], sO[kFsRING];
  double2 pu[kFsPF], ps[kFsPF];
  float2 pr[kFsPF];  // the density's pairs in flight, in place of ps (RHO)
  const double *uin, *s;
  const float *rho;  // (RHO) s formed from the density (fr_source), not read
  double mean, cA, K;
  double *uout, *lds;
  int n, i0, ci, qend;
  size_t nn;
  __device__ __forceinline__ int wrap_plane(int q) const { return q < 0 ? q + n : (q >= n ? q - n : q); }
  // plane q into prefetch slot P; with RHO the density is kept as loaded and turned into
  // s only when the slot is used, so the loads stay in flight
  template <bool RHO>
  __device__ __forceinline__ void load(int q, int P) {
    const size_t plane = (size_t)wrap_plane(q) * nn;
    pu[P] = *reinterpret_cast<const double2 *>(uin + plane + col);
    if constexpr (RHO)
      pr[P] = *reinterpret_cast<const float2 *>(rho + plane + col);
    else
      ps[P] = *reinterpret_cast<const double2 *>(s + plane + col);
  }
  template <bool RHO>
  __device__ __forceinline__ double2 source_pair(int P) const {
    if constexpr (RHO)
      return make_double2(fr_source(pr[P].x, mean, cA, K), fr_source(pr[P].y, mean, cA, K));
    else
      return ps[P];
  }
};

template <int R>
constexpr int fs_ring(int d) {
  return ((R - d) % kFsRING + kFsRING) % kFsRING;
}

// half-sweep S (1, 2) of the step with q = R mod RING: plane q - S, in-plane neighbours
// from the LDS slot of S (the other points of the plane, as published this step)
template <int R, int S, int NE>
__device__ __forceinline__ void fs_half(FrStream &c, const FrLevel &L) {
  constexpr int cs = fs_ring<R>(S), cm = fs_ring<R>(S + 1), cp = fs_ring<R>(S - 1);
  const double *LE = c.lds + ((R & 1) * kFsH + S - 1) * kFsSLOT, *LO = LE + kFsARR;
  const int e = c.li;
  if constexpr ((R & 1) == 0) {
    // update E (k-neighbours in the O array at e - 1 + offe, e + offe)
    const int k = c.swp ? e : e - 1;
    const double nb =
        nb6<NE>(c.uE[cm], c.uE[cp], LO[e - kFsRK2], LO[e + kFsRK2], LO[k], LO[k + 1]);
    const double p = fma(nb, -1.0 / 6.0, L.ps * c.sE[cs]);
    c.uE[cs] = NE == 1 ? root3(p, L.q) : root4(p, L.q);
  } else {
    const int k = c.swp ? e - 1 : e;
    const double nb =
        nb6<NE>(c.uO[cm], c.uO[cp], LE[e - kFsRK2], LE[e + kFsRK2], LE[k], LE[k + 1]);
    const double p = fma(nb, -1.0 / 6.0, L.ps * c.sO[cs]);
    c.uO[cs] = NE == 1 ? root3(p, L.q) : root4(p, L.q);
  }
}

template <int R, int NE, bool RHO>
__device__ __forceinline__ void fs_step(FrStream &c, const FrLevel &L, int q) {
  constexpr int P = R % kFsPF, c0 = fs_ring<R>(0), cH = fs_ring<R>(kFsH);
  {
    const double2 u = c.pu[P], sv = c.template source_pair<RHO>(P);
    c.uE[c0] = c.swp ? u.y : u.x;
    c.uO[c0] = c.swp ? u.x : u.y;
    c.sE[c0] = c.swp ? sv.y : sv.x;
    c.sO[c0] = c.swp ? sv.x : sv.y;
  }
  c.template load<RHO>(min(q + kFsPF, c.qend - 1), P);  // past the end: a harmless reload
  // half-sweep S acts on plane q - S; it reads the points of that plane it does not
  // change, published here (E values when it updates O, and the reverse)
#pragma unroll
  for (int S = 1; S <= kFsH; ++S) {
    double *LE = c.lds + ((R & 1) * kFsH + S - 1) * kFsSLOT, *LO = LE + kFsARR;
    const int cs = ((R - S) % kFsRING + kFsRING) % kFsRING;
    if ((R & 1) == 1) LE[c.li] = c.uE[cs];
    if ((R & 1) == 0) LO[c.li] = c.uO[cs];
  }
  __syncthreads();
  fs_half<R, 1, NE>(c, L);
  fs_half<R, 2, NE>(c, L);
  const int pout = q - kFsH;  // final
  if (c.inside && pout >= c.i0 && pout < c.i0 + c.ci) {
    const double a = c.uE[cH], b = c.uO[cH];
    *reinterpret_cast<double2 *>(c.uout + (size_t)pout * c.nn + c.col) =
        c.swp ? make_double2(b, a) : make_double2(a, b);
  }
}

template <int R, bool GUARD, int NE, bool RHO>
__device__ __forceinline__ void fs_steps(FrStream &c, const FrLevel &L, int q) {
  if constexpr (R < kFsRING) {
    if (!GUARD || q + R < c.qend) fs_step<R, NE, RHO>(c, L, q + R);
    fs_steps<R + 1, GUARD, NE, RHO>(c, L, q);
  }
}

template <int NE, bool RHO>
__global__ __launch_bounds__(kFsNT) void k_fr_sweep_stream(const double *__restrict__ uin,
                                                           double *__restrict__ uout,
                                                           const double *__restrict__ s,
                                                           const float *__restrict__ rho,
                                                           const double *__restrict__ mean,
                                                           double cA, double K, FrLevel L,
                                                           int ci, int first_colour) {
  static_assert(kFsRING % 2 == 0 && kFsRING % kFsPF == 0, "ring parity and prefetch slots");
  // two sets (steps of even and odd q) of kFsH slots: a set is rewritten two steps after
  // it was read, behind the barrier that ended those reads
  __shared__ double lds[2 * kFsH * kFsSLOT];
  const unsigned lin = xcd_block(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                                 gridDim.x * gridDim.y * gridDim.z);
  const int bx = lin % gridDim.x, by = (lin / gridDim.x) % gridDim.y,
            bz = lin / (gridDim.x * gridDim.y);
  const int n = L.n, k0 = bx * kFsSK, j0 = by * kFsSJ;
  FrStream c;
  c.uin = uin;
  c.s = s;
  c.rho = rho;
  c.mean = RHO ? mean[0] : 0.0;
  c.cA = cA;
  c.K = K;
  c.uout = uout;
  c.lds = lds;
  c.n = n;
  c.i0 = bz * ci;
  c.ci = ci;
  c.qend = c.i0 + ci + kFsH;
  c.nn = (size_t)n * n;
  for (int e = threadIdx.x; e < kFsPAD; e += kFsNT)
    for (int a = 0; a < 4 * kFsH; ++a) {
      lds[a * kFsARR + e] = 1.0;
      lds[a * kFsARR + kFsPAD + kFsNPAIR + e] = 1.0;
    }
  {
    const int e = threadIdx.x;
    const bool v = e < kFsNPAIR;
    const int rj = v ? e / kFsRK2 : 0, r2 = v ? e % kFsRK2 : 0;
    const int gj = j0 - kFsH + rj, gk = k0 - kFsH + 2 * r2;  // gk even
    c.swp = ((gj + first_colour) & 1) == 0;  // E = the point with j + k + first_colour odd
    // a thread without a pair works on the trailing padding (its values reach only halo
    // points), so every lane runs the same code
    c.li = v ? kFsPAD + e : kFsPAD + kFsNPAIR + 1;
    c.col = v ? (wrapn(gj < 0 ? gj + n : (gj >= n ? gj - n : gj), n) * n +
                 (gk < 0 ? gk + n : (gk >= n ? gk - n : gk)))
              : 0;
    c.inside = v && rj >= kFsH && rj < kFsH + kFsSJ && 2 * r2 >= kFsH && 2 * r2 < kFsH + kFsSK;
#pragma unroll
    for (int a = 0; a < kFsRING; ++a) c.uE[a] = c.uO[a] = c.sE[a] = c.sO[a] = 1.0;
  }
  const int qbeg = c.i0 - kFsH;  // even (ci even): step R of a ring period has q = R mod 2
#pragma unroll
  for (int a = 0; a < kFsPF; ++a) c.template load<RHO>(qbeg + a, a);
  int q = qbeg;
  for (; q + kFsRING <= c.qend; q += kFsRING) fs_steps<0, false, NE, RHO>(c, L, q);
  fs_steps<0, true, NE, RHO>(c, L, q);
}

// d = s - N_h(u)
__global__ __launch_bounds__(kFrThreads) void k_fr_residual(const double *__restrict__ u,
                                                            const double *__restrict__ s,
                                                            FrLevel L, double K, int ne,
                                                            double *__restrict__ d) {
  const int n = L.n;
  const unsigned c = fr_thread();
  if (c >= (unsigned)n * n * n) return;
  int i, j, k;
  cell_ijk(c, n, i, j, k);
  const double uc = u[c];
  const double op = L.a_op * (nb_sum(u, n, i, j, k, ne) - 6.0 * pow_n1(uc, ne)) - K / uc;
  d[c] = s[c] - op;
}

// full weighting of u and d onto the grid of side n/2: per axis (1, 3, 3, 1) / 8 over the
// fine cells 2J-1 .. 2J+2; u0 = uH = R u, sH = R d
__global__ __launch_bounds__(kFrThreads) void k_fr_restrict(const double *__restrict__ u,
                                                            const double *__restrict__ d, int n,
                                                            double *__restrict__ u0,
                                                            double *__restrict__ uH,
                                                            double *__restrict__ sH) {
  const int N = n >> 1;
  const unsigned c = fr_thread();
  if (c >= (unsigned)N * N * N) return;
  int I, J, Kc;
  cell_ijk(c, N, I, J, Kc);
  constexpr double w[4] = {0.125, 0.375, 0.375, 0.125};
  double su = 0.0, sd = 0.0;
  for (int a = 0; a < 4; ++a) {
    const size_t ra = (size_t)wrapn(2 * I - 1 + a, n) * n;
    for (int b = 0; b < 4; ++b) {
      const size_t rb = (ra + wrapn(2 * J - 1 + b, n)) * n;
      const double wab = w[a] * w[b];
      double tu = 0.0, td = 0.0;
      for (int e = 0; e < 4; ++e) {
        const size_t f = rb + wrapn(2 * Kc - 1 + e, n);
        tu += w[e] * u[f];
        td += w[e] * d[f];
      }
      su += wab * tu;
      sd += wab * td;
    }
  }
  u0[c] = su;
  uH[c] = su;
  sH[c] = sd;
}

// Residual and restriction in one pass over the fine grid (fine grids of at least 256
// cells per side, the coarse side a multiple of 16): u0 = uH = R u and sH = R d with d = s - N_h(u), the full weighting of
// k_fr_restrict and the residual of k_fr_residual, without writing d. A block owns a
// 16 x 16 tile of coarse (J, K) columns and a chunk of coarse planes, and walks through
// the fine planes once: iteration t publishes u of plane t in LDS, forms d of plane
// t - 1 from it (the i-neighbours in registers) and restricts u and d of plane t - 2 in
// the plane; each fine plane adds to two coarse planes (three accumulator slots). u
// planes rotate through three LDS buffers and d planes through two, so one barrier per
// iteration orders every buffer's reuse.
constexpr int kRrCJ = 16, kRrCK = 16, kRrT = 256;
constexpr int kRrUJ = 2 * kRrCJ + 4, kRrUK = 2 * kRrCK + 4, kRrNP = kRrUJ * kRrUK;
constexpr int kRrPer = (kRrNP + kRrT - 1) / kRrT;  // region points per thread
static_assert(kRrCJ * kRrCK == kRrT, "one coarse column per thread");

template <int NE, bool RHO>
__global__ __launch_bounds__(kRrT) void k_fr_rr(const double *__restrict__ u,
                                                const double *__restrict__ s,
                                                const float *__restrict__ rho,
                                                const double *__restrict__ mean, double cA,
                                                FrLevel L, double K, int cic,
                                                double *__restrict__ u0,
                                                double *__restrict__ uH,
                                                double *__restrict__ sH) {
  __shared__ double Lu[3][kRrNP];
  __shared__ double Ld[2][kRrNP];
  const int n = L.n, N = n >> 1;
  const unsigned lin = xcd_block(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                                 gridDim.x * gridDim.y * gridDim.z);
  const int bx = lin % gridDim.x, by = (lin / gridDim.x) % gridDim.y,
            bz = lin / (gridDim.x * gridDim.y);
  const int K0 = bx * kRrCK, J0 = by * kRrCJ, I0 = bz * cic;
  const int fj0 = 2 * J0 - 2, fk0 = 2 * K0 - 2;  // fine region origin
  const size_t nn = (size_t)n * n;
  int rj[kRrPer], rk[kRrPer];
  unsigned col[kRrPer];
#pragma unroll
  for (int v = 0; v < kRrPer; ++v) {
    const int e = threadIdx.x + v * kRrT;
    rj[v] = e < kRrNP ? e / kRrUK : -100;
    rk[v] = e < kRrNP ? e % kRrUK : -100;
    col[v] = e < kRrNP ? (unsigned)(wrapn(((fj0 + rj[v]) % n + n) % n, n) * n +
                                    ((fk0 + rk[v]) % n + n) % n)
                       : 0u;
  }
  double um[kRrPer], uc[kRrPer], up[kRrPer], nu[kRrPer], sc[kRrPer], sn[kRrPer];
#pragma unroll
  for (int v = 0; v < kRrPer; ++v) um[v] = uc[v] = up[v] = nu[v] = sc[v] = sn[v] = 1.0;
  double au[3] = {0.0, 0.0, 0.0}, ad[3] = {0.0, 0.0, 0.0};  // coarse planes, slot I mod 3
  // fine planes restricted: 2 I0 - 1 .. 2 (I0 + cic), i.e. [pbeg, pend)
  const int pbeg = 2 * I0 - 1, pend = 2 * (I0 + cic) + 1;
  // RHO: the finest grid's s formed from the density (fr_source) when a plane moves into
  // place, the loads kept in flight as loaded
  const double mv = RHO ? mean[0] : 0.0;
  float rn[kRrPer];
#pragma unroll
  for (int v = 0; v < kRrPer; ++v) rn[v] = 0.0f;
  auto plane_of = [&](int q) { return (size_t)(((q % n) + n) % n) * nn; };
  auto prefetch = [&](int q) {  // u of plane q, s of plane q - 1
    const size_t pu = plane_of(q), ps = plane_of(q - 1);
#pragma unroll
    for (int v = 0; v < kRrPer; ++v)
      if (rj[v] >= 0) {
        nu[v] = u[pu + col[v]];
        if constexpr (RHO)
          rn[v] = rho[ps + col[v]];
        else
          sn[v] = s[ps + col[v]];
      }
  };
  constexpr double w[4] = {0.125, 0.375, 0.375, 0.125};
  const int cj = threadIdx.x / kRrCK, ck = threadIdx.x % kRrCK;
  prefetch(pbeg - 1);
  for (int t = pbeg - 1; t <= pend + 1; ++t) {
#pragma unroll
    for (int v = 0; v < kRrPer; ++v) {
      um[v] = uc[v];
      uc[v] = up[v];
      up[v] = nu[v];  // u of plane t
      sc[v] = RHO ? fr_source(rn[v], mv, cA, K) : sn[v];  // s of plane t - 1
    }
    if (t < pend) prefetch(t + 1);
    const int su = ((t % 3) + 3) % 3;
    if (t >= pbeg - 1 && t < pend) {
      // (plane pbeg - 1 too: the residual of plane pbeg needs it only through registers,
      // but publishing it keeps the buffer rotation uniform)
#pragma unroll
      for (int v = 0; v < kRrPer; ++v)
        if (rj[v] >= 0) Lu[su][rj[v] * kRrUK + rk[v]] = up[v];
    }
    if (t - 1 >= pbeg && t - 1 < pend) {
      // d of plane t - 1 on the region less its outer ring (centre uc, i-neighbours um, up)
      const double *lu = Lu[((t - 1) % 3 + 3) % 3];
      double *ld = Ld[((t - 1) & 1)];
#pragma unroll
      for (int v = 0; v < kRrPer; ++v) {
        const int a = rj[v], b = rk[v];
        if (a < 1 || a >= kRrUJ - 1 || b < 1 || b >= kRrUK - 1) continue;
        const int e = a * kRrUK + b;
        const double c = uc[v];
        const double nb = pow_n1(um[v], NE) + pow_n1(up[v], NE) + pow_n1(lu[e - kRrUK], NE) +
                          pow_n1(lu[e + kRrUK], NE) + pow_n1(lu[e - 1], NE) +
                          pow_n1(lu[e + 1], NE);
        const double op = L.a_op * (nb - 6.0 * pow_n1(c, NE)) - K / c;
        ld[e] = sc[v] - op;
      }
    }
    const int p = t - 2;
    if (p >= pbeg && p < pend) {
      const double *lu = Lu[((p % 3) + 3) % 3];
      const double *ld = Ld[p & 1];
      double tu = 0.0, td = 0.0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int row = (2 * cj + 1 + b) * kRrUK + 2 * ck + 1;
        double ru = 0.0, rd = 0.0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          ru += w[e] * lu[row + e];
          rd += w[e] * ld[row + e];
        }
        tu += w[b] * ru;
        td += w[b] * rd;
      }
      // fine plane p adds to coarse planes I = p/2 (weight 3/8) and the next one on its
      // side (1/8); only coarse planes of this block accumulate
      const int Ip = (p >= 0) ? p / 2 : -((1 - p) / 2);
      const int Io = (p & 1) ? Ip + 1 : Ip - 1;
      if (Ip >= I0 && Ip < I0 + cic) {
        au[Ip % 3] += 0.375 * tu;
        ad[Ip % 3] += 0.375 * td;
      }
      if (Io >= I0 && Io < I0 + cic) {
        au[Io % 3] += 0.125 * tu;
        ad[Io % 3] += 0.125 * td;
      }
      // coarse plane I complete after fine plane 2 I + 2
      if ((p & 1) == 0 && p >= 2 * I0 + 2) {
        const int I = p / 2 - 1, sl = I % 3;
        const int J = J0 + cj, Kc = K0 + ck;
        if (J < N && Kc < N) {
          const size_t ci = ((size_t)I * N + J) * N + Kc;
          u0[ci] = au[sl];
          uH[ci] = au[sl];
          sH[ci] = ad[sl];
        }
        au[sl] = 0.0;
        ad[sl] = 0.0;
      }
    }
    __syncthreads();
  }
}

// sH += N_H(u0): the coarse right-hand side N_H(R u) + R d
__global__ __launch_bounds__(kFrThreads) void k_fr_coarse_rhs(const double *__restrict__ u0,
                                                              FrLevel L, double K, int ne,
                                                              double *__restrict__ sH) {
  const int n = L.n;
  const unsigned c = fr_thread();
  if (c >= (unsigned)n * n * n) return;
  int i, j, k;
  cell_ijk(c, n, i, j, k);
  const double uc = u0[c];
  sH[c] += L.a_op * (nb_sum(u0, n, i, j, k, ne) - 6.0 * pow_n1(uc, ne)) - K / uc;
}

// uout = uin + P(uH - u0) on the fine grid of side n: per axis 3/4 of the nearest coarse
// centre and 1/4 of the next one. A thread owns a coarse column (J, K) over `ch`
// consecutive coarse planes I and updates the 8 fine children (2I+a, 2J+b, 2K+c) of each;
// the differences e = uH - u0 of the 3 x 3 (J, K) neighbourhood sit in a ring of three
// planes (I-1, I, I+1) in registers, so each coarse value is loaded 9 times instead of
// 27 (a thread per coarse cell) or 64 (a thread per fine cell), and the next plane is in
// flight while the current one is written.
// VEC: uin and uout 16-byte aligned, each pair of fine children (2K, 2K+1) loaded and
// stored as one double2
template <bool VEC>
__global__ __launch_bounds__(kFrThreads) void k_fr_prolong(const double *uin, double *uout,
                                                           int n, int ch,
                                                           const double *__restrict__ uH,
                                                           const double *__restrict__ u0) {
  const int N = n >> 1;
  const unsigned t = fr_thread();
  if (t >= (unsigned)N * N * (unsigned)(N / ch)) return;
  int ic, J, K;
  cell_ijk(t, N, ic, J, K);
  const size_t NN = (size_t)N * N;
  const size_t jr[3] = {(size_t)wrapn(J - 1, N) * N, (size_t)J * N, (size_t)wrapn(J + 1, N) * N};
  const int kx[3] = {wrapn(K - 1, N), K, wrapn(K + 1, N)};
  constexpr double w[2] = {0.75, 0.25};
  const auto load_plane = [&](int I, double(&d)[3][3]) {
    const size_t r0 = (size_t)wrapn(I, N) * NN;
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int q = 0; q < 3; ++q) d[b][q] = uH[r0 + jr[b] + kx[q]] - u0[r0 + jr[b] + kx[q]];
  };
  const int I0 = ic * ch;
  double e[3][3][3];  // planes I - 1, I, I + 1
  load_plane(I0 - 1, e[0]);
  load_plane(I0, e[1]);
  load_plane(I0 + 1, e[2]);
  const size_t nn = (size_t)n * n;
  for (int I = I0; I < I0 + ch; ++I) {
    double nx[3][3];
    if (I + 1 < I0 + ch) load_plane(I + 2, nx);
#pragma unroll
    for (int ai = 0; ai < 2; ++ai) {      // fine plane 2I + ai: near coarse plane 1, far 0 or 2
      const int af = ai ? 2 : 0;
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {    // fine row 2J + bj
        const int bf = bj ? 2 : 0;
        double out[2];
#pragma unroll
        for (int ck = 0; ck < 2; ++ck) {  // fine column 2K + ck
          const int kf = ck ? 2 : 0;
          // planes (near, far) x rows (near, far), each the k-interpolation
          // w0 e_near + w1 e_far
          const int pa[2] = {1, af}, pb[2] = {1, bf};
          double v = 0.0;
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
              const double tk = w[0] * e[pa[a]][pb[b]][1] + w[1] * e[pa[a]][pb[b]][kf];
              v += w[a] * w[b] * tk;
            }
          out[ck] = v;
        }
        const size_t o = (size_t)(2 * I + ai) * nn + (size_t)(2 * J + bj) * n + 2 * K;
        // (in place when uout == uin)
        if constexpr (VEC) {
          const double2 v = *reinterpret_cast<const double2 *>(uin + o);
          *reinterpret_cast<double2 *>(uout + o) = make_double2(v.x + out[0], v.y + out[1]);
        } else {
          uout[o] = uin[o] + out[0];
          uout[o + 1] = uin[o + 1] + out[1];
        }
      }
    }
    if (I + 1 < I0 + ch) {
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          e[0][b][q] = e[1][b][q];
          e[1][b][q] = e[2][b][q];
          e[2][b][q] = nx[b][q];
        }
    }
  }
}

// the coarsest grid (n^3 <= kFrCoarseMax, n even): `sweeps` red-black sweeps in LDS
template <int NE>
__global__ __launch_bounds__(kFrCoarseThreads) void k_fr_coarse(double *__restrict__ u,
                                                                const double *__restrict__ s,
                                                                FrLevel L, int sweeps) {
  constexpr int kCC = kFrCoarseMax / kFrCoarseThreads;  // cells per thread at most
  __shared__ double su[kFrCoarseMax];
  __shared__ double ss[kFrCoarseMax];
  const int n = L.n, cells = n * n * n;
  // a thread's cells, their colours and neighbours' places, decoded once for all sweeps
  int cell[kCC], colour_of[kCC], nbr[kCC][6];
#pragma unroll
  for (int m = 0; m < kCC; ++m) {
    const int c = (int)threadIdx.x + m * kFrCoarseThreads;
    cell[m] = c < cells ? c : -1;
    const int cv = c < cells ? c : 0;
    const int i = cv / (n * n), j = (cv / n) % n, k = cv % n;
    colour_of[m] = (i + j + k) & 1;
    const int ri = i * n * n, rj = j * n;
    nbr[m][0] = wrapn(i - 1, n) * n * n + rj + k;
    nbr[m][1] = wrapn(i + 1, n) * n * n + rj + k;
    nbr[m][2] = ri + wrapn(j - 1, n) * n + k;
    nbr[m][3] = ri + wrapn(j + 1, n) * n + k;
    nbr[m][4] = ri + rj + wrapn(k - 1, n);
    nbr[m][5] = ri + rj + wrapn(k + 1, n);
    if (c < cells) {
      su[c] = u[c];
      ss[c] = s[c];
    }
  }
  __syncthreads();
  for (int it = 0; it < sweeps; ++it)
    for (int colour = 0; colour < 2; ++colour) {
#pragma unroll
      for (int m = 0; m < kCC; ++m) {
        const int c = cell[m];
        if (c < 0 || colour_of[m] != colour) continue;
        const double nb = nb6<NE>(su[nbr[m][0]], su[nbr[m][1]], su[nbr[m][2]], su[nbr[m][3]],
                                  su[nbr[m][4]], su[nbr[m][5]]);
        const double p = fma(nb, -1.0 / 6.0, L.ps * ss[c]);
        su[c] = NE == 1 ? root3(p, L.q) : root4(p, L.q);
      }
      __syncthreads();
    }
#pragma unroll
  for (int m = 0; m < kCC; ++m)
    if (cell[m] >= 0) u[cell[m]] = su[cell[m]];
}

// s = -cA (rho - mean) - K
__global__ __launch_bounds__(kFrThreads) void k_fr_source(const float *__restrict__ rho,
                                                          const double *__restrict__ mean,
                                                          int64_t count, double cA, double K,
                                                          double *__restrict__ s) {
  const int64_t c = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kFrThreads + threadIdx.x;
  if (c >= count) return;
  s[c] = fr_source(rho[c], mean[0], cA, K);
}

__global__ __launch_bounds__(kFrThreads) void k_fill_d(double *__restrict__ x, double v,
                                                       int64_t count) {
  const int64_t c = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kFrThreads + threadIdx.x;
  if (c < count) x[c] = v;
}

// the potential of the force: phi_N - (c~^2 / 2) f~_bar u^(n+1)
__global__ __launch_bounds__(kFrThreads) void k_fr_phi(const float *__restrict__ phin,
                                                       const double *__restrict__ u,
                                                       int64_t count, double coef, int ne,
                                                       float *__restrict__ out) {
  const int64_t c = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kFrThreads + threadIdx.x;
  if (c >= count) return;
  out[c] = (float)((double)phin[c] - coef * pow_n1(u[c], ne));
}

// per-block sums of d^2 and s^2 (two doubles per block, grid-stride)
__global__ __launch_bounds__(kFrThreads) void k_fr_norms(const double *__restrict__ d,
                                                         const double *__restrict__ s,
                                                         int64_t count,
                                                         double *__restrict__ partial) {
  double a = 0.0, b = 0.0;
  for (int64_t c = (int64_t)blockIdx.x * kFrThreads + threadIdx.x; c < count;
       c += (int64_t)gridDim.x * kFrThreads) {
    a += d[c] * d[c];
    b += s[c] * s[c];
  }
  __shared__ double la[kFrThreads], lb[kFrThreads];
  la[threadIdx.x] = a;
  lb[threadIdx.x] = b;
  __syncthreads();
  for (int o = kFrThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      la[threadIdx.x] += la[threadIdx.x + o];
      lb[threadIdx.x] += lb[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = la[0];
    partial[2 * blockIdx.x + 1] = lb[0];
  }
}

__global__ __launch_bounds__(kFrThreads) void k_fr_norms_final(const double *__restrict__ partial,
                                                               int nblocks,
                                                               double *__restrict__ out) {
  __shared__ double la[kFrThreads], lb[kFrThreads];
  double a = 0.0, b = 0.0;
  for (int q = threadIdx.x; q < nblocks; q += kFrThreads) {
    a += partial[2 * q];
    b += partial[2 * q + 1];
  }
  la[threadIdx.x] = a;
  lb[threadIdx.x] = b;
  __syncthreads();
  for (int o = kFrThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      la[threadIdx.x] += la[threadIdx.x + o];
      lb[threadIdx.x] += lb[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = la[0];
    out[1] = lb[0];
  }
}

unsigned blocks(int64_t count) { return (unsigned)((count + kFrThreads - 1) / kFrThreads); }

bool fr_is_coarsest(int n) { return n <= 4 || n % 4 != 0; }

struct FrRun {
  pm_ctx *ctx;
  const pm_step_params *p;
  double fbar, K;
  int ne;
  hipStream_t s;
  // non-null: the finest grid reads the density in place of its s (streaming levels)
  const float *rho0 = nullptr;
  const double *mean0 = nullptr;
  double cA = 0.0;

  FrLevel level(int l) const {
    const int n = ctx->fr_lev[l].n;
    const double h = 1.0 / n;
    FrLevel L;
    L.n = n;
    L.h2 = h * h;
    L.q = L.h2 * K / (6.0 * fbar);
    L.ps = L.h2 / (6.0 * fbar);
    L.a_op = fbar / L.h2;
    return L;
  }

  hipError_t sweep(int l, double *u, int first) {
    const FrLevel L = level(l);
    const int64_t half = (int64_t)L.n * L.n * L.n / 2;
    const double *sv = ctx->fr_lev[l].s;
    if (l == 0) pm_kt_begin(ctx, PM_KERNEL_FR_SWEEP, s);
    for (int colour : {first, 1 - first}) {
      if (ne == 1)
        k_fr_sweep<1><<<blocks(half), kFrThreads, 0, s>>>(u, sv, L, colour);
      else
        k_fr_sweep<2><<<blocks(half), kFrThreads, 0, s>>>(u, sv, L, colour);
    }
    if (l == 0) pm_kt_end(ctx, PM_KERNEL_FR_SWEEP, s, 32.0 * 2.0 * (double)half);
    return hipGetLastError();
  }

  // the streaming sweep (out of place) on level l: grids of at least 256 cells per side
  // in 16 x 64 tiles, when the pre- and post-sweeps and the out-of-place prolongation
  // leave the iterate in the caller's array (an odd pre + post count) and u is 16-byte
  // aligned for the paired loads
  bool streams(int l, const double *u) const {
    const int n = ctx->fr_lev[l].n;
    return ctx->fr_lev[l].alt && n >= 256 && n % kFsSK == 0 &&
           (p->fr_pre + p->fr_post) % 2 == 1 && (reinterpret_cast<uintptr_t>(u) & 15) == 0;
  }

  void prolong(int l, const double *in, double *out) {
    const FrLevel L = level(l);
    const pm_fr_level &C = ctx->fr_lev[l + 1];
    // coarse planes per thread: up to 16, a divisor of N, with at least 2048 workgroups
    const int N = L.n / 2;
    int ch = 16;
    while (ch > 1 && (N % ch != 0 || (int64_t)N * N * (N / ch) < 2048 * kFrThreads)) ch /= 2;
    const int64_t threads = (int64_t)N * N * (N / ch);
    if (((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15) == 0)
      k_fr_prolong<true><<<blocks(threads), kFrThreads, 0, s>>>(in, out, L.n, ch, C.u, C.u0);
    else
      k_fr_prolong<false><<<blocks(threads), kFrThreads, 0, s>>>(in, out, L.n, ch, C.u, C.u0);
  }

  hipError_t stream_sweep(int l, const double *in, double *out, int first) {
    const FrLevel L = level(l);
    const int n = L.n, tiles = (n / kFsSJ) * (n / kFsSK);
    int ci = n;
    while (ci / 2 >= 16 && tiles * (n / ci) < 512 && n % (ci / 2) == 0) ci /= 2;
    const dim3 grid(n / kFsSK, n / kFsSJ, n / ci);
    const float *src = l == 0 ? rho0 : nullptr;
    if (l == 0) pm_kt_begin(ctx, PM_KERNEL_FR_SWEEP, s);
    const double *sv = ctx->fr_lev[l].s;
    if (ne == 1 && src)
      k_fr_sweep_stream<1, true><<<grid, kFsNT, 0, s>>>(in, out, sv, src, mean0, cA, K, L, ci, first);
    else if (ne == 1)
      k_fr_sweep_stream<1, false><<<grid, kFsNT, 0, s>>>(in, out, sv, src, mean0, cA, K, L, ci, first);
    else if (src)
      k_fr_sweep_stream<2, true><<<grid, kFsNT, 0, s>>>(in, out, sv, src, mean0, cA, K, L, ci, first);
    else
      k_fr_sweep_stream<2, false><<<grid, kFsNT, 0, s>>>(in, out, sv, src, mean0, cA, K, L, ci, first);
    if (l == 0) pm_kt_end(ctx, PM_KERNEL_FR_SWEEP, s, 32.0 * (double)n * n * n);
    return hipGetLastError();
  }

  hipError_t coarsest(int l, double *u) {
    const FrLevel L = level(l);
    if ((int64_t)L.n * L.n * L.n <= kFrCoarseMax) {
      if (ne == 1)
        k_fr_coarse<1><<<1, kFrCoarseThreads, 0, s>>>(u, ctx->fr_lev[l].s, L, p->fr_coarse_sweeps);
      else
        k_fr_coarse<2><<<1, kFrCoarseThreads, 0, s>>>(u, ctx->fr_lev[l].s, L, p->fr_coarse_sweeps);
      return hipGetLastError();
    }
    for (int it = 0; it < p->fr_coarse_sweeps; ++it)
      if (hipError_t e = sweep(l, u, 0)) return e;
    return hipSuccess;
  }

  hipError_t cycle(int l, double *u, int kind) {
    if (l == ctx->fr_nlev - 1) return coarsest(l, u);
    const FrLevel L = level(l);
    const int64_t cells = (int64_t)L.n * L.n * L.n;
    // streaming levels ping-pong between u and alt (cur holds the iterate)
    const bool st = streams(l, u);
    double *cur = u, *oth = st ? ctx->fr_lev[l].alt : nullptr;
    for (int it = 0; it < p->fr_pre; ++it) {
      if (st) {
        if (hipError_t e = stream_sweep(l, cur, oth, 0)) return e;
        std::swap(cur, oth);
      } else if (hipError_t e = sweep(l, u, 0)) {
        return e;
      }
    }
    pm_fr_level &C = ctx->fr_lev[l + 1];
    const int64_t cc = (int64_t)C.n * C.n * C.n;
    if (C.n >= 128 && C.n % kRrCJ == 0) {
      // one streaming pass: residual and restriction (chunks of coarse planes sized for
      // about 2048 blocks); on smaller grids a block would walk its planes with too few
      // blocks beside it, and the two plain kernels are faster (45 against 10 us at 64^3)
      const int tiles = (C.n / kRrCJ) * (C.n / kRrCK);
      int cic = C.n;
      while (cic / 2 >= 8 && tiles * (C.n / cic) < 2048 && C.n % (cic / 2) == 0) cic /= 2;
      const dim3 grid(C.n / kRrCK, C.n / kRrCJ, C.n / cic);
      const double *sv = ctx->fr_lev[l].s;
      const float *src = l == 0 ? rho0 : nullptr;
      if (ne == 1 && src)
        k_fr_rr<1, true><<<grid, kRrT, 0, s>>>(cur, sv, src, mean0, cA, L, K, cic, C.u0, C.u, C.s);
      else if (ne == 1)
        k_fr_rr<1, false><<<grid, kRrT, 0, s>>>(cur, sv, src, mean0, cA, L, K, cic, C.u0, C.u, C.s);
      else if (src)
        k_fr_rr<2, true><<<grid, kRrT, 0, s>>>(cur, sv, src, mean0, cA, L, K, cic, C.u0, C.u, C.s);
      else
        k_fr_rr<2, false><<<grid, kRrT, 0, s>>>(cur, sv, src, mean0, cA, L, K, cic, C.u0, C.u, C.s);
    } else {
      double *d = ctx->fr_lev[l].d;
      k_fr_residual<<<blocks(cells), kFrThreads, 0, s>>>(cur, ctx->fr_lev[l].s, L, K, ne, d);
      k_fr_restrict<<<blocks(cc), kFrThreads, 0, s>>>(cur, d, L.n, C.u0, C.u, C.s);
    }
    k_fr_coarse_rhs<<<blocks(cc), kFrThreads, 0, s>>>(C.u0, level(l + 1), K, ne, C.s);
    if (hipError_t e = hipGetLastError()) return e;
    const int inner[2] = {kind == PM_CYCLE_W ? PM_CYCLE_W : (kind == PM_CYCLE_F ? PM_CYCLE_F
                                                                                : PM_CYCLE_V),
                          kind == PM_CYCLE_W ? PM_CYCLE_W : PM_CYCLE_V};
    const int visits = kind == PM_CYCLE_V ? 1 : 2;
    for (int v = 0; v < visits; ++v)
      if (hipError_t e = cycle(l + 1, C.u, inner[v])) return e;
    if (st) {
      prolong(l, cur, oth);
      std::swap(cur, oth);
    } else {
      prolong(l, u, u);
    }
    for (int it = 0; it < p->fr_post; ++it) {
      if (st) {
        if (hipError_t e = stream_sweep(l, cur, oth, 1)) return e;
        std::swap(cur, oth);
      } else if (hipError_t e = sweep(l, u, 1)) {
        return e;
      }
    }
    // (an odd pre + post count brings the iterate back to u)
    return hipGetLastError();
  }

  // ||s - N(u)||^2 and ||s||^2 on the finest grid into out[0..1] (device)
  hipError_t norms(double *u, double *out) {
    const FrLevel L = level(0);
    const int64_t cells = (int64_t)L.n * L.n * L.n;
    double *d = ctx->fr_lev[0].d;
    k_fr_residual<<<blocks(cells), kFrThreads, 0, s>>>(u, ctx->fr_lev[0].s, L, K, ne, d);
    const int nb = (int)std::min<int64_t>(RED_BLOCKS, blocks(cells));
    k_fr_norms<<<nb, kFrThreads, 0, s>>>(d, ctx->fr_lev[0].s, cells, ctx->red_partial);
    k_fr_norms_final<<<1, kFrThreads, 0, s>>>(ctx->red_partial, nb, out);
    return hipGetLastError();
  }
};

}  // namespace

// R_bar in units of H0^2 / c^2 and the scalaron background (Sect. 2.5)
static double fr_rbar(double om, double ol, double a) { return 3.0 * (om / (a * a * a) + 4.0 * ol); }

void pm_fr_constants(const pm_step_params *p, double a, double *fbar, double *K, double *cA) {
  const double rb = fr_rbar(p->omega_m, p->omega_l, a);
  const double f = std::pow(fr_rbar(p->omega_m, p->omega_l, 1.0) / rb, p->fr_n + 1) * p->fr_f0;
  *fbar = a * a * f;
  *K = a * a * a * a * rb / (3.0 * p->fr_c2);
  *cA = p->omega_m * a / p->fr_c2;
}

int pm_fr_setup(pm_ctx *ctx) {
  if (ctx->fr_nlev > 0) return PM_OK;
  int n = ctx->n, nl = 0;
  pm_fr_level lev[PM_MAX_LEVELS] = {};
  while (true) {
    if (nl >= PM_MAX_LEVELS) return pm_fail(ctx, PM_ERR_SHAPE, "too many FAS levels");
    lev[nl].n = n;
    ++nl;
    if (fr_is_coarsest(n)) break;
    n /= 2;
  }
  for (int l = 0; l < nl; ++l) {
    const size_t bytes = sizeof(double) * (size_t)lev[l].n * lev[l].n * lev[l].n;
    bool ok = hipMalloc(&lev[l].s, bytes) == hipSuccess && hipMalloc(&lev[l].d, bytes) == hipSuccess;
    if (ok && l > 0)
      ok = hipMalloc(&lev[l].u, bytes) == hipSuccess && hipMalloc(&lev[l].u0, bytes) == hipSuccess;
    if (ok && lev[l].n >= 256 && lev[l].n % kFsSK == 0)
      ok = hipMalloc(&lev[l].alt, bytes) == hipSuccess;
    if (!ok) {
      for (int m = 0; m <= l; ++m) {
        for (double *q : {lev[m].s, lev[m].d, lev[m].u, lev[m].u0, lev[m].alt})
          if (q) (void)hipFree(q);
      }
      (void)hipGetLastError();
      return pm_fail(ctx, PM_ERR_NOMEM, "FAS level allocation failed");
    }
  }
  for (int l = 0; l < nl; ++l) ctx->fr_lev[l] = lev[l];
  ctx->fr_nlev = nl;
  return PM_OK;
}

void pm_fr_free(pm_ctx *ctx) {
  for (int l = 0; l < ctx->fr_nlev; ++l)
    for (double *q : {ctx->fr_lev[l].s, ctx->fr_lev[l].d, ctx->fr_lev[l].u, ctx->fr_lev[l].u0,
                      ctx->fr_lev[l].alt})
      if (q) (void)hipFree(q);
  ctx->fr_nlev = 0;
  if (ctx->fr_u) (void)hipFree(ctx->fr_u);
  if (ctx->fr_phi) (void)hipFree(ctx->fr_phi);
  ctx->fr_u = nullptr;
  ctx->fr_phi = nullptr;
}

int pm_fr_solve(pm_ctx *ctx, const float *rho, double a, const pm_step_params *p, double *u,
                double *relres, hipStream_t s) {
  if (int st = pm_fr_setup(ctx)) return st;
  const int n = ctx->n;
  const int64_t cells = (int64_t)n * n * n;
  FrRun run{ctx, p, 0.0, 0.0, p->fr_n, s};
  double cA;
  pm_fr_constants(p, a, &run.fbar, &run.K, &cA);
  // the density's mean in FP64 (red_result[2])
  PM_HIP(ctx, launch_sum_moments(rho, cells, ctx->red_partial, ctx->red_result, nullptr, s));
  // a streaming finest grid (its passes read rho in pairs: 8-byte aligned) forms s from
  // the density where it needs it; s itself is written only for the other passes and for
  // the residual norms
  if (run.streams(0, u) && (reinterpret_cast<uintptr_t>(rho) & 7) == 0) {
    run.rho0 = rho;
    run.mean0 = ctx->red_result + 2;
    run.cA = cA;
  }
  if (!run.rho0 || relres) {
    k_fr_source<<<blocks(cells), kFrThreads, 0, s>>>(rho, ctx->red_result + 2, cells, cA, run.K,
                                                     ctx->fr_lev[0].s);
    PM_HIP(ctx, hipGetLastError());
  }
  if (relres) PM_HIP(ctx, run.norms(u, ctx->red_result));
  if (relres) PM_HIP(ctx, hipMemcpyAsync(ctx->host_result + 2, ctx->red_result, 2 * sizeof(double),
                                         hipMemcpyDeviceToHost, s));
  for (int c = 0; c < p->fr_cycles; ++c) PM_HIP(ctx, run.cycle(0, u, p->fr_cycle));
  if (relres) {
    PM_HIP(ctx, run.norms(u, ctx->red_result));
    PM_HIP(ctx, hipMemcpyAsync(ctx->host_result, ctx->red_result, 2 * sizeof(double),
                               hipMemcpyDeviceToHost, s));
    PM_HIP(ctx, hipStreamSynchronize(s));
    const double s2 = ctx->host_result[1];
    relres[0] = s2 > 0.0 ? std::sqrt(ctx->host_result[2] / s2) : 0.0;
    relres[1] = s2 > 0.0 ? std::sqrt(ctx->host_result[0] / s2) : 0.0;
  }
  return PM_OK;
}

hipError_t launch_fill_double(double *x, double v, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  k_fill_d<<<blocks(count), kFrThreads, 0, s>>>(x, v, count);
  return hipGetLastError();
}

int pm_fr_force_potential(pm_ctx *ctx, const float *rho, double a, const pm_step_params *p,
                          bool warm, const float *phin, hipStream_t s) {
  const int n = ctx->n;
  const int64_t cells = (int64_t)n * n * n;
  if (!ctx->fr_u) {
    if (hipMalloc(&ctx->fr_u, sizeof(double) * cells) != hipSuccess) {
      ctx->fr_u = nullptr;
      (void)hipGetLastError();
      return pm_fail(ctx, PM_ERR_NOMEM, "f(R) scalaron allocation failed");
    }
    ctx->fr_valid = false;
  }
  if (!ctx->fr_phi) {
    if (hipMalloc(&ctx->fr_phi, sizeof(float) * cells) != hipSuccess) {
      ctx->fr_phi = nullptr;
      (void)hipGetLastError();
      return pm_fail(ctx, PM_ERR_NOMEM, "f(R) potential allocation failed");
    }
  }
  if (!warm || !ctx->fr_valid) PM_HIP(ctx, launch_fill_double(ctx->fr_u, 1.0, cells, s));
  ctx->fr_valid = false;
  if (int st = pm_fr_solve(ctx, rho, a, p, ctx->fr_u, nullptr, s)) return st;
  ctx->fr_valid = true;
  double fbar, K, cA;
  pm_fr_constants(p, a, &fbar, &K, &cA);
  k_fr_phi<<<blocks(cells), kFrThreads, 0, s>>>(phin, ctx->fr_u, cells, 0.5 * p->fr_c2 * fbar,
                                                p->fr_n, ctx->fr_phi);
  PM_HIP(ctx, hipGetLastError());
  return PM_OK;
}
