// Initial conditions by Lagrangian perturbation theory and the power-spectrum estimator
// (paper Sect. 3.3 and App. A; the estimator of Sect. 4).
//
// pm_ic_lpt: the linear density at a = 1 from a white-noise grid and a P(k) table,
// DFT[delta] = sqrt(N) sqrt(P(k)) DFT[w] (unit box, N = n^3), with the k = 0 mode and
// the Nyquist planes zero; then, with every derivative taken in Fourier space,
//   Psi(1) = -grad phi(1),        phi(1) = lap^-1 delta
//   Psi(2) =  grad phi(2),        lap phi(2) = sum_{i<j} phi(1)_ii phi(1)_jj - phi(1)_ij^2
//   Psi(3a) = grad phi(3a),       lap phi(3a) = det phi(1)_ij
//   Psi(3b) = grad phi(3b),       lap phi(3b) = [tr phi(2)_ij tr phi(1)_ij
//                                                - phi(2)_ij phi(1)_ij] / 2
//   Psi(3c) = curl A(3c),         lap A(3c) = sum_i grad phi(2)_,i x grad phi(1)_,i
// and x = q + sum D^(k) Psi^(k), v = a^(1/2) sum k D^(k) Psi^(k) with the
// Einstein-de Sitter growth factors D = a, D2 = -3/7 D^2, D3a = -1/3 D^3,
// D3b = 10/21 D^3, D3c = -1/7 D^3. Products of fields are formed pointwise on a grid of
// m = n (dealias 0) or m = 2n (dealias 1: zero-padded spectra, free of aliasing for the
// quadratic and cubic terms) cells per side and truncated back to the band of the n grid.
//
// Every spectral step is one elementwise pass k_spec_op from one half spectrum to
// another (the two grids may differ: padding and truncation are index maps) followed
// by the inverse passes of fft.hip, or a forward transform of a real product field.
#include <cmath>
#include <vector>

#include "internal.h"

namespace {

constexpr int kT = 256;
constexpr double kTwoPi = 6.283185307179586;

inline unsigned blocks_for(int64_t count, int threads) {
  return (unsigned)((count + threads - 1) / threads);
}

// dst = scale * (i)^imag * k_ka * k_kb / k^2 (inv_k2) * sqrt(P(|k|)) (pk) * src
struct SpecOp {
  float scale;
  int ka, kb;      // axes of the k factors (-1: none)
  int inv_k2;      // divide by k^2 (the k = 0 mode becomes 0)
  int imag;        // multiply by i
  int pk;          // multiply by sqrt(P(|k|)) from the table
  int accumulate;  // dst += instead of dst =
};

// log-log interpolation of the table, constant beyond its ends
__device__ double table_sqrt_p(double k, const double *__restrict__ lk, const double *__restrict__ lp,
                               int nt) {
  const double x = log(k);
  if (x <= lk[0]) return exp(0.5 * lp[0]);
  if (x >= lk[nt - 1]) return exp(0.5 * lp[nt - 1]);
  int lo = 0, hi = nt - 1;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (lk[mid] <= x) lo = mid;
    else hi = mid;
  }
  const double t = (x - lk[lo]) / (lk[hi] - lk[lo]);
  return exp(0.5 * (lp[lo] + t * (lp[hi] - lp[lo])));
}

// One thread per mode of the destination half spectrum (gd cells per side, pitch Pd).
// A mode is kept when it lies inside the band of the n grid, |m_d| < n/2 on every axis
// (so the n grid's Nyquist planes are dropped); its source is the same wavevector on the
// source grid (gs cells per side, pitch Ps).
__global__ __launch_bounds__(kT) void k_spec_op(const float2 *__restrict__ src, int gs, int Ps,
                                                float2 *__restrict__ dst, int gd, int Pd, int nband,
                                                SpecOp op, const double *__restrict__ lk,
                                                const double *__restrict__ lp, int nt) {
  const int hz = gd / 2 + 1;
  const int64_t count = (int64_t)gd * gd * hz;
  const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (t >= count) return;
  const int iz = (int)(t % hz);
  const int iy = (int)((t / hz) % gd);
  const int ix = (int)(t / ((int64_t)hz * gd));
  const int mx = ix < gd / 2 ? ix : ix - gd;
  const int my = iy < gd / 2 ? iy : iy - gd;
  const int mz = iz;
  const int h = nband / 2;
  const bool keep = mx > -h && mx < h && my > -h && my < h && mz < h;
  float2 *out = dst + ((int64_t)ix * gd + iy) * Pd + iz;
  float2 r = make_float2(0.f, 0.f);
  if (keep) {
    const int sx = mx >= 0 ? mx : mx + gs, sy = my >= 0 ? my : my + gs;
    const float2 v = src[((int64_t)sx * gs + sy) * Ps + mz];
    const double k[3] = {kTwoPi * mx, kTwoPi * my, kTwoPi * mz};
    const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    double mult = (double)op.scale;
    if (op.ka >= 0) mult *= k[op.ka];
    if (op.kb >= 0) mult *= k[op.kb];
    if (op.inv_k2) mult = k2 > 0.0 ? mult / k2 : 0.0;
    if (op.pk) mult = k2 > 0.0 ? mult * table_sqrt_p(sqrt(k2), lk, lp, nt) : 0.0;
    const float fm = (float)mult;
    r = op.imag ? make_float2(-fm * v.y, fm * v.x) : make_float2(fm * v.x, fm * v.y);
  }
  if (op.accumulate) {
    const float2 o = *out;
    *out = make_float2(o.x + r.x, o.y + r.y);
  } else {
    *out = r;
  }
}

// The six distinct second derivatives of a potential, a[0..5] = xx, yy, zz, xy, xz, yz.
struct Hess {
  const float *a[6];
};

enum { kSrcS2 = 0, kSrcDet = 1, kSrcS3b = 2, kSrcRx = 3, kSrcRy = 4, kSrcRz = 5 };

// The pointwise sources of the higher orders (paper Sect. 3.3, explicit forms), from the
// second derivatives of phi(1) (A) and of phi(2) (B).
__global__ __launch_bounds__(kT) void k_lpt_source(Hess A, Hess B, int which, int64_t count,
                                                   float *__restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p >= count) return;
  const float axx = A.a[0][p], ayy = A.a[1][p], azz = A.a[2][p];
  const float axy = A.a[3][p], axz = A.a[4][p], ayz = A.a[5][p];
  float v = 0.0f;
  if (which == kSrcS2) {
    v = axx * (ayy + azz) + ayy * azz - axy * axy - axz * axz - ayz * ayz;
  } else if (which == kSrcDet) {
    v = axx * ayy * azz + 2.0f * axy * axz * ayz - ayz * ayz * axx - axz * axz * ayy -
        axy * axy * azz;
  } else {
    const float bxx = B.a[0][p], byy = B.a[1][p], bzz = B.a[2][p];
    const float bxy = B.a[3][p], bxz = B.a[4][p], byz = B.a[5][p];
    if (which == kSrcS3b)
      v = 0.5f * axx * (byy + bzz) + 0.5f * ayy * (bxx + bzz) + 0.5f * azz * (bxx + byy) -
          axy * bxy - axz * bxz - ayz * byz;
    else if (which == kSrcRx)
      v = bxy * axz - bxz * axy + ayz * (byy - bzz) - byz * (ayy - azz);
    else if (which == kSrcRy)
      v = byz * axy - bxy * ayz + axz * (bzz - bxx) - bxz * (azz - axx);
    else
      v = bxz * ayz - byz * axz + axy * (bxx - byy) - bxy * (axx - ayy);
  }
  out[p] = v;
}

// disp[p][comp] += cd f[p]; vel[p][comp] += cv f[p]
__global__ __launch_bounds__(kT) void k_lpt_add(const float *__restrict__ f, int comp, float cd,
                                                float cv, int64_t count, float *__restrict__ disp,
                                                float *__restrict__ vel) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p >= count) return;
  const float v = f[p];
  disp[3 * p + comp] = fmaf(cd, v, disp[3 * p + comp]);
  vel[3 * p + comp] = fmaf(cv, v, vel[3 * p + comp]);
}

// Particle p = (i n + j) n + k starts at the cell centre q = ((i, j, k) + 1/2) / n;
// pos holds its displacement on entry and the position on exit: box units wrapped into
// [0, 1) (cell == NULL), or the in-cell offset with the cell index carried.
__global__ __launch_bounds__(kT) void k_lpt_finish(float *__restrict__ pos,
                                                   int32_t *__restrict__ cell, int n,
                                                   int64_t count) {
  const int64_t p = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (p >= count) return;
  const int ijk[3] = {(int)(p / ((int64_t)n * n)), (int)((p / n) % n), (int)(p % n)};
  int c[3];
  const float fn = (float)n;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float dp = pos[3 * p + d];
    if (!cell) {
      float x = ((float)ijk[d] + 0.5f) / fn + dp;
      x -= floorf(x);
      pos[3 * p + d] = x >= 1.0f ? 0.0f : x;
    } else {
      const float s = fmaf(dp, fn, 0.5f);
      float fl = floorf(s);
      float o = s - fl;
      if (o >= 1.0f) {
        o = 0.0f;
        fl += 1.0f;
      }
      int ci = (ijk[d] + (int)fl) % n;
      c[d] = ci < 0 ? ci + n : ci;
      pos[3 * p + d] = o;
    }
  }
  if (cell) cell[p] = (c[0] * n + c[1]) * n + c[2];
}

// P(k) shells: per mode |F|^2 / (N mean)^2 / W^2 with W = prod_d sinc(pi m_d / n)^deconv,
// weight 2 for 0 < kz < n/2 (the mode and its conjugate), shell b = rint(|m|) in
// 1 .. nbins; per-block sums in LDS, then one FP64 atomic per shell and block.
constexpr int kPkMaxBins = 1024;

__global__ __launch_bounds__(kT) void k_pk_bins(const float2 *__restrict__ spec, int n, int P,
                                                int deconv, const double *__restrict__ mean,
                                                int nbins, double *__restrict__ acc) {
  __shared__ double s_p[kPkMaxBins], s_k[kPkMaxBins], s_c[kPkMaxBins];
  for (int b = threadIdx.x; b < nbins; b += kT) s_p[b] = s_k[b] = s_c[b] = 0.0;
  __syncthreads();
  const int hz = n / 2 + 1;
  const int64_t count = (int64_t)n * n * hz;
  const double norm = 1.0 / ((double)n * n * n * mean[0]);
  for (int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x; t < count; t += (int64_t)gridDim.x * kT) {
    const int iz = (int)(t % hz);
    const int iy = (int)((t / hz) % n);
    const int ix = (int)(t / ((int64_t)hz * n));
    const int mx = ix < n / 2 ? ix : ix - n;
    const int my = iy < n / 2 ? iy : iy - n;
    const double mm = sqrt((double)mx * mx + (double)my * my + (double)iz * iz);
    const int b = (int)rint(mm);
    if (b < 1 || b > nbins) continue;
    const float2 v = spec[((int64_t)ix * n + iy) * P + iz];
    double w = 1.0;
    const int md[3] = {mx, my, iz};
    for (int d = 0; d < 3; ++d) {
      if (md[d] != 0) {
        const double x = M_PI * md[d] / n;
        w *= pow(sin(x) / x, (double)deconv);
      }
    }
    const double re = v.x * norm, im = v.y * norm;
    const double pw = (re * re + im * im) / (w * w);
    const double wt = (iz == 0 || 2 * iz == n) ? 1.0 : 2.0;
    atomicAdd(&s_p[b - 1], wt * pw);
    atomicAdd(&s_k[b - 1], wt * kTwoPi * mm);
    atomicAdd(&s_c[b - 1], wt);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbins; b += kT) {
    if (s_c[b] != 0.0) {
      atomicAdd(&acc[3 * b], s_p[b]);
      atomicAdd(&acc[3 * b + 1], s_k[b]);
      atomicAdd(&acc[3 * b + 2], s_c[b]);
    }
  }
}

// Device scratch of one pm_ic_lpt call (allocated for the call and released after it).
struct IcScratch {
  std::vector<void *> owned;
  hipError_t alloc(void **p, size_t bytes) {
    const hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess) owned.push_back(*p);
    return e;
  }
  ~IcScratch() {
    // queued work may still read the buffers (an early error return): wait for it
    if (!owned.empty()) (void)hipDeviceSynchronize();
    for (void *p : owned) (void)hipFree(p);
  }
};

}  // namespace

extern "C" {

int pm_ic_lpt(pm_ctx *ctx, const float *noise, int ntab, const double *k_tab, const double *p_tab,
              int order, int dealias, double a0, float *pos, int32_t *cell, float *vel,
              pm_stream stream) {
  if (!ctx) return PM_ERR_ARG;
  if (!noise || !pos || !vel || !k_tab || !p_tab) return pm_fail(ctx, PM_ERR_ARG, "null pointer");
  if (order < 1 || order > 3) return pm_fail(ctx, PM_ERR_ARG, "order must be 1, 2 or 3");
  if (dealias != 0 && dealias != 1) return pm_fail(ctx, PM_ERR_ARG, "dealias must be 0 or 1");
  if (!(a0 > 0.0) || !std::isfinite(a0)) return pm_fail(ctx, PM_ERR_ARG, "scale factor must be > 0");
  if (ntab < 2 || ntab > 65536) return pm_fail(ctx, PM_ERR_ARG, "the P(k) table needs 2 .. 65536 points");
  std::vector<double> lt(2 * (size_t)ntab);
  for (int i = 0; i < ntab; ++i) {
    if (!(k_tab[i] > 0.0) || !(p_tab[i] > 0.0) || !std::isfinite(k_tab[i]) ||
        !std::isfinite(p_tab[i]) || (i > 0 && !(k_tab[i] > k_tab[i - 1])))
      return pm_fail(ctx, PM_ERR_ARG, "P(k) table: k ascending, k and P positive and finite");
    lt[i] = std::log(k_tab[i]);
    lt[ntab + i] = std::log(p_tab[i]);
  }
  const int n = ctx->n;
  const int m = dealias ? 2 * n : n;
  if ((n & (n - 1)) != 0 || m > 1024)
    return pm_fail(ctx, PM_ERR_SHAPE, "initial conditions need a power-of-two grid (2n <= 1024 "
                                      "with dealiasing)");
  const hipStream_t s = (hipStream_t)stream;
  const int64_t N = (int64_t)n * n * n, M = (int64_t)m * m * m;
  IcScratch sc;
  double *d_tab = nullptr;
  float2 *spec_n = nullptr, *spec_d = nullptr, *spec_m = nullptr;
  float2 *src_sp[6] = {};
  float *fn_real = nullptr, *tmp_m = nullptr;
  float *h1[6] = {}, *h2[6] = {};
  float2 *tw_n = nullptr, *tw_m = nullptr;
  float *tab_n = nullptr, *tab_m = nullptr;
  const size_t en = fft_spec_elems(n), em = fft_spec_elems(m);
  const int nsrc = order == 1 ? 0 : (order == 2 ? 1 : 6);
  bool ok = sc.alloc((void **)&d_tab, sizeof(double) * 2 * ntab) == hipSuccess &&
            sc.alloc((void **)&spec_n, sizeof(float2) * en) == hipSuccess &&
            sc.alloc((void **)&spec_d, sizeof(float2) * en) == hipSuccess &&
            sc.alloc((void **)&fn_real, sizeof(float) * N) == hipSuccess &&
            sc.alloc((void **)&tw_n, sizeof(float2) * n) == hipSuccess &&
            sc.alloc((void **)&tab_n, sizeof(float) * 3 * n) == hipSuccess;
  if (ok && order >= 2) {
    ok = sc.alloc((void **)&spec_m, sizeof(float2) * em) == hipSuccess &&
         sc.alloc((void **)&tmp_m, sizeof(float) * M) == hipSuccess &&
         sc.alloc((void **)&tw_m, sizeof(float2) * m) == hipSuccess &&
         sc.alloc((void **)&tab_m, sizeof(float) * 3 * m) == hipSuccess;
    for (int i = 0; ok && i < 6; ++i) ok = sc.alloc((void **)&h1[i], sizeof(float) * M) == hipSuccess;
    for (int i = 0; ok && i < nsrc; ++i)
      ok = sc.alloc((void **)&src_sp[i], sizeof(float2) * en) == hipSuccess;
    for (int i = 0; ok && order == 3 && i < 6; ++i)
      ok = sc.alloc((void **)&h2[i], sizeof(float) * M) == hipSuccess;
  }
  if (!ok) return pm_fail(ctx, PM_ERR_NOMEM, "initial-condition scratch allocation failed");
  PM_HIP(ctx, hipMemcpyAsync(d_tab, lt.data(), sizeof(double) * 2 * ntab, hipMemcpyHostToDevice, s));
  const double *lk = d_tab, *lp = d_tab + ntab;
  FftBufs bn{spec_n, nullptr, tw_n, tab_n}, bm{spec_m, nullptr, tw_m, tab_m};
  PM_HIP(ctx, fft_tables(bn, n, 0, 0, s));
  if (order >= 2) PM_HIP(ctx, fft_tables(bm, m, 0, 0, s));
  const int Pn = fft_pitch(n), Pm = fft_pitch(m);
  const unsigned gn = blocks_for((int64_t)n * n * (n / 2 + 1), kT);
  const unsigned gm = blocks_for((int64_t)m * m * (m / 2 + 1), kT);
  auto op_n = [&](const float2 *src, int gs, int Ps, SpecOp op) {  // into spec_n
    k_spec_op<<<gn, kT, 0, s>>>(src, gs, Ps, spec_n, n, Pn, n, op, lk, lp, ntab);
  };
  auto op_m = [&](const float2 *src, int gs, int Ps, SpecOp op) {  // into spec_m
    k_spec_op<<<gm, kT, 0, s>>>(src, gs, Ps, spec_m, m, Pm, n, op, lk, lp, ntab);
  };
  const float invN = (float)(1.0 / (double)N);
  const float trunc = (float)((double)N / (double)M);  // DFT on the m grid -> n-grid units
  // linear density at a = 1: DFT[delta] = sqrt(N) sqrt(P) DFT[w]
  PM_HIP(ctx, fft_forward(bn, n, noise, nullptr, s));
  k_spec_op<<<gn, kT, 0, s>>>(spec_n, n, Pn, spec_d, n, Pn, n,
                              SpecOp{(float)std::sqrt((double)N), -1, -1, 0, 0, 1, 0}, lk, lp, ntab);
  PM_HIP(ctx, hipGetLastError());
  PM_HIP(ctx, launch_fill(pos, 0.0f, 3 * N, s));
  PM_HIP(ctx, launch_fill(vel, 0.0f, 3 * N, s));
  const double ra = std::sqrt(a0);
  // add sum_d grad-like fields: spectrum op into spec_n, inverse, then disp += cd f, vel += cv f
  auto add_field = [&](int comp, double cd, double cv) -> hipError_t {
    hipError_t e = fft_inverse(bn, n, fn_real, 1, 0, s);
    if (e != hipSuccess) return e;
    k_lpt_add<<<blocks_for(N, kT), kT, 0, s>>>(fn_real, comp, (float)cd, (float)cv, N, pos, vel);
    return hipGetLastError();
  };
  // first order: Psi(1)_d = IDFT[i k_d delta / k^2] / N
  for (int d = 0; d < 3; ++d) {
    op_n(spec_d, n, Pn, SpecOp{invN, d, -1, 1, 1, 0, 0});
    PM_HIP(ctx, add_field(d, a0, ra * a0));
  }
  if (order >= 2) {
    static const int hi[6] = {0, 1, 2, 0, 0, 1}, hj[6] = {0, 1, 2, 1, 2, 2};
    // phi(1)_ij = IDFT[k_i k_j delta / k^2] / N on the product grid
    for (int c = 0; c < 6; ++c) {
      op_m(spec_d, n, Pn, SpecOp{invN, hi[c], hj[c], 1, 0, 0, 0});
      PM_HIP(ctx, fft_inverse(bm, m, h1[c], 1, 0, s));
    }
    Hess A{{h1[0], h1[1], h1[2], h1[3], h1[4], h1[5]}};
    Hess B{{h2[0], h2[1], h2[2], h2[3], h2[4], h2[5]}};
    // a source on the product grid -> its spectrum truncated to the n band (n-grid units)
    auto source = [&](int which, float2 *dst) -> hipError_t {
      k_lpt_source<<<blocks_for(M, kT), kT, 0, s>>>(A, B, which, M, tmp_m);
      hipError_t e = fft_forward(bm, m, tmp_m, nullptr, s);
      if (e != hipSuccess) return e;
      k_spec_op<<<gn, kT, 0, s>>>(spec_m, m, Pm, dst, n, Pn, n, SpecOp{trunc, -1, -1, 0, 0, 0, 0},
                                  lk, lp, ntab);
      return hipGetLastError();
    };
    PM_HIP(ctx, source(kSrcS2, src_sp[0]));
    // phi(2) = -lap^-1 S2: Psi(2)_d = IDFT[i k_d phi2] / N = IDFT[-i k_d S2 / k^2] / N
    const double d2 = -3.0 / 7.0 * a0 * a0;
    for (int d = 0; d < 3; ++d) {
      op_n(src_sp[0], n, Pn, SpecOp{-invN, d, -1, 1, 1, 0, 0});
      PM_HIP(ctx, add_field(d, d2, ra * 2.0 * d2));
    }
    if (order == 3) {
      // phi(2)_ij = IDFT[-k_i k_j phi2] = IDFT[k_i k_j S2 / k^2] / N on the product grid
      for (int c = 0; c < 6; ++c) {
        op_m(src_sp[0], n, Pn, SpecOp{invN, hi[c], hj[c], 1, 0, 0, 0});
        PM_HIP(ctx, fft_inverse(bm, m, h2[c], 1, 0, s));
      }
      PM_HIP(ctx, source(kSrcDet, src_sp[1]));
      PM_HIP(ctx, source(kSrcS3b, src_sp[2]));
      PM_HIP(ctx, source(kSrcRx, src_sp[3]));
      PM_HIP(ctx, source(kSrcRy, src_sp[4]));
      PM_HIP(ctx, source(kSrcRz, src_sp[5]));
      const double d3a = -1.0 / 3.0 * a0 * a0 * a0, d3b = 10.0 / 21.0 * a0 * a0 * a0;
      const double d3c = -1.0 / 7.0 * a0 * a0 * a0;
      // Psi(3a), Psi(3b) = grad lap^-1 S: IDFT[-i k_d S / k^2] / N
      for (int d = 0; d < 3; ++d) {
        op_n(src_sp[1], n, Pn, SpecOp{-invN, d, -1, 1, 1, 0, 0});
        PM_HIP(ctx, add_field(d, d3a, ra * 3.0 * d3a));
        op_n(src_sp[2], n, Pn, SpecOp{-invN, d, -1, 1, 1, 0, 0});
        PM_HIP(ctx, add_field(d, d3b, ra * 3.0 * d3b));
      }
      // Psi(3c) = curl A, A = -lap^-1 R: (curl A)_d = i (k_e A_f - k_f A_e) for the cyclic
      // (d, e, f), i.e. IDFT[-i (k_e R_f - k_f R_e) / k^2] / N
      for (int d = 0; d < 3; ++d) {
        const int e = (d + 1) % 3, f = (d + 2) % 3;
        op_n(src_sp[3 + f], n, Pn, SpecOp{-invN, e, -1, 1, 1, 0, 0});
        op_n(src_sp[3 + e], n, Pn, SpecOp{invN, f, -1, 1, 1, 0, 1});
        PM_HIP(ctx, add_field(d, d3c, ra * 3.0 * d3c));
      }
    }
  }
  k_lpt_finish<<<blocks_for(N, kT), kT, 0, s>>>(pos, cell, n, N);
  PM_HIP(ctx, hipGetLastError());
  // the scratch is released when the call returns: wait for the work that reads it
  PM_HIP(ctx, hipStreamSynchronize(s));
  return PM_OK;
}

int pm_power_spectrum(pm_ctx *ctx, const float *rho, int deconv, int nbins, double *pk,
                      double *kmean, int64_t *nmodes, pm_stream stream) {
  if (!ctx) return PM_ERR_ARG;
  if (!rho || !pk) return pm_fail(ctx, PM_ERR_ARG, "null pointer");
  if (deconv < 0 || deconv > 3) return pm_fail(ctx, PM_ERR_ARG, "deconv must be 0 .. 3");
  if (nbins < 1 || nbins > kPkMaxBins) return pm_fail(ctx, PM_ERR_ARG, "nbins must be 1 .. 1024");
  const int n = ctx->n;
  if ((n & (n - 1)) != 0)
    return pm_fail(ctx, PM_ERR_SHAPE, "the power spectrum needs a power-of-two grid");
  const hipStream_t s = (hipStream_t)stream;
  const int64_t N = (int64_t)n * n * n;
  if (!ctx->spec) {
    if (hipMalloc(&ctx->spec, sizeof(float2) * fft_spec_elems(n)) != hipSuccess ||
        hipMalloc(&ctx->twiddle, sizeof(float2) * n) != hipSuccess ||
        hipMalloc(&ctx->fft_tab, sizeof(float) * 3 * n) != hipSuccess)
      return pm_fail(ctx, PM_ERR_NOMEM, "FFT scratch allocation failed");
  }
  // FP64 mean in red_result[2], FP32 mean (subtracted before the transform) in mean_f[2]
  PM_HIP(ctx, launch_sum_moments(rho, N, ctx->red_partial, ctx->red_result, ctx->mean_f + 2, s));
  FftBufs b{(float2 *)ctx->spec, nullptr, ctx->twiddle, ctx->fft_tab};
  PM_HIP(ctx, fft_tables(b, n, 0, 0, s));
  PM_HIP(ctx, fft_forward(b, n, rho, ctx->mean_f + 2, s));
  // shell sums in the partial buffer (3 doubles per shell, within its 3 * 65536 doubles)
  double *acc = ctx->red_partial;
  PM_HIP(ctx, hipMemsetAsync(acc, 0, sizeof(double) * 3 * nbins, s));
  const int64_t modes = (int64_t)n * n * (n / 2 + 1);
  const unsigned grid = (unsigned)std::min<int64_t>(blocks_for(modes, kT), 2048);
  k_pk_bins<<<grid, kT, 0, s>>>(b.spec, n, fft_pitch(n), deconv, ctx->red_result + 2, nbins, acc);
  PM_HIP(ctx, hipGetLastError());
  std::vector<double> h(3 * (size_t)nbins);
  PM_HIP(ctx, hipMemcpyAsync(h.data(), acc, sizeof(double) * 3 * nbins, hipMemcpyDeviceToHost, s));
  PM_HIP(ctx, hipStreamSynchronize(s));
  for (int b2 = 0; b2 < nbins; ++b2) {
    const double c = h[3 * b2 + 2];
    pk[b2] = c > 0.0 ? h[3 * b2] / c : 0.0;
    if (kmean) kmean[b2] = c > 0.0 ? h[3 * b2 + 1] / c : 0.0;
    if (nmodes) nmodes[b2] = (int64_t)std::llround(c);
  }
  return PM_OK;
}

}  // extern "C"
