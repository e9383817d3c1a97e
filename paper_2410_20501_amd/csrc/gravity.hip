// Background expansion, parametrised gravity and QUMOND (paper Sects. 2.3, 2.4, 3.1,
// 3.10).
//
// Host: the supercomoving time step and the linear growth factor of a background of
// matter, curvature and a cosmological constant, and the force coefficient
// (3/2) Omega_m a mu(a). Device: the QUMOND source, the divergence of
// nu(|grad phi_N| / g0) grad phi_N on the cell faces (Eq. QUMOND_Poisson_MOND_discrete).
#include <cmath>

#include "internal.h"

namespace {

// 5-point Gauss-Legendre rule on [-1, 1]
constexpr double kGLx[5] = {-0.9061798459386640, -0.5384693101056831, 0.0, 0.5384693101056831,
                            0.9061798459386640};
constexpr double kGLw[5] = {0.2369268850561891, 0.4786286704993665, 0.5688888888888889,
                            0.4786286704993665, 0.2369268850561891};
constexpr int kPanels = 256;

template <class F>
double gauss_legendre(F f, double lo, double hi) {
  const double w = (hi - lo) / kPanels;
  double sum = 0.0;
  for (int p = 0; p < kPanels; ++p) {
    const double c = lo + (p + 0.5) * w;
    for (int q = 0; q < 5; ++q) sum += kGLw[q] * f(c + 0.5 * w * kGLx[q]);
  }
  return 0.5 * w * sum;
}

// E(a)^2 = H(a)^2 / H0^2
double e2(double om, double ol, double a) {
  return om / (a * a * a) + (1.0 - om - ol) / (a * a) + ol;
}

// nu(y) of the QUMOND families (Sect. 2.3)
__device__ __forceinline__ float nu_of(float y, int family, float par) {
  switch (family) {
    case PM_NU_N:
      return powf(0.5f + 0.5f * sqrtf(1.0f + 4.0f / powf(y, par)), 1.0f / par);
    case PM_NU_BETA:
      return rsqrtf(1.0f - expf(-y)) + par * expf(-y);
    case PM_NU_GAMMA: {
      const float e = expf(-powf(y, 0.5f * par));
      return powf(1.0f - e, -1.0f / par) + (1.0f - 1.0f / par) * e;
    }
    case PM_NU_DELTA:
      return powf(1.0f - expf(-powf(y, 0.5f * par)), -1.0f / par);
    default:
      return 0.5f + 0.5f * sqrtf(1.0f + 4.0f / y);
  }
}

// nu g_n at the face between cell c and c + e_axis: the normal component g_n is the
// two-point difference across the face; each transverse component averages the
// centred differences of the two cells (Sect. 3.10). nu g_n -> 0 where the gradient
// vanishes (nu grows at most as y^-1/2).
__device__ float face_flux(const float *__restrict__ phi, int n, int i, int j, int k, int axis,
                           float inv_h, float inv_g0, int family, float par) {
  auto at = [&](int a, int b, int c) -> float {
    a = a < 0 ? a + n : (a >= n ? a - n : a);
    b = b < 0 ? b + n : (b >= n ? b - n : b);
    c = c < 0 ? c + n : (c >= n ? c - n : c);
    return phi[((size_t)a * n + b) * n + c];
  };
  const int e[3] = {axis == 0, axis == 1, axis == 2};
  const float p0 = at(i, j, k), p1 = at(i + e[0], j + e[1], k + e[2]);
  const float gn = (p1 - p0) * inv_h;
  float g2 = gn * gn;
  for (int t = 0; t < 3; ++t) {
    if (t == axis) continue;
    const int f[3] = {t == 0, t == 1, t == 2};
    const float du = at(i + e[0] + f[0], j + e[1] + f[1], k + e[2] + f[2]) -
                     at(i + e[0] - f[0], j + e[1] - f[1], k + e[2] - f[2]);
    const float dc = at(i + f[0], j + f[1], k + f[2]) - at(i - f[0], j - f[1], k - f[2]);
    const float gt = (du + dc) * (0.25f * inv_h);
    g2 += gt * gt;
  }
  if (!(g2 > 0.0f)) return 0.0f;
  return nu_of(sqrtf(g2) * inv_g0, family, par) * gn;
}

__global__ __launch_bounds__(256) void k_qumond_source(const float *__restrict__ phin, int n,
                                                       float inv_h, float inv_g0, int family,
                                                       float par, float *__restrict__ out) {
  const int64_t c = (int64_t)xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  const int64_t count = (int64_t)n * n * n;
  if (c >= count) return;
  const int i = (int)(c / ((int64_t)n * n)), j = (int)((c / n) % n), k = (int)(c % n);
  float s = 0.0f;
  for (int axis = 0; axis < 3; ++axis) {
    const float fb = face_flux(phin, n, i, j, k, axis, inv_h, inv_g0, family, par);
    const float fa = face_flux(phin, n, i - (axis == 0), j - (axis == 1), k - (axis == 2), axis,
                               inv_h, inv_g0, family, par);
    s += fb - fa;
  }
  out[c] = s * inv_h;
}

}  // namespace

double pm_bg_tau(double om, double ol, double a0, double a1) {
  if (ol == 0.0 && om == 1.0) return 2.0 * (1.0 / std::sqrt(a0) - 1.0 / std::sqrt(a1));
  // with s = a^-1/2 (a = s^-2): dt~ = 2 ds / sqrt(Omega_m + Omega_k a + Omega_L a^3),
  // a smooth integrand on [a1^-1/2, a0^-1/2]
  auto f = [&](double s) {
    const double a = 1.0 / (s * s);
    return 2.0 / std::sqrt(om + (1.0 - om - ol) * a + ol * a * a * a);
  };
  return gauss_legendre(f, 1.0 / std::sqrt(a1), 1.0 / std::sqrt(a0));
}

double pm_bg_growth(double om, double ol, double a) {
  if (ol == 0.0 && om == 1.0) return a;
  // growing mode of matter with curvature and a cosmological constant:
  // D(a) proportional to E(a) * integral_0^a da' / (a' E(a'))^3; with a' = t^2 the
  // integrand 2 t / (t^2 E(t^2))^3 is smooth at 0
  auto f = [&](double t) {
    const double ap = t * t;
    const double ae = ap * std::sqrt(e2(om, ol, ap));
    return 2.0 * t / (ae * ae * ae);
  };
  return std::sqrt(e2(om, ol, a)) * gauss_legendre(f, 0.0, std::sqrt(a));
}

double pm_bg_coef(const pm_step_params *p, double a) {
  double mu = 1.0;
  if (p->gravity == PM_GRAVITY_MU) mu = 1.0 + p->mu0 / e2(p->omega_m, p->omega_l, a);
  return 1.5 * a * p->omega_m * mu;
}

double pm_bg_warm_scale(const pm_step_params *p, double a0, double a1) {
  // the supercomoving potential grows as a D(a) in the linear regime
  return (a1 * pm_bg_growth(p->omega_m, p->omega_l, a1)) /
         (a0 * pm_bg_growth(p->omega_m, p->omega_l, a0));
}

hipError_t launch_qumond_source(const float *phin, int n, float g0, int family, float param,
                                float *out, hipStream_t s) {
  const int64_t count = (int64_t)n * n * n;
  const unsigned nb = (unsigned)((count + 255) / 256);
  k_qumond_source<<<nb, 256, 0, s>>>(phin, n, (float)n, 1.0f / g0, family, param, out);
  return hipGetLastError();
}

extern "C" double pm_supercomoving_time(double omega_m, double omega_l, double a0, double a1) {
  if (!(a0 > 0.0) || !(a1 > 0.0) || !std::isfinite(a0) || !std::isfinite(a1) ||
      !std::isfinite(omega_m) || !std::isfinite(omega_l) || !(omega_m > 0.0))
    return std::nan("");
  // the expansion rate must stay real on the interval (no recollapse before a1)
  const double lo = std::min(a0, a1), hi = std::max(a0, a1);
  for (int q = 0; q <= 64; ++q) {
    const double a = lo + (hi - lo) * q / 64.0;
    if (!(omega_m + (1.0 - omega_m - omega_l) * a + omega_l * a * a * a > 0.0)) return std::nan("");
  }
  return pm_bg_tau(omega_m, omega_l, a0, a1);
}
