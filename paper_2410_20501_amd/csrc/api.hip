// C ABI entry points: argument validation, context and scratch management,
// and the orchestration of the particle-mesh stages on the caller's stream.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "internal.h"

void pm_kt_begin(pm_ctx *ctx, int kernel, hipStream_t s) {
  if (ctx->kt_kernel != kernel || kernel == PM_KERNEL_NONE) return;
  if (ctx->kt_used >= ctx->kt_cap) {
    ++ctx->kt_dropped;
    return;
  }
  (void)hipEventRecord(ctx->kt_ev[2 * ctx->kt_used], s);
}

void pm_kt_end(pm_ctx *ctx, int kernel, hipStream_t s, double bytes) {
  if (ctx->kt_kernel != kernel || kernel == PM_KERNEL_NONE || ctx->kt_used >= ctx->kt_cap) return;
  (void)hipEventRecord(ctx->kt_ev[2 * ctx->kt_used + 1], s);
  ctx->kt_used++;
  ctx->kt_bytes += bytes;
}

int pm_fail(pm_ctx *ctx, int code, const std::string &msg) {
  if (ctx) ctx->err = msg;
  return code;
}

int pm_hip_check(pm_ctx *ctx, hipError_t e, const char *what) {
  if (e == hipSuccess) return PM_OK;
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return pm_fail(ctx, e == hipErrorOutOfMemory ? PM_ERR_NOMEM : PM_ERR_HIP, m);
}

namespace {

bool valid_mas(int m) { return m == PM_NGP || m == PM_CIC || m == PM_TSC; }
// reverse mode needs the window's position derivative: CIC or TSC
bool valid_mas_vjp(int m) { return m == PM_CIC || m == PM_TSC; }
bool is_fft(int solver) {
  return solver == PM_SOLVER_FFT || solver == PM_SOLVER_FFT_7PT || solver == PM_SOLVER_FULL_FFT;
}
bool valid_poskind(int k) { return k == PM_POS_BOX || k == PM_POS_CELLOFF; }

int check_particles(pm_ctx *ctx, const void *pos, const int32_t *cell, int64_t np, int poskind) {
  if (np < 0) return pm_fail(ctx, PM_ERR_ARG, "negative particle count");
  if (!valid_poskind(poskind)) return pm_fail(ctx, PM_ERR_ARG, "bad poskind");
  if (np > 0 && !pos) return pm_fail(ctx, PM_ERR_ARG, "null pos");
  if (np > 0 && poskind == PM_POS_CELLOFF && !cell)
    return pm_fail(ctx, PM_ERR_ARG, "null cell array with PM_POS_CELLOFF");
  return PM_OK;
}

// with PM_CREATE_CHECK_FINITE: PM_ERR_NONFINITE if a position (or velocity) is not
// finite, found before any other kernel reads them (one pass and a host sync)
int check_finite(pm_ctx *ctx, const float *pos, const float *vel, int64_t np, hipStream_t s) {
  if (!(ctx->flags & PM_CREATE_CHECK_FINITE) || np == 0) return PM_OK;
  auto *cnt = reinterpret_cast<unsigned long long *>(ctx->red_result + 3);
  PM_HIP(ctx, hipMemsetAsync(cnt, 0, sizeof(unsigned long long), s));
  PM_HIP(ctx, launch_count_nonfinite(pos, 3 * np, cnt, s));
  if (vel) PM_HIP(ctx, launch_count_nonfinite(vel, 3 * np, cnt, s));
  PM_HIP(ctx, hipMemcpyAsync(ctx->host_result + 3, cnt, sizeof(unsigned long long),
                             hipMemcpyDeviceToHost, s));
  PM_HIP(ctx, hipStreamSynchronize(s));
  unsigned long long found;
  std::memcpy(&found, ctx->host_result + 3, sizeof(found));
  if (found) return pm_fail(ctx, PM_ERR_NONFINITE, "non-finite particle positions or velocities");
  return PM_OK;
}

int check_mg(pm_ctx *ctx, const pm_mg_params *p) {
  if (!p) return pm_fail(ctx, PM_ERR_ARG, "null multigrid params");
  if (p->pre < 0 || p->post < 0 || p->pre > 16 || p->post > 16)
    return pm_fail(ctx, PM_ERR_ARG, "sweep counts must be in [0, 16]");
  if (!(p->omega > 0.0f && p->omega < 2.0f)) return pm_fail(ctx, PM_ERR_ARG, "omega must be in (0, 2)");
  if (p->fixed_cycles < 0 || p->fixed_cycles > 1000)
    return pm_fail(ctx, PM_ERR_ARG, "fixed_cycles must be in [0, 1000]");
  if (p->fixed_cycles == 0 && (p->max_cycles < 1 || p->max_cycles > 63))
    return pm_fail(ctx, PM_ERR_ARG, "max_cycles must be in [1, 63]");
  if (p->fixed_cycles == 0 && !(p->tol >= 0.0f)) return pm_fail(ctx, PM_ERR_ARG, "bad tol");
  if (!(p->alpha >= 0.0f) || !std::isfinite(p->alpha))
    return pm_fail(ctx, PM_ERR_ARG, "alpha must be finite and >= 0");
  if (p->cycle != PM_CYCLE_V && p->cycle != PM_CYCLE_W && p->cycle != PM_CYCLE_F)
    return pm_fail(ctx, PM_ERR_ARG, "bad cycle");
  if (p->restrict_kind != PM_RESTRICT_FW && p->restrict_kind != PM_RESTRICT_AVG)
    return pm_fail(ctx, PM_ERR_ARG, "bad restrict_kind");
  if (p->guess != PM_GUESS_JACOBI && p->guess != PM_GUESS_WARM &&
      p->guess != PM_GUESS_WARM_RESCALED && p->guess != PM_GUESS_EXTRAPOLATED)
    return pm_fail(ctx, PM_ERR_ARG, "bad guess");
  return PM_OK;
}

// the f(R) fields of the step parameters (pm_solve_fr and PM_GRAVITY_FR)
int check_fr(pm_ctx *ctx, const pm_step_params *p) {
  if (!(p->omega_m > 0.0) || !std::isfinite(p->omega_m) || !std::isfinite(p->omega_l))
    return pm_fail(ctx, PM_ERR_ARG, "Omega_m must be > 0 and Omega_L finite");
  if (!(p->fr_f0 < 0.0) || !std::isfinite(p->fr_f0))
    return pm_fail(ctx, PM_ERR_ARG, "f(R) needs a finite f_R0 < 0");
  if (!(p->fr_c2 > 0.0) || !std::isfinite(p->fr_c2))
    return pm_fail(ctx, PM_ERR_ARG, "f(R) needs a finite c~^2 > 0");
  if (p->fr_n != 1 && p->fr_n != 2) return pm_fail(ctx, PM_ERR_ARG, "Hu-Sawicki n must be 1 or 2");
  if (p->fr_cycles < 1 || p->fr_cycles > 64)
    return pm_fail(ctx, PM_ERR_ARG, "fr_cycles must be 1 .. 64");
  if (p->fr_cycle != PM_CYCLE_V && p->fr_cycle != PM_CYCLE_W && p->fr_cycle != PM_CYCLE_F)
    return pm_fail(ctx, PM_ERR_ARG, "bad FAS cycle");
  if (p->fr_pre < 1 || p->fr_pre > 64 || p->fr_post < 1 || p->fr_post > 64)
    return pm_fail(ctx, PM_ERR_ARG, "FAS pre- and post-smoothing must be 1 .. 64 sweeps");
  if (p->fr_coarse_sweeps < 1 || p->fr_coarse_sweeps > 4096)
    return pm_fail(ctx, PM_ERR_ARG, "fr_coarse_sweeps must be 1 .. 4096");
  return PM_OK;
}

int check_gravity(pm_ctx *ctx, const pm_step_params *p) {
  if (!(p->omega_m > 0.0) || !std::isfinite(p->omega_m) || !std::isfinite(p->omega_l))
    return pm_fail(ctx, PM_ERR_ARG, "Omega_m must be > 0 and Omega_L finite");
  if (p->gravity != PM_GRAVITY_NEWTON && p->gravity != PM_GRAVITY_MU &&
      p->gravity != PM_GRAVITY_QUMOND && p->gravity != PM_GRAVITY_FR)
    return pm_fail(ctx, PM_ERR_ARG, "bad gravity");
  if (p->gravity == PM_GRAVITY_FR) {
    if (int st = check_fr(ctx, p)) return st;
    if (p->solver == PM_SOLVER_FULL_FFT)
      return pm_fail(ctx, PM_ERR_ARG, "f(R) needs a potential: not the FULL_FFT solver");
  }
  if (p->gravity == PM_GRAVITY_MU && (!std::isfinite(p->mu0) || !(p->omega_l > 0.0)))
    return pm_fail(ctx, PM_ERR_ARG, "parametrised gravity needs a finite mu0 and Omega_L > 0");
  if (p->gravity == PM_GRAVITY_QUMOND) {
    if (!(p->mond_g0 > 0.0) || !std::isfinite(p->mond_g0) || !std::isfinite(p->mond_g0_exp))
      return pm_fail(ctx, PM_ERR_ARG, "QUMOND needs g0 > 0 and a finite exponent");
    if (p->mond_family < PM_NU_SIMPLE || p->mond_family > PM_NU_DELTA)
      return pm_fail(ctx, PM_ERR_ARG, "bad nu family");
    if (p->mond_family != PM_NU_SIMPLE && p->mond_family != PM_NU_BETA &&
        !(p->mond_param > 0.0))
      return pm_fail(ctx, PM_ERR_ARG, "the nu family's parameter must be > 0");
    if (p->mond_family == PM_NU_BETA && !std::isfinite(p->mond_param))
      return pm_fail(ctx, PM_ERR_ARG, "bad beta");
    if (p->solver != PM_SOLVER_MG && p->solver != PM_SOLVER_FFT_7PT)
      return pm_fail(ctx, PM_ERR_ARG, "QUMOND takes the multigrid or FFT_7pt solver");
  }
  return PM_OK;
}

int check_step(pm_ctx *ctx, const pm_step_params *p) {
  if (!p) return pm_fail(ctx, PM_ERR_ARG, "null step params");
  if (!valid_mas(p->mas)) return pm_fail(ctx, PM_ERR_ARG, "bad mas");
  if (int g = check_gravity(ctx, p)) return g;
  if (p->order != PM_DEPOSIT_ATOMIC && p->order != PM_DEPOSIT_SORTED)
    return pm_fail(ctx, PM_ERR_ARG, "bad deposit order");
  if (p->solver != PM_SOLVER_MG && !is_fft(p->solver))
    return pm_fail(ctx, PM_ERR_ARG, "bad solver");
  if (p->solver == PM_SOLVER_MG) return check_mg(ctx, &p->mg);
  if (p->fft_deconv < 0 || p->fft_deconv > 3)
    return pm_fail(ctx, PM_ERR_ARG, "fft_deconv must be 0, 1, 2 or 3");
  return PM_OK;
}

// reverse mode: the window needs a position derivative and the force a potential
int check_step_vjp(pm_ctx *ctx, const pm_step_params *p) {
  const int st = check_step(ctx, p);
  if (st != PM_OK) return st;
  if (!valid_mas_vjp(p->mas)) return pm_fail(ctx, PM_ERR_ARG, "reverse mode takes CIC or TSC");
  if (p->solver == PM_SOLVER_FULL_FFT)
    return pm_fail(ctx, PM_ERR_ARG, "reverse mode does not take the FULL_FFT solver");
  if (p->gravity == PM_GRAVITY_QUMOND || p->gravity == PM_GRAVITY_FR)
    return pm_fail(ctx, PM_ERR_ARG, "reverse mode takes Newtonian or parametrised gravity");
  return PM_OK;
}

int ensure_sort_scratch(pm_ctx *ctx, int64_t np) {
  if (np > INT32_MAX) return pm_fail(ctx, PM_ERR_SHAPE, "sorted deposit supports < 2^31 particles");
  const int64_t ncell = (int64_t)ctx->n * ctx->n * ctx->n;
  if (!ctx->cell_count) {
    const size_t len = (size_t)ncell + 1;
    const int64_t nblk = scan_blocks_needed((int64_t)len);
    if (hipMalloc(&ctx->cell_count, sizeof(int32_t) * len) != hipSuccess ||
        hipMalloc(&ctx->scan_partial, sizeof(int32_t) * (size_t)nblk) != hipSuccess)
      return pm_fail(ctx, PM_ERR_NOMEM, "sort scratch allocation failed");
  }
  if (ctx->sort_cap < np) {
    if (ctx->perm) (void)hipFree(ctx->perm);
    if (ctx->pcell) (void)hipFree(ctx->pcell);
    ctx->perm = ctx->pcell = nullptr;
    const int64_t cap = std::max<int64_t>(np, ctx->np_max);
    if (hipMalloc(&ctx->perm, sizeof(int32_t) * (size_t)std::max<int64_t>(cap, 1)) != hipSuccess ||
        hipMalloc(&ctx->pcell, sizeof(int32_t) * (size_t)std::max<int64_t>(cap, 1)) != hipSuccess)
      return pm_fail(ctx, PM_ERR_NOMEM, "sort scratch allocation failed");
    ctx->sort_cap = cap;
  }
  if (ctx->n % 8 == 0 && !ctx->cell_count2) {
    const size_t len = (size_t)ncell / 512 + 1;
    if (hipMalloc(&ctx->cell_count2, sizeof(int32_t) * len) != hipSuccess) {
      ctx->cell_count2 = nullptr;
      return pm_fail(ctx, PM_ERR_NOMEM, "sort scratch allocation failed");
    }
  }
  return PM_OK;
}

int deposit_impl(pm_ctx *ctx, const float *pos, const int32_t *cell, int64_t np, int poskind,
                 int mas, int order, float *rho, hipStream_t s, bool *mean_ready = nullptr) {
  if (mean_ready) *mean_ready = false;
  const int n = ctx->n;
  const int64_t ncell = (int64_t)n * n * n;
  const float mass = np > 0 ? (float)((double)ncell / (double)np) : 0.0f;
  if (order == PM_DEPOSIT_SORTED) {
    int st = ensure_sort_scratch(ctx, np);
    if (st != PM_OK) return st;
    const bool tiles = (n % 8) == 0;
    if (tiles && !ctx->tile_box) {
      // 10^3 values per 8^3 tile (every non-empty tile overwrites its box)
      if (hipMalloc(&ctx->tile_box, sizeof(float) * 1000 * (size_t)(ncell / 512)) !=
          hipSuccess) {
        ctx->tile_box = nullptr;
        return pm_fail(ctx, PM_ERR_NOMEM, "tile box allocation failed");
      }
    }
    bool hist = tiles && ctx->hist_ready;
    if (tiles && !hist && ctx->hist_next && ctx->hist_pos == pos && ctx->hist_cell == cell &&
        ctx->hist_np == np) {
      // histogram and keys made by the previous chained step's fused drift
      PM_HIP(ctx, hipMemcpyAsync(ctx->cell_count, ctx->cell_count2,
                                 sizeof(int32_t) * (size_t)(ncell / 512 + 1),
                                 hipMemcpyDeviceToDevice, s));
      hist = true;
    }
    ctx->hist_ready = false;
    ctx->hist_next = false;
    PM_HIP(ctx, launch_sort_by_cell(ctx, pos, cell, np, poskind, s, tiles ? 2 : 0, hist));
    pm_kt_begin(ctx, PM_KERNEL_DEPOSIT, s);
    if (tiles)
    {
      // the mean of rho comes exactly from the fixed-point sums when the caller wants it
      PM_HIP(ctx, launch_deposit_own(ctx, pos, cell, poskind, mas, mass, rho,
                                     mean_ready ? ctx->mean_f : nullptr, s));
      if (mean_ready) *mean_ready = true;
    }
    else
      PM_HIP(ctx, launch_deposit_pull(ctx, pos, np, poskind, mas, mass, rho, s));
    // algorithmic bytes: in-cell offsets (12 B per particle) + the density (4 B per cell)
    pm_kt_end(ctx, PM_KERNEL_DEPOSIT, s, 12.0 * (double)np + 4.0 * (double)ncell);
    return PM_OK;
  }
  PM_HIP(ctx, hipMemsetAsync(rho, 0, sizeof(float) * (size_t)ncell, s));
  PM_HIP(ctx, launch_deposit_atomic(pos, cell, np, poskind, mas, n, mass, rho, s));
  return PM_OK;
}

int solve_impl(pm_ctx *ctx, const pm_step_params *p, const float *rho, float coef, float *phi,
               pm_mg_stats *st, hipStream_t s, float warm_scale, bool rho_mean_ready = false) {
  // the sorted deposit leaves the density's mean in mean_f[0]
  const float *mean = rho_mean_ready ? ctx->mean_f : nullptr;
  if (p->solver == PM_SOLVER_FFT) return pm_fft_solve(ctx, rho, coef, p->fft_deconv, phi, s, mean);
  if (p->solver == PM_SOLVER_FFT_7PT)
    return pm_fft_solve_kind(ctx, rho, coef, 0, PM_FFT_7PT, phi, s, mean);
  return pm_mg_solve(ctx, rho, coef, phi, &p->mg, st, s, warm_scale, rho_mean_ready);
}

// PM_GUESS_EXTRAPOLATED: with two earlier solves on this phi (at a_p < a_c < a), phi
// becomes the linear extrapolation in supercomoving time of psi = phi / (a D) and
// *warm_scale 1; with one, the current potential is kept as the previous one and the
// solve starts from the rescaled one (*warm_scale as given)
int extrapolate_guess(pm_ctx *ctx, float *phi, double a, const pm_step_params *p,
                      float *warm_scale, hipStream_t s) {
  const int64_t count = (int64_t)ctx->n * ctx->n * ctx->n;
  const bool have_cur = ctx->ex_phi == phi && ctx->ex_a_cur > 0.0 && ctx->ex_a_cur < a;
  if (!have_cur) {
    ctx->ex_has_prev = false;
    return PM_OK;
  }
  if (!ctx->ex_prev) {
    if (hipMalloc(&ctx->ex_prev, sizeof(float) * (size_t)count) != hipSuccess) {
      ctx->ex_prev = nullptr;
      (void)hipGetLastError();
      return pm_fail(ctx, PM_ERR_NOMEM, "extrapolated warm start allocation failed");
    }
    ctx->ex_has_prev = false;
  }
  const double ap = ctx->ex_a_prev, ac = ctx->ex_a_cur;
  if (ctx->ex_has_prev && ap < ac) {
    const double om = p->omega_m, ol = p->omega_l;
    const double gp = ap * pm_bg_growth(om, ol, ap), gc = ac * pm_bg_growth(om, ol, ac),
                 gn = a * pm_bg_growth(om, ol, a);
    const double theta = pm_bg_tau(om, ol, ac, a) / pm_bg_tau(om, ol, ap, ac);
    PM_HIP(ctx, launch_extrapolate(phi, ctx->ex_prev, count, (float)(gn / gc * (1.0 + theta)),
                                   (float)(-gn / gp * theta), s));
    *warm_scale = 1.0f;
  } else {
    PM_HIP(ctx, hipMemcpyAsync(ctx->ex_prev, phi, sizeof(float) * (size_t)count,
                               hipMemcpyDeviceToDevice, s));
  }
  ctx->ex_a_prev = ac;
  ctx->ex_has_prev = true;
  return PM_OK;
}

// deposit -> solve -> gradient -> interp (+ optional kick on vel)
// the next step of a chain of leapfrog steps: its opening half-kick and its drift
struct ChainNext {
  float kick, dt;
};

int accel_impl(pm_ctx *ctx, const float *pos, const int32_t *cell, int64_t np, int poskind,
               double a, const pm_step_params *p, float *phi, float *acc, float *vel, float kick,
               pm_step_stats *stats, hipStream_t s, bool timing, float warm_scale,
               const ChainNext *next) {
  if (timing) PM_HIP(ctx, hipEventRecord(ctx->ev[1], s));
  bool mean_ready = false;
  int st = deposit_impl(ctx, pos, cell, np, poskind, p->mas, p->order, ctx->rho, s, &mean_ready);
  if (st != PM_OK) return st;
  if (timing) PM_HIP(ctx, hipEventRecord(ctx->ev[2], s));
  const float coef = (float)pm_bg_coef(p, a);
  const bool full_fft = p->solver == PM_SOLVER_FULL_FFT;
  int sst;
  if (full_fft) {
    // FULL_FFT: the force grid comes straight from Fourier space (no potential, no stencil)
    sst = pm_fft_solve_kind(ctx, ctx->rho, coef, p->fft_deconv, PM_FFT_FULL, ctx->g, s,
                            mean_ready ? ctx->mean_f : nullptr);
  } else if (p->gravity == PM_GRAVITY_QUMOND) {
    // QUMOND: the Newtonian potential (warm-started from the previous one), the MOND
    // source on the cell faces, and the MOND potential (phi, warm-started as usual)
    const size_t bytes = sizeof(float) * (size_t)ctx->n * ctx->n * ctx->n;
    if (!ctx->mond_phin) {
      if (hipMalloc(&ctx->mond_phin, bytes) != hipSuccess ||
          hipMalloc(&ctx->mond_src, bytes) != hipSuccess)
        return pm_fail(ctx, PM_ERR_NOMEM, "QUMOND scratch allocation failed");
      ctx->mond_valid = false;
    }
    pm_step_params pn = *p;
    if (!ctx->mond_valid) pn.mg.guess = PM_GUESS_JACOBI;
    sst = solve_impl(ctx, &pn, ctx->rho, coef, ctx->mond_phin, nullptr, s, warm_scale,
                     mean_ready);
    if (sst < 0) return sst;
    ctx->mond_valid = true;
    const double g0 = p->mond_g0 * std::pow(a, p->mond_g0_exp);
    PM_HIP(ctx, launch_qumond_source(ctx->mond_phin, ctx->n, (float)g0, p->mond_family,
                                     (float)p->mond_param, ctx->mond_src, s));
    sst = solve_impl(ctx, p, ctx->mond_src, 1.0f, phi, stats ? &stats->mg : nullptr, s,
                     warm_scale, false);
  } else {
    float ws = warm_scale;
    const bool mg = p->solver == PM_SOLVER_MG;
    // extrapolation only for tolerance-driven solves: a fixed cycle count must not depend
    // on a history the caller does not see
    const bool extrap = mg && p->mg.guess == PM_GUESS_EXTRAPOLATED && p->mg.fixed_cycles == 0;
    if (extrap) {
      if (int est = extrapolate_guess(ctx, phi, a, p, &ws, s)) return est;
    } else {
      ctx->ex_has_prev = false;  // ex_prev is not this solve's predecessor
    }
    sst = solve_impl(ctx, p, ctx->rho, coef, phi, stats ? &stats->mg : nullptr, s, ws,
                     mean_ready);
    // the solve history of the extrapolated warm start (multigrid solves on this phi)
    ctx->ex_phi = mg ? phi : nullptr;
    ctx->ex_a_cur = a;
  }
  if (p->gravity == PM_GRAVITY_QUMOND || full_fft) ctx->ex_phi = nullptr;
  if (sst < 0) return sst;
  // f(R): the scalaron (from the previous one unless the guess is Jacobi) and the force
  // potential phi_N - (c~^2 / 2) f~; phi keeps the Newtonian potential
  const float *phif = phi;
  if (p->gravity == PM_GRAVITY_FR) {
    if (int fst = pm_fr_force_potential(ctx, ctx->rho, a, p, p->mg.guess != PM_GUESS_JACOBI,
                                        phi, s))
      return fst;
    phif = ctx->fr_phi;
  }
  if (timing) PM_HIP(ctx, hipEventRecord(ctx->ev[3], s));
  // with the tile buckets of these positions (sorted deposit on tiles), the gradient is
  // formed per tile inside the interpolation kernel
  const bool tiles = p->order == PM_DEPOSIT_SORTED && ctx->n % 8 == 0 && !full_fft;
  if (!tiles && !full_fft) PM_HIP(ctx, launch_gradient(phif, ctx->n, 5, ctx->g, s));
  if (timing) PM_HIP(ctx, hipEventRecord(ctx->ev[4], s));
  pm_kt_begin(ctx, PM_KERNEL_INTERP, s);
  double bytes;
  if (tiles && next && np > 0) {
    // the closing kick of this step and the opening kick and drift of the next one, in
    // the interpolation kernel; the next sort's tile histogram comes with the drift
    float *wpos = const_cast<float *>(pos);
    int32_t *wcell = const_cast<int32_t *>(cell);
    const int64_t ntiles = (int64_t)ctx->n * ctx->n * ctx->n / 512;
    PM_HIP(ctx, hipMemsetAsync(ctx->cell_count2, 0, sizeof(int32_t) * (size_t)(ntiles + 1), s));
    PM_HIP(ctx, launch_interp_tile_phi(ctx, wpos, wcell, poskind, p->mas, phif, nullptr, vel,
                                       kick + next->kick, next->dt, ctx->pcell, ctx->cell_count2,
                                       s));
    ctx->hist_next = true;
    ctx->hist_pos = pos;
    ctx->hist_cell = cell;
    ctx->hist_np = np;
    // position (+ cell index) and velocity in and out, tile key out
    bytes = (double)np * (2.0 * (12.0 + (poskind == PM_POS_CELLOFF ? 4.0 : 0.0)) + 24.0 + 4.0) +
            4.0 * (double)ctx->n * ctx->n * ctx->n;
  } else {
    if (tiles)
      PM_HIP(ctx, launch_interp_tile_phi(ctx, const_cast<float *>(pos), const_cast<int32_t *>(cell),
                                         poskind, p->mas, phif, acc, vel, kick, 0.0f, nullptr,
                                         nullptr, s));
    else
      PM_HIP(ctx, launch_interp(pos, cell, np, poskind, p->mas, ctx->n, ctx->g, acc, vel, kick, s));
    // algorithmic bytes: position (12 B, + 4 B cell index), velocity in/out (24 B),
    // acceleration out (12 B) per particle, and the force grid once (12 B per cell) or,
    // with the gradient fused, the potential once (4 B per cell)
    bytes = (double)np * (48.0 + (poskind == PM_POS_CELLOFF ? 4.0 : 0.0)) +
            (tiles ? 4.0 : 12.0) * (double)ctx->n * ctx->n * ctx->n;
  }
  pm_kt_end(ctx, PM_KERNEL_INTERP, s, bytes);
  if (next && !tiles && np > 0)
    PM_HIP(ctx, launch_kick_drift(const_cast<float *>(pos), const_cast<int32_t *>(cell), vel, acc,
                                  np, poskind, ctx->n, next->kick, next->dt, s));
  if (timing) PM_HIP(ctx, hipEventRecord(ctx->ev[5], s));
  return sst;
}

void fill_timing(pm_ctx *ctx, pm_step_stats *stats, bool with_drift) {
  if (!stats) return;
  if (hipEventSynchronize(ctx->ev[5]) != hipSuccess) return;
  float t = 0.f;
  stats->ms_drift = 0.f;
  if (with_drift && hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[1]) == hipSuccess) stats->ms_drift = t;
  if (hipEventElapsedTime(&t, ctx->ev[1], ctx->ev[2]) == hipSuccess) stats->ms_deposit = t;
  if (hipEventElapsedTime(&t, ctx->ev[2], ctx->ev[3]) == hipSuccess) stats->ms_solve = t;
  if (hipEventElapsedTime(&t, ctx->ev[3], ctx->ev[4]) == hipSuccess) stats->ms_gradient = t;
  if (hipEventElapsedTime(&t, ctx->ev[4], ctx->ev[5]) == hipSuccess) stats->ms_interp = t;
}

int ensure_adjoint_scratch(pm_ctx *ctx) {
  if (ctx->adj_gbar) return PM_OK;
  const size_t ncell = (size_t)ctx->n * ctx->n * ctx->n;
  if (hipMalloc(&ctx->adj_gbar, 3 * sizeof(float) * ncell) != hipSuccess ||
      hipMalloc(&ctx->adj_phibar, sizeof(float) * ncell) != hipSuccess ||
      hipMalloc(&ctx->adj_rhobar, sizeof(float) * ncell) != hipSuccess) {
    if (ctx->adj_gbar) (void)hipFree(ctx->adj_gbar);
    if (ctx->adj_phibar) (void)hipFree(ctx->adj_phibar);
    ctx->adj_gbar = ctx->adj_phibar = nullptr;
    return pm_fail(ctx, PM_ERR_NOMEM, "adjoint scratch allocation failed");
  }
  ctx->adj_warm = false;
  return PM_OK;
}

// interp^T: through the tile buckets of a tile sort of the positions when the grid has
// 8^3 tiles (the sort overwrites the deposit's sort scratch, so the histogram a fused
// drift left there is dropped), else per chunk of consecutive particles
int interp_vjp_impl(pm_ctx *ctx, const float *pos, const int32_t *cell, int64_t np, int poskind,
                    int mas, const float *g, const float *lam, float pscale, float gscale,
                    float *g_bar, float *pos_bar, hipStream_t s) {
  const int n = ctx->n;
  if (n % 8 == 0 && np > 0 && np <= INT32_MAX) {
    int st = ensure_sort_scratch(ctx, np);
    if (st != PM_OK) return st;
    ctx->hist_ready = false;
    ctx->hist_next = false;
    PM_HIP(ctx, launch_sort_by_cell(ctx, pos, cell, np, poskind, s, 2, false));
    PM_HIP(ctx, launch_interp_vjp_tile(pos, cell, np, poskind, mas, n, ctx->cell_count,
                                       ctx->perm, g, lam, pscale, gscale, g_bar, pos_bar, s));
    return PM_OK;
  }
  PM_HIP(ctx, launch_interp_vjp(pos, cell, np, poskind, mas, n, g, lam, pscale, gscale, g_bar,
                                pos_bar, s));
  return PM_OK;
}

// pos_bar += scale * J(pos)^T lam, J = d accel / d pos at scale factor a (box units).
// phi is the potential of pos at a. Uses ctx->g (force grid), the adjoint scratch and
// ctx->rho (cotangent of the density).
int accel_vjp_impl(pm_ctx *ctx, const float *pos, const int32_t *cell, int64_t np, int poskind,
                   double a, const pm_step_params *p, const float *phi, const float *lam,
                   float scale, float *pos_bar, pm_mg_stats *stats, hipStream_t s) {
  const int n = ctx->n;
  const int64_t ncell = (int64_t)n * n * n;
  const float mass = np > 0 ? (float)((double)ncell / (double)np) : 0.0f;
  PM_HIP(ctx, launch_gradient(phi, n, 5, ctx->g, s));
  PM_HIP(ctx, launch_fill(ctx->adj_gbar, 0.0f, 3 * ncell, s));
  // g_bar = interp^T lam, and the position term sum_c grad W (g_c . lam_p)
  if (int st = interp_vjp_impl(ctx, pos, cell, np, poskind, p->mas, ctx->g, lam, scale * (float)n,
                               1.0f, ctx->adj_gbar, pos_bar, s))
    return st;
  // phi_bar = sum_d D_d g_bar_d
  PM_HIP(ctx, launch_divergence(ctx->adj_gbar, n, 5, false, ctx->adj_phibar, s));
  // rho_bar = coef L^+ (phi_bar - mean): the solve is self-adjoint
  const double coefd = pm_bg_coef(p, a);
  const float coef = (float)coefd;
  float *rho_bar = ctx->adj_rhobar;
  int sst;
  if (p->solver == PM_SOLVER_FFT) {
    sst = pm_fft_solve(ctx, ctx->adj_phibar, coef, p->fft_deconv, rho_bar, s);
  } else if (p->solver == PM_SOLVER_FFT_7PT) {
    sst = pm_fft_solve_kind(ctx, ctx->adj_phibar, coef, 0, PM_FFT_7PT, rho_bar, s);
  } else {
    // tolerance-driven solves start from the previous adjoint solve, rescaled by the
    // ratio of the source coefficients (the cotangents of consecutive reversed steps
    // change little); a fixed cycle count starts from the Jacobi guess, so that its
    // result does not depend on the calls before it
    pm_mg_params mg = p->mg;
    const bool warm = ctx->adj_warm && mg.fixed_cycles == 0 && ctx->adj_coef != 0.0;
    mg.guess = warm ? PM_GUESS_WARM : PM_GUESS_JACOBI;
    sst = pm_mg_solve(ctx, ctx->adj_phibar, coef, rho_bar, &mg, stats, s,
                      warm ? (float)(coefd / ctx->adj_coef) : 1.0f);
  }
  if (sst < 0) {
    ctx->adj_warm = false;
    return sst;
  }
  ctx->adj_warm = true;
  ctx->adj_coef = coefd;
  PM_HIP(ctx, launch_deposit_vjp(pos, cell, np, poskind, p->mas, n, rho_bar,
                                 scale * mass * (float)n, pos_bar, s));
  return sst;
}

}  // namespace

extern "C" {

void pm_default_step_params(pm_step_params *p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->mas = PM_TSC;
  p->order = PM_DEPOSIT_ATOMIC;
  p->solver = PM_SOLVER_MG;
  p->fft_deconv = 3;
  p->omega_m = 1.0;
  p->mg.pre = 2;
  p->mg.post = 2;
  p->mg.omega = 1.0f;
  p->mg.tol = 1e-6f;
  p->mg.max_cycles = 50;
  p->mg.restrict_kind = PM_RESTRICT_FW;
  p->mg.guess = PM_GUESS_JACOBI;
  p->mg.fixed_cycles = 0;
  p->mg.alpha = 0.0f;
  p->mg.cycle = PM_CYCLE_V;
  p->timing = 0;
  p->omega_l = 0.0;
  p->gravity = PM_GRAVITY_NEWTON;
  p->mond_family = PM_NU_SIMPLE;
  p->mu0 = 0.0;
  p->mond_g0 = 0.0;
  p->mond_g0_exp = 0.0;
  p->mond_param = 1.0;
  p->fr_f0 = -1e-5;
  p->fr_c2 = 29.9792458 * 29.9792458;  // a 100 Mpc/h box
  p->fr_n = 1;
  p->fr_cycles = 1;
  p->fr_cycle = PM_CYCLE_F;
  p->fr_pre = 2;
  p->fr_post = 1;
  p->fr_coarse_sweeps = 32;
}

int pm_create(pm_ctx **out, int n, int64_t np_max, int flags) {
  if (!out) return PM_ERR_ARG;
  *out = nullptr;
  if (np_max < 0) return PM_ERR_ARG;
  if (n < 8 || n > 1024 || (n & 1)) return PM_ERR_SHAPE;
  if (flags & ~(PM_CREATE_REFERENCE_KERNELS | PM_CREATE_CHECK_FINITE)) return PM_ERR_ARG;
  pm_ctx *ctx = new pm_ctx();  // value-initialised: every pointer starts null
  ctx->n = n;
  ctx->np_max = np_max;
  ctx->flags = flags;
  if (hipGetDevice(&ctx->device) != hipSuccess) {
    delete ctx;
    return PM_ERR_HIP;
  }
  const size_t ncell = (size_t)n * n * n;
  int st = PM_OK;
  if (hipMalloc(&ctx->rho, sizeof(float) * ncell) != hipSuccess ||
      hipMalloc(&ctx->g, 3 * sizeof(float) * ncell) != hipSuccess ||
      hipMalloc(&ctx->red_partial, 3 * sizeof(double) * RED_PARTIAL_CAP) != hipSuccess ||
      hipMalloc(&ctx->red_result, 4 * sizeof(double)) != hipSuccess ||
      hipMalloc(&ctx->mean_f, 4 * sizeof(float)) != hipSuccess ||
      hipHostMalloc(&ctx->host_result, 4 * sizeof(double), hipHostMallocDefault) != hipSuccess)
    st = PM_ERR_NOMEM;
  if (st == PM_OK) st = pm_mg_setup(ctx);
  for (int i = 0; st == PM_OK && i < 8; ++i)
    if (hipEventCreate(&ctx->ev[i]) != hipSuccess) st = PM_ERR_HIP;
  if (st != PM_OK) {
    pm_destroy(ctx);
    return st;
  }
  *out = ctx;
  return PM_OK;
}

void pm_destroy(pm_ctx *ctx) {
  if (!ctx) return;
  (void)hipDeviceSynchronize();
  auto fr = [](void *p) {
    if (p) (void)hipFree(p);
  };
  fr(ctx->rho);
  fr(ctx->g);
  fr(ctx->red_partial);
  fr(ctx->red_result);
  fr(ctx->mean_f);
  if (ctx->host_result) (void)hipHostFree(ctx->host_result);
  for (int l = 0; l < ctx->nlevels; ++l) {
    if (l > 0) {
      fr(ctx->lev[l].u);
      fr(ctx->lev[l].f);
    }
    fr(ctx->lev[l].alt);
    fr(ctx->lev[l].res);
  }
  fr(ctx->spec);
  fr(ctx->spec2);
  fr(ctx->twiddle);
  fr(ctx->fft_tab);
  fr(ctx->cell_count);
  fr(ctx->perm);
  fr(ctx->pcell);
  fr(ctx->scan_partial);
  fr(ctx->reorder_tmp);
  fr(ctx->tile_box);
  fr(ctx->cell_count2);
  fr(ctx->adj_gbar);
  fr(ctx->adj_phibar);
  fr(ctx->adj_rhobar);
  fr(ctx->mond_phin);
  fr(ctx->mond_src);
  fr(ctx->ex_prev);
  pm_fr_free(ctx);
  for (int i = 0; i < 8; ++i)
    if (ctx->ev[i]) (void)hipEventDestroy(ctx->ev[i]);
  for (int i = 0; i < 2 * ctx->kt_cap; ++i) (void)hipEventDestroy(ctx->kt_ev[i]);
  delete[] ctx->kt_ev;
  delete ctx;
}

const char *pm_last_error(const pm_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int pm_deposit(pm_ctx *ctx, const float *pos, const int32_t *cell, int64_t np, int poskind,
               int mas, int order, float *rho, pm_stream stream) {
  if (!ctx) return PM_ERR_ARG;
  int st = check_particles(ctx, pos, cell, np, poskind);
  if (st != PM_OK) return st;
  if (!valid_mas(mas)) return pm_fail(ctx, PM_ERR_ARG, "bad mas");
  if (order != PM_DEPOSIT_ATOMIC && order != PM_DEPOSIT_SORTED)
    return pm_fail(ctx, PM_ERR_ARG, "bad deposit order");
  if (!rho) return pm_fail(ctx, PM_ERR_ARG, "null rho");
  return deposit_impl(ctx, pos, cell, np, poskind, mas, order, rho, (hipStream_t)stream);
}

int pm_solve_mg(pm_ctx *ctx, const float *rho, float coef, float *phi,
                const pm_mg_params *params, pm_mg_stats *stats, pm_stream stream) {
  if (!ctx) return PM_ERR_ARG;
  if (!rho || !phi) return pm_fail(ctx, PM_ERR_ARG, "null grid");
  int st = check_mg(ctx, params);
  if (st != PM_OK) return st;
  if (!std::isfinite(coef)) return pm_fail(ctx, PM_ERR_NONFINITE, "non-finite coef");
  return pm_mg_solve(ctx, rho, coef, phi, params, stats, (hipStream_t)stream, 1.0f);
}

int pm_solve_fft(pm_ctx *ctx, const float *rho, float coef, int deconv, float *phi,
                 pm_stream stream) {
  if (!ctx) return PM_ERR_ARG;
  if (!rho || !phi) return pm_fail(ctx, PM_ERR_ARG, "null grid");
  if (deconv < 0 || deconv > 3) return pm_fail(ctx, PM_ERR_ARG, "deconv must be 0, 1, 2 or 3");
  if (!std::isfinite(coef)) return pm_fail(ctx, PM_ERR_NONFINITE, "non-finite coef");
  return pm_fft_solve(ctx, rho, coef, deconv, phi, (hipStream_t)stream);
}

int pm_solve_fft_kernel(pm_ctx *ctx, const float *rho, float coef, int kernel, int deconv,
                        float *out, pm_stream stream) {
  if (!ctx) return PM_ERR_ARG;
  if (!rho || !out) return pm_fail(ctx, PM_ERR_ARG, "null grid");
  if (kernel != PM_FFT_GREEN && kernel != PM_FFT_7PT && kernel != PM_FFT_FULL)
    return pm_fail(ctx, PM_ERR_ARG, "bad FFT kernel");
  if (deconv < 0 || deconv > 3) return pm_fail(ctx, PM_ERR_ARG, "deconv must be 0, 1, 2 or 3");
  if (!std::isfinite(coef)) return pm_fail(ctx, PM_ERR_NONFINITE, "non-finite coef");
  return pm_fft_solve_kind(ctx, rho, coef, kernel == PM_FFT_7PT ? 0 : deconv, kernel, out,
                           (hipStream_t)stream);
}

int pm_solve_fr(pm_ctx *ctx, const float *rho, double a, const pm_step_params *params,
                double *u, double *relres, pm_stream stream) {
  if (!ctx) return PM_ERR_ARG;
  if (!rho || !u || !params) return pm_fail(ctx, PM_ERR_ARG, "null pointer");
  if (!(a > 0.0) || !std::isfinite(a)) return pm_fail(ctx, PM_ERR_ARG, "a must be finite and > 0");
  if (int st = check_fr(ctx, params)) return st;
  return pm_fr_solve(ctx, rho, a, params, u, relres, (hipStream_t)stream);
}

int pm_gradient(pm_ctx *ctx, const float *phi, int points, float *g, pm_stream stream) {
  if (!ctx) return PM_ERR_ARG;
  if (!phi || !g) return pm_fail(ctx, PM_ERR_ARG, "null grid");
  if (points != 3 && points != 5 && points != 7)
    return pm_fail(ctx, PM_ERR_ARG, "points must be 3, 5 or 7");
  PM_HIP(ctx, launch_gradient(phi, ctx->n, points, g, (hipStream_t)stream));
  return PM_OK;
}

int pm_interp(pm_ctx *ctx, const float *pos, const int32_t *cell, int64_t np, int poskind,
              int mas, const float *g, float *acc, pm_stream stream) {
  if (!ctx) return PM_ERR_ARG;
  int st = check_particles(ctx, pos, cell, np, poskind);
  if (st != PM_OK) return st;
  if (!valid_mas(mas)) return pm_fail(ctx, PM_ERR_ARG, "bad mas");
  if (!g || (np > 0 && !acc)) return pm_fail(ctx, PM_ERR_ARG, "null pointer");
  PM_HIP(ctx, launch_interp(pos, cell, np, poskind, mas, ctx->n, g, acc, nullptr, 0.f,
                            (hipStream_t)stream));
  return PM_OK;
}

int pm_accel(pm_ctx *ctx, const float *pos, const int32_t *cell, int64_t np, int poskind,
             double a, const pm_step_params *params, float *phi, float *acc,
             pm_step_stats *stats, pm_stream stream) {
  if (!ctx) return PM_ERR_ARG;
  int st = check_particles(ctx, pos, cell, np, poskind);
  if (st != PM_OK) return st;
  st = check_step(ctx, params);
  if (st != PM_OK) return st;
  if (!phi || (np > 0 && !acc)) return pm_fail(ctx, PM_ERR_ARG, "null pointer");
  if (!(a > 0.0) || !std::isfinite(a)) return pm_fail(ctx, PM_ERR_ARG, "scale factor must be > 0");
  hipStream_t s = (hipStream_t)stream;
  if ((st = check_finite(ctx, pos, nullptr, np, s)) != PM_OK) return st;
  const bool timing = params->timing && stats;
  st = accel_impl(ctx, pos, cell, np, poskind, a, params, phi, acc, nullptr, 0.f, stats, s, timing,
                  1.0f, nullptr);
  if (st >= 0 && timing) fill_timing(ctx, stats, false);
  return st;
}

int pm_kernel_timer(pm_ctx *ctx, int kernel, int capacity) {
  if (!ctx) return PM_ERR_ARG;
  if (kernel < PM_KERNEL_NONE || kernel > PM_KERNEL_FR_SWEEP)
    return pm_fail(ctx, PM_ERR_ARG, "unknown kernel id");
  if (capacity < 0 || capacity > (1 << 20)) return pm_fail(ctx, PM_ERR_ARG, "bad capacity");
  if (capacity > ctx->kt_cap) {
    hipEvent_t *ev = new hipEvent_t[2 * capacity];
    for (int i = 0; i < 2 * ctx->kt_cap; ++i) ev[i] = ctx->kt_ev[i];
    for (int i = 2 * ctx->kt_cap; i < 2 * capacity; ++i)
      if (hipEventCreate(&ev[i]) != hipSuccess) {
        for (int j = 2 * ctx->kt_cap; j < i; ++j) (void)hipEventDestroy(ev[j]);
        delete[] ev;
        return pm_fail(ctx, PM_ERR_HIP, "event creation failed");
      }
    delete[] ctx->kt_ev;
    ctx->kt_ev = ev;
    ctx->kt_cap = capacity;
  }
  ctx->kt_kernel = kernel;
  ctx->kt_used = 0;
  ctx->kt_bytes = 0.0;
  ctx->kt_dropped = 0;
  return PM_OK;
}

int pm_kernel_timer_read(pm_ctx *ctx, double *ms, int64_t *launches, double *bytes) {
  if (!ctx || !ms || !launches || !bytes) return PM_ERR_ARG;
  double total = 0.0;
  for (int i = 0; i < ctx->kt_used; ++i) {
    float t = 0.f;
    PM_HIP(ctx, hipEventSynchronize(ctx->kt_ev[2 * i + 1]));
    PM_HIP(ctx, hipEventElapsedTime(&t, ctx->kt_ev[2 * i], ctx->kt_ev[2 * i + 1]));
    total += t;
  }
  *ms = total;
  *launches = ctx->kt_used;
  *bytes = ctx->kt_bytes;
  return ctx->kt_dropped ? pm_fail(ctx, PM_WARN_NOT_CONVERGED, "kernel timer pool overflowed")
                         : PM_OK;
}

int pm_reorder(pm_ctx *ctx, float *pos, int32_t *cell, float *vel, float *acc, int64_t *ids,
               int64_t np, int poskind, pm_stream stream) {
  if (!ctx) return PM_ERR_ARG;
  int st = check_particles(ctx, pos, cell, np, poskind);
  if (st != PM_OK) return st;
  if (np == 0) return PM_OK;
  st = ensure_sort_scratch(ctx, np);
  if (st != PM_OK) return st;
  if (ctx->reorder_cap < np) {
    if (ctx->reorder_tmp) (void)hipFree(ctx->reorder_tmp);
    ctx->reorder_tmp = nullptr;
    const int64_t cap = std::max<int64_t>(np, ctx->np_max);
    if (hipMalloc(&ctx->reorder_tmp, 12 * (size_t)cap) != hipSuccess)
      return pm_fail(ctx, PM_ERR_NOMEM, "reorder scratch allocation failed");
    ctx->reorder_cap = cap;
  }
  hipStream_t s = (hipStream_t)stream;
  int32_t *cell_arr = poskind == PM_POS_CELLOFF ? cell : nullptr;
  if (ctx->n % 8 == 0) {
    // tile-major cell order in two levels: bucket by 8^3 tile (with the tile histogram
    // and keys a chained step's drift made for these arrays, when it did), then order
    // each tile's bucket by cell in LDS
    bool hist = false;
    if (ctx->hist_next && ctx->hist_pos == pos && ctx->hist_cell == cell && ctx->hist_np == np) {
      PM_HIP(ctx, hipMemcpyAsync(ctx->cell_count, ctx->cell_count2,
                                 sizeof(int32_t) * (size_t)(ctx->n / 8 * (ctx->n / 8) * (ctx->n / 8) + 1),
                                 hipMemcpyDeviceToDevice, s));
      hist = true;
    }
    ctx->hist_next = false;  // the particles move: the tile keys are stale afterwards
    ctx->hist_ready = false;
    PM_HIP(ctx, launch_sort_by_cell(ctx, pos, cell, np, poskind, s, 2, hist));
    PM_HIP(ctx, launch_tile_cell_sort(ctx, pos, cell, poskind, ctx->pcell, s));
    PM_HIP(ctx, launch_apply_perm(ctx, ctx->pcell, pos, cell_arr, vel, acc, ids, np, s));
  } else {
    ctx->hist_next = false;
    ctx->hist_ready = false;
    PM_HIP(ctx, launch_sort_by_cell(ctx, pos, cell, np, poskind, s, 0));
    PM_HIP(ctx, launch_apply_perm(ctx, ctx->perm, pos, cell_arr, vel, acc, ids, np, s));
  }
  return PM_OK;
}

int pm_kdk(pm_ctx *ctx, float *pos, int32_t *cell, float *vel, int64_t np, int poskind,
           double a0, double a1, const pm_step_params *params, float *phi, float *acc,
           pm_step_stats *stats, pm_stream stream) {
  if (!ctx) return PM_ERR_ARG;
  int st = check_particles(ctx, pos, cell, np, poskind);
  if (st != PM_OK) return st;
  st = check_step(ctx, params);
  if (st != PM_OK) return st;
  if (np > 0 && (!vel || !acc)) return pm_fail(ctx, PM_ERR_ARG, "null vel or acc");
  if (!phi) return pm_fail(ctx, PM_ERR_ARG, "null phi");
  if (!(a0 > 0.0) || !(a1 > 0.0) || !std::isfinite(a0) || !std::isfinite(a1))
    return pm_fail(ctx, PM_ERR_ARG, "scale factors must be > 0");
  hipStream_t s = (hipStream_t)stream;
  if ((st = check_finite(ctx, pos, vel, np, s)) != PM_OK) return st;
  const bool timing = params->timing && stats;
  const double tau = pm_bg_tau(params->omega_m, params->omega_l, a0, a1);
  if (!std::isfinite(tau)) return pm_fail(ctx, PM_ERR_ARG, "the background has no real time step");
  const float half = (float)(0.5 * tau);
  if (timing) PM_HIP(ctx, hipEventRecord(ctx->ev[0], s));
  // with the sorted deposit on tiles, the drift also makes the tile histogram of the new
  // positions (the first pass of the deposit's sort)
  const bool fuse_hist = params->order == PM_DEPOSIT_SORTED && ctx->n % 8 == 0 && np > 0;
  int32_t *pcell = nullptr, *count = nullptr;
  if (fuse_hist) {
    st = ensure_sort_scratch(ctx, np);
    if (st != PM_OK) return st;
    const int64_t ntiles = (int64_t)(ctx->n / 8) * (ctx->n / 8) * (ctx->n / 8);
    PM_HIP(ctx, hipMemsetAsync(ctx->cell_count, 0, sizeof(int32_t) * (size_t)(ntiles + 1), s));
    pcell = ctx->pcell;
    count = ctx->cell_count;
  }
  PM_HIP(ctx, launch_kick_drift(pos, cell, vel, acc, np, poskind, ctx->n, half, (float)tau, s,
                                pcell, count));
  ctx->hist_ready = fuse_hist;
  // growth rescaling of the previous potential: phi~ grows as a D(a) (a^2 in EdS)
  const float warm_scale = params->mg.guess == PM_GUESS_WARM_RESCALED ||
                                   params->mg.guess == PM_GUESS_EXTRAPOLATED
                               ? (float)pm_bg_warm_scale(params, a0, a1) : 1.0f;
  st = accel_impl(ctx, pos, cell, np, poskind, a1, params, phi, acc, vel, half, stats, s, timing,
                  warm_scale, nullptr);
  if (st >= 0 && timing) fill_timing(ctx, stats, true);
  return st;
}

int pm_kdk_chain(pm_ctx *ctx, float *pos, int32_t *cell, float *vel, int64_t np, int poskind,
                 double a0, double a1, double a2, int stage, const pm_step_params *params,
                 float *phi, float *acc, pm_step_stats *stats, pm_stream stream) {
  if (!ctx) return PM_ERR_ARG;
  int st = check_particles(ctx, pos, cell, np, poskind);
  if (st != PM_OK) return st;
  st = check_step(ctx, params);
  if (st != PM_OK) return st;
  if (np > 0 && (!vel || !acc)) return pm_fail(ctx, PM_ERR_ARG, "null vel or acc");
  if (!phi) return pm_fail(ctx, PM_ERR_ARG, "null phi");
  if (stage != PM_CHAIN_FIRST && stage != PM_CHAIN_NEXT)
    return pm_fail(ctx, PM_ERR_ARG, "stage must be PM_CHAIN_FIRST or PM_CHAIN_NEXT");
  if (!(a0 > 0.0) || !(a1 > 0.0) || !std::isfinite(a0) || !std::isfinite(a1) || !std::isfinite(a2))
    return pm_fail(ctx, PM_ERR_ARG, "scale factors must be > 0 and finite");
  const bool more = a2 > a1;
  hipStream_t s = (hipStream_t)stream;
  if ((st = check_finite(ctx, pos, vel, np, s)) != PM_OK) return st;
  const bool timing = params->timing && stats;
  const double tau = pm_bg_tau(params->omega_m, params->omega_l, a0, a1);
  if (!std::isfinite(tau)) return pm_fail(ctx, PM_ERR_ARG, "the background has no real time step");
  const float half = (float)(0.5 * tau);
  if (timing) PM_HIP(ctx, hipEventRecord(ctx->ev[0], s));
  if (stage == PM_CHAIN_FIRST) {
    // synchronised state at a0: the opening half-kick and the drift, as in pm_kdk
    const bool fuse_hist = params->order == PM_DEPOSIT_SORTED && ctx->n % 8 == 0 && np > 0;
    int32_t *pcell = nullptr, *count = nullptr;
    if (fuse_hist) {
      st = ensure_sort_scratch(ctx, np);
      if (st != PM_OK) return st;
      const int64_t ntiles = (int64_t)(ctx->n / 8) * (ctx->n / 8) * (ctx->n / 8);
      PM_HIP(ctx, hipMemsetAsync(ctx->cell_count, 0, sizeof(int32_t) * (size_t)(ntiles + 1), s));
      pcell = ctx->pcell;
      count = ctx->cell_count;
    }
    PM_HIP(ctx, launch_kick_drift(pos, cell, vel, acc, np, poskind, ctx->n, half, (float)tau, s,
                                  pcell, count));
    ctx->hist_ready = fuse_hist;
  }
  const float warm_scale = params->mg.guess == PM_GUESS_WARM_RESCALED ||
                                   params->mg.guess == PM_GUESS_EXTRAPOLATED
                               ? (float)pm_bg_warm_scale(params, a0, a1) : 1.0f;
  ChainNext next{};
  if (more) {
    const double tau2 = pm_bg_tau(params->omega_m, params->omega_l, a1, a2);
    next.kick = (float)(0.5 * tau2);
    next.dt = (float)tau2;
  }
  st = accel_impl(ctx, pos, cell, np, poskind, a1, params, phi, acc, vel, half, stats, s, timing,
                  warm_scale, more ? &next : nullptr);
  if (st >= 0 && timing) fill_timing(ctx, stats, stage == PM_CHAIN_FIRST);
  return st;
}

int pm_deposit_vjp(pm_ctx *ctx, const float *pos, const int32_t *cell, int64_t np, int poskind,
                   int mas, const float *rho_bar, float *pos_bar, pm_stream stream) {
  if (!ctx) return PM_ERR_ARG;
  int st = check_particles(ctx, pos, cell, np, poskind);
  if (st != PM_OK) return st;
  if (!valid_mas_vjp(mas)) return pm_fail(ctx, PM_ERR_ARG, "reverse mode takes CIC or TSC");
  if (!rho_bar || (np > 0 && !pos_bar)) return pm_fail(ctx, PM_ERR_ARG, "null pointer");
  const int n = ctx->n;
  const float mass = np > 0 ? (float)((double)n * n * n / (double)np) : 0.0f;
  PM_HIP(ctx, launch_deposit_vjp(pos, cell, np, poskind, mas, n, rho_bar, mass * (float)n, pos_bar,
                                 (hipStream_t)stream));
  return PM_OK;
}

int pm_interp_vjp(pm_ctx *ctx, const float *pos, const int32_t *cell, int64_t np, int poskind,
                  int mas, const float *g, const float *lam, float *g_bar, float *pos_bar,
                  pm_stream stream) {
  if (!ctx) return PM_ERR_ARG;
  int st = check_particles(ctx, pos, cell, np, poskind);
  if (st != PM_OK) return st;
  if (!valid_mas_vjp(mas)) return pm_fail(ctx, PM_ERR_ARG, "reverse mode takes CIC or TSC");
  if (np > 0 && !lam) return pm_fail(ctx, PM_ERR_ARG, "null lam");
  if (!g_bar && !pos_bar) return pm_fail(ctx, PM_ERR_ARG, "both outputs null");
  if (pos_bar && !g) return pm_fail(ctx, PM_ERR_ARG, "pos_bar needs g");
  return interp_vjp_impl(ctx, pos, cell, np, poskind, mas, g, lam, (float)ctx->n, 1.0f, g_bar,
                         pos_bar, (hipStream_t)stream);
}

int pm_gradient_vjp(pm_ctx *ctx, const float *g_bar, int points, float *phi_bar,
                    pm_stream stream) {
  if (!ctx) return PM_ERR_ARG;
  if (!g_bar || !phi_bar) return pm_fail(ctx, PM_ERR_ARG, "null grid");
  if (points != 3 && points != 5 && points != 7)
    return pm_fail(ctx, PM_ERR_ARG, "points must be 3, 5 or 7");
  PM_HIP(ctx, launch_divergence(g_bar, ctx->n, points, true, phi_bar, (hipStream_t)stream));
  return PM_OK;
}

int pm_accel_vjp(pm_ctx *ctx, const float *pos, const int32_t *cell, int64_t np, int poskind,
                 double a, const pm_step_params *params, const float *phi, const float *lam,
                 float scale, float *pos_bar, pm_mg_stats *stats, pm_stream stream) {
  if (!ctx) return PM_ERR_ARG;
  int st = check_particles(ctx, pos, cell, np, poskind);
  if (st != PM_OK) return st;
  st = check_step_vjp(ctx, params);
  if (st != PM_OK) return st;
  if (!phi || (np > 0 && (!lam || !pos_bar))) return pm_fail(ctx, PM_ERR_ARG, "null pointer");
  if (!(a > 0.0) || !std::isfinite(a)) return pm_fail(ctx, PM_ERR_ARG, "scale factor must be > 0");
  if (!std::isfinite(scale)) return pm_fail(ctx, PM_ERR_NONFINITE, "non-finite scale");
  st = ensure_adjoint_scratch(ctx);
  if (st != PM_OK) return st;
  return accel_vjp_impl(ctx, pos, cell, np, poskind, a, params, phi, lam, scale, pos_bar, stats,
                        (hipStream_t)stream);
}

int pm_kdk_adjoint(pm_ctx *ctx, const float *pos0, const int32_t *cell0, const float *phi0,
                   const float *pos1, const int32_t *cell1, const float *phi1, int64_t np,
                   int poskind, double a_prev, double a0, double a1, const pm_step_params *params,
                   int flags, float *pos_bar, float *vel_bar, pm_step_stats *stats,
                   pm_stream stream) {
  if (!ctx) return PM_ERR_ARG;
  if (flags & ~PM_ADJ_CLOSING_MERGED) return pm_fail(ctx, PM_ERR_ARG, "bad flags");
  const bool closing = !(flags & PM_ADJ_CLOSING_MERGED);
  int st = check_particles(ctx, pos0, cell0, np, poskind);
  if (st == PM_OK && closing) st = check_particles(ctx, pos1, cell1, np, poskind);
  if (st != PM_OK) return st;
  st = check_step_vjp(ctx, params);
  if (st != PM_OK) return st;
  if (np > 0 && (!pos_bar || !vel_bar)) return pm_fail(ctx, PM_ERR_ARG, "null cotangent");
  if (!phi0 || (closing && !phi1)) return pm_fail(ctx, PM_ERR_ARG, "null potential");
  if (!(a0 > 0.0) || !(a1 > 0.0) || !std::isfinite(a0) || !std::isfinite(a1) ||
      !std::isfinite(a_prev))
    return pm_fail(ctx, PM_ERR_ARG, "scale factors must be > 0 and finite");
  if (a_prev > 0.0 && !(a_prev < a0)) return pm_fail(ctx, PM_ERR_ARG, "a_prev must be < a0");
  st = ensure_adjoint_scratch(ctx);
  if (st != PM_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  // supercomoving time steps of the background (Sect. 3.1)
  const double tau = pm_bg_tau(params->omega_m, params->omega_l, a0, a1);
  const double tau_prev = a_prev > 0.0 ? pm_bg_tau(params->omega_m, params->omega_l, a_prev, a0) : 0.0;
  if (!std::isfinite(tau) || !std::isfinite(tau_prev))
    return pm_fail(ctx, PM_ERR_ARG, "the background has no real time step");
  const double kick0 = 0.5 * (tau + tau_prev);
  pm_mg_stats *ms = stats ? &stats->mg : nullptr;
  int worst = PM_OK;
  if (closing) {
    st = accel_vjp_impl(ctx, pos1, cell1, np, poskind, a1, params, phi1, vel_bar,
                        (float)(0.5 * tau), pos_bar, ms, s);
    if (st < 0) return st;
    worst = std::max(worst, st);
  }
  PM_HIP(ctx, launch_axpy(vel_bar, pos_bar, (float)tau, 3 * np, s));
  st = accel_vjp_impl(ctx, pos0, cell0, np, poskind, a0, params, phi0, vel_bar, (float)kick0,
                      pos_bar, ms, s);
  if (st < 0) return st;
  worst = std::max(worst, st);
  return worst;
}

int pm_density_loss(pm_ctx *ctx, const float *pos, const int32_t *cell, int64_t np, int poskind,
                    int mas, int order, const float *w, double *loss, float *pos_bar,
                    pm_stream stream) {
  if (!ctx) return PM_ERR_ARG;
  int st = check_particles(ctx, pos, cell, np, poskind);
  if (st != PM_OK) return st;
  if (!valid_mas(mas)) return pm_fail(ctx, PM_ERR_ARG, "bad mas");
  if (pos_bar && !valid_mas_vjp(mas)) return pm_fail(ctx, PM_ERR_ARG, "reverse mode takes CIC or TSC");
  if (order != PM_DEPOSIT_ATOMIC && order != PM_DEPOSIT_SORTED)
    return pm_fail(ctx, PM_ERR_ARG, "bad deposit order");
  if (!w) return pm_fail(ctx, PM_ERR_ARG, "null weight grid");
  hipStream_t s = (hipStream_t)stream;
  const int n = ctx->n;
  const int64_t ncell = (int64_t)n * n * n;
  st = deposit_impl(ctx, pos, cell, np, poskind, mas, order, ctx->rho, s);
  if (st != PM_OK) return st;
  PM_HIP(ctx, launch_density_loss(ctx->rho, w, ncell, ctx->red_partial, ctx->red_result, s));
  if (pos_bar) {
    const float mass = np > 0 ? (float)((double)ncell / (double)np) : 0.0f;
    PM_HIP(ctx, launch_deposit_vjp(pos, cell, np, poskind, mas, n, ctx->rho, mass * (float)n,
                                   pos_bar, s));
  }
  if (loss) {
    PM_HIP(ctx, hipMemcpyAsync(ctx->host_result, ctx->red_result, sizeof(double),
                               hipMemcpyDeviceToHost, s));
    PM_HIP(ctx, hipStreamSynchronize(s));
    *loss = ctx->host_result[0];
  }
  return PM_OK;
}

int pm_ic_state(pm_ctx *ctx, const float *q, const float *psi, int64_t np, double a0, float *pos,
                int32_t *cell, float *vel, pm_stream stream) {
  if (!ctx) return PM_ERR_ARG;
  if (np < 0) return pm_fail(ctx, PM_ERR_ARG, "negative particle count");
  if (np > 0 && (!q || !psi || !pos || !vel)) return pm_fail(ctx, PM_ERR_ARG, "null pointer");
  if (!(a0 > 0.0) || !std::isfinite(a0)) return pm_fail(ctx, PM_ERR_ARG, "scale factor must be > 0");
  PM_HIP(ctx, launch_ic_state(q, psi, np, ctx->n, (float)std::sqrt(a0), pos, cell, vel,
                              (hipStream_t)stream));
  return PM_OK;
}

int pm_ic_vjp(pm_ctx *ctx, const float *pos_bar, const float *vel_bar, int64_t np, double a0,
              float *psi_bar, pm_stream stream) {
  if (!ctx) return PM_ERR_ARG;
  if (np < 0) return pm_fail(ctx, PM_ERR_ARG, "negative particle count");
  if (np > 0 && (!pos_bar || !vel_bar || !psi_bar)) return pm_fail(ctx, PM_ERR_ARG, "null pointer");
  if (!(a0 > 0.0) || !std::isfinite(a0)) return pm_fail(ctx, PM_ERR_ARG, "scale factor must be > 0");
  PM_HIP(ctx, launch_ic_vjp(pos_bar, vel_bar, np, (float)std::sqrt(a0), psi_bar,
                            (hipStream_t)stream));
  return PM_OK;
}

}  // extern "C"
