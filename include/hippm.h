/*
 * hippm.h -- C ABI of the MI355X (gfx950) particle-mesh force-and-step library.
 *
 * The library implements the particle-mesh loop of Breton, "PySCo: A fast
 * particle-mesh N-body code for modified gravity simulations in Python"
 * (arXiv:2410.20501): mass assignment (Sect. 3.5), the Poisson solve by
 * multigrid (Sects. 3.6-3.7) or FFT (Sect. 3.8), the central finite-difference
 * gradient (Sect. 3.5, gradient table), interpolation back to particles
 * (Sect. 3.5) and the kick-drift-kick leapfrog (Sect. 3.4), in the
 * supercomoving units of Sect. 3.1.
 *
 * Conventions shared by every entry point
 *   - Periodic unit box with n cells per side, cell size h = 1/n; cell (i,j,k)
 *     has its centre at ((i,j,k) + 1/2) h. Scalar grids are float [n][n][n]
 *     row-major (k fastest); vector grids are float [n][n][n][3]; particle
 *     arrays are float [np][3] (Sect. 3.2).
 *   - Positions come in one of two forms (pm_poskind):
 *       PM_POS_BOX     pos[np][3] in box units, [0, 1);
 *       PM_POS_CELLOFF pos[np][3] is the in-cell offset in [0, 1) (cell units)
 *                      and cell[np] the int32 linear index (i*n + j)*n + k.
 *     Velocities are in box units per unit of supercomoving time in both forms.
 *   - All array pointers are DEVICE pointers owned by the caller; the library
 *     never frees them. Calls are asynchronous on `stream` (a hipStream_t; NULL
 *     is the null stream); outputs are valid once the stream has reached the
 *     call. Host pointers (params, stats) are read or written before return.
 *   - A pm_ctx owns every scratch buffer (density and force grids, multigrid
 *     hierarchy, FFT spectrum, sort arrays, reduction partials). Scratch is
 *     allocated by pm_create, except the FFT spectrum and the sort arrays,
 *     which are allocated on the first call that needs them; later calls do
 *     not allocate. A context serves one stream at a time: calls that overlap
 *     on different streams race on its scratch.
 *   - Return value: PM_OK (0); a warning (> 0) when a result was produced but a
 *     solver target was missed; an error (< 0) when nothing usable was
 *     produced. Argument and shape errors are detected before any launch and
 *     leave every buffer untouched. pm_last_error(ctx) describes the most
 *     recent error or warning of that context.
 */
#ifndef HIPPM_H
#define HIPPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pm_ctx pm_ctx;
typedef void *pm_stream; /* hipStream_t */

enum pm_status {
  PM_OK = 0,
  PM_WARN_NOT_CONVERGED = 1, /* multigrid stopped at max_cycles above tol */
  PM_WARN_FLOOR = 2,         /* multigrid reached the FP32 rounding floor above tol: below
                                a relative residual of 1e-4 a V-cycle gained less than 1.5x */
  PM_ERR_ARG = -1,           /* null pointer, bad enum, negative count */
  PM_ERR_SHAPE = -2,         /* grid size or particle count not supported */
  PM_ERR_NOMEM = -3,         /* device allocation failed */
  PM_ERR_HIP = -4,           /* a HIP runtime call failed (text in pm_last_error) */
  PM_ERR_NONFINITE = -5      /* a non-finite value was found where checked */
};

/* Mass-assignment window (Sect. 3.5): p of the window W^p, the number of cells it
 * covers per axis. NGP serves deposit, interpolation and the forward steps; the
 * reverse-mode and batched entry points take CIC or TSC (NGP has no position
 * derivative). */
enum pm_mas { PM_NGP = 1, PM_CIC = 2, PM_TSC = 3 };
enum pm_order { PM_DEPOSIT_ATOMIC = 0, PM_DEPOSIT_SORTED = 1 };
enum pm_poskind { PM_POS_BOX = 0, PM_POS_CELLOFF = 1 };
enum pm_restrict { PM_RESTRICT_FW = 0, PM_RESTRICT_AVG = 1 };
/* Multigrid cycle shape (Sect. 3.7.1, App. C): the coarse error equation of every
 * level is treated by one V cycle (V), by two W cycles in a row (W), or by an F
 * cycle followed by a V cycle (F). */
enum pm_cycle { PM_CYCLE_V = 0, PM_CYCLE_W = 1, PM_CYCLE_F = 2 };
/* Poisson solver of a force evaluation (Sects. 3.7, 3.8): multigrid; FFT with the
 * Green's function -1/k^2 and window deconvolution (fft_deconv); FFT_7pt, the
 * seven-point Laplacian's eigenvalue in Fourier space (the system multigrid
 * solves, no deconvolution); FULL_FFT, the force itself taken in Fourier space
 * (no finite-difference gradient; the potential is then not written). */
enum pm_solver { PM_SOLVER_MG = 0, PM_SOLVER_FFT = 1, PM_SOLVER_FFT_7PT = 2,
                 PM_SOLVER_FULL_FFT = 3 };
/* Fourier-space kernels of pm_solve_fft_kernel (Sect. 3.8). */
enum pm_fft_kernel { PM_FFT_GREEN = 0, PM_FFT_7PT = 1, PM_FFT_FULL = 2 };
/* Starting guess of the multigrid solve (Sects. 3.7.1 and 3.9): the Jacobi step
 * -h^2 f / 6, the potential passed in phi, or (in pm_kdk) that potential scaled
 * by the linear growth of the supercomoving potential between the two scale
 * factors. The paper writes the rescaling factor as (1+z1) D1 / ((1+z0) D0);
 * with the supercomoving Poisson equation of Sect. 3.1 the potential grows as
 * a D, so the factor used is a1 D1 / (a0 D0) = (a1 / a0)^2 in Einstein-de
 * Sitter. pm_solve_mg and pm_accel treat PM_GUESS_WARM_RESCALED as
 * PM_GUESS_WARM (they have no second scale factor).
 * PM_GUESS_EXTRAPOLATED (multigrid steps, Newtonian or parametrised gravity): the
 * growth-normalised potential psi = phi / (a D) of the last two solves on the same phi
 * array, at a_p < a_c, extrapolated linearly in supercomoving time to the new scale
 * factor a: phi = a D(a) [psi_c + theta (psi_c - psi_p)], theta = tau(a_c, a) /
 * tau(a_p, a_c). The context keeps the previous potential (4 bytes per cell,
 * allocated on first use). The history is the last two solves on this phi array in a
 * run of consecutive PM_GUESS_EXTRAPOLATED steps (the solve before the run may have any
 * guess); without it, when a does not increase, or with fixed_cycles > 0, the step acts
 * as PM_GUESS_WARM_RESCALED. Not a method of the paper: a better
 * starting point for the same tolerance-driven solve (one V-cycle fewer per step at
 * 512^3). pm_solve_mg treats it as PM_GUESS_WARM; the batched step as
 * PM_GUESS_WARM_RESCALED. */
enum pm_guess {
  PM_GUESS_JACOBI = 0,
  PM_GUESS_WARM = 1,
  PM_GUESS_WARM_RESCALED = 2,
  PM_GUESS_EXTRAPOLATED = 3
};

/* pm_create flags */
enum pm_create_flags {
  /* Run every multigrid level with the plain one-kernel-per-half-sweep kernels
   * instead of the fused streaming kernels (a reference for testing; slower). */
  PM_CREATE_REFERENCE_KERNELS = 1,
  /* pm_accel, pm_kdk and pm_kdk_chain first count the non-finite values of the
   * positions (and velocities) they are given, one pass over those arrays and a host
   * synchronisation per call, and return PM_ERR_NONFINITE before any other kernel
   * reads them (without the flag, non-finite positions are undefined behaviour) */
  PM_CREATE_CHECK_FINITE = 2
};

/* Multigrid settings (paper Sect. 3.7.1). */
typedef struct {
  int pre;            /* pre-smoothing red-black Gauss-Seidel sweeps (>= 0) */
  int post;           /* post-smoothing sweeps (>= 0) */
  float omega;        /* over-relaxation factor; 1 = plain Gauss-Seidel */
  float tol;          /* stop when ||f - L phi||_2 / ||f||_2 < tol */
  int max_cycles;     /* at most this many V-cycles (1 .. 63) */
  int restrict_kind;  /* pm_restrict */
  int guess;          /* pm_guess: Jacobi step -h^2 f/6, or phi as given */
  int fixed_cycles;   /* > 0: run exactly this many cycles, no convergence test
                         and no host synchronisation (graph-capturable) */
  float alpha;        /* > 0: the paper's rule (Sect. 3.7.1, Eq. multigrid_threshold)
                         instead of tol: stop when ||f - L phi||_2 (over the fine
                         cells) < alpha ||tau||_2 (over the coarse cells), with the
                         truncation-error estimate tau = L_H(R phi) - R(L_h phi),
                         H = 2h and R the cycle's restriction (the paper's value is
                         0.005); costs two extra grid passes and a host
                         synchronisation per test; needs n > 16; 0: the tol rule.
                         Ignored by the batched step (fixed cycles). */
  int cycle;          /* pm_cycle (the batched step always runs V cycles) */
} pm_mg_params;

typedef struct {
  int cycles;         /* V-cycles run */
  int status;         /* PM_OK, PM_WARN_NOT_CONVERGED or PM_WARN_FLOOR */
  double relres[64];  /* relres[0] of the starting guess, relres[c] after cycle c
                         (not filled when fixed_cycles > 0) */
} pm_mg_stats;

/* Theory of gravity of a force evaluation (Sects. 2.3, 2.4, 3.10). */
enum pm_gravity {
  PM_GRAVITY_NEWTON = 0,  /* lap phi = (3/2) Omega_m a (rho - mean rho) */
  PM_GRAVITY_MU = 1,      /* parametrised: the source times mu(a) = 1 + mu0 Omega_L(a) /
                             Omega_L0 (Eq. mu_parametrized_gravity), Omega_L0 > 0 */
  PM_GRAVITY_QUMOND = 2,  /* QUMOND: the Newtonian potential phi_N, then lap phi =
                             div[nu(|grad phi_N| / g0) grad phi_N] discretised on cell
                             faces as Eq. QUMOND_Poisson_MOND_discrete; multigrid or
                             FFT_7pt solver */
  PM_GRAVITY_FR = 3       /* f(R) (Hu-Sawicki, Sects. 2.5, 3.11): the Newtonian potential
                             phi_N (any solver but FULL_FFT) and the scalaron f~ by
                             non-linear multigrid (pm_solve_fr); the force is the
                             gradient of phi_N - (c~^2 / 2) f~ (F = F_N + c~^2/2 grad f~) */
};
/* QUMOND interpolating functions nu(y) (Sect. 2.3): simple 1/2 + sqrt(1 + 4/y) / 2; the
 * n-family [1/2 + sqrt(1 + 4/y^n) / 2]^(1/n); the beta-family (1 - e^-y)^-1/2 + beta e^-y;
 * the gamma-family (1 - e^(-y^(g/2)))^(-1/g) + (1 - 1/g) e^(-y^(g/2)); the delta-family
 * (1 - e^(-y^(d/2)))^(-1/d). mond_param is n, beta, gamma or delta. */
enum pm_nu { PM_NU_SIMPLE = 0, PM_NU_N = 1, PM_NU_BETA = 2, PM_NU_GAMMA = 3, PM_NU_DELTA = 4 };

typedef struct {
  int mas;            /* pm_mas for deposit and interpolation */
  int order;          /* pm_order of the deposit */
  int solver;         /* pm_solver */
  int fft_deconv;     /* FFT and FULL_FFT solvers: window power to deconvolve (0 none,
                         1 NGP, 2 CIC, 3 TSC) */
  double omega_m;     /* matter density parameter today (1 = Einstein-de Sitter) */
  pm_mg_params mg;
  int timing;         /* 1: record per-stage times into pm_step_stats (adds events) */
  /* Background and gravity (Sects. 2.3, 2.4, 3.1, 3.10). The supercomoving time of a
   * step a0 -> a1 is the integral of da / sqrt(Omega_m a^3 + Omega_k a^4 + Omega_L a^6),
   * Omega_k = 1 - Omega_m - Omega_L (Einstein-de Sitter: 2 (a0^-1/2 - a1^-1/2)). */
  double omega_l;     /* cosmological constant today (0 = Einstein-de Sitter) */
  int gravity;        /* pm_gravity */
  int mond_family;    /* pm_nu (QUMOND) */
  double mu0;         /* PM_GRAVITY_MU: the coupling today */
  double mond_g0;     /* PM_GRAVITY_QUMOND: acceleration scale g0 (> 0) in the code's
                         supercomoving units, used as g0 a^mond_g0_exp */
  double mond_g0_exp; /* exponent N of the time-dependent scale g0 a^N (paper default 0) */
  double mond_param;  /* n, beta, gamma or delta of the nu family */
  /* PM_GRAVITY_FR (Sects. 2.5, 3.7.2, 3.11). Units: curvature in H0^2 / c^2, the
   * scalaron f~ = a^2 f_R, the speed of light c~ = c / (H0 L_box) = 2997.92458 / L_box
   * for a box of L_box Mpc/h. */
  double fr_f0;       /* f_R0, the scalaron today (< 0) */
  double fr_c2;       /* c~^2 (> 0) */
  int fr_n;           /* Hu-Sawicki exponent n: 1 (cubic) or 2 (quartic) */
  int fr_cycles;      /* FAS cycles per force evaluation (1 .. 64; paper default 1) */
  int fr_cycle;       /* pm_cycle of the FAS (paper default PM_CYCLE_F) */
  int fr_pre;         /* non-linear Gauss-Seidel sweeps before the coarse correction
                         (>= 1) */
  int fr_post;        /* ... and after it (>= 1) */
  int fr_coarse_sweeps; /* sweeps on the coarsest FAS grid (1 .. 4096) */
} pm_step_params;

typedef struct {
  pm_mg_stats mg;
  float ms_drift, ms_deposit, ms_solve, ms_gradient, ms_interp; /* when timing */
} pm_step_stats;

/* Default parameters: TSC, atomic deposit, multigrid 2/2 sweeps, omega 1,
 * tol 1e-6 (alpha 0), 50 V cycles, full-weighting restriction, Jacobi guess,
 * Omega_m 1, Omega_L 0, Newtonian gravity. */
void pm_default_step_params(pm_step_params *p);

/* Supercomoving time between scale factors a0 < a1 (Sect. 3.1: dt~ = H0 dt / a^2) for
 * matter Omega_m, a cosmological constant Omega_L and curvature 1 - Omega_m - Omega_L:
 * the integral of da / sqrt(Omega_m a^3 + Omega_k a^4 + Omega_L a^6) (composite
 * Gauss-Legendre quadrature in FP64; the closed form in Einstein-de Sitter). The step
 * functions take their tau from it. Returns NaN for invalid arguments. Host only. */
double pm_supercomoving_time(double omega_m, double omega_l, double a0, double a1);

/* Create a context for an n^3 grid and up to np_max particles.
 * n must be even, 8 <= n <= 1024, and halving n while it exceeds 16 and is a
 * multiple of 4 must end at most at 20 (the coarsest multigrid level).
 * flags: 0 or a combination of pm_create_flags.
 * Errors: PM_ERR_ARG, PM_ERR_SHAPE, PM_ERR_NOMEM, PM_ERR_HIP. */
int pm_create(pm_ctx **ctx, int n, int64_t np_max, int flags);
void pm_destroy(pm_ctx *ctx);
const char *pm_last_error(const pm_ctx *ctx);

/* Mass assignment (paper Sect. 3.5): rho[c] = w sum_p prod_d W(u_pd - (c_d + 1/2))
 * with the CIC (8 cells) or TSC (27 cells) window, u = position in cell units,
 * and particle weight w = n^3 / np (mean density 1, the paper's normalisation
 * when np = n^3). rho is overwritten.
 * order PM_DEPOSIT_ATOMIC: chunks of 2048 consecutive particles are sorted by
 *   cell in on-chip memory, every cell of the chunk's box sums its weights in
 *   registers, and the box is added to rho with one FP32 atomic per cell (the
 *   sum order across chunks, hence the last bits, may differ between runs).
 *   Fast when neighbours in memory are neighbours in space (see pm_reorder);
 *   chunks spread over more than 4096 cells use one atomic per weight.
 * order PM_DEPOSIT_SORTED: particles are bucketed (a counting sort into context
 *   scratch; the caller's arrays are not reordered). With n % 8 == 0 the buckets
 *   are 8^3-cell tiles: each tile adds its particles' weights into a box of the
 *   tile plus a one-cell halo on chip, in 64-bit fixed point, and stores the box
 *   (10^3 values, each rounded once to FP32, per tile of context scratch,
 *   allocated on first use); a second pass sums for every cell the boxes that
 *   cover it in FP64 in a fixed order, with one write per cell. Otherwise the
 *   buckets are cells and every cell gathers the contributions of the particles
 *   in its 27 (8, 1) neighbour cells in 64-bit fixed point. Either way the result
 *   is bitwise identical for any particle order and any run. */
int pm_deposit(pm_ctx *ctx, const float *pos, const int32_t *cell, int64_t np,
               int poskind, int mas, int order, float *rho, pm_stream stream);

/* Multigrid Poisson solve of the seven-point system (Sects. 3.5-3.7, 3.9):
 *   (sum of 6 neighbours - 6 phi) / h^2 = coef (rho - mean rho)
 * with coef = (3/2) a Omega_m for the supercomoving Poisson equation.
 * phi: in = starting guess when params->guess == PM_GUESS_WARM; out = the
 * solution with its mean removed. V-cycles of red-black Gauss-Seidel
 * smoothing, restriction to a grid twice as coarse, recursion down to at most
 * 16 cells per side, trilinear prolongation-correction. Unless fixed_cycles is
 * set, the residual norm is checked after every cycle (one host sync each).
 * Returns PM_OK, or a warning if tol was not reached; stats may be NULL. */
int pm_solve_mg(pm_ctx *ctx, const float *rho, float coef, float *phi,
                const pm_mg_params *params, pm_mg_stats *stats, pm_stream stream);

/* FFT Poisson solve (Sect. 3.8, 'FFT'): phi(k) = -coef rho(k) / (k^2 W(k)^2),
 * W = [prod_d sinc(k_d h / 2)]^deconv with deconv = 0 (none), 1 (NGP), 2 (CIC) or
 * 3 (TSC), k = 2 pi m in the unit box with m in [-n/2, n/2); phi(0) = 0. n must
 * be a power of two (8 .. 1024). Same as pm_solve_fft_kernel with PM_FFT_GREEN. */
int pm_solve_fft(pm_ctx *ctx, const float *rho, float coef, int deconv, float *phi,
                 pm_stream stream);

/* FFT solve with the Fourier-space kernel of the paper's three FFT methods (Sect. 3.8):
 *   PM_FFT_GREEN  out = phi [n][n][n]: as pm_solve_fft (deconv 0 .. 3);
 *   PM_FFT_7PT    out = phi: phi(k) = -coef rho(k) / lambda(k), lambda the seven-point
 *                 Laplacian's eigenvalue (4/h^2) sum_d sin^2(k_d h / 2) (the paper's
 *                 printed form of it is garbled; this is the eigenvalue of the stencil
 *                 it names); no deconvolution (deconv ignored). This is the system the
 *                 multigrid solver converges to;
 *   PM_FFT_FULL   out = g [n][n][n][3] = -grad phi taken in Fourier space
 *                 (Eq. exact_fullfft_kernel): g_d(k) = i k_d coef rho(k) / (k^2 W^2),
 *                 with k_d = 0 on the Nyquist plane of axis d; deconv as for GREEN.
 * n must be a power of two (8 .. 1024). FULL uses three more spectra of context
 * scratch (one per force component, about 14 bytes per cell in all, allocated on first
 * use). */
int pm_solve_fft_kernel(pm_ctx *ctx, const float *rho, float coef, int kernel, int deconv,
                        float *out, pm_stream stream);

/* pm_solve_fft without a context and without allocating, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc). The spectrum, tables and the mean's partial sums live in a
 * statically sized device array of the library (about 12.6 MiB, held on each GPU the
 * library runs on until the process ends); n must be a power of two, 8 .. 128
 * (PM_ERR_SHAPE otherwise). Same kernels and result as pm_solve_fft with the same n,
 * coef and deconv (0 .. 3). rho and phi: device arrays [n][n][n] owned by the caller.
 * Every call on one GPU shares that array: calls that overlap on one GPU (different
 * streams or threads) race. Errors: PM_ERR_ARG (null pointer, bad deconv),
 * PM_ERR_NONFINITE (coef), PM_ERR_SHAPE, PM_ERR_HIP (returned as codes; there is no
 * context for a message). */
int pm_solve_fft_noalloc(const float *rho, int n, float coef, int deconv, float *phi,
                         pm_stream stream);

/* f(R) scalaron by non-linear multigrid (Sects. 3.7.2, 3.11). With
 * u = (f~ / f~_bar)^(1/(n+1)) (1 in the background; f~_bar = a^2 f_R_bar(a),
 * f_R_bar = (R_bar(1) / R_bar(a))^(n+1) f_R0, R_bar = 3 (Omega_m a^-3 + 4 Omega_L)) the
 * seven-point discretisation of Eq. fr_sim_2 is, per cell,
 *   (f~_bar / h^2) [sum of 6 neighbours of u^(n+1) - 6 u^(n+1)] - K / u = s,
 *   K = a^4 R_bar / (3 c~^2),  s = -(Omega_m a / c~^2)(rho - mean rho) - K,
 * which for u given its neighbours is the depressed polynomial u^(n+2) + p u + q = 0
 * solved by the paper's closed forms (cubic for n = 1, quartic for n = 2) in FP64 (the
 * cubic's forms evaluated in FP32 and polished to FP64 rounding by two Newton steps).
 * Full-approximation-storage cycles (params->fr_cycle, fr_cycles of them) of red-black
 * non-linear Gauss-Seidel (fr_pre sweeps red first, fr_post sweeps black first),
 * full-weighting restriction of u and of the residual, coarse problem
 * N_H(u_H) = N_H(R u) + R d, trilinear prolongation of u_H - R u; grids are halved while
 * the side exceeds 4 and is a multiple of 4, and the coarsest gets fr_coarse_sweeps
 * sweeps. Uses params->omega_m, omega_l and the fr_ fields.
 * rho: device [n][n][n] density (its mean is measured). u: device FP64 [n][n][n], in =
 * starting guess (all ones for the background), out = the result. Grids of 256 cells per
 * side and more (a multiple of 64) sweep in one streaming pass per sweep when u is
 * 16-byte aligned and fr_pre + fr_post is odd, the iterate alternating with a buffer of
 * the context; otherwise in two colour passes; both give the same bits.
 * relres: host double[2] or NULL; when given, ||s - N(u)||_2 / ||s||_2 before and after
 * the cycles (host synchronisation). Errors: PM_ERR_ARG (bad pointer or parameter),
 * PM_ERR_NOMEM (first call allocates the FAS levels: 32 bytes per cell in total, and
 * 9 more per cell for the streaming grids' second buffers). */
int pm_solve_fr(pm_ctx *ctx, const float *rho, double a, const pm_step_params *params,
                double *u, double *relres, pm_stream stream);

/* Acceleration grid g = -grad phi with the central difference of the given
 * number of points (3, 5 or 7; paper gradient table). g is [n][n][n][3]. */
int pm_gradient(pm_ctx *ctx, const float *phi, int points, float *g, pm_stream stream);

/* Interpolation (Sect. 3.5): acc[p] = sum_c W(u_p - (c + 1/2)) g[c], same window
 * as the deposit. acc is [np][3]. */
int pm_interp(pm_ctx *ctx, const float *pos, const int32_t *cell, int64_t np, int poskind,
              int mas, const float *g, float *acc, pm_stream stream);

/* Accelerations of the particles at scale factor a: deposit, solve with
 * coef = 1.5 a Omega_m, 5-point gradient, interpolation. phi is the potential
 * (warm-start input when the multigrid guess is PM_GUESS_WARM; output).
 * With PM_GRAVITY_FR phi is the Newtonian potential; the context keeps the scalaron's
 * u (FP64, n^3), which the next evaluation starts from unless the multigrid guess is
 * PM_GUESS_JACOBI (then from u = 1, the background), as the paper starts each step's
 * scalaron from the previous step's without rescaling (Sect. 3.11). */
int pm_accel(pm_ctx *ctx, const float *pos, const int32_t *cell, int64_t np, int poskind,
             double a, const pm_step_params *params, float *phi, float *acc,
             pm_step_stats *stats, pm_stream stream);

/* Reorder the particle arrays in place by cell (paper Sect. 3.2 and App. E:
 * particles are periodically re-sorted so that neighbours in memory are
 * neighbours in space; the paper uses a Morton curve). The order is tile-major:
 * 8^3-cell tiles in row-major order and row-major cells inside a tile (plain
 * row-major cells when n is not a multiple of 8); particles in the same cell
 * keep no particular order. pos (and cell for PM_POS_CELLOFF), vel, acc and ids
 * are permuted together; vel, acc and ids may be NULL. ids is an int64 tag per
 * particle that lets the caller follow particle identity. Scratch: 12 bytes per
 * particle plus the sort arrays, allocated on first use. */
int pm_reorder(pm_ctx *ctx, float *pos, int32_t *cell, float *vel, float *acc, int64_t *ids,
               int64_t np, int poskind, pm_stream stream);

/* One kick-drift-kick step (Sect. 3.4) from scale factor a0 to a1 in
 * Einstein-de Sitter supercomoving time, tau = 2 (a0^-1/2 - a1^-1/2):
 *   v += (tau/2) acc;  x = wrap(x + tau v);  acc = accel(x, a1);  v += (tau/2) acc.
 * acc: in = accelerations at (x, a0); out = at (x_new, a1). pos/cell are
 * updated in place (offsets carried into the cell index for PM_POS_CELLOFF).
 * phi: warm start in, potential at a1 out. */
int pm_kdk(pm_ctx *ctx, float *pos, int32_t *cell, float *vel, int64_t np, int poskind,
           double a0, double a1, const pm_step_params *params, float *phi, float *acc,
           pm_step_stats *stats, pm_stream stream);

/* Stages of a chain of kick-drift-kick steps (pm_kdk_chain). */
enum { PM_CHAIN_FIRST = 0, PM_CHAIN_NEXT = 1 };

/* One step a0 -> a1 of a chain of kick-drift-kick steps a0 < a1 < a2 < ... (Sect. 3.4).
 * The closing half-kick of a step and the opening half-kick of the next one use the
 * same accelerations (at x(a1)), so the chain applies them together with the next
 * drift in one pass over the particles: the same arithmetic as consecutive pm_kdk
 * calls up to FP32 rounding order.
 *   stage PM_CHAIN_FIRST: state synchronised at a0 (x(a0), v(a0), acc at a0), as for
 *     pm_kdk; PM_CHAIN_NEXT: the previous call of the chain left x(a1) and the
 *     mid-step velocities of [a0, a1].
 *   a2 > a1: the call ends with x(a2) and the mid-step velocities of [a1, a2] (the
 *     next call passes PM_CHAIN_NEXT and a1, a2, a3); acc is not written (with the
 *     sorted deposit on 8^3 tiles) or holds the accelerations at x(a1).
 *   a2 <= a1 (for example 0): last step; ends synchronised at a1 with acc at x(a1).
 * Between the calls of a chain the particle arrays must change only through
 * pm_reorder. Arguments, ownership and errors as for pm_kdk. */
int pm_kdk_chain(pm_ctx *ctx, float *pos, int32_t *cell, float *vel, int64_t np, int poskind,
                 double a0, double a1, double a2, int stage, const pm_step_params *params,
                 float *phi, float *acc, pm_step_stats *stats, pm_stream stream);

/* ------------------------------------------------------------------ reverse mode
 * Vector-Jacobian products of the steps above, for differentiating a run with
 * respect to its initial conditions (the use the paper gives for
 * differentiable PM in its introduction). Every "_bar" output is ACCUMULATED
 * (the call adds to it) unless stated otherwise, so a caller zeroes it once.
 * Particle cotangents are with respect to box-unit positions x in both
 * position forms (for PM_POS_CELLOFF, x = (cell + offset) / n). The window
 * derivatives are exact: TSC is continuously differentiable, CIC piecewise
 * linear (its derivative is taken inside the cell, like the forward window).
 */

/* Transpose of pm_deposit (Sect. 3.5):
 *   pos_bar[p] += sum_c rho_bar[c] d rho[c] / d x_p
 *              =  w n sum_c rho_bar[c] grad_u W(u_p - (c + 1/2)),  w = n^3 / np.
 * A gather (one thread per particle, no atomics); deterministic. */
int pm_deposit_vjp(pm_ctx *ctx, const float *pos, const int32_t *cell, int64_t np,
                   int poskind, int mas, const float *rho_bar, float *pos_bar,
                   pm_stream stream);

/* Transpose of pm_interp against a particle cotangent lam [np][3]:
 *   g_bar[c]   += sum_p W(u_p - (c + 1/2)) lam[p]             (if g_bar != NULL)
 *   pos_bar[p] += n sum_c grad_u W(u_p - (c + 1/2)) (g[c] . lam[p])  (if pos_bar != NULL;
 *                                                                     needs g)
 * g_bar is [n][n][n][3]; its sum order (FP32 atomics) may differ between runs. */
int pm_interp_vjp(pm_ctx *ctx, const float *pos, const int32_t *cell, int64_t np,
                  int poskind, int mas, const float *g, const float *lam, float *g_bar,
                  float *pos_bar, pm_stream stream);

/* Transpose of pm_gradient: g = -D phi with D the antisymmetric periodic central
 * difference of the gradient table, so phi_bar += sum_d D_d g_bar_d (D^T = -D). */
int pm_gradient_vjp(pm_ctx *ctx, const float *g_bar, int points, float *phi_bar,
                    pm_stream stream);

/* The Poisson solves are self-adjoint: phi = L^+ coef (rho - mean rho) with L
 * the symmetric seven-point operator (or the even FFT kernel) gives
 *   rho_bar = coef L^+ (phi_bar - mean phi_bar),
 * which is pm_solve_mg / pm_solve_fft applied to phi_bar; there is no separate
 * entry point. */

/* J(x)^T of the acceleration map of pm_accel at scale factor a, applied to lam:
 *   pos_bar += scale (d acc / d x)^T lam
 * phi: the potential of these positions at a (as pm_accel / pm_kdk return it);
 * read only. Computes g = -D phi, g_bar = interp^T lam, phi_bar = D g_bar,
 * rho_bar = solve(phi_bar) (multigrid from the Jacobi guess with params->mg,
 * or FFT), then the two position terms (interpolation weights against g . lam,
 * deposit weights against rho_bar). Uses 16 bytes per cell of context scratch
 * (allocated on first use) and the context's density and force grids.
 * Returns the status of the adjoint solve; stats may be NULL. */
int pm_accel_vjp(pm_ctx *ctx, const float *pos, const int32_t *cell, int64_t np, int poskind,
                 double a, const pm_step_params *params, const float *phi, const float *lam,
                 float scale, float *pos_bar, pm_mg_stats *stats, pm_stream stream);

/* Flags of pm_kdk_adjoint. */
enum pm_adjoint_flags {
  /* The closing half-kick term of this step (at x1) was already applied, merged
   * into the opening term of the step after it (see a_prev below): it is skipped,
   * and pos1, cell1 and phi1 may be NULL. */
  PM_ADJ_CLOSING_MERGED = 1
};

/* Reverse of one pm_kdk step from a0 to a1 (Sect. 3.4 leapfrog, transposed), with
 * tau = 2 (a0^-1/2 - a1^-1/2) the step's supercomoving time:
 *   pos_bar += (tau/2) J(x1)^T vel_bar;  vel_bar += tau pos_bar;
 *   pos_bar += w0 J(x0)^T vel_bar
 * where J(x) = d accel / d x at the scale factor of x. (pos0, cell0, phi0) is the
 * state at a0 before the step and (pos1, cell1, phi1) the state after it.
 * When a chain of steps a_prev -> a0 -> a1 is reversed, the closing term of the
 * step a_prev -> a0 acts on the same positions (x0) and the same vel_bar as the
 * opening term of this one, so the library merges them:
 *   a_prev > 0 (a_prev < a0): w0 = (tau(a_prev, a0) + tau(a0, a1)) / 2, and the
 *     caller reverses the step a_prev -> a0 next with PM_ADJ_CLOSING_MERGED;
 *   a_prev <= 0: w0 = tau / 2 (the exact transpose of this step alone).
 * A chain of N steps so costs N + 1 transposed force evaluations instead of 2N.
 * flags: 0 or PM_ADJ_CLOSING_MERGED. Updates pos_bar and vel_bar in place; stats
 * (may be NULL) receives the last adjoint solve's record.
 * Errors: PM_ERR_ARG (null pointers, a_prev >= a0 > 0, bad scale factors, bad
 * flags). */
int pm_kdk_adjoint(pm_ctx *ctx, const float *pos0, const int32_t *cell0, const float *phi0,
                   const float *pos1, const int32_t *cell1, const float *phi1, int64_t np,
                   int poskind, double a_prev, double a0, double a1,
                   const pm_step_params *params, int flags, float *pos_bar, float *vel_bar,
                   pm_step_stats *stats, pm_stream stream);

/* Density objective for inference of initial conditions:
 *   L = sum_c w[c] (rho[c] - 1)^2,  rho = pm_deposit(pos) (mean 1 when np = n^3),
 * summed in FP64 in a fixed order. If loss != NULL it receives L (the call then
 * synchronises the stream); if pos_bar != NULL, pos_bar += dL/dx, through
 * rho_bar = 2 w (rho - 1) and the deposit transpose. Uses the context's density
 * grid. */
int pm_density_loss(pm_ctx *ctx, const float *pos, const int32_t *cell, int64_t np,
                    int poskind, int mas, int order, const float *w, double *loss,
                    float *pos_bar, pm_stream stream);

/* Zel'dovich initial state (Sect. 3.3) from a displacement field psi [np][3] (box
 * units) at lattice points q [np][3]: pos = wrap(q + psi), vel = a0^{1/2} psi, the
 * growing mode in Einstein-de Sitter supercomoving units (D = a). With cell == NULL
 * pos is in box units (PM_POS_BOX); otherwise the state is written in cell-offset
 * form (PM_POS_CELLOFF): every q must then be a cell centre (c + 1/2) / n, and
 * u = c + 1/2 + n psi is split into cell[p] and the offset pos[p] in [0, 1). */
int pm_ic_state(pm_ctx *ctx, const float *q, const float *psi, int64_t np, double a0,
                float *pos, int32_t *cell, float *vel, pm_stream stream);

/* Transpose of pm_ic_state: psi_bar = pos_bar + a0^{1/2} vel_bar (overwritten, not
 * accumulated; the periodic wrap has unit derivative). */
int pm_ic_vjp(pm_ctx *ctx, const float *pos_bar, const float *vel_bar, int64_t np, double a0,
              float *psi_bar, pm_stream stream);

/* ------------------------------------------------------------------ initial conditions
 * and the power spectrum */

/* Initial conditions by Lagrangian perturbation theory (Sect. 3.3, Eqs. x_ini_LPT and
 * v_ini_LPT; growth factors of App. A in Einstein-de Sitter) for np = n^3 particles on
 * the lattice of cell centres, particle p = (i n + j) n + k at ((i, j, k) + 1/2) / n.
 *   noise: [n][n][n] white noise, N(0, 1) per cell (the caller draws it; device);
 *   k_tab, p_tab: host table of the linear P(k) at a = 1 (k = 2 pi m in the unit box,
 *     ascending, 2 .. 65536 points), interpolated linearly in log k - log P and held
 *     constant beyond its ends; DFT[delta] = sqrt(n^3) sqrt(P(k)) DFT[noise], with the
 *     k = 0 mode and the Nyquist planes zero;
 *   order 1 (Zel'dovich), 2 or 3: Psi = a Psi(1) - 3/7 a^2 Psi(2) - 1/3 a^3 Psi(3a)
 *     + 10/21 a^3 Psi(3b) - 1/7 a^3 Psi(3c), the Psi(k) from Fourier-space derivatives
 *     of delta as the paper writes them; velocities in supercomoving units
 *     v = a^(1/2) sum k D^(k) Psi^(k) (an order-k term grows as a^k);
 *   dealias 1: products of fields formed on a 2n grid from zero-padded spectra and
 *     truncated back (free of aliasing for the quadratic and cubic terms; the paper uses
 *     Orszag's 3/2 rule, which this equals for the quadratic ones); 0: on the n grid;
 *   pos [np][3]: box units (cell == NULL) or in-cell offsets with cell [np]; vel [np][3].
 * n must be a power of two (2n <= 1024 with dealiasing). The call allocates its working
 * fields (up to 12 grids of (2n)^3 floats at third order) for its own duration and
 * synchronises the stream before it returns. Errors: PM_ERR_ARG, PM_ERR_SHAPE,
 * PM_ERR_NOMEM, PM_ERR_HIP. */
int pm_ic_lpt(pm_ctx *ctx, const float *noise, int ntab, const double *k_tab,
              const double *p_tab, int order, int dealias, double a0, float *pos,
              int32_t *cell, float *vel, pm_stream stream);

/* Power spectrum of a density grid (the estimator behind the paper's Sect. 4 results):
 * delta = rho / mean(rho) - 1, delta_k = DFT[delta] / n^3 divided by the window
 * W = prod_d sinc(k_d h / 2)^deconv (deconv 0 .. 3, the deposit's p), and
 *   pk[b - 1] = mean of |delta_k|^2 over the modes of shell b = rint(|m|), b = 1 .. nbins,
 * counting the whole sphere of wavevectors (a half-spectrum mode with 0 < k_z < n/2
 * counts twice). kmean (may be NULL) receives the mean |k| = 2 pi |m| per shell, nmodes
 * (may be NULL) the number of modes; empty shells give 0. Host outputs of nbins
 * entries (1 .. 1024); the call synchronises the stream. n must be a power of two. */
int pm_power_spectrum(pm_ctx *ctx, const float *rho, int deconv, int nbins, double *pk,
                      double *kmean, int64_t *nmodes, pm_stream stream);

/* ------------------------------------------------------------------ batched ensembles
 * Many independent periodic boxes of different grid sizes advanced together
 * (the paper's purpose is large suites of simulations; introduction and
 * conclusions). Box b has an n[b]^3 grid and np[b] particles in box units; the
 * caller packs the particle arrays of all boxes into pos, vel, acc of
 * [sum np][3] (box b at rows p_off[b] .. p_off[b+1]) and the potentials into
 * phi of [sum n^3] (box b at c_off[b], row-major [n][n][n]); pm_batch_layout
 * returns both offset tables (exclusive prefix sums). Every stage of a step is
 * one launch for the whole batch: the kernels walk work lists of (box, block)
 * items with a persistent grid. The multigrid solve runs a fixed number of
 * V-cycles (mg.fixed_cycles >= 1; same smoother, restriction, prolongation and
 * coarsest-level solve as pm_solve_mg, levels halved down to at most 16 cells
 * per side), so a step never synchronises with the host and can be captured
 * as a graph. Deposit is the chunked form with its sums in 64-bit fixed point
 * (integer atomics into a per-cell fixed-point arena, then one conversion pass), so a
 * step is bitwise reproducible. The batch owns the density, fixed-point, force and
 * multigrid arenas (about 29 bytes per cell). */
typedef struct pm_batch pm_batch;

/* n[b]: even, 8 .. 1024, halving while > 16 and a multiple of 4 must end at <= 20;
 * np[b] >= 1. flags: 0. Errors: PM_ERR_ARG, PM_ERR_SHAPE, PM_ERR_NOMEM. */
int pm_batch_create(pm_batch **batch, int nboxes, const int *n, const int64_t *np, int flags);
void pm_batch_destroy(pm_batch *batch);
const char *pm_batch_last_error(const pm_batch *batch);
/* p_off[nboxes + 1], c_off[nboxes + 1] (host arrays) receive the packing offsets. */
int pm_batch_layout(const pm_batch *batch, int64_t *p_off, int64_t *c_off);

/* Accelerations of every box at scale factor a (deposit, solve with coef
 * 1.5 a Omega_m, 5-point gradient, interpolation). phi is the starting guess
 * when params->mg.guess is PM_GUESS_WARM(_RESCALED), else the Jacobi guess is
 * used; out: the potentials. relres (host, [nboxes], may be NULL) receives each
 * box's final ||f - L phi|| / ||f|| (the call then synchronises the stream). */
int pm_batch_accel(pm_batch *batch, const float *pos, float *acc, float *phi, double a,
                   const pm_step_params *params, double *relres, pm_stream stream);

/* nsteps kick-drift-kick steps a[i] -> a[i+1] (a: host array of nsteps + 1) of
 * every box, as pm_kdk does for one box; acc must hold the accelerations at
 * a[0] (pm_batch_accel) and phi the potentials (warm start). With
 * use_graph != 0 each step replays the graph recorded by pm_graph_capture_step
 * (same buffers and parameters required; at most 1024 steps per call). */
int pm_batch_kdk(pm_batch *batch, float *pos, float *vel, float *acc, float *phi, int nsteps,
                 const double *a, const pm_step_params *params, int use_graph,
                 pm_stream stream);

/* Record one batched step on `stream` (not the null stream) as a HIP graph for
 * pm_batch_kdk(..., use_graph = 1). The graph holds the buffer addresses and
 * the parameters; per-step scalars come from a device table that
 * pm_batch_kdk fills, indexed by a device step counter the graph advances.
 * The graph clears its grids with kernels (no memset nodes). */
int pm_graph_capture_step(pm_batch *batch, float *pos, float *vel, float *acc, float *phi,
                          const pm_step_params *params, pm_stream stream);

/* Autotuner for the stencil tile shapes of the batch (rows of the plane each
 * thread owns in the red-black smoother and in the gradient: 1, 2 or 4): times
 * every usable shape on the batch's own finest grids with HIP events and keeps
 * the fastest; choice (host, [2], may be NULL) receives the smoother and
 * gradient picks. pos supplies a density; phi is used as scratch and
 * overwritten. Drops a captured step graph (capture again afterwards). */
int pm_tune(pm_batch *batch, float *pos, float *phi, const pm_step_params *params, int *choice,
            pm_stream stream);

/* Per-kernel timing (measurement support). pm_kernel_timer(ctx, kernel, cap)
 * starts recording a pair of HIP events on the caller's stream around every
 * launch of one kernel (at most cap launches; resets the previous record):
 *   PM_KERNEL_DEPOSIT  the deposit kernels of PM_DEPOSIT_SORTED (the tile
 *                      pass and the gather pass, or the cell gather);
 *                      algorithmic bytes 12 per particle + 4 per cell
 *   PM_KERNEL_SMOOTH   the streaming smoother on the finest grid (n >= 256);
 *                      algorithmic bytes 12 per cell per red-black sweep (a pass
 *                      fuses two sweeps: 24 per cell), + 0.5 per cell for the
 *                      post-smoothing pass that adds the prolongation
 *   PM_KERNEL_INTERP   interpolation (+ kick) in pm_accel/pm_kdk/pm_kdk_chain;
 *                      algorithmic bytes 48 per particle (+4 with cell indices)
 *                      + 12 per cell (force grid), or + 4 per cell with the
 *                      gradient fused (sorted deposit on 8^3 tiles); in a chain,
 *                      52 per particle (+8 with cell indices) + 4 per cell
 *   PM_KERNEL_FR_SWEEP the f(R) non-linear Gauss-Seidel sweep on the finest grid
 *                      (both colours, FP64): algorithmic bytes 32 per cell (u read
 *                      by each colour's pass, s read and u written once)
 * pm_kernel_timer_read synchronises on the recorded events and returns the
 * summed elapsed time, the number of launches and the summed algorithmic
 * bytes; PM_WARN_NOT_CONVERGED if launches exceeded the pool. */
enum pm_kernel_id { PM_KERNEL_NONE = 0, PM_KERNEL_DEPOSIT = 1, PM_KERNEL_SMOOTH = 2,
                    PM_KERNEL_INTERP = 3, PM_KERNEL_FR_SWEEP = 4 };
int pm_kernel_timer(pm_ctx *ctx, int kernel, int capacity);
int pm_kernel_timer_read(pm_ctx *ctx, double *ms, int64_t *launches, double *bytes);

#ifdef __cplusplus
}
#endif
#endif /* HIPPM_H */
