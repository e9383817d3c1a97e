// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/hippm.h"

#define PM_MAX_LEVELS 12

struct pm_level {
  int n;          // cells per side
  float *u;       // solution / error (level 0: caller's phi)
  float *f;       // right-hand side (level 0: NULL, the source is read from rho)
  float *alt;     // second buffer for the out-of-place streaming smoother (or NULL)
  float *res;     // residual scratch of the two-pass restriction (levels below streaming)
};

#ifndef PM_STREAM_MIN_N
#define PM_STREAM_MIN_N 128   // levels at least this large use the streaming kernels
#endif

// one grid of the f(R) full-approximation-storage hierarchy (FP64)
struct pm_fr_level {
  int n;
  double *u;   // iterate (level 0: the caller's or the context's scalaron)
  double *s;   // right-hand side
  double *u0;  // R u of the finer grid (levels > 0)
  double *d;   // residual scratch
  double *alt; // second iterate buffer of the streaming sweeps (levels of >= 256 cells)
};

struct pm_ctx {
  int n;
  int64_t np_max;
  int flags;
  int device;
  std::string err;
  // grids
  float *rho;            // [n^3] density scratch (pm_accel / pm_kdk)
  float *g;              // [n^3 * 3] acceleration grid scratch
  // multigrid hierarchy (level 0 fields are the caller's)
  int nlevels;
  pm_level lev[PM_MAX_LEVELS];
  // reductions
  double *red_partial;   // [RED_MAX_BLOCKS * 2]
  double *red_result;    // [4] device: {sum0, sum1, mean, spare}
  double *host_result;   // pinned [4]
  float *mean_f;         // [4] device: [0] FP32 mean of the current source grid,
                         // [1] mean of the solve's final iterate (gauge), [2] mean of the
                         // FFT solve's input
  // FFT spectrum (lazy)
  void *spec;            // complex float [n][n][fft_pitch(n)]
  void *spec2;           // three spectra of the Fourier-space force (lazy)
  float2 *twiddle;       // [n] e^{-2 pi i m / n}, m = 0 .. n-1
  float *fft_tab;        // [3n] per-axis tables: k^2 part, window part, k_d
  // counting sort (lazy)
  int32_t *cell_count;   // [n^3 + 1] counts -> starts -> ends (end of c = start of c + 1)
  int32_t *perm;         // [np_max] particle indices bucketed by cell
  int32_t *pcell;        // [np_max] cell of each particle
  int32_t *scan_partial; // [SCAN_MAX_BLOCKS]
  int64_t sort_cap;
  void *reorder_tmp;     // [np_max * 12 bytes] permutation staging (lazy)
  float *tile_box;       // [n^3 / 512][10^3] tile boxes of the sorted deposit (lazy)
  bool hist_ready;       // tile histogram and keys of the current positions already made
  // a chained step's fused drift leaves the next sort's tile histogram in cell_count2
  // and its keys in pcell, valid for the particle arrays it names until they move
  int32_t *cell_count2;  // [n^3 / 512 + 1]
  bool hist_next;
  const void *hist_pos, *hist_cell;
  int64_t hist_np;
  int64_t reorder_cap;
  // reverse mode (lazy)
  float *adj_gbar;       // [n^3 * 3] cotangent of the force grid
  float *adj_phibar;     // [n^3] cotangent of the potential
  float *adj_rhobar;     // [n^3] cotangent of the density: the last adjoint solve's result
  bool adj_warm;         // adj_rhobar holds a solve result (multigrid warm start)
  double adj_coef;       // source coefficient of that solve
  // QUMOND (lazy): the Newtonian potential (kept as the next solve's warm start) and the
  // MOND source
  float *mond_phin;      // [n^3]
  float *mond_src;       // [n^3]
  bool mond_valid;       // mond_phin holds a solution
  // f(R) (lazy): the FAS levels, the scalaron's u of the force evaluations (kept as the
  // next one's starting guess) and the potential of the force
  int fr_nlev;
  pm_fr_level fr_lev[PM_MAX_LEVELS];
  double *fr_u;          // [n^3]
  float *fr_phi;         // [n^3] phi_N - (c~^2 / 2) f~
  bool fr_valid;         // fr_u holds a result
  // extrapolated warm start (lazy): the potential of the solve before the last one on
  // the phi array ex_phi, and the scale factors of those two solves
  float *ex_prev;        // [n^3]
  const float *ex_phi;
  double ex_a_prev, ex_a_cur;
  bool ex_has_prev;
  // timing events
  hipEvent_t ev[8];
  // per-kernel timer: event pairs around every launch of one kernel
  int kt_kernel;
  int kt_cap, kt_used;
  hipEvent_t *kt_ev;     // [2 * kt_cap]
  double kt_bytes;       // algorithmic bytes of the recorded launches
  int64_t kt_dropped;    // launches beyond the pool (not timed)
};

// kernel-timer hooks (api.hip): bracket one launch of `kernel` on stream s
void pm_kt_begin(pm_ctx *ctx, int kernel, hipStream_t s);
void pm_kt_end(pm_ctx *ctx, int kernel, hipStream_t s, double bytes);

// Workgroups are dispatched round-robin over the 8 XCDs of an MI355X, each with its
// own L2. Remapping the block index so that every XCD walks a contiguous range of
// logical blocks keeps spatial neighbours (shared halos, planes) in the same L2.
__device__ __forceinline__ unsigned xcd_block(unsigned bid, unsigned nblocks) {
  const unsigned x = bid & 7u, k = bid >> 3;
  const unsigned per = nblocks >> 3, rem = nblocks & 7u;
  return x * per + (x < rem ? x : rem) + k;
}

#define RED_BLOCKS 1024
#define RED_PARTIAL_CAP 65536  // partial-sum slots (smoother blocks or reduction blocks)
#define RED_THREADS 256

// ---------------------------------------------------------------- helpers
int pm_fail(pm_ctx *ctx, int code, const std::string &msg);
int pm_hip_check(pm_ctx *ctx, hipError_t e, const char *what);
#define PM_HIP(ctx, call)                                   \
  do {                                                      \
    hipError_t _e = (call);                                 \
    if (_e != hipSuccess) return pm_hip_check(ctx, _e, #call); \
  } while (0)

// ---------------------------------------------------------------- launchers
// particles.hip
hipError_t launch_deposit_atomic(const float *pos, const int32_t *cell, int64_t np, int poskind,
                                 int mas, int n, float mass, float *rho, hipStream_t s);
// keymode: 0 row-major cells, 2 tiles of 8^3 cells (n % 8 == 0);
// hist_done: the counts and keys were already made (by the fused kick-drift)
hipError_t launch_sort_by_cell(pm_ctx *ctx, const float *pos, const int32_t *cell, int64_t np,
                               int poskind, hipStream_t s, int keymode, bool hist_done = false);
// second level of the tile-major cell sort: the tile buckets left by keymode 2 ordered
// by cell within each tile; out[i] = particle at place i (n % 8 == 0)
hipError_t launch_tile_cell_sort(pm_ctx *ctx, const float *pos, const int32_t *cell,
                                 int poskind, int32_t *out, hipStream_t s);
// arrays[i] = arrays[order[i]] for every array given (NULL: skipped)
hipError_t launch_apply_perm(pm_ctx *ctx, const int32_t *order, float *pos, int32_t *cell,
                             float *vel, float *acc, int64_t *ids, int64_t np, hipStream_t s);
hipError_t launch_deposit_pull(pm_ctx *ctx, const float *pos, int64_t np, int poskind, int mas,
                               float mass, float *rho, hipStream_t s);
hipError_t launch_deposit_own(pm_ctx *ctx, const float *pos, const int32_t *cell, int poskind,
                              int mas, float mass, float *rho, float *mean, hipStream_t s);
// interpolation (+ kick) through the tile buckets left by the sorted deposit of the
// same positions (n % 8 == 0)
hipError_t launch_interp_tile(pm_ctx *ctx, const float *pos, const int32_t *cell, int poskind,
                              int mas, const float *g, float *acc, float *vel, float kick,
                              hipStream_t s);
// the same with the 5-point gradient of phi formed per tile in LDS (no force grid);
// with count != NULL the kicked particles also drift by dt, and their new tile keys
// (pcell) and tile histogram (count, zeroed by the caller) are those of the next sort;
// acc may be NULL (not written)
hipError_t launch_interp_tile_phi(pm_ctx *ctx, float *pos, int32_t *cell, int poskind, int mas,
                                  const float *phi, float *acc, float *vel, float kick, float dt,
                                  int32_t *pcell, int32_t *count, hipStream_t s);
hipError_t launch_interp(const float *pos, const int32_t *cell, int64_t np, int poskind, int mas,
                         int n, const float *g, float *acc, float *vel, float kick,
                         hipStream_t s);
hipError_t launch_kick_drift(float *pos, int32_t *cell, float *vel, const float *acc, int64_t np,
                             int poskind, int n, float kick, float dt, hipStream_t s,
                             int32_t *pcell = nullptr, int32_t *count = nullptr);

// adjoint.hip
hipError_t launch_deposit_vjp(const float *pos, const int32_t *cell, int64_t np, int poskind,
                              int mas, int n, const float *rho_bar, float scale, float *pos_bar,
                              hipStream_t s);
hipError_t launch_interp_vjp(const float *pos, const int32_t *cell, int64_t np, int poskind,
                             int mas, int n, const float *g, const float *lam, float pscale,
                             float gscale, float *g_bar, float *pos_bar, hipStream_t s);
// the same through the 8^3-tile buckets (end, perm) of a tile sort of these positions
// (n % 8 == 0)
hipError_t launch_interp_vjp_tile(const float *pos, const int32_t *cell, int64_t np, int poskind,
                                  int mas, int n, const int32_t *end, const int32_t *perm,
                                  const float *g, const float *lam, float pscale, float gscale,
                                  float *g_bar, float *pos_bar, hipStream_t s);
hipError_t launch_divergence(const float *gb, int n, int points, bool accumulate, float *phib,
                             hipStream_t s);
hipError_t launch_axpy(float *y, const float *x, float alpha, int64_t count, hipStream_t s);
hipError_t launch_fill(float *y, float value, int64_t count, hipStream_t s);
hipError_t launch_density_loss(float *rho, const float *w, int64_t count, double *partial,
                               double *result, hipStream_t s);
hipError_t launch_ic_state(const float *q, const float *psi, int64_t np, int n, float vfac,
                           float *pos, int32_t *cell, float *vel, hipStream_t s);
hipError_t launch_ic_vjp(const float *xbar, const float *vbar, int64_t np, float vfac,
                         float *psibar, hipStream_t s);

// grid.hip
hipError_t launch_gradient(const float *phi, int n, int points, float *g, hipStream_t s);
hipError_t launch_sum_moments(const float *x, int64_t count, double *partial, double *result,
                              float *mean_out, hipStream_t s);
// phi = c1 phi + c2 prev and prev = the old phi, per cell
hipError_t launch_extrapolate(float *phi, float *prev, int64_t count, float c1, float c2,
                              hipStream_t s);
// *out += number of non-finite values of x[0 .. count)
hipError_t launch_count_nonfinite(const float *x, int64_t count, unsigned long long *out,
                                  hipStream_t s);

// mg.hip
// rho_mean_ready: ctx->mean_f[0] already holds the mean of rho (the sorted deposit's
// gather pass sums its exact fixed-point values), so the solve does not re-read rho
int pm_mg_solve(pm_ctx *ctx, const float *rho, float coef, float *phi, const pm_mg_params *p,
                pm_mg_stats *stats, hipStream_t s, float warm_scale = 1.0f,
                bool rho_mean_ready = false);
int pm_mg_setup(pm_ctx *ctx);

// mg_stream.hip
int64_t smooth_stream_blocks(int n);
// partial != NULL: the pass also sums ||f - L u||^2, ||f||^2 and sum u of its input,
// three doubles per block; uscale multiplies the input as it is read; ec != NULL (not
// with partial): the input is uin + P ec, the trilinear prolongation of the coarse
// correction ec ((n/2)^3) added as each plane is read
hipError_t launch_smooth_stream(const float *uin, float *uout, const float *f, float fscale,
                                const float *fmean, int n, float h2, float omega,
                                int first_colour, int half_sweeps, double *partial,
                                float uscale, const float *ec, hipStream_t s);
// residual + restriction in one streaming pass; with ucg != NULL also the coarse
// starting guess ucg = gscale * fc
hipError_t launch_rr_stream(const float *u, const float *f, float fscale, const float *fmean,
                            int n, float inv_h2, int kind, float *fc, float *ucg, float gscale,
                            hipStream_t s);

// gravity.hip: background of matter, curvature and a cosmological constant
double pm_bg_tau(double omega_m, double omega_l, double a0, double a1);   // supercomoving time
double pm_bg_growth(double omega_m, double omega_l, double a);            // D(a), any normalisation
double pm_bg_coef(const pm_step_params *p, double a);       // (3/2) Omega_m a mu(a)
double pm_bg_warm_scale(const pm_step_params *p, double a0, double a1);  // a1 D1 / (a0 D0)
// fr.hip: f(R) scalaron by non-linear multigrid (FP64)
int pm_fr_solve(pm_ctx *ctx, const float *rho, double a, const pm_step_params *p, double *u,
                double *relres, hipStream_t s);
// the scalaron of a force evaluation (ctx->fr_u, from the previous one when warm) and
// ctx->fr_phi = phin - (c~^2 / 2) f~
int pm_fr_force_potential(pm_ctx *ctx, const float *rho, double a, const pm_step_params *p,
                          bool warm, const float *phin, hipStream_t s);
void pm_fr_free(pm_ctx *ctx);
// QUMOND source div[nu(|grad phi_N| / g0) grad phi_N] on cell faces (n^3 grids)
hipError_t launch_qumond_source(const float *phin, int n, float g0, int family, float param,
                                float *out, hipStream_t s);

// fft.hip
struct FftBufs {
  float2 *spec, *spec2;  // half spectra [n][n][fft_pitch(n)] (spec2: three, PM_FFT_FULL only)
  float2 *twiddle;       // [n]
  float *tab;            // [3n]
};
#ifndef PM_FFT_TL
#define PM_FFT_TL 4096  // complex elements an FFT workgroup holds in LDS
#endif
// row pitch of the half spectrum: n/2 + 1 columns rounded up to a whole column tile
// (PM_FFT_TL / n columns)
constexpr int fft_pitch_of(int n) {
  return ((n / 2 + 1 + PM_FFT_TL / n - 1) / (PM_FFT_TL / n)) * (PM_FFT_TL / n);
}
int fft_pitch(int n);
size_t fft_spec_elems(int n);
// kind: a pm_fft_kernel; out: phi [n^3] (PM_FFT_GREEN, PM_FFT_7PT) or g [n^3 * 3] (PM_FFT_FULL);
// mean (device, may be NULL): subtracted from rho before the transform
hipError_t fft_run(const FftBufs &b, int n, const float *rho, const float *mean, float coef,
                   int deconv, int kind, float *out, hipStream_t s);
// separate passes over one grid: the twiddles and tables of b for an n^3 grid; the
// forward transform of the real grid x (mean subtracted when given) into b.spec (full
// half spectrum, unnormalised); the inverse of b.spec (consumed) into out[(p * stride) +
// comp] (unnormalised: no 1 / n^3)
hipError_t fft_tables(const FftBufs &b, int n, int deconv, int kind, hipStream_t s);
hipError_t fft_forward(const FftBufs &b, int n, const float *x, const float *mean, hipStream_t s);
hipError_t fft_inverse(const FftBufs &b, int n, float *out, int stride, int comp, hipStream_t s);
// mean: the device mean of rho when known (the sorted deposit's), else computed here
int pm_fft_solve(pm_ctx *ctx, const float *rho, float coef, int deconv, float *phi,
                 hipStream_t s, const float *mean = nullptr);
int pm_fft_solve_kind(pm_ctx *ctx, const float *rho, float coef, int deconv, int kind, float *out,
                      hipStream_t s, const float *mean = nullptr);
int64_t scan_blocks_needed(int64_t len);
