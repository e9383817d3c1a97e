// FFT Poisson solver (paper Sect. 3.8, 'FFT' kernel with mass-assignment
// deconvolution, and the seven-point eigenvalue variant).
//
// phi = IDFT[ G(k) DFT[rho] ] with G = -coef / (k^2 W(k)^2), W = prod_d sinc(k_d h/2)^p.
//
// Layout: the half spectrum is kept as complex float spec[i][j][kc],
// kc = 0 .. n/2, row pitch P (a multiple of the column-tile width).
// Five passes over HBM, each a batch of 1D transforms staged in LDS:
//   A  rows along k, real -> half complex (length-n/2 complex FFT + split)
//   B  columns along j, forward
//   C  columns along i: forward, multiply by G, inverse (one kernel)
//   D  columns along j, inverse
//   E  rows along k, half complex -> real
// The 1D transforms are Stockham autosort radix-4 (+ one radix-2) stages
// with twiddles from an FP64-computed table.
#include <cmath>
#include <vector>

#include "internal.h"

namespace {

constexpr int FT = 256;   // threads per block
constexpr int TL = 4096;  // complex elements held in LDS per block

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }

template <int R, bool INV>
__device__ __forceinline__ void butterfly(float2 *v) {
  if constexpr (R == 2) {
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else {
    const float2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    const float2 a2 = cadd(v[1], v[3]), d = csub(v[1], v[3]);
    // forward: d * (-i); inverse: d * (+i)
    const float2 a3 = INV ? make_float2(-d.y, d.x) : make_float2(d.y, -d.x);
    v[0] = cadd(a0, a2);
    v[1] = cadd(a1, a3);
    v[2] = csub(a0, a2);
    v[3] = csub(a1, a3);
  }
}

// One Stockham stage on T independent length-L sequences in LDS.
// Element (col, idx) lives at col*L + idx (ROWS) or idx*T + col (!ROWS).
// Butterfly j of sub-transform size Ns: inputs x[j + r L/R], twiddle
// W_{Ns R}^{r (j mod Ns)}, outputs y[(j/Ns) Ns R + (j mod Ns) + r Ns].
template <int R, bool INV, bool ROWS>
__device__ __forceinline__ void fft_stage(float2 *buf, int L, int T, int Ns, int logNs,
                                          const float2 *__restrict__ tw, int twstep) {
  constexpr int PER = TL / (R * FT);
  const int nb = L / R;
  float2 v[PER][R];
  int jj[PER], cc[PER];
#pragma unroll
  for (int b = 0; b < PER; ++b) {
    const int w = threadIdx.x + b * FT;
    int j, col;
    if constexpr (ROWS) {
      j = w % nb;
      col = w / nb;
    } else {
      col = w % T;
      j = w / T;
    }
    jj[b] = j;
    cc[b] = col;
#pragma unroll
    for (int r = 0; r < R; ++r) v[b][r] = buf[ROWS ? col * L + j + r * nb : (j + r * nb) * T + col];
  }
  __syncthreads();
  const int step = (L / (Ns * R)) * twstep;
#pragma unroll
  for (int b = 0; b < PER; ++b) {
    const int j = jj[b], col = cc[b];
    const int k = j & (Ns - 1);
#pragma unroll
    for (int r = 1; r < R; ++r) {
      float2 t = tw[r * k * step];
      if (INV) t.y = -t.y;
      v[b][r] = cmul(v[b][r], t);
    }
    butterfly<R, INV>(v[b]);
    const int base = ((j >> logNs) << logNs) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int o = base + r * Ns;
      buf[ROWS ? col * L + o : o * T + col] = v[b][r];
    }
  }
  __syncthreads();
}

template <bool INV, bool ROWS>
__device__ void lds_fft(float2 *buf, int L, int T, const float2 *__restrict__ tw, int twstep) {
  int Ns = 1, logNs = 0;
  while (L / Ns >= 4) {
    fft_stage<4, INV, ROWS>(buf, L, T, Ns, logNs, tw, twstep);
    Ns *= 4;
    logNs += 2;
  }
  if (Ns < L) fft_stage<2, INV, ROWS>(buf, L, T, Ns, logNs, tw, twstep);
}

// Pass A: each row x[0..n) -> X[0..n/2]. z_m = x_{2m} + i x_{2m+1}, Z = FFT_{n/2}(z),
// E_k = (Z_k + conj Z_{n/2-k}) / 2, O_k = -i (Z_k - conj Z_{n/2-k}) / 2, X_k = E_k + w^k O_k.
__global__ __launch_bounds__(FT) void k_rows_r2c(const float *__restrict__ x,
                                                 float2 *__restrict__ spec, int n, int P,
                                                 const float2 *__restrict__ tw) {
  __shared__ float2 buf[TL];
  const int L = n / 2, T = TL / L;
  const int64_t rows = (int64_t)n * n;
  const int64_t row0 = (int64_t)blockIdx.x * T;
  for (int e = threadIdx.x; e < TL; e += FT) {
    const int col = e / L, m = e % L;
    const int64_t row = row0 + col;
    buf[e] = row < rows ? reinterpret_cast<const float2 *>(x + row * n)[m] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  lds_fft<false, true>(buf, L, T, tw, 2);
  for (int e = threadIdx.x; e < T * (L + 1); e += FT) {
    const int col = e / (L + 1), k = e % (L + 1);
    const int64_t row = row0 + col;
    if (row >= rows) continue;
    const float2 zk = buf[col * L + (k == L ? 0 : k)];
    const float2 zm = conjf2(buf[col * L + (k == 0 ? 0 : L - k)]);
    const float2 E = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y + zm.y));
    const float2 D = csub(zk, zm);
    const float2 O = make_float2(0.5f * D.y, -0.5f * D.x);  // -i D / 2
    spec[row * P + k] = cadd(E, cmul(tw[k], O));
  }
}

// Pass E: X[0..n/2] -> x[0..n). Z~_k = (X_k + conj X_{n/2-k}) + i conj(w^k) (X_k - conj X_{n/2-k}),
// z = unnormalised inverse FFT_{n/2}(Z~) = n (x_{2m} + i x_{2m+1}); the 1/n^3 is in G.
__global__ __launch_bounds__(FT) void k_rows_c2r(const float2 *__restrict__ spec,
                                                 float *__restrict__ x, int n, int P,
                                                 const float2 *__restrict__ tw) {
  __shared__ float2 buf[TL];
  const int L = n / 2, T = TL / L;
  const int64_t rows = (int64_t)n * n;
  const int64_t row0 = (int64_t)blockIdx.x * T;
  for (int e = threadIdx.x; e < TL; e += FT) {
    const int col = e / L, k = e % L;
    const int64_t row = row0 + col;
    float2 z = make_float2(0.f, 0.f);
    if (row < rows) {
      const float2 xk = spec[row * P + k];
      const float2 xm = conjf2(spec[row * P + (L - k)]);
      const float2 Et = cadd(xk, xm);
      const float2 Ot = cmul(conjf2(tw[k]), csub(xk, xm));
      z = make_float2(Et.x - Ot.y, Et.y + Ot.x);  // Et + i Ot
    }
    buf[e] = z;
  }
  __syncthreads();
  lds_fft<true, true>(buf, L, T, tw, 2);
  for (int e = threadIdx.x; e < TL; e += FT) {
    const int col = e / L, m = e % L;
    const int64_t row = row0 + col;
    if (row < rows) reinterpret_cast<float2 *>(x + row * n)[m] = buf[e];
  }
}

// Passes B, C, D: length-n transforms along j (AXIS 1) or i (AXIS 0) over a tile of
// T consecutive kc columns. MODE 0 forward, 1 forward * G then inverse, 2 inverse.
template <int AXIS, int MODE>
__global__ __launch_bounds__(FT) void k_cols(float2 *__restrict__ spec, int n, int P,
                                             const float2 *__restrict__ tw,
                                             const float *__restrict__ tab, float scale) {
  __shared__ float2 buf[TL];
  const int L = n, T = TL / n;
  const int kc0 = blockIdx.x * T;
  const int outer = blockIdx.y;
  auto gidx = [&](int idx, int col) -> int64_t {
    if constexpr (AXIS == 1)
      return ((int64_t)outer * n + idx) * P + kc0 + col;
    else
      return ((int64_t)idx * n + outer) * P + kc0 + col;
  };
  for (int e = threadIdx.x; e < TL; e += FT) {
    const int idx = e / T, col = e % T;
    buf[e] = spec[gidx(idx, col)];
  }
  __syncthreads();
  if constexpr (MODE == 2) {
    lds_fft<true, false>(buf, L, T, tw, 1);
  } else {
    lds_fft<false, false>(buf, L, T, tw, 1);
  }
  if constexpr (MODE == 1) {
    // G(mx, my, kz) = -scale / ((t0[mx] + t0[my] + t0[kz]) * t1[mx] * t1[my] * t1[kz])
    const float *t0 = tab, *t1 = tab + n;
    const int my = outer;
    for (int e = threadIdx.x; e < TL; e += FT) {
      const int mx = e / T, kz = kc0 + e % T;
      float gval = 0.0f;
      if (kz <= n / 2 && (mx | my | kz) != 0)
        gval = -scale / ((t0[mx] + t0[my] + t0[kz]) * (t1[mx] * t1[my] * t1[kz]));
      const float2 v = buf[e];
      buf[e] = make_float2(v.x * gval, v.y * gval);
    }
    __syncthreads();
    lds_fft<true, false>(buf, L, T, tw, 1);
  }
  for (int e = threadIdx.x; e < TL; e += FT) {
    const int idx = e / T, col = e % T;
    spec[gidx(idx, col)] = buf[e];
  }
}

}  // namespace

// kind 0: continuous Laplacian with window power `deconv`; kind 1: seven-point eigenvalue.
static int fft_prepare(pm_ctx *ctx, int deconv, int kind) {
  const int n = ctx->n;
  const int T = TL / n;
  if (!ctx->spec) {
    ctx->spec_pitch = ((n / 2 + 1 + T - 1) / T) * T;
    const size_t bytes = sizeof(float2) * (size_t)n * n * ctx->spec_pitch;
    if (hipMalloc(&ctx->spec, bytes) != hipSuccess)
      return pm_fail(ctx, PM_ERR_NOMEM, "FFT spectrum allocation failed");
    if (hipMemset(ctx->spec, 0, bytes) != hipSuccess)
      return pm_fail(ctx, PM_ERR_HIP, "FFT spectrum clear failed");
    std::vector<float2> tw(n);
    for (int m = 0; m < n; ++m) {
      const double ang = -2.0 * M_PI * (double)m / (double)n;
      tw[m] = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }
    if (hipMalloc(&ctx->twiddle, sizeof(float2) * n) != hipSuccess ||
        hipMalloc(&ctx->fft_tab, sizeof(float) * 2 * n) != hipSuccess)
      return pm_fail(ctx, PM_ERR_NOMEM, "FFT table allocation failed");
    if (hipMemcpy(ctx->twiddle, tw.data(), sizeof(float2) * n, hipMemcpyHostToDevice) != hipSuccess)
      return pm_fail(ctx, PM_ERR_HIP, "twiddle upload failed");
    ctx->fft_tab_key = -1;
  }
  const int key = kind * 16 + deconv;
  if (ctx->fft_tab_key != key) {
    std::vector<float> tab(2 * n);
    for (int i = 0; i < n; ++i) {
      const int m = i < n / 2 ? i : i - n;
      const double half = M_PI * (double)m / (double)n;  // omega / 2
      if (kind == 1) {
        const double s = std::sin(half);
        tab[i] = (float)(4.0 * (double)n * n * s * s);
        tab[n + i] = 1.0f;
      } else {
        const double k = 2.0 * M_PI * (double)m;
        const double sinc = (m == 0) ? 1.0 : std::sin(half) / half;
        tab[i] = (float)(k * k);
        tab[n + i] = (float)std::pow(sinc, 2.0 * deconv);
      }
    }
    if (hipMemcpy(ctx->fft_tab, tab.data(), sizeof(float) * 2 * n, hipMemcpyHostToDevice) !=
        hipSuccess)
      return pm_fail(ctx, PM_ERR_HIP, "Green table upload failed");
    ctx->fft_tab_key = key;
  }
  return PM_OK;
}

int pm_fft_solve_kind(pm_ctx *ctx, const float *rho, float coef, int deconv, int kind, float *phi,
                      hipStream_t s) {
  const int n = ctx->n;
  if (n < 8 || (n & (n - 1)) != 0)
    return pm_fail(ctx, PM_ERR_SHAPE, "FFT solver needs a power-of-two grid (8 .. 1024)");
  int st = fft_prepare(ctx, deconv, kind);
  if (st != PM_OK) return st;
  const int P = ctx->spec_pitch;
  float2 *spec = (float2 *)ctx->spec;
  const int Trow = TL / (n / 2), Tcol = TL / n;
  const unsigned row_blocks = (unsigned)(((int64_t)n * n + Trow - 1) / Trow);
  const dim3 col_grid(P / Tcol, n);
  const float scale = (float)((double)coef / ((double)n * n * n));
  k_rows_r2c<<<row_blocks, FT, 0, s>>>(rho, spec, n, P, ctx->twiddle);
  k_cols<1, 0><<<col_grid, FT, 0, s>>>(spec, n, P, ctx->twiddle, ctx->fft_tab, scale);
  k_cols<0, 1><<<col_grid, FT, 0, s>>>(spec, n, P, ctx->twiddle, ctx->fft_tab, scale);
  k_cols<1, 2><<<col_grid, FT, 0, s>>>(spec, n, P, ctx->twiddle, ctx->fft_tab, scale);
  k_rows_c2r<<<row_blocks, FT, 0, s>>>(spec, phi, n, P, ctx->twiddle);
  PM_HIP(ctx, hipGetLastError());
  return PM_OK;
}

int pm_fft_solve(pm_ctx *ctx, const float *rho, float coef, int deconv, float *phi, hipStream_t s) {
  return pm_fft_solve_kind(ctx, rho, coef, deconv, 0, phi, s);
}
