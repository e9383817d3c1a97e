// FFT Poisson solvers of paper Sect. 3.8:
//   FFT      phi = IDFT[ G(k) DFT[rho] ], G = -coef / (k^2 W(k)^2), W = prod_d sinc(k_d h/2)^p;
//   FFT_7pt  the same with the seven-point eigenvalue (4/h^2) sum_d sin^2(k_d h/2) in place
//            of k^2 and no deconvolution;
//   FULL_FFT the force g = -grad phi taken in Fourier space, g_d = IDFT[-i k_d G DFT[rho]]
//            (Eq. exact_fullfft_kernel), with k_d = 0 on the Nyquist plane of axis d.
//
// Layout: the half spectrum is kept as complex float spec[i][j][kc],
// kc = 0 .. n/2, row pitch P (a multiple of the column-tile width).
// Five passes over HBM, each a batch of 1D transforms staged in LDS:
//   A  rows along k, real -> half complex (length-n/2 complex FFT + split)
//   B  columns along j, forward
//   C  columns along i: forward, multiply by G, inverse (one kernel)
//   D  columns along j, inverse
//   E  rows along k, half complex -> real
// (FULL_FFT: C stores G F; then per force component the i pass multiplies by -i k_d
// and inverts into a spectrum of its own, followed by D; one E pass over the three
// spectra writes whole (x, y, z) cells.)
// The 1D transforms are Stockham autosort radix-4 (+ one radix-2) stages
// with twiddles from a table computed in FP64 on the device.
#include <cmath>

#include "internal.h"

namespace {

#ifndef PM_FFT_THREADS
#define PM_FFT_THREADS 256
#endif
constexpr int FT = PM_FFT_THREADS;  // threads per block
constexpr int TL = PM_FFT_TL;       // complex elements held in LDS per block

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
// The mean of x (mean != NULL) is subtracted as it is read: the k = 0 mode is dropped by
// every kernel anyway, and a large mean would otherwise set the scale of the FP32
// rounding of every other mode (a density of mean 1 with fluctuations of 0.3 loses
// about a factor 1 / 0.3 in relative accuracy at 512^3).
__global__ __launch_bounds__(FT) void k_rows_r2c(const float *__restrict__ x,
                                                 float2 *__restrict__ spec, int n, int P,
                                                 const float2 *__restrict__ tw,
                                                 const float *__restrict__ mean) {
  __shared__ float2 buf[TL];
  const int L = n / 2, T = TL / L;
  const int64_t rows = (int64_t)n * n;
  const int64_t row0 = (int64_t)blockIdx.x * T;
  const float mu = mean ? *mean : 0.0f;
  for (int e = threadIdx.x; e < TL; e += FT) {
    const int col = e / L, m = e % L;
    const int64_t row = row0 + col;
    float2 v = make_float2(0.f, 0.f);
    if (row < rows) {
      v = reinterpret_cast<const float2 *>(x + row * n)[m];
      v.x -= mu;
      v.y -= mu;
    }
    buf[e] = v;
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
// The output element of row r and position m goes to x[(r n + m) * stride + comp]
// (stride 1: a scalar grid; stride 3: one component of a vector grid). With ncomp > 1
// the block also takes the same rows of the next spectra (cstride elements apart) into
// components comp + 1 ..: the components of a cell are written close together in time,
// so the interleaved grid's cache lines are whole when they leave L2.
__global__ __launch_bounds__(FT) void k_rows_c2r(const float2 *__restrict__ spec0,
                                                 float *__restrict__ x, int n, int P,
                                                 const float2 *__restrict__ tw, int stride,
                                                 int comp0, int ncomp, int64_t cstride) {
  __shared__ float2 buf[TL];
  const int L = n / 2, T = TL / L;
  const int64_t rows = (int64_t)n * n;
  const int64_t row0 = (int64_t)blockIdx.x * T;
  for (int d = 0; d < ncomp; ++d) {
    const float2 *__restrict__ spec = spec0 + d * cstride;
    const int comp = comp0 + d;
    if (d > 0) __syncthreads();  // the previous component's reads of buf are done
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
    if (stride == 1) {
      for (int e = threadIdx.x; e < TL; e += FT) {
        const int col = e / L, m = e % L;
        const int64_t row = row0 + col;
        if (row < rows) reinterpret_cast<float2 *>(x + row * n)[m] = buf[e];
      }
    } else {
      for (int e = threadIdx.x; e < 2 * TL; e += FT) {
        const int col = e / n, m = e % n;   // m: real position along the row
        const int64_t row = row0 + col;
        if (row < rows) {
          const float2 v = buf[col * L + (m >> 1)];
          x[(row * n + m) * stride + comp] = (m & 1) ? v.y : v.x;
        }
      }
    }
  }
}

// Passes B, C, D: length-n transforms along j (AXIS 1) or i (AXIS 0) over a tile of
// T consecutive kc columns, from src to dst (the same buffer, or not). MODE:
//   0 forward; 1 forward, times G, inverse; 2 inverse; 3 forward, times G;
//   4 times -i k_d, inverse (d = deriv: 0 the i axis, 1 the j axis, 2 the k axis).
// G(mx, my, kz) = -scale / ((t0[mx] + t0[my] + t0[kz]) t1[mx] t1[my] t1[kz]) with the
// per-axis tables t0 = tab[0 .. n), t1 = tab[n .. 2n); k_d = tab[2n + m_d].
template <int AXIS, int MODE>
__global__ __launch_bounds__(FT) void k_cols(const float2 *src, float2 *dst, int n, int P,
                                             const float2 *__restrict__ tw,
                                             const float *__restrict__ tab, float scale,
                                             int deriv) {
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
    buf[e] = src[gidx(idx, col)];
  }
  __syncthreads();
  if constexpr (MODE == 0 || MODE == 1 || MODE == 3) lds_fft<false, false>(buf, L, T, tw, 1);
  if constexpr (MODE == 1 || MODE == 3) {
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
  }
  if constexpr (MODE == 4) {
    // AXIS 0 pass: the element (idx = mx, col) sits at (mx, my = outer, kz = kc0 + col)
    const float *kv = tab + 2 * n;
    const int my = outer;
    for (int e = threadIdx.x; e < TL; e += FT) {
      const int mx = e / T, kz = kc0 + e % T;
      const float k = kv[deriv == 0 ? mx : (deriv == 1 ? my : min(kz, n - 1))];
      const float2 v = buf[e];
      buf[e] = make_float2(k * v.y, -k * v.x);  // (-i k) v
    }
    __syncthreads();
  }
  if constexpr (MODE == 1 || MODE == 2 || MODE == 4) lds_fft<true, false>(buf, L, T, tw, 1);
  for (int e = threadIdx.x; e < TL; e += FT) {
    const int idx = e / T, col = e % T;
    dst[gidx(idx, col)] = buf[e];
  }
}

// Length-256 column passes (n = 256) as a four-step transform in registers: a length-256
// DFT is 16 DFTs of length 16 over the stride-16 subsequences, twiddles W_256^(j k1),
// a transpose through LDS and 16 DFTs of length 16 again. A column is handled by 16
// threads; thread j holds the elements j, j + 16, ... before a transform and the
// elements j, j + 16, ... of the result after it, which is also the input order of the
// next transform, so a pass with the kernel between the forward and the inverse
// transform needs two transposes. The same tile of 16 columns and the same modes and
// tables as k_cols.
// 16-point DFT in registers, natural order in and out: a radix-4 pass over the four
// stride-4 subsequences, twiddles W_16^(n2 k1), a radix-4 pass across them.
__device__ __forceinline__ float2 w16(int m, bool inv) {
  // e^{-2 pi i m / 16} (forward), its conjugate (inverse), m = 0 .. 9
  constexpr float c[10] = {1.0f, 0.92387953251128674f, 0.70710678118654752f,
                           0.38268343236508977f, 0.0f, -0.38268343236508977f,
                           -0.70710678118654752f, -0.92387953251128674f, -1.0f,
                           -0.92387953251128674f};
  constexpr float sn[10] = {0.0f, 0.38268343236508977f, 0.70710678118654752f,
                            0.92387953251128674f, 1.0f, 0.92387953251128674f,
                            0.70710678118654752f, 0.38268343236508977f, 0.0f,
                            -0.38268343236508977f};
  return make_float2(c[m], inv ? sn[m] : -sn[m]);
}

template <bool INV>
__device__ __forceinline__ void dft16(float2 (&x)[16]) {
  float2 y[4][4];  // y[n2][k1]: DFT over n1 of x[4 n1 + n2]
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    float2 v[4] = {x[n2], x[4 + n2], x[8 + n2], x[12 + n2]};
    butterfly<4, INV>(v);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) y[n2][k1] = (n2 * k1 == 0) ? v[k1] : cmul(v[k1], w16(n2 * k1, INV));
  }
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 v[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
    butterfly<4, INV>(v);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) x[k1 + 4 * k2] = v[k2];
  }
}

constexpr int kC256Pad = 17;  // LDS row of 16 values plus one (bank spread)

// x: this thread's 16 inputs (elements j + 16 n1 of its column, in order of n1); out:
// elements j + 16 k2 of the transform (thread j of the column, c its column in the tile)
template <bool INV>
__device__ __forceinline__ void fft256_cols(float2 (&x)[16], float2 *lds, int c, int j,
                                            const float2 *__restrict__ tw) {
  dft16<INV>(x);  // x[k1] = DFT over n1 of the subsequence j
#pragma unroll
  for (int k1 = 1; k1 < 16; ++k1) {
    float2 t = tw[j * k1];
    if (INV) t.y = -t.y;
    x[k1] = cmul(x[k1], t);
  }
  __syncthreads();  // the previous transpose's reads are done
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) lds[(c * 16 + k1) * kC256Pad + j] = x[k1];
  __syncthreads();
#pragma unroll
  for (int n2 = 0; n2 < 16; ++n2) x[n2] = lds[(c * 16 + j) * kC256Pad + n2];
  dft16<INV>(x);  // x[k2] = element j + 16 k2
}

template <int AXIS, int MODE>
__global__ __launch_bounds__(FT) void k_cols256(const float2 *src, float2 *dst, int P,
                                                const float2 *__restrict__ tw,
                                                const float *__restrict__ tab, float scale,
                                                int deriv) {
  constexpr int n = 256, T = 16;
  static_assert(FT == T * 16, "16 threads per column");
  __shared__ float2 lds[T * 16 * kC256Pad];
  const int c = threadIdx.x & 15, j = threadIdx.x >> 4;
  const int kc0 = blockIdx.x * T;
  const int outer = blockIdx.y;
  auto gidx = [&](int idx) -> int64_t {
    if constexpr (AXIS == 1)
      return ((int64_t)outer * n + idx) * P + kc0 + c;
    else
      return ((int64_t)idx * n + outer) * P + kc0 + c;
  };
  float2 x[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) x[q] = src[gidx(j + 16 * q)];
  if constexpr (MODE == 4) {
    // (-i k_d) v before the inverse transform; element j + 16 q sits at mx = j + 16 q
    const float *kv = tab + 2 * n;
    const int kz = kc0 + c;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int mx = j + 16 * q;
      const float k = kv[deriv == 0 ? mx : (deriv == 1 ? outer : min(kz, n - 1))];
      x[q] = make_float2(k * x[q].y, -k * x[q].x);
    }
  }
  if constexpr (MODE == 0 || MODE == 1 || MODE == 3) fft256_cols<false>(x, lds, c, j, tw);
  if constexpr (MODE == 1 || MODE == 3) {
    const float *t0 = tab, *t1 = tab + n;
    const int my = outer, kz = kc0 + c;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int mx = j + 16 * q;
      float gval = 0.0f;
      if (kz <= n / 2 && (mx | my | kz) != 0)
        gval = -scale / ((t0[mx] + t0[my] + t0[kz]) * (t1[mx] * t1[my] * t1[kz]));
      x[q] = make_float2(x[q].x * gval, x[q].y * gval);
    }
  }
  if constexpr (MODE == 1 || MODE == 2 || MODE == 4) fft256_cols<true>(x, lds, c, j, tw);
#pragma unroll
  for (int q = 0; q < 16; ++q) dst[gidx(j + 16 * q)] = x[q];
}

// 8-point DFT in registers, natural order in and out (radix 4 over the two stride-2
// subsequences, twiddles W_8^(n2 k1), radix 2 across)
template <bool INV>
__device__ __forceinline__ void dft8(float2 (&x)[8]) {
  constexpr float h = 0.70710678118654752f;
  float2 v0[4] = {x[0], x[2], x[4], x[6]}, v1[4] = {x[1], x[3], x[5], x[7]};
  butterfly<4, INV>(v0);
  butterfly<4, INV>(v1);
  // W_8^k1 for k1 = 1, 2, 3 (forward e^{-i pi k1 / 4}; inverse conjugate)
  const float s = INV ? 1.0f : -1.0f;
  v1[1] = cmul(v1[1], make_float2(h, s * h));
  v1[2] = make_float2(-s * v1[2].y, s * v1[2].x);  // times (0, s)
  v1[3] = cmul(v1[3], make_float2(-h, s * h));
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    x[k1] = cadd(v0[k1], v1[k1]);
    x[k1 + 4] = csub(v0[k1], v1[k1]);
  }
}

// In-place length-128 transforms of the 32 rows of buf (row r at r * kRowPitch128,
// natural order in and out), as 16 x 8 four-step transforms: thread t = 0 .. 7 of a row
// takes the 16-point DFT of the stride-8 subsequence t, the twiddles W_128^(t k1), and
// after a transpose the two 8-point DFTs of k1 = t and t + 8. tw is the table of n = 256
// (W_128^m = tw[2 m]).
constexpr int kRowPitch128 = 132;  // 128 values plus 4 (spreads the rows over the banks)

template <bool INV>
__device__ __forceinline__ void fft128_rows(float2 *buf, const float2 *__restrict__ tw) {
  const int r = threadIdx.x >> 3, t = threadIdx.x & 7;
  float2 *row = buf + r * kRowPitch128;
  float2 x[16];
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) x[n1] = row[8 * n1 + t];
  dft16<INV>(x);
#pragma unroll
  for (int k1 = 1; k1 < 16; ++k1) {
    float2 w = tw[2 * t * k1];
    if (INV) w.y = -w.y;
    x[k1] = cmul(x[k1], w);
  }
  __syncthreads();
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) row[k1 * 8 + t] = x[k1];
  __syncthreads();
  float2 a[8], b[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    a[j] = row[t * 8 + j];
    b[j] = row[(t + 8) * 8 + j];
  }
  dft8<INV>(a);
  dft8<INV>(b);
  __syncthreads();
#pragma unroll
  for (int k2 = 0; k2 < 8; ++k2) {
    row[t + 16 * k2] = a[k2];
    row[t + 8 + 16 * k2] = b[k2];
  }
  __syncthreads();
}

// k_rows_r2c for n = 256 (32 rows per block) with the register transform
__global__ __launch_bounds__(FT) void k_rows_r2c256(const float *__restrict__ x,
                                                    float2 *__restrict__ spec, int P,
                                                    const float2 *__restrict__ tw,
                                                    const float *__restrict__ mean) {
  constexpr int n = 256, L = 128, T = 32;
  static_assert(FT == T * 8, "8 threads per row");
  __shared__ float2 buf[T * kRowPitch128];
  const int64_t rows = (int64_t)n * n;
  const int64_t row0 = (int64_t)blockIdx.x * T;
  const float mu = mean ? *mean : 0.0f;
  for (int e = threadIdx.x; e < T * L; e += FT) {
    const int col = e / L, m = e % L;
    const int64_t row = row0 + col;
    float2 v = make_float2(0.f, 0.f);
    if (row < rows) {
      v = reinterpret_cast<const float2 *>(x + row * n)[m];
      v.x -= mu;
      v.y -= mu;
    }
    buf[col * kRowPitch128 + m] = v;
  }
  __syncthreads();
  fft128_rows<false>(buf, tw);
  for (int e = threadIdx.x; e < T * (L + 1); e += FT) {
    const int col = e / (L + 1), k = e % (L + 1);
    const int64_t row = row0 + col;
    if (row >= rows) continue;
    const float2 *b = buf + col * kRowPitch128;
    const float2 zk = b[k == L ? 0 : k];
    const float2 zm = conjf2(b[k == 0 ? 0 : L - k]);
    const float2 E = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y + zm.y));
    const float2 D = csub(zk, zm);
    const float2 O = make_float2(0.5f * D.y, -0.5f * D.x);  // -i D / 2
    spec[row * P + k] = cadd(E, cmul(tw[k], O));
  }
}

// k_rows_c2r for n = 256 with the register transform
__global__ __launch_bounds__(FT) void k_rows_c2r256(const float2 *__restrict__ spec0,
                                                    float *__restrict__ x, int P,
                                                    const float2 *__restrict__ tw, int stride,
                                                    int comp0, int ncomp, int64_t cstride) {
  constexpr int n = 256, L = 128, T = 32;
  __shared__ float2 buf[T * kRowPitch128];
  const int64_t rows = (int64_t)n * n;
  const int64_t row0 = (int64_t)blockIdx.x * T;
  for (int d = 0; d < ncomp; ++d) {
    const float2 *__restrict__ spec = spec0 + d * cstride;
    const int comp = comp0 + d;
    if (d > 0) __syncthreads();  // the previous component's reads of buf are done
    // the rows' half spectra (L + 1 values each) read once, coalesced, then Z~ formed from
    // X_k and X_{L-k} in LDS
    for (int e = threadIdx.x; e < T * (L + 1); e += FT) {
      const int col = e / (L + 1), k = e % (L + 1);
      const int64_t row = row0 + col;
      buf[col * kRowPitch128 + k] = row < rows ? spec[row * P + k] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    constexpr int kPer = T * L / FT;
    float2 z[kPer];
  #pragma unroll
    for (int it = 0; it < kPer; ++it) {
      const int e = threadIdx.x + it * FT, col = e / L, k = e % L;
      const float2 *b = buf + col * kRowPitch128;
      const float2 xk = b[k];
      const float2 xm = conjf2(b[L - k]);
      const float2 Et = cadd(xk, xm);
      const float2 Ot = cmul(conjf2(tw[k]), csub(xk, xm));
      z[it] = make_float2(Et.x - Ot.y, Et.y + Ot.x);  // Et + i Ot
    }
    __syncthreads();
  #pragma unroll
    for (int it = 0; it < kPer; ++it) {
      const int e = threadIdx.x + it * FT, col = e / L, k = e % L;
      buf[col * kRowPitch128 + k] = z[it];
    }
    __syncthreads();
    fft128_rows<true>(buf, tw);
    if (stride == 1) {
      for (int e = threadIdx.x; e < T * L; e += FT) {
        const int col = e / L, m = e % L;
        const int64_t row = row0 + col;
        if (row < rows) reinterpret_cast<float2 *>(x + row * n)[m] = buf[col * kRowPitch128 + m];
      }
    } else {
      for (int e = threadIdx.x; e < 2 * T * L; e += FT) {
        const int col = e / n, m = e % n;  // m: real position along the row
        const int64_t row = row0 + col;
        if (row < rows) {
          const float2 v = buf[col * kRowPitch128 + (m >> 1)];
          x[(row * n + m) * stride + comp] = (m & 1) ? v.y : v.x;
        }
      }
    }
  }
}

// a column pass: the register four-step kernel for n = 256 (16-column tiles), the LDS
// Stockham kernel otherwise
template <int AXIS, int MODE>
void launch_cols(dim3 grid, hipStream_t s, const float2 *src, float2 *dst, int n, int P,
                 const float2 *tw, const float *tab, float scale, int deriv) {
  if (n == 256 && TL / n == 16)
    k_cols256<AXIS, MODE><<<grid, FT, 0, s>>>(src, dst, P, tw, tab, scale, deriv);
  else
    k_cols<AXIS, MODE><<<grid, FT, 0, s>>>(src, dst, n, P, tw, tab, scale, deriv);
}

// Twiddles tw[m] = e^{-2 pi i m / n} and the per-axis tables of the kernel, in FP64 on
// the device and rounded once. For wavenumber index i (m = i, or i - n above n/2):
//   kind 0 (Green's function with window deconvolution): t0 = k^2, k = 2 pi m (unit
//     box), t1 = sinc(omega/2)^(2 deconv), omega = k h = 2 pi m / n;
//   kind 1 (seven-point eigenvalue): t0 = (4 / h^2) sin^2(omega/2), t1 = 1;
//   kd = k, except 0 at the Nyquist index n/2 (the derivative of a self-conjugate mode).
__global__ void k_fft_tables(float2 *__restrict__ tw, float *__restrict__ tab, int n, int deconv,
                             int kind) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double sn, cs;
  sincospi(-2.0 * (double)i / (double)n, &sn, &cs);
  tw[i] = make_float2((float)cs, (float)sn);
  const int m = i < n / 2 ? i : i - n;
  const double half = (double)m / (double)n;  // omega / (2 pi)
  const double sh = sinpi(half);
  if (kind == 1) {
    tab[i] = (float)(4.0 * (double)n * n * sh * sh);
    tab[n + i] = 1.0f;
  } else {
    const double k = 2.0 * M_PI * (double)m;
    const double sinc = (m == 0) ? 1.0 : sh / (M_PI * half);
    tab[i] = (float)(k * k);
    tab[n + i] = (float)pow(sinc, 2.0 * deconv);
  }
  tab[2 * n + i] = (i == n / 2) ? 0.0f : (float)(2.0 * M_PI * (double)m);
}

}  // namespace

int fft_pitch(int n) { return fft_pitch_of(n); }

size_t fft_spec_elems(int n) { return (size_t)n * n * fft_pitch(n); }

hipError_t fft_run(const FftBufs &b, int n, const float *rho, const float *mean, float coef,
                   int deconv, int kind, float *out, hipStream_t s) {
  const int P = fft_pitch(n);
  const int Trow = TL / (n / 2), Tcol = TL / n;
  const unsigned row_blocks = (unsigned)(((int64_t)n * n + Trow - 1) / Trow);
  const dim3 col_grid(P / Tcol, n);
  const float scale = (float)((double)coef / ((double)n * n * n));
  float2 *spec = b.spec;
  k_fft_tables<<<(n + 255) / 256, 256, 0, s>>>(b.twiddle, b.tab, n, deconv,
                                               kind == PM_FFT_7PT ? 1 : 0);
  if (n == 256 && Trow == 32)
    k_rows_r2c256<<<row_blocks, FT, 0, s>>>(rho, spec, P, b.twiddle, mean);
  else
    k_rows_r2c<<<row_blocks, FT, 0, s>>>(rho, spec, n, P, b.twiddle, mean);
  launch_cols<1, 0>(col_grid, s, spec, spec, n, P, b.twiddle, b.tab, scale, 0);
  if (kind != PM_FFT_FULL) {
    launch_cols<0, 1>(col_grid, s, spec, spec, n, P, b.twiddle, b.tab, scale, 0);
    launch_cols<1, 2>(col_grid, s, spec, spec, n, P, b.twiddle, b.tab, scale, 0);
    if (n == 256 && Trow == 32)
      k_rows_c2r256<<<row_blocks, FT, 0, s>>>(spec, out, P, b.twiddle, 1, 0, 1, 0);
    else
      k_rows_c2r<<<row_blocks, FT, 0, s>>>(spec, out, n, P, b.twiddle, 1, 0, 1, 0);
    return hipGetLastError();
  }
  // force in Fourier space: spec <- G F once, then per component d the inverse of
  // -i k_d G F along i and j into spectrum d of spec2 (three spectra), and one row pass
  // over the three writing whole (x, y, z) cells of the force grid
  launch_cols<0, 3>(col_grid, s, spec, spec, n, P, b.twiddle, b.tab, scale, 0);
  const int64_t elems = (int64_t)fft_spec_elems(n);
  for (int d = 0; d < 3; ++d) {
    float2 *sd = b.spec2 + d * elems;
    launch_cols<0, 4>(col_grid, s, spec, sd, n, P, b.twiddle, b.tab, scale, d);
    launch_cols<1, 2>(col_grid, s, sd, sd, n, P, b.twiddle, b.tab, scale, 0);
  }
  if (n == 256 && Trow == 32)
    k_rows_c2r256<<<row_blocks, FT, 0, s>>>(b.spec2, out, P, b.twiddle, 3, 0, 3, elems);
  else
    k_rows_c2r<<<row_blocks, FT, 0, s>>>(b.spec2, out, n, P, b.twiddle, 3, 0, 3, elems);
  return hipGetLastError();
}

hipError_t fft_tables(const FftBufs &b, int n, int deconv, int kind, hipStream_t s) {
  k_fft_tables<<<(n + 255) / 256, 256, 0, s>>>(b.twiddle, b.tab, n, deconv, kind);
  return hipGetLastError();
}

hipError_t fft_forward(const FftBufs &b, int n, const float *x, const float *mean, hipStream_t s) {
  const int P = fft_pitch(n);
  const int Trow = TL / (n / 2), Tcol = TL / n;
  const unsigned row_blocks = (unsigned)(((int64_t)n * n + Trow - 1) / Trow);
  const dim3 col_grid(P / Tcol, n);
  if (n == 256 && Trow == 32)
    k_rows_r2c256<<<row_blocks, FT, 0, s>>>(x, b.spec, P, b.twiddle, mean);
  else
    k_rows_r2c<<<row_blocks, FT, 0, s>>>(x, b.spec, n, P, b.twiddle, mean);
  launch_cols<1, 0>(col_grid, s, b.spec, b.spec, n, P, b.twiddle, b.tab, 0.0f, 0);
  launch_cols<0, 0>(col_grid, s, b.spec, b.spec, n, P, b.twiddle, b.tab, 0.0f, 0);
  return hipGetLastError();
}

hipError_t fft_inverse(const FftBufs &b, int n, float *out, int stride, int comp, hipStream_t s) {
  const int P = fft_pitch(n);
  const int Trow = TL / (n / 2), Tcol = TL / n;
  const unsigned row_blocks = (unsigned)(((int64_t)n * n + Trow - 1) / Trow);
  const dim3 col_grid(P / Tcol, n);
  launch_cols<0, 2>(col_grid, s, b.spec, b.spec, n, P, b.twiddle, b.tab, 0.0f, 0);
  launch_cols<1, 2>(col_grid, s, b.spec, b.spec, n, P, b.twiddle, b.tab, 0.0f, 0);
  if (n == 256 && Trow == 32)
    k_rows_c2r256<<<row_blocks, FT, 0, s>>>(b.spec, out, P, b.twiddle, stride, comp, 1, 0);
  else
    k_rows_c2r<<<row_blocks, FT, 0, s>>>(b.spec, out, n, P, b.twiddle, stride, comp, 1, 0);
  return hipGetLastError();
}

int pm_fft_solve_kind(pm_ctx *ctx, const float *rho, float coef, int deconv, int kind, float *out,
                      hipStream_t s, const float *mean) {
  const int n = ctx->n;
  if (n < 8 || (n & (n - 1)) != 0)
    return pm_fail(ctx, PM_ERR_SHAPE, "FFT solver needs a power-of-two grid (8 .. 1024)");
  const size_t elems = fft_spec_elems(n);
  if (!ctx->spec) {
    if (hipMalloc(&ctx->spec, sizeof(float2) * elems) != hipSuccess ||
        hipMalloc(&ctx->twiddle, sizeof(float2) * n) != hipSuccess ||
        hipMalloc(&ctx->fft_tab, sizeof(float) * 3 * n) != hipSuccess)
      return pm_fail(ctx, PM_ERR_NOMEM, "FFT scratch allocation failed");
  }
  if (kind == PM_FFT_FULL && !ctx->spec2) {
    // three spectra: one per force component
    if (hipMalloc(&ctx->spec2, 3 * sizeof(float2) * elems) != hipSuccess) {
      ctx->spec2 = nullptr;
      return pm_fail(ctx, PM_ERR_NOMEM, "FFT scratch allocation failed");
    }
  }
  if (!mean) {
    // the mean of rho, subtracted before the transform
    PM_HIP(ctx, launch_sum_moments(rho, (int64_t)n * n * n, ctx->red_partial, ctx->red_result,
                                   ctx->mean_f + 2, s));
    mean = ctx->mean_f + 2;
  }
  FftBufs b{(float2 *)ctx->spec, (float2 *)ctx->spec2, ctx->twiddle, ctx->fft_tab};
  PM_HIP(ctx, fft_run(b, n, rho, mean, coef, deconv, kind, out, s));
  return PM_OK;
}

int pm_fft_solve(pm_ctx *ctx, const float *rho, float coef, int deconv, float *phi, hipStream_t s,
                 const float *mean) {
  return pm_fft_solve_kind(ctx, rho, coef, deconv, PM_FFT_GREEN, phi, s, mean);
}
