// Allocation-free FFT Poisson solve (pm_solve_fft_noalloc): the same kernels as
// pm_solve_fft (fft.hip), with the spectrum and the tables in a statically sized
// device array instead of context scratch, for callers that cannot allocate.
#include <cmath>
#include <mutex>

#include "internal.h"

// pm_solve_fft_noalloc keeps its spectrum and tables in one statically sized device
// array (allocated with the code object, per device, until the process ends) instead
// of context scratch. Grids up to kNoAllocMaxN per side.
namespace {

constexpr int kNoAllocMaxN = 128;
constexpr int kNoAllocMaxDevices = 64;
// spectrum of the largest grid (smaller power-of-two grids need fewer elements), then n
// twiddles, 3n table floats, the partial sums of the mean (2 doubles per reduction
// block) and its result (4 doubles, then the FP32 mean), each part 256-byte aligned
// (32 float2)
constexpr size_t kNoAllocSpec = (size_t)kNoAllocMaxN * kNoAllocMaxN * fft_pitch_of(kNoAllocMaxN);
constexpr size_t kNoAllocRed = 2 * RED_BLOCKS + 32;
constexpr size_t kNoAllocElems = kNoAllocSpec + kNoAllocMaxN + 2 * kNoAllocMaxN + kNoAllocRed + 64;

static __device__ __align__(256) float2 scratch[kNoAllocElems];

// device address of `scratch` per device (the host-side name is only a stand-in)
float2 *g_scratch_addr[kNoAllocMaxDevices];
hipError_t g_scratch_status[kNoAllocMaxDevices];
std::once_flag g_scratch_once[kNoAllocMaxDevices];

size_t round_up32(size_t x) { return (x + 31) / 32 * 32; }

}  // namespace

extern "C" int pm_solve_fft_noalloc(const float *rho, int n, float coef, int deconv, float *phi,
                                    pm_stream stream) {
  if (!rho || !phi) return PM_ERR_ARG;
  if (deconv < 0 || deconv > 3) return PM_ERR_ARG;
  if (!std::isfinite(coef)) return PM_ERR_NONFINITE;
  if (n < 8 || n > kNoAllocMaxN || (n & (n - 1)) != 0) return PM_ERR_SHAPE;
  if (fft_spec_elems(n) > kNoAllocSpec) return PM_ERR_SHAPE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoAllocMaxDevices) return PM_ERR_HIP;
  std::call_once(g_scratch_once[dev], [dev]() {
    void *p = nullptr;
    g_scratch_status[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_addr[dev] = g_scratch_status[dev] == hipSuccess ? (float2 *)p : nullptr;
  });
  if (g_scratch_status[dev] != hipSuccess || !g_scratch_addr[dev]) return PM_ERR_HIP;
  float2 *base = g_scratch_addr[dev];
  const size_t tw_off = round_up32(fft_spec_elems(n));
  const size_t tab_off = tw_off + round_up32((size_t)n);
  const size_t red_off = tab_off + round_up32((3 * (size_t)n + 1) / 2);
  if (red_off + kNoAllocRed > kNoAllocElems) return PM_ERR_SHAPE;
  FftBufs b{base, nullptr, base + tw_off, reinterpret_cast<float *>(base + tab_off)};
  double *partial = reinterpret_cast<double *>(base + red_off);
  double *result = partial + 2 * RED_BLOCKS;
  float *mean = reinterpret_cast<float *>(result + 4);
  const hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_sum_moments(rho, (int64_t)n * n * n, partial, result, mean, s);
  if (e == hipSuccess) e = fft_run(b, n, rho, mean, coef, deconv, PM_FFT_GREEN, phi, s);
  return e == hipSuccess ? PM_OK : PM_ERR_HIP;
}
