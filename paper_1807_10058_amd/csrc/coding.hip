// Spectrum quantiser for block-wise volumetric coding (the application the
// paper motivates in Sec. I and Sec. V: FCC spectra of volume blocks are
// thresholded and quantised, and the blocks rebuilt by the inverse transform).
//
// For every complex coefficient X = (re, im):
//   keep  = re*re + im*im >= threshold^2      (FP32, each operation rounded once)
//   code  = keep ? (rint(re / step), rint(im / step)) : (0, 0), saturated to int16
//   Xq    = step * code                        (the dequantised coefficient)
// and the number of kept coefficients is added to a counter.  The operations
// are unfused single roundings so that any IEEE FP32 implementation takes the
// same decisions.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "fcc_dct.h"

namespace {

__device__ __forceinline__ int16_t sat16(float v) {
  return int16_t(fminf(fmaxf(v, -32768.0f), 32767.0f));
}

__global__ __launch_bounds__(256) void k_quantise(const float2* __restrict__ X, long long count, float thr2, float step,
                                                  short2* __restrict__ codes, float2* __restrict__ Xq,
                                                  unsigned long long* __restrict__ kept) {
  unsigned long long mine = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x) {
    const float2 v = X[i];
    const float m2 = __fadd_rn(__fmul_rn(v.x, v.x), __fmul_rn(v.y, v.y));
    short2 c = make_short2(0, 0);
    if (m2 >= thr2) {
      c.x = sat16(rintf(__fdiv_rn(v.x, step)));
      c.y = sat16(rintf(__fdiv_rn(v.y, step)));
      ++mine;
    }
    if (codes) codes[i] = c;
    if (Xq) Xq[i] = make_float2(__fmul_rn(step, float(c.x)), __fmul_rn(step, float(c.y)));
  }
  // wave sum, then one atomic per wave
  for (int off = 32; off > 0; off >>= 1) mine += __shfl_down(mine, off);
  if ((threadIdx.x & 63) == 0 && mine) atomicAdd(kept, mine);
}

__global__ void k_zero1(unsigned long long* p) { *p = 0ull; }

}  // namespace

extern "C" {

fcc_status fcc_spectrum_quantise(const void* X, long long count, float threshold, float step, void* codes, void* Xq,
                                 unsigned long long* kept, void* hip_stream) {
  if (!X || count < 0 || !kept || !(step > 0.0f) || !(threshold >= 0.0f) || !std::isfinite(step) ||
      !std::isfinite(threshold))
    return FCC_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(X) & 7u) || (reinterpret_cast<uintptr_t>(Xq) & 7u) ||
      (reinterpret_cast<uintptr_t>(codes) & 3u) || (reinterpret_cast<uintptr_t>(kept) & 7u))
    return FCC_ERR_INVALID_ARG;
  if (Xq == X) return FCC_ERR_UNSUPPORTED;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_zero1, dim3(1), dim3(1), 0, st, kept);
  if (count > 0) {
    const float thr2 = threshold * threshold;
    const long long blocks = std::min<long long>((count + 255) / 256, 8192);
    hipLaunchKernelGGL(k_quantise, dim3(unsigned(blocks)), dim3(256), 0, st, static_cast<const float2*>(X), count,
                       thr2, step, static_cast<short2*>(codes), static_cast<float2*>(Xq), kept);
  }
  return hipGetLastError() == hipSuccess ? FCC_OK : FCC_ERR_HIP;
}

}  // extern "C"
