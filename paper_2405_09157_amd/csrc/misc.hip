// Small non-iterative kernels: resuming a test from given running sums and
// the FP32 -> BF16 storage conversion.
#include <algorithm>

#include "mwu_kernels.hpp"

namespace scpmwu {

// Continue a test from given running sums: ybar = S / t.
__global__ __launch_bounds__(kBlock) void set_state_kernel(PassArgs a, int problem, int64_t t,
                                                           double S1, double S2) {
  __shared__ double s_red[kWavesPerBlock];
  DevState *st = a.st;
  const int d = (int)a.d;
  const int tid = threadIdx.x;
  double wn = 0.0;
  if (t > 0)
    for (int c = tid; c < d; c += kBlock) {
      const double y = a.vec[kVecS * d + c] / (double)t;
      a.vec[kVecMean * d + c] = y;
      wn += y * y;
    }
  wn = block_sum<kBlock>(wn, s_red);
  if (tid == 0) {
    st->t = t;
    if (problem == kSVM) {
      st->S1 = S1;
      st->S2 = S2;
      st->s1bar = t > 0 ? S1 / (double)t : 0.0;
      st->s2bar = t > 0 ? S2 / (double)t : 0.0;
      st->wbar_norm = sqrt(wn);
    }
  }
}

// FP32 -> BF16, round to nearest even; NaN stays NaN.
__global__ __launch_bounds__(kBlock) void cast_bf16_kernel(const float *src, uint16_t *dst, int64_t n,
                                                          int64_t d, int64_t ld_src, int64_t ld_dst) {
  const int64_t total = n * d;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * kBlock) {
    const int64_t r = i / d, c = i - r * d;
    const uint32_t b = __float_as_uint(src[r * ld_src + c]);
    uint32_t h;
    if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu) != 0u)
      h = (b >> 16) | 0x40u;
    else
      h = (b + 0x7FFFu + ((b >> 16) & 1u)) >> 16;
    dst[r * ld_dst + c] = (uint16_t)h;
  }
}

hipError_t launch_set_state_k(const PassArgs &a, int problem, int64_t t, double S1, double S2,
                              hipStream_t s) {
  hipLaunchKernelGGL(set_state_kernel, dim3(1), dim3(kBlock), 0, s, a, problem, t, S1, S2);
  return hipGetLastError();
}

hipError_t launch_cast(const float *src, uint16_t *dst, int64_t n, int64_t d, int64_t ld_src,
                       int64_t ld_dst, hipStream_t s) {
  const int64_t total = n * d;
  const int64_t blocks = std::min<int64_t>((total + kBlock - 1) / kBlock, 65536);
  hipLaunchKernelGGL(cast_bf16_kernel, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(kBlock), 0, s,
                     src, dst, n, d, ld_src, ld_dst);
  return hipGetLastError();
}

}  // namespace scpmwu
