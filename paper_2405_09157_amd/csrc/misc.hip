// Small non-iterative kernels: resuming a test from given running sums, the
// FP32 -> BF16 and FP32 -> FP8 (per-row scaled) storage conversions, and a
// plain streaming read of a buffer (the achievable-read-bandwidth reference
// the streaming pass is held to).
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

// Streaming read, no arithmetic on the data: each wave moves chunks of
// kReadChunk bytes into a two-stage LDS ring with buffer-to-LDS loads (16 B
// per lane), the next chunk in flight while the previous one is consumed.
// A resource per chunk bounds it (its tail reads zeros); nothing is written
// unless an impossible sum appears, so the loads cannot be elided.
constexpr int kReadU = 4;                      // 1 KB loads per chunk
constexpr int kReadChunk = kReadU * 1024;      // bytes per wave per stage
typedef __attribute__((address_space(3))) void lds_void_t;

__global__ __launch_bounds__(kPassBlock) void read_reference_kernel(const char *buf, int64_t bytes, float *sink) {
  __shared__ __attribute__((aligned(16))) float4 ring[kPassWaves * 2 * kReadU * 64];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int64_t nchunks = (bytes + kReadChunk - 1) / kReadChunk;
  const int64_t gw = (int64_t)gridDim.x * kPassWaves;
  float4 *mine = ring + wave * 2 * kReadU * 64;
  auto issue = [&](int64_t c, int stage) {
    const int64_t base = c * kReadChunk;
    const int64_t left = bytes - base;
    const __amdgpu_buffer_rsrc_t r = uniform_rsrc(buf + base, (int32_t)(left < kReadChunk ? left : kReadChunk));
#pragma unroll
    for (int u = 0; u < kReadU; ++u)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_void_t *)(mine + (stage * kReadU + u) * 64), 16,
                                               (unsigned)(lane * 16 + u * 1024), 0, 0, 0);
  };
  float acc = 0.f;
  int stage = 0;
  int64_t c = (int64_t)blockIdx.x * kPassWaves + wave;
  if (c < nchunks) issue(c, 0);
  for (; c < nchunks; c += gw) {
    __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0): this wave's chunk is in LDS
    __builtin_amdgcn_wave_barrier();
    float4 v[kReadU];
#pragma unroll
    for (int u = 0; u < kReadU; ++u) v[u] = mine[(stage * kReadU + u) * 64 + lane];
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the stage is free again
    if (c + gw < nchunks) issue(c + gw, stage ^ 1);
#pragma unroll
    for (int u = 0; u < kReadU; ++u) acc += v[u].x + v[u].y + v[u].z + v[u].w;
    stage ^= 1;
  }
  if (acc == 1.2345e-30f) sink[blockIdx.x & 15] = acc;
}

hipError_t launch_read_reference(const void *buf, int64_t bytes, int grid, float *sink, hipStream_t s) {
  hipLaunchKernelGGL(read_reference_kernel, dim3(grid), dim3(kPassBlock), 0, s, reinterpret_cast<const char *>(buf),
                     bytes, sink);
  return hipGetLastError();
}

// FP32 -> FP8 E4M3 code (sign, 4 exponent bits with bias 7, 3 mantissa
// bits, no infinities): round to nearest, ties to even; magnitudes from 464
// (the tie above the largest finite value 448) up saturate to 448; NaN gives
// 0x7F with its sign.
__device__ inline uint32_t fp8_encode(float v) {
  const uint32_t sign = (__float_as_uint(v) >> 24) & 0x80u;
  const float a = fabsf(v);
  uint32_t code;
  if (!(a == a)) {
    code = 0x7Fu;
  } else if (a >= 464.f) {
    code = 0x7Eu;
  } else if (a < 0.015625f) {
    // below the smallest normal 2^-6: multiples of 2^-9 (the scaling is exact)
    code = (uint32_t)rintf(a * 512.f);
  } else {
    const uint32_t ab = __float_as_uint(a);
    int e = (int)(ab >> 23) - 127;
    uint32_t m3 = (ab >> 20) & 7u;
    const uint32_t rem = ab & 0xFFFFFu;
    if (rem > 0x80000u || (rem == 0x80000u && (m3 & 1u))) ++m3;
    if (m3 == 8u) {
      m3 = 0u;
      ++e;
    }
    code = ((uint32_t)(e + 7) << 3) | m3;
    if (code > 0x7Eu) code = 0x7Eu;
  }
  return code | sign;
}

// Per-row scaled FP8 storage: one wave per row; the scale is the row's
// largest magnitude over 448 (binary32 division; 1 for an all-zero row), the
// codes encode x / scale (binary32 division).  Codes are stored with row
// stride d.
__global__ __launch_bounds__(kBlock) void quantize_fp8_kernel(const float *__restrict__ src, int64_t n, int64_t d,
                                                             int64_t ld, uint8_t *__restrict__ codes,
                                                             float *__restrict__ scales) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t r = (int64_t)blockIdx.x * kWavesPerBlock + wave; r < n; r += (int64_t)gridDim.x * kWavesPerBlock) {
    const float *row = src + r * ld;
    float m = 0.f;
    for (int64_t c = lane; c < d; c += kWave) m = fmaxf(m, fabsf(row[c]));
    m = (float)wave_max((double)m);
    const float sc = m > 0.f ? m / 448.f : 1.f;
    for (int64_t c = lane; c < d; c += kWave) codes[r * d + c] = (uint8_t)fp8_encode(row[c] / sc);
    if (lane == 0) scales[r] = sc;
  }
}

hipError_t launch_quantize_fp8(const float *src, int64_t n, int64_t d, int64_t ld, uint8_t *codes, float *scales,
                               hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((n + kWavesPerBlock - 1) / kWavesPerBlock, 65536);
  hipLaunchKernelGGL(quantize_fp8_kernel, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(kBlock), 0, s, src, n,
                     d, ld, codes, scales);
  return hipGetLastError();
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
