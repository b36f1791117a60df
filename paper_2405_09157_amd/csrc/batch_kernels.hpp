// Batched smallest-enclosing-sphere problems: many independent SES instances
// advanced together, one launch per column layout for the streaming pass and
// one launch for all epilogues per MWU iteration.  Each instance keeps its own
// PassArgs (points, state, vectors, records); the per-instance arithmetic is
// exactly that of the single-problem kernels, whose bodies run here with a
// virtual workgroup index.
#pragma once

#include "mwu_kernels.hpp"

namespace scpmwu {

// Streaming pass: workgroup blockIdx.x runs tile tiles[blockIdx.x], i.e.
// workgroup vb of the vg workgroups of instance inst.  Tiles of an instance
// are contiguous and its vg records are written to its own record block.
template <typename T, int EPL, int VEC>
__global__ __launch_bounds__(kPassBlock) __attribute__((amdgpu_waves_per_eu(SCPMWU_PASS_WAVES)))
void ses_pass_batch_kernel(const PassArgs *__restrict__ args, const BatchTile *__restrict__ tiles) {
  const BatchTile tl = tiles[blockIdx.x];
  const PassArgs a = args[tl.inst];
  ses_pass_body<T, EPL, VEC, false, kPrefetchNone>(a, tl.vb, tl.vg);
}

// Epilogue of every instance (workgroup k sums instance k's nrec[k] records;
// an instance whose test has ended only reads its state).
template <typename T>
__global__ __launch_bounds__(kCombBlock) void epilogue_batch_kernel(const PassArgs *__restrict__ args,
                                                                    const int32_t *__restrict__ nrec) {
  const PassArgs a = args[blockIdx.x];
  epilogue_body<T, kSES, false>(a, nrec[blockIdx.x]);
}

// (Re)start the alpha-tests of the instances list[0 .. count) with params[j].
template <typename T>
__global__ __launch_bounds__(kBlock) void ftp_init_batch_kernel(const PassArgs *__restrict__ args,
                                                                const int32_t *__restrict__ list,
                                                                const InitParams *__restrict__ params) {
  const int j = blockIdx.x;
  const PassArgs a = args[list[j]];
  const InitParams p = params[j];
  ftp_init_body<T>(a, p, kSES);
}

// D of every instance: the largest distance from row v1 (binary64, on the
// stored values); a non-finite distance makes it +inf.  One workgroup per
// instance.
template <typename T>
__global__ __launch_bounds__(kBlock) void diameter_batch_kernel(const PassArgs *__restrict__ args,
                                                                double *__restrict__ D) {
  __shared__ double s_v1[kMaxD];
  __shared__ double s_red[kWavesPerBlock];
  const PassArgs a = args[blockIdx.x];
  const int d = (int)a.d, tid = threadIdx.x;
  for (int c = tid; c < d; c += kBlock) s_v1[c] = row_value<T>(a, a.v1, c);
  __syncthreads();
  double m = 0.0;
  for (int64_t i = tid; i < a.n; i += kBlock) {
    double s = 0.0;
    for (int c = 0; c < d; ++c) {
      const double df = row_value<T>(a, i, c) - s_v1[c];
      s = fma(df, df, s);
    }
    const double r = sqrt(s);
    m = fmax(m, isfinite(r) ? r : INFINITY);
  }
  m = wave_max(m);
  if ((tid & 63) == 0) s_red[tid >> 6] = m;
  __syncthreads();
  if (tid == 0) {
    double r = s_red[0];
    for (int w = 1; w < kWavesPerBlock; ++w) r = fmax(r, s_red[w]);
    D[blockIdx.x] = r;
  }
}

template <typename T, int EPL>
hipError_t launch_pass_batch_v(int vec, int ntiles, const PassArgs *args, const BatchTile *tiles, hipStream_t s) {
  constexpr int VF = (16 / (int)sizeof(T)) < EPL ? (16 / (int)sizeof(T)) : EPL;
  if (vec == VF) {
    hipLaunchKernelGGL((ses_pass_batch_kernel<T, EPL, VF>), dim3(ntiles), dim3(kPassBlock), 0, s, args, tiles);
    return hipGetLastError();
  }
  if constexpr (VF >= 4) {
    if (vec == VF / 2) {
      hipLaunchKernelGGL((ses_pass_batch_kernel<T, EPL, VF / 2>), dim3(ntiles), dim3(kPassBlock), 0, s, args, tiles);
      return hipGetLastError();
    }
  }
  if constexpr (VF > 1) {
    if (vec == 1) {
      hipLaunchKernelGGL((ses_pass_batch_kernel<T, EPL, 1>), dim3(ntiles), dim3(kPassBlock), 0, s, args, tiles);
      return hipGetLastError();
    }
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_pass_batch_typed(int epl, int vec, int ntiles, const PassArgs *args, const BatchTile *tiles,
                                   hipStream_t s) {
  switch (epl) {
    case 1: return launch_pass_batch_v<T, 1>(vec, ntiles, args, tiles, s);
    case 2: return launch_pass_batch_v<T, 2>(vec, ntiles, args, tiles, s);
    case 4: return launch_pass_batch_v<T, 4>(vec, ntiles, args, tiles, s);
    case 8: return launch_pass_batch_v<T, 8>(vec, ntiles, args, tiles, s);
    case 16: return launch_pass_batch_v<T, 16>(vec, ntiles, args, tiles, s);
    case 32: return launch_pass_batch_v<T, 32>(vec, ntiles, args, tiles, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_epilogue_batch_typed(int m, const PassArgs *args, const int32_t *nrec, hipStream_t s) {
  hipLaunchKernelGGL((epilogue_batch_kernel<T>), dim3(m), dim3(kCombBlock), 0, s, args, nrec);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_init_batch_typed(int count, const PassArgs *args, const int32_t *list, const InitParams *params,
                                   hipStream_t s) {
  hipLaunchKernelGGL((ftp_init_batch_kernel<T>), dim3(count), dim3(kBlock), 0, s, args, list, params);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_diameter_batch_typed(int m, const PassArgs *args, double *D, hipStream_t s) {
  hipLaunchKernelGGL((diameter_batch_kernel<T>), dim3(m), dim3(kBlock), 0, s, args, D);
  return hipGetLastError();
}

}  // namespace scpmwu
