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

// The k-way search's KS tests over one point set (instances 0 .. KS-1 share
// the rows): each batch of rows is loaded once and every running test
// computes its own distances, weights and sums from the registers; test j's
// record goes to instance j's record block (workgroup vb of vg = gridDim.x).
template <int KS>
struct KwayPrologue {
  const PassArgs *args;
  __device__ __forceinline__ void pre() {}
  __device__ __forceinline__ PassIn post() { return state_pass_in(args[0]); }
  __device__ __forceinline__ PassIn slot(int j) { return state_pass_in(args[j]); }
};

template <typename T, int EPL, int VEC, int KS>
__global__ __launch_bounds__(kPassBlock) __attribute__((amdgpu_waves_per_eu(SCPMWU_PASS_WAVES)))
void ses_kway_batch_kernel(const PassArgs *__restrict__ args) {
  const PassArgs a = args[0];
  KwayPrologue<KS> pro{args};
  ses_pass_body<T, EPL, VEC, false, kPrefetchNone, KwayPrologue<KS>, KS>(a, (int)blockIdx.x, (int)gridDim.x, pro);
}

template <typename T, int EPL, int VEC>
hipError_t launch_kway_v(int ks, int grid, const PassArgs *args, hipStream_t s) {
  switch (ks) {
    case 2: hipLaunchKernelGGL((ses_kway_batch_kernel<T, EPL, VEC, 2>), dim3(grid), dim3(kPassBlock), 0, s, args); break;
    case 3: hipLaunchKernelGGL((ses_kway_batch_kernel<T, EPL, VEC, 3>), dim3(grid), dim3(kPassBlock), 0, s, args); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int EPL>
hipError_t launch_kway_e(int vec, int ks, int grid, const PassArgs *args, hipStream_t s) {
  constexpr int VF = (16 / (int)sizeof(T)) < EPL ? (16 / (int)sizeof(T)) : EPL;
  if (vec == VF) return launch_kway_v<T, EPL, VF>(ks, grid, args, s);
  if constexpr (VF >= 4) {
    if (vec == VF / 2) return launch_kway_v<T, EPL, VF / 2>(ks, grid, args, s);
  }
  if constexpr (VF > 1) {
    if (vec == 1) return launch_kway_v<T, EPL, 1>(ks, grid, args, s);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_kway_batch_typed(int epl, int vec, int ks, int grid, const PassArgs *args, hipStream_t s) {
  switch (epl) {
    case 1: return launch_kway_e<T, 1>(vec, ks, grid, args, s);
    case 2: return launch_kway_e<T, 2>(vec, ks, grid, args, s);
    case 4: return launch_kway_e<T, 4>(vec, ks, grid, args, s);
    case 8: return launch_kway_e<T, 8>(vec, ks, grid, args, s);
    default: return hipErrorInvalidValue;
  }
}

// Row-per-lane SES pass for instances with d <= DM <= 16 columns: every lane
// owns RL = 2 whole rows of a batch (a wave batch is 128 rows), so a row's
// squared distance is summed inside the lane and the binary64 chains of the
// per-row phase (sqrt, exp, expm1, division) of RL rows run side by side; the
// weighted sums are kept per lane and reduced once per workgroup.  Point sets
// only (no radii).  Arithmetic is binary64 per element for every storage
// type; with BF16 storage the weighted sums are taken about fl32(ubar), the
// origin its epilogue expects: summed about ubar and moved to fl32(ubar) once
// per lane, sum a_i (x_i - fl32(ubar)) = sum a_i (x_i - ubar) + (ubar -
// fl32(ubar)) sum a_i, which keeps a second copy of the mean out of the
// registers.  The record has the layout of ses_pass_body's.
template <typename T, int DM, int VEC>
__device__ __forceinline__ void ses_rows_body(const PassArgs &a, int vb, int vg) {
  static_assert(DM % VEC == 0 && DM <= 16, "row layout");
  constexpr int RL = 2;
  constexpr int NQ = DM / VEC;
  constexpr int B = kWave * RL;
  constexpr bool M32 = sizeof(T) <= 2;
  __shared__ double s_vec[kPassWaves][DM];
  __shared__ double s_sc[kPassWaves][8];

  DevState *st = a.st;
  const int32_t status0 = __builtin_amdgcn_readfirstlane(st->status);  // uniform over the instance
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t n = a.n, ld = a.ld;
  const int d = (int)a.d;
  const T *__restrict__ X = reinterpret_cast<const T *>(a.X);
  const double kappa = st->kscale * (double)st->t;
  const double Gb = st->shift_bound;
  const int64_t v1 = a.v1;
  double ub[DM], acc[DM];
#pragma unroll
  for (int c = 0; c < DM; ++c) {
    ub[c] = c < d ? a.vec[kVecMean * d + c] : 0.0;
    acc[c] = 0.0;
  }
  double asum = 0.0, bsum = 0.0, esum = 0.0, gmax = -INFINITY, fall = -INFINITY;

  const int64_t nb = (n + B - 1) / B;
  const int64_t GW = (int64_t)vg * kPassWaves;
  // byte offsets of lane row j's column chunks within a batch; chunks past
  // column d get an offset beyond any batch (read as zero)
  int32_t voff[RL][NQ];
#pragma unroll
  for (int j = 0; j < RL; ++j)
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      voff[j][q] = q * VEC < d ? (int32_t)(((int64_t)(lane + kWave * j) * ld + q * VEC) * (int64_t)sizeof(T))
                               : kOffInvalid;
  const int64_t b0 = (int64_t)vb * kPassWaves + wave;
  __syncthreads();
  for (int64_t b = b0; b < nb; b += GW) {
    const int64_t r0 = b * B;
    const int64_t rows = n - r0 < B ? n - r0 : B;
    const __amdgpu_buffer_rsrc_t rs = rows_rsrc<T>(X, r0, rows, ld, d);
    VecT<T, VEC> x[RL][NQ];
#pragma unroll
    for (int j = 0; j < RL; ++j)
#pragma unroll
      for (int q = 0; q < NQ; ++q) x[j][q] = buf_load<T, VEC>(rs, voff[j][q], 0);
    // the first batch's loads go out before the state word is waited on
    if (b == b0 && status0 != kRunning) return;
#pragma unroll
    for (int j = 0; j < RL; ++j) {
      double dsq = 0.0;
#pragma unroll
      for (int c = 0; c < DM; ++c) {
        const double df = to_f64(x[j][c / VEC].v[c % VEC]) - ub[c];
        dsq = fma(df, df, dsq);
      }
      const int64_t row = r0 + lane + kWave * j;
      const bool valid = row < n;
      const bool incl = valid && row != v1;
      // the cone exponential of ses_pass_body for a point (gamma_i = 0)
      const double di = sqrt(dsq);
      const double ep = exp(kappa * (di - Gb));
      const double om = -expm1(-2.0 * kappa * di);
      double aw = di > 0.0 ? ep * om / di : 2.0 * kappa * ep;
      double bw = ep * (2.0 - om);
      double ew = ep * om * di;
      if (!incl) aw = bw = ew = 0.0;
      asum += aw;
      bsum += bw;
      esum += ew;
      if (incl) gmax = fmax(gmax, di);
      if (valid) fall = fmax(fall, di);
#pragma unroll
      for (int c = 0; c < DM; ++c) {
        const double xv = to_f64(x[j][c / VEC].v[c % VEC]);
        acc[c] = fma(aw, M32 ? xv - ub[c] : xv, acc[c]);
      }
    }
  }
  if (status0 != kRunning) return;

  // ---- workgroup record: sums, maxima
#pragma unroll
  for (int c = 0; c < DM; ++c) {
    if constexpr (M32) acc[c] = fma(ub[c] - (double)(float)ub[c], asum, acc[c]);
    const double v = wave_sum(acc[c]);
    if (lane == 0) s_vec[wave][c] = v;
  }
  asum = wave_sum(asum);
  bsum = wave_sum(bsum);
  esum = wave_sum(esum);
  gmax = wave_max(gmax);
  fall = wave_max(fall);
  if (lane == 0) {
    s_sc[wave][0] = bsum;
    s_sc[wave][1] = esum;
    s_sc[wave][2] = 0.0;  // sum gamma_i b_i: no radii
    s_sc[wave][3] = 0.0;  // no certificate
    s_sc[wave][4] = asum;
    s_sc[wave][5] = gmax;
    s_sc[wave][6] = fall;
  }
  __syncthreads();
  double *rec = a.partials + (int64_t)vb * rec_width(d);
  const int dp = rec_dp(d);
  if (tid < d) rec[tid] = sum_waves(s_vec, tid);
  if (tid < 8) {
    double v;
    if (tid < 5)
      v = sum_waves(s_sc, tid);
    else if (tid < 7)
      v = max_waves(s_sc, tid);
    else
      v = -INFINITY;
    rec[dp + tid] = v;
  }
}

// With at most 4 columns per lane the kernel fits 128 VGPRs, i.e. four waves
// per SIMD (two workgroups per compute unit) to hide the per-row latency.
template <typename T, int DM, int VEC>
__global__ __launch_bounds__(kPassBlock) __attribute__((amdgpu_waves_per_eu(DM <= 4 ? 4 : SCPMWU_PASS_WAVES)))
void ses_rows_batch_kernel(const PassArgs *__restrict__ args, const BatchTile *__restrict__ tiles) {
  const BatchTile tl = tiles[blockIdx.x];
  const PassArgs a = args[tl.inst];
  ses_rows_body<T, DM, VEC>(a, tl.vb, tl.vg);
}

// Epilogue of every instance (workgroup k sums instance k's nrec[k] records;
// an instance whose test has ended only reads its state).
constexpr int kBatchEpiBlock = 256;
template <typename T>
__global__ __launch_bounds__(kBatchEpiBlock) void epilogue_batch_kernel(const PassArgs *__restrict__ args,
                                                                        const int32_t *__restrict__ nrec) {
  const PassArgs a = args[blockIdx.x];
  epilogue_body<T, kSES, false, kBatchEpiBlock>(a, nrec[blockIdx.x]);
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

template <typename T, int DM>
hipError_t launch_rows_batch_v(int vec, int ntiles, const PassArgs *args, const BatchTile *tiles, hipStream_t s) {
  constexpr int VF = (16 / (int)sizeof(T)) < DM ? (16 / (int)sizeof(T)) : DM;
  if (vec == VF) {
    hipLaunchKernelGGL((ses_rows_batch_kernel<T, DM, VF>), dim3(ntiles), dim3(kPassBlock), 0, s, args, tiles);
    return hipGetLastError();
  }
  if constexpr (VF >= 2) {
    if (vec == VF / 2) {
      hipLaunchKernelGGL((ses_rows_batch_kernel<T, DM, VF / 2>), dim3(ntiles), dim3(kPassBlock), 0, s, args, tiles);
      return hipGetLastError();
    }
  }
  if constexpr (VF > 2) {
    if (vec == 1) {
      hipLaunchKernelGGL((ses_rows_batch_kernel<T, DM, 1>), dim3(ntiles), dim3(kPassBlock), 0, s, args, tiles);
      return hipGetLastError();
    }
  }
  return hipErrorInvalidValue;
}

// Row-per-lane layout: dm = columns held per lane (2, 4, 8 or 16 >= d).
template <typename T>
hipError_t launch_rows_batch_typed(int dm, int vec, int ntiles, const PassArgs *args, const BatchTile *tiles,
                                   hipStream_t s) {
  switch (dm) {
    case 2: return launch_rows_batch_v<T, 2>(vec, ntiles, args, tiles, s);
    case 3:  // exactly three columns, one value per load
      if (vec != 1) return hipErrorInvalidValue;
      hipLaunchKernelGGL((ses_rows_batch_kernel<T, 3, 1>), dim3(ntiles), dim3(kPassBlock), 0, s, args, tiles);
      return hipGetLastError();
    case 4: return launch_rows_batch_v<T, 4>(vec, ntiles, args, tiles, s);
    case 8: return launch_rows_batch_v<T, 8>(vec, ntiles, args, tiles, s);
    case 16: return launch_rows_batch_v<T, 16>(vec, ntiles, args, tiles, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_epilogue_batch_typed(int m, const PassArgs *args, const int32_t *nrec, hipStream_t s) {
  hipLaunchKernelGGL((epilogue_batch_kernel<T>), dim3(m), dim3(kBatchEpiBlock), 0, s, args, nrec);
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
