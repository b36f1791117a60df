// Streaming-pass kernels of the primal-dual symmetric-cone MWU iteration for
// SES (product of second-order cones) and SVM (orthant), gfx950.
//
// One launch = one MWU iteration t of the alpha-feasibility test (Section 3
// meta-algorithm): it reads the n x d point matrix once and, for every point,
//   SES  diff_i = v_i - ubar(t-1), d_i = ||diff_i||; the SOC block of the
//        cumulative loss -(eta (t-1)/rho)(ubar - v_i ; alpha - gamma_i)
//        (eq. implement) has spectral values
//        lambda_{+-} = kappa (+-d_i - alpha + gamma_i), kappa = eta (t-1)/(rho sqrt2),
//        (Section 2.1: (u0 +- ||u||)/sqrt2), and its Loewner exponential is
//        (1/sqrt2)((e+ - e-) diff_i/d_i ; e+ + e-) (Section 2.1, Loewner
//        extension).  The pass accumulates W = sum_{i != v1} a_i diff_i with
//        a_i = (e+ - e-)/d_i, the trace sum B = sum (e+ + e-), and the terms
//        of the ORACLE objective of eq.(ses_oracle);
//   SVM  slack_i = z_i.wbar - sbar_c(i) (z_i = +-x_i by class), weight
//        e_i = exp(-(eta (t-1)/rho) slack_i) (eq. min_implement on the
//        orthant), and the class sums A_P = sum_P e_i x_i, A_Q = sum_Q e_i x_i,
//        T1 = sum_P e_i, T2 = sum_Q e_i of eq.(svm_oracle);
// plus the f(t-1) monitor of Section 5 (max distance / class extremes).  The
// trace normaliser is never applied per point: every exponent is shifted by a
// bound M on its maximum carried from the previous iteration, which cancels
// in the ORACLE (a common factor) and is added back to ln C.
//
// Data flow inside a wavefront (64 lanes):
//   phase 1  lanes over columns: 16 lanes per row, EPL columns per lane,
//            4 rows per load step, SB steps per batch of B = 4*SB rows; the
//            per-lane FP64 partial of the row reduction goes to LDS;
//   phase 2  lanes over rows: lane j of the batch sums row j's 16 partials
//            and evaluates the cone exponential (one sqrt/exp/expm1 per row);
//            the row weight goes back to LDS;
//   phase 3  lanes over columns: weighted accumulation of the rows still held
//            in registers (one FMA per element).
// Workgroup partials are reduced by a two-level, fixed-order combine (the
// last finisher of each group of kGroup workgroups, then the last group),
// whose final workgroup runs the FP64 epilogue: ORACLE closed form, the
// separation test, the running mean and the early-exit rules.  All
// arithmetic on point data is binary64; results are bitwise reproducible for
// a fixed grid.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "mwu_common.hpp"

namespace scpmwu {

// ------------------------------------------------------------ element types
template <typename T>
__device__ __forceinline__ double to_f64(T x);
template <>
__device__ __forceinline__ double to_f64<float>(float x) {
  return (double)x;
}
template <>
__device__ __forceinline__ double to_f64<uint16_t>(uint16_t h) {
  return (double)__uint_as_float(((uint32_t)h) << 16);
}
template <>
__device__ __forceinline__ double to_f64<double>(double x) {
  return x;
}

template <typename T, int V>
struct alignas(sizeof(T) * V) VecT {
  T v[V];
};

// Type a row element is held in between the phases: binary32 holds F32 and
// BF16 storage exactly at half the registers of binary64.
template <typename T>
struct RegT {
  using type = float;
};
template <>
struct RegT<double> {
  using type = double;
};
template <typename T>
__device__ __forceinline__ typename RegT<T>::type to_reg(T x);
template <>
__device__ __forceinline__ float to_reg<float>(float x) {
  return x;
}
template <>
__device__ __forceinline__ float to_reg<uint16_t>(uint16_t h) {
  return __uint_as_float(((uint32_t)h) << 16);
}
template <>
__device__ __forceinline__ double to_reg<double>(double x) {
  return x;
}

// Occupancy target of the streaming pass (waves per SIMD): caps the
// register budget at 512 / target VGPRs so that enough waves are resident
// to keep loads in flight.
#ifndef SCPMWU_PASS_WAVES
#define SCPMWU_PASS_WAVES 2
#endif

// Batch shape: SB load steps of 4 rows; the batch's row data (SB * EPL
// elements per lane, 64 VGPRs) stays in registers through the three phases.
template <int EPL, int ESZ, int PROB = kSES>
struct Shape {
  // SVM keeps two binary64 class accumulators per column: half the batch.
  static constexpr int LIM = (ESZ == 8 ? 32 : 64) / (PROB == kSVM ? 2 : 1);
  static constexpr int SB = (LIM / EPL) < 8 ? ((LIM / EPL) > 0 ? LIM / EPL : 1) : 8;
  static constexpr int B = SB * kRowsPerStep;  // rows per batch (<= 32)
};

// Forces the compiler to keep x in its (narrow) register type across the
// per-row phase instead of caching its binary64 conversion: the widened copy
// of a whole batch would double the live registers.
template <typename R, int SB, int EPL>
__device__ __forceinline__ void opaque(R (&x)[SB][EPL]) {
#pragma unroll
  for (int s = 0; s < SB; ++s)
#pragma unroll
    for (int k = 0; k < EPL; ++k) asm volatile("" : "+v"(x[s][k]));
}

// Lanes of one wavefront exchange data through LDS only: DS instructions of a
// wave execute in order, so a compiler barrier is all that is needed.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m));
  return v;
}

// Fixed-order sum / max over the waves of a pass workgroup.
template <int W>
__device__ __forceinline__ double sum_waves(const double (*v)[W], int c) {
  double r = 0.0;
#pragma unroll
  for (int w = 0; w < kPassWaves; ++w) r += v[w][c];
  return r;
}
template <int W>
__device__ __forceinline__ double max_waves(const double (*v)[W], int c) {
  double r = -INFINITY;
#pragma unroll
  for (int w = 0; w < kPassWaves; ++w) r = fmax(r, v[w][c]);
  return r;
}

// Sum over a workgroup of NT threads; every thread must call it; all get the
// same value (fixed order).
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *s_red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) r += s_red[w];
  return r;
}

// Load one row's EPL columns owned by lane `cl` (zeros outside [0,n) x [0,d)).
template <typename T, int EPL, int VEC>
__device__ __forceinline__ void load_row(const T *__restrict__ X, int64_t row, int64_t n, int d,
                                         int64_t ld, int cl, VecT<T, VEC> (&raw)[EPL / VEC]) {
  const bool rv = row < n;
  const T *rp = X + row * ld + (int64_t)cl * EPL;
#pragma unroll
  for (int q = 0; q < EPL / VEC; ++q) {
    VecT<T, VEC> v;
#pragma unroll
    for (int e = 0; e < VEC; ++e) v.v[e] = T(0);
    if (rv && (cl * EPL + q * VEC) < d) v = *reinterpret_cast<const VecT<T, VEC> *>(rp + q * VEC);
    raw[q] = v;
  }
}

// Section 5 monitor for a mean evaluated by this pass (iteration k-1 >= 1).
// `better` means f improves on f_best; `beat` means f is already better than
// alpha.  Runs on one thread; returns the new status.
__device__ __forceinline__ int monitor_rules(DevState *st, int64_t k, double f, bool better,
                                             bool beat, int *copy_best) {
  int status = kRunning;
  st->f_last = f;
  if (!isfinite(f)) return kNumeric;
  if (better) {
    st->f_best = f;
    st->t_best = k - 1;
    *copy_best = 1;
  }
  if (st->early) {
    if (beat) {
      status = kBeat;
    } else {
      if (st->f_prev >= 0.0) {  // a previous monitored iteration exists
        if (st->f_prev > 0.0 && fabs(f - st->f_prev) / st->f_prev < st->delta)
          st->cnt += 1;
        else
          st->cnt = 0;
      }
      st->f_prev = f;
      if (st->cnt >= st->patience) status = kStabilized;
    }
  }
  if (status == kRunning && k - 1 >= st->T) status = kTReached;
  return status;
}

// =========================================================== SES pass
template <typename T, int NT>
__device__ void ses_epilogue(const PassArgs &a, const double *comb, bool cert, double *s_red,
                             int *s_int) {
  DevState *st = a.st;
  const int d = (int)a.d;
  const int tid = threadIdx.x;
  double *Sv = a.vec + kVecS * d;
  double *ybar = a.vec + kVecMean * d;
  double *best = a.vec + kVecBest * d;
  double *last = a.vec + kVecLast * d;
  const int64_t k = st->t + 1;  // iteration index of this pass
  const double Bsum = comb[2 * d + 0], Esum = comb[2 * d + 1], Gsum = comb[2 * d + 2];
  const double BD2 = comb[2 * d + 3], Asum = comb[2 * d + 4], gmax = comb[2 * d + 5];
  const double fall = comb[2 * d + 6];
  if (tid == 0) {
    int status = kRunning, copy = 0;
    if (k >= 2) status = monitor_rules(st, k, fall, fall < st->f_best, fall < st->alpha, &copy);
    s_int[0] = status;
    s_int[1] = copy;
  }
  __syncthreads();
  if (s_int[1])
    for (int c = tid; c < d; c += NT) best[c] = ybar[c];
  if (s_int[0] != kRunning) {
    if (tid == 0) {
      st->status = s_int[0];
      st->t_end = k - 1;
    }
    return;
  }
  // W = sum_i a_i (v_i - ubar) from the pass's sum a_i v_i and sum a_i.
  double Wr[(kMaxD + NT - 1) / NT];
  double p = 0.0;
#pragma unroll
  for (int j = 0; j < (kMaxD + NT - 1) / NT; ++j) {
    const int c = tid + j * NT;
    Wr[j] = c < d ? comb[c] - Asum * ybar[c] : 0.0;
    p += Wr[j] * Wr[j];
  }
  const double nW = sqrt(block_sum<NT>(p, s_red));
  const double alpha = st->alpha, g1 = st->gamma1;
  const T *v1 = reinterpret_cast<const T *>(a.X) + a.v1 * a.ld;
  double u[(kMaxD + NT - 1) / NT];
  double q = 0.0;
#pragma unroll
  for (int j = 0; j < (kMaxD + NT - 1) / NT; ++j) {
    const int c = tid + j * NT;
    u[j] = 0.0;
    if (c < d) {
      const double v1c = to_f64(v1[c]);
      u[j] = nW > 0.0 ? v1c + (alpha - g1) * (Wr[j] / nW) : v1c;
      q += (u[j] - ybar[c]) * Wr[j];
    }
  }
  // sum_i (u - v_i).w_i + (alpha - gamma_i) s_i, scaled by sqrt2 C e^{-M}:
  // (u - ubar).W - sum (e+ - e-) d_i + alpha sum b_i - sum gamma_i b_i.
  const double dotp = block_sum<NT>(q, s_red);
  const double obj = dotp - Esum + alpha * Bsum - Gsum;
  const double scale = alpha * (nW + Bsum);
  double lb2 = 0.0;
  if (cert) {
    double cc = 0.0;
    for (int c = tid; c < d; c += NT) {
      const double cv = comb[d + c] - Bsum * ybar[c];  // sum_i b_i (v_i - ubar)
      cc += cv * cv;
    }
    const double cn2 = block_sum<NT>(cc, s_red);
    lb2 = BD2 / Bsum - cn2 / (Bsum * Bsum);
  }
  const bool bad = !isfinite(obj) || !(Bsum > 0.0) || !isfinite(nW);
  const bool separated = obj < -st->tau * scale;
  if (tid == 0) {
    const double M = st->kscale * (double)st->t * (st->shift_bound - alpha);
    st->value = obj / (M_SQRT2 * Bsum);
    st->scale = scale / (M_SQRT2 * Bsum);
    st->log_trace = M + log(Bsum);
    st->degenerate = !(nW > 0.0);
    st->cert = cert ? 1 : 0;
    if (cert && a.radii == nullptr) st->bound = fmax(st->bound, sqrt(fmax(lb2, 0.0)));
  }
#pragma unroll
  for (int j = 0; j < (kMaxD + NT - 1) / NT; ++j) {
    const int c = tid + j * NT;
    if (c < d) last[c] = u[j];
  }
  if (bad || separated) {
    if (tid == 0) {
      st->status = bad ? kNumeric : kSeparated;
      st->t_end = k;
    }
    return;
  }
  double dl = 0.0;
#pragma unroll
  for (int j = 0; j < (kMaxD + NT - 1) / NT; ++j) {
    const int c = tid + j * NT;
    if (c < d) {
      const double s = Sv[c] + u[j];
      Sv[c] = s;
      const double yn = s / (double)k;
      const double dd = yn - ybar[c];
      dl += dd * dd;
      ybar[c] = yn;
    }
  }
  const double Delta = sqrt(block_sum<NT>(dl, s_red));
  if (tid == 0) {
    // ||v_i - ubar(k)|| <= ||v_i - ubar(k-1)|| + ||ubar(k) - ubar(k-1)||
    st->shift_bound = gmax + Delta;
    st->t = k;
  }
}

template <typename T, int EPL, int VEC, bool CERT>
__global__ __launch_bounds__(kPassBlock) __attribute__((amdgpu_waves_per_eu(SCPMWU_PASS_WAVES)))
void ses_pass_kernel(PassArgs a) {
  using Sh = Shape<EPL, (int)sizeof(typename RegT<T>::type)>;
  constexpr int SB = Sh::SB, B = Sh::B;
  __shared__ double s_part[kPassWaves][B][kG + 1];
  __shared__ double s_wa[kPassWaves][B];
  __shared__ double s_wb[kPassWaves][CERT ? B : 1];
  __shared__ double s_vec[kPassWaves][kG * EPL];
  __shared__ double s_sc[kPassWaves][8];

  DevState *st = a.st;
  if (st->status != kRunning) return;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, cl = lane & 15;
  const int64_t n = a.n, ld = a.ld;
  const int d = (int)a.d;
  const T *__restrict__ X = reinterpret_cast<const T *>(a.X);
  const double kappa = st->kscale * (double)st->t;
  const double Gb = st->shift_bound;
  const double *ybar = a.vec + kVecMean * d;
  const double *__restrict__ radii = a.radii;
  const int64_t v1 = a.v1;

  double ub[EPL];
#pragma unroll
  for (int k = 0; k < EPL; ++k) {
    const int c = cl * EPL + k;
    ub[k] = c < d ? ybar[c] : 0.0;
  }
  double wacc[EPL], cacc[CERT ? EPL : 1];
#pragma unroll
  for (int k = 0; k < EPL; ++k) wacc[k] = 0.0;
#pragma unroll
  for (int k = 0; k < (CERT ? EPL : 1); ++k) cacc[k] = 0.0;
  double asum = 0.0, bsum = 0.0, esum = 0.0, gsum = 0.0, bd2 = 0.0, gmax = -INFINITY, fall = -INFINITY;

  const int64_t nb = (n + B - 1) / B;
  const int64_t GW = (int64_t)gridDim.x * kPassWaves;
  for (int64_t b = (int64_t)blockIdx.x * kPassWaves + wave; b < nb; b += GW) {
    const int64_t r0 = b * B;
    using R = typename RegT<T>::type;
    R xs[SB][EPL];
#pragma unroll
    for (int s = 0; s < SB; ++s) {
      VecT<T, VEC> raw[EPL / VEC];
      load_row<T, EPL, VEC>(X, r0 + s * kRowsPerStep + g, n, d, ld, cl, raw);
#pragma unroll
      for (int q = 0; q < EPL / VEC; ++q)
#pragma unroll
        for (int e = 0; e < VEC; ++e) xs[s][q * VEC + e] = to_reg(raw[q].v[e]);
    }
#pragma unroll
    for (int s = 0; s < SB; ++s) {
      double dsq = 0.0;
#pragma unroll
      for (int k = 0; k < EPL; ++k) {
        const double df = (double)xs[s][k] - ub[k];
        dsq = fma(df, df, dsq);
      }
      s_part[wave][s * kRowsPerStep + g][cl] = dsq;
    }
    wave_lds_sync();
    if (lane < B) {
      double dsq = 0.0;
#pragma unroll
      for (int c = 0; c < kG; ++c) dsq += s_part[wave][lane][c];
      const int64_t row = r0 + lane;
      const bool valid = row < n;
      const bool incl = valid && row != v1;
      const double di = sqrt(dsq);
      const double gi = (valid && radii != nullptr) ? radii[row] : 0.0;
      const double h = di + gi;
      // shifted lambda_+ = kappa (h - alpha) - kappa (G - alpha) <= ~0
      const double ep = exp(kappa * (h - Gb));
      const double om = -expm1(-2.0 * kappa * di);  // 1 - e^{lambda_- - lambda_+}
      double aw = di > 0.0 ? ep * om / di : 2.0 * kappa * ep;
      double bw = ep * (2.0 - om);
      double ew = ep * om * di;
      if (!incl) aw = bw = ew = 0.0;
      asum += aw;
      bsum += bw;
      esum += ew;
      gsum += gi * bw;
      if (CERT) bd2 += bw * dsq;
      if (incl) gmax = fmax(gmax, h);
      if (valid) fall = fmax(fall, h);
      s_wa[wave][lane] = aw;
      if (CERT) s_wb[wave][lane] = bw;
    }
    wave_lds_sync();
    opaque(xs);
    // sum_i a_i x_i (and sum_i b_i x_i); the epilogue subtracts (sum a_i) ubar
#pragma unroll
    for (int s = 0; s < SB; ++s) {
      const double ar = s_wa[wave][s * kRowsPerStep + g];
#pragma unroll
      for (int k = 0; k < EPL; ++k) wacc[k] = fma(ar, (double)xs[s][k], wacc[k]);
      if (CERT) {
        const double br = s_wb[wave][s * kRowsPerStep + g];
#pragma unroll
        for (int k = 0; k < EPL; ++k) cacc[k] = fma(br, (double)xs[s][k], cacc[k]);
      }
    }
    wave_lds_sync();
  }

  // ---- workgroup record: W, C(cert), sums, maxima
#pragma unroll
  for (int k = 0; k < EPL; ++k) {
    wacc[k] += __shfl_xor(wacc[k], 16);
    wacc[k] += __shfl_xor(wacc[k], 32);
  }
  const int pw = partial_width(d);
  if (g == 0)
#pragma unroll
    for (int k = 0; k < EPL; ++k) s_vec[wave][cl * EPL + k] = wacc[k];
  asum = wave_sum(asum);
  bsum = wave_sum(bsum);
  esum = wave_sum(esum);
  gsum = wave_sum(gsum);
  bd2 = wave_sum(bd2);
  gmax = wave_max(gmax);
  fall = wave_max(fall);
  if (lane == 0) {
    s_sc[wave][0] = bsum;
    s_sc[wave][1] = esum;
    s_sc[wave][2] = gsum;
    s_sc[wave][3] = bd2;
    s_sc[wave][4] = asum;
    s_sc[wave][5] = gmax;
    s_sc[wave][6] = fall;
  }
  __syncthreads();
  double *rec = a.partials + (int64_t)blockIdx.x * pw;
  for (int c = tid; c < d; c += kPassBlock) rec[c] = sum_waves(s_vec, c);
  __syncthreads();
  if (CERT) {
#pragma unroll
    for (int k = 0; k < EPL; ++k) {
      cacc[k] += __shfl_xor(cacc[k], 16);
      cacc[k] += __shfl_xor(cacc[k], 32);
    }
    if (g == 0)
#pragma unroll
      for (int k = 0; k < EPL; ++k) s_vec[wave][cl * EPL + k] = cacc[k];
    __syncthreads();
    for (int c = tid; c < d; c += kPassBlock) rec[d + c] = sum_waves(s_vec, c);
  } else {
    for (int c = tid; c < d; c += kPassBlock) rec[d + c] = 0.0;
  }
  if (tid < 8) {
    double v;
    if (tid < 5)
      v = sum_waves(s_sc, tid);
    else if (tid < 7)
      v = max_waves(s_sc, tid);
    else
      v = -INFINITY;
    rec[2 * d + tid] = v;
  }
}

// =========================================================== SVM pass
template <typename T, int NT>
__device__ void svm_epilogue(const PassArgs &a, const double *comb, double *s_red, int *s_int) {
  DevState *st = a.st;
  const int d = (int)a.d;
  const int tid = threadIdx.x;
  double *Sv = a.vec + kVecS * d;
  double *wbar = a.vec + kVecMean * d;
  double *best = a.vec + kVecBest * d;
  double *last = a.vec + kVecLast * d;
  const int64_t k = st->t + 1;
  const double T1 = comb[2 * d + 0], T2 = comb[2 * d + 1];
  const double minP = -comb[2 * d + 4], maxQ = comb[2 * d + 5], slmin = -comb[2 * d + 6];
  if (tid == 0) {
    int status = kRunning, copy = 0;
    if (k >= 2) {
      const double nw = st->wbar_norm;
      const double f = nw > 0.0 ? fmax((minP - maxQ) / nw, 0.0) : 0.0;
      status = monitor_rules(st, k, f, f > st->f_best, f > st->alpha, &copy);
    }
    s_int[0] = status;
    s_int[1] = copy;
  }
  __syncthreads();
  if (s_int[1])
    for (int c = tid; c < d; c += NT) best[c] = wbar[c];
  if (s_int[0] != kRunning) {
    if (tid == 0) {
      st->status = s_int[0];
      st->t_end = k - 1;
    }
    return;
  }
  // ORACLE of eq.(svm_oracle): w = V/||V||, V = P mu - Q gamma.
  const double *AP = comb, *AQ = comb + d;
  double p = 0.0, pu = 0.0;
  const bool both = T1 > 0.0 && T2 > 0.0;
  for (int c = tid; c < d; c += NT) {
    const double V = AP[c] - AQ[c];
    p += V * V;
    if (both) {
      const double U = AP[c] / T1 - AQ[c] / T2;
      pu += U * U;
    }
  }
  const double nV = sqrt(block_sum<NT>(p, s_red));
  const double ub = both ? sqrt(block_sum<NT>(pu, s_red)) : INFINITY;
  const double alpha = st->alpha, D = st->D;
  const double s1 = (T1 <= T2) ? D : alpha - D;
  const double s2 = alpha - s1;
  const double obj = nV - T1 * s1 - T2 * s2;
  const double scale = nV + T1 * fabs(s1) + T2 * fabs(s2);
  const bool bad = !isfinite(obj) || !(T1 + T2 > 0.0);
  const bool separated = obj < -st->tau * scale;
  if (tid == 0) {
    const double M = -st->kscale * (double)st->t * st->shift_bound;
    st->value = obj / (T1 + T2);
    st->scale = scale / (T1 + T2);
    st->log_trace = M + log(T1 + T2);
    st->degenerate = !(nV > 0.0);
    st->bound = fmin(st->bound, ub);
    st->s1_last = s1;
    st->s2_last = s2;
  }
  double w[(kMaxD + NT - 1) / NT];
#pragma unroll
  for (int j = 0; j < (kMaxD + NT - 1) / NT; ++j) {
    const int c = tid + j * NT;
    w[j] = 0.0;
    if (c < d) {
      w[j] = nV > 0.0 ? (AP[c] - AQ[c]) / nV : 0.0;
      last[c] = w[j];
    }
  }
  if (bad || separated) {
    if (tid == 0) {
      st->status = bad ? kNumeric : kSeparated;
      st->t_end = k;
    }
    return;
  }
  double dl = 0.0, wn = 0.0;
#pragma unroll
  for (int j = 0; j < (kMaxD + NT - 1) / NT; ++j) {
    const int c = tid + j * NT;
    if (c < d) {
      const double s = Sv[c] + w[j];
      Sv[c] = s;
      const double yn = s / (double)k;
      const double dd = yn - wbar[c];
      dl += dd * dd;
      wn += yn * yn;
      wbar[c] = yn;
    }
  }
  const double Dw = sqrt(block_sum<NT>(dl, s_red));
  const double nwb = sqrt(block_sum<NT>(wn, s_red));
  if (tid == 0) {
    st->S1 += s1;
    st->S2 += s2;
    const double n1 = st->S1 / (double)k, n2 = st->S2 / (double)k;
    const double ds = fmax(fabs(n1 - st->s1bar), fabs(n2 - st->s2bar));
    st->s1bar = n1;
    st->s2bar = n2;
    st->wbar_norm = nwb;
    // slack_i(k) >= slack_i(k-1) - ||x_i|| ||dwbar|| - |dsbar_c|, ||x_i|| <= D
    st->shift_bound = slmin - D * Dw - ds;
    st->t = k;
  }
}

template <typename T, int EPL, int VEC>
__global__ __launch_bounds__(kPassBlock) __attribute__((amdgpu_waves_per_eu(SCPMWU_PASS_WAVES)))
void svm_pass_kernel(PassArgs a) {
  using Sh = Shape<EPL, (int)sizeof(typename RegT<T>::type), kSVM>;
  constexpr int SB = Sh::SB, B = Sh::B;
  __shared__ double s_part[kPassWaves][B][kG + 1];
  __shared__ double s_wa[kPassWaves][B];
  __shared__ double s_vec[kPassWaves][kG * EPL];
  __shared__ double s_sc[kPassWaves][8];

  DevState *st = a.st;
  if (st->status != kRunning) return;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, cl = lane & 15;
  const int64_t n = a.n, ld = a.ld, n_pos = a.n_pos;
  const int d = (int)a.d;
  const T *__restrict__ X = reinterpret_cast<const T *>(a.X);
  const double kappa = st->kscale * (double)st->t;
  const double slb = st->shift_bound;
  const double s1b = st->s1bar, s2b = st->s2bar;
  const double *wbar = a.vec + kVecMean * d;

  double wb[EPL];
#pragma unroll
  for (int k = 0; k < EPL; ++k) {
    const int c = cl * EPL + k;
    wb[k] = c < d ? wbar[c] : 0.0;
  }
  double accP[EPL], accQ[EPL];
#pragma unroll
  for (int k = 0; k < EPL; ++k) accP[k] = accQ[k] = 0.0;
  double t1 = 0.0, t2 = 0.0, nminP = -INFINITY, maxQ = -INFINITY, nslmin = -INFINITY;

  const int64_t nb = (n + B - 1) / B;
  const int64_t GW = (int64_t)gridDim.x * kPassWaves;
  for (int64_t b = (int64_t)blockIdx.x * kPassWaves + wave; b < nb; b += GW) {
    const int64_t r0 = b * B;
    using R = typename RegT<T>::type;
    R xv[SB][EPL];
#pragma unroll
    for (int s = 0; s < SB; ++s) {
      VecT<T, VEC> raw[EPL / VEC];
      load_row<T, EPL, VEC>(X, r0 + s * kRowsPerStep + g, n, d, ld, cl, raw);
#pragma unroll
      for (int q = 0; q < EPL / VEC; ++q)
#pragma unroll
        for (int e = 0; e < VEC; ++e) xv[s][q * VEC + e] = to_reg(raw[q].v[e]);
    }
#pragma unroll
    for (int s = 0; s < SB; ++s) {
      double dot = 0.0;
#pragma unroll
      for (int k = 0; k < EPL; ++k) dot = fma((double)xv[s][k], wb[k], dot);
      s_part[wave][s * kRowsPerStep + g][cl] = dot;
    }
    wave_lds_sync();
    if (lane < B) {
      double dot = 0.0;
#pragma unroll
      for (int c = 0; c < kG; ++c) dot += s_part[wave][lane][c];
      const int64_t row = r0 + lane;
      const bool valid = row < n;
      const bool isP = row < n_pos;
      const double sl = (isP ? dot : -dot) - (isP ? s1b : s2b);
      // weight exp(-kappa' slack) shifted by the lower bound on the slack
      const double e = valid ? exp(-kappa * (sl - slb)) : 0.0;
      if (isP) t1 += e; else t2 += e;
      if (valid) {
        if (isP) nminP = fmax(nminP, -dot); else maxQ = fmax(maxQ, dot);
        nslmin = fmax(nslmin, -sl);
      }
      s_wa[wave][lane] = e;
    }
    wave_lds_sync();
    opaque(xv);
    if (r0 + B <= n_pos) {
#pragma unroll
      for (int s = 0; s < SB; ++s) {
        const double er = s_wa[wave][s * kRowsPerStep + g];
#pragma unroll
        for (int k = 0; k < EPL; ++k) accP[k] = fma(er, (double)xv[s][k], accP[k]);
      }
    } else if (r0 >= n_pos) {
#pragma unroll
      for (int s = 0; s < SB; ++s) {
        const double er = s_wa[wave][s * kRowsPerStep + g];
#pragma unroll
        for (int k = 0; k < EPL; ++k) accQ[k] = fma(er, (double)xv[s][k], accQ[k]);
      }
    } else {
#pragma unroll
      for (int s = 0; s < SB; ++s) {
        const double er = s_wa[wave][s * kRowsPerStep + g];
        const bool rp = (r0 + s * kRowsPerStep + g) < n_pos;
        const double eP = rp ? er : 0.0, eQ = rp ? 0.0 : er;
#pragma unroll
        for (int k = 0; k < EPL; ++k) {
          accP[k] = fma(eP, (double)xv[s][k], accP[k]);
          accQ[k] = fma(eQ, (double)xv[s][k], accQ[k]);
        }
      }
    }
    wave_lds_sync();
  }

#pragma unroll
  for (int k = 0; k < EPL; ++k) {
    accP[k] += __shfl_xor(accP[k], 16);
    accP[k] += __shfl_xor(accP[k], 32);
    accQ[k] += __shfl_xor(accQ[k], 16);
    accQ[k] += __shfl_xor(accQ[k], 32);
  }
  const int pw = partial_width(d);
  if (g == 0)
#pragma unroll
    for (int k = 0; k < EPL; ++k) s_vec[wave][cl * EPL + k] = accP[k];
  t1 = wave_sum(t1);
  t2 = wave_sum(t2);
  nminP = wave_max(nminP);
  maxQ = wave_max(maxQ);
  nslmin = wave_max(nslmin);
  if (lane == 0) {
    s_sc[wave][0] = t1;
    s_sc[wave][1] = t2;
    s_sc[wave][4] = nminP;
    s_sc[wave][5] = maxQ;
    s_sc[wave][6] = nslmin;
  }
  __syncthreads();
  double *rec = a.partials + (int64_t)blockIdx.x * pw;
  for (int c = tid; c < d; c += kPassBlock) rec[c] = sum_waves(s_vec, c);
  __syncthreads();
  if (g == 0)
#pragma unroll
    for (int k = 0; k < EPL; ++k) s_vec[wave][cl * EPL + k] = accQ[k];
  __syncthreads();
  for (int c = tid; c < d; c += kPassBlock) rec[d + c] = sum_waves(s_vec, c);
  if (tid < 8) {
    double v;
    if (tid < 2)
      v = sum_waves(s_sc, tid);
    else if (tid < 4)
      v = 0.0;
    else if (tid < 7)
      v = max_waves(s_sc, tid);
    else
      v = -INFINITY;
    rec[2 * d + tid] = v;
  }
}

// ===================================================== combine + epilogue
// One workgroup: sums the per-workgroup records of the pass that just ran
// (fixed order: a transposed pass over record pairs, then over the row
// groups) and runs the FP64 epilogue of the iteration.  The kernel boundary
// after the pass makes every record visible; no fences are needed.
template <typename T, int PROB, bool CERT>
__global__ __launch_bounds__(kCombBlock) void epilogue_kernel(PassArgs a, int P) {
  __shared__ double s_acc[2 * kCombBlock];
  __shared__ double s_comb[2 * kMaxD + 8];
  __shared__ double s_red[kCombBlock / 64];
  __shared__ int s_int[4];
  DevState *st = a.st;
  if (st->status != kRunning) return;
  const int d = (int)a.d;
  const int pw = partial_width(d);
  const int nsum = PROB == kSES ? 2 * d + 5 : 2 * d + 4;
  const int npairs = pw / 2;
  const int groups = kCombBlock / npairs;
  const int tid = threadIdx.x;
  const int j = tid % npairs, grp = tid / npairs;
  if (grp < groups) {
    const int c0 = 2 * j;
    const bool s0 = c0 < nsum, s1 = c0 + 1 < nsum;
    double acc0 = s0 ? 0.0 : -INFINITY, acc1 = s1 ? 0.0 : -INFINITY;
#pragma unroll 8
    for (int b = grp; b < P; b += groups) {
      const double2 v = *reinterpret_cast<const double2 *>(a.partials + (int64_t)b * pw + c0);
      acc0 = s0 ? acc0 + v.x : fmax(acc0, v.x);
      acc1 = s1 ? acc1 + v.y : fmax(acc1, v.y);
    }
    s_acc[grp * pw + c0] = acc0;
    s_acc[grp * pw + c0 + 1] = acc1;
  }
  __syncthreads();
  for (int c = tid; c < pw; c += kCombBlock) {
    const bool sm = c < nsum;
    double r = sm ? 0.0 : -INFINITY;
    for (int g = 0; g < groups; ++g) r = sm ? r + s_acc[g * pw + c] : fmax(r, s_acc[g * pw + c]);
    s_comb[c] = r;
  }
  __syncthreads();
  if (PROB == kSES)
    ses_epilogue<T, kCombBlock>(a, s_comb, CERT, s_red, s_int);
  else
    svm_epilogue<T, kCombBlock>(a, s_comb, s_red, s_int);
}

// ========================================================== monitor pass
// Per workgroup over its rows: mode 0 (distance to `center`): out[0] = max
// over rows != exclude of ||x_i - c|| + gamma_i, out[1] = the same over all
// rows; mode 1 (dot with `center`): out[2] = -min over rows < n_pos of x.c,
// out[3] = max over rows >= n_pos of x.c.  Not on the iteration path (used
// for D and after set_state), so it uses a simple generic layout.
template <typename T>
__global__ __launch_bounds__(kBlock) void monitor_kernel(PassArgs a, const double *center,
                                                         int64_t exclude, int mode, double *out) {
  __shared__ double s_sc[kWavesPerBlock][4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, cl = lane & 15;
  const int64_t n = a.n, ld = a.ld;
  const int d = (int)a.d;
  const T *X = reinterpret_cast<const T *>(a.X);
  double r0 = -INFINITY, r1 = -INFINITY, r2 = -INFINITY, r3 = -INFINITY;
  const int64_t GR = (int64_t)gridDim.x * kWavesPerBlock * kRowsPerStep;
  // the whole wave iterates together; rows >= n contribute nothing
  for (int64_t base = ((int64_t)blockIdx.x * kWavesPerBlock + wave) * kRowsPerStep; base < n;
       base += GR) {
    const int64_t row = base + g;
    double acc = 0.0;
    if (row < n)
      for (int c = cl; c < d; c += kG) {
        const double x = to_f64(X[row * ld + c]);
        if (mode == 0) {
          const double df = x - center[c];
          acc = fma(df, df, acc);
        } else {
          acc = fma(x, center[c], acc);
        }
      }
    acc += __shfl_xor(acc, 8, 16);
    acc += __shfl_xor(acc, 4, 16);
    acc += __shfl_xor(acc, 2, 16);
    acc += __shfl_xor(acc, 1, 16);
    if (row < n) {
      if (mode == 0) {
        const double h = sqrt(acc) + (a.radii ? a.radii[row] : 0.0);
        if (row != exclude) r0 = fmax(r0, h);
        r1 = fmax(r1, h);
      } else {
        if (row < a.n_pos) r2 = fmax(r2, -acc); else r3 = fmax(r3, acc);
      }
    }
  }
  r0 = wave_max(r0);
  r1 = wave_max(r1);
  r2 = wave_max(r2);
  r3 = wave_max(r3);
  if (lane == 0) {
    s_sc[wave][0] = r0;
    s_sc[wave][1] = r1;
    s_sc[wave][2] = r2;
    s_sc[wave][3] = r3;
  }
  __syncthreads();
  if (tid < 4)
    out[(int64_t)blockIdx.x * 4 + tid] =
        fmax(fmax(s_sc[0][tid], s_sc[1][tid]), fmax(s_sc[2][tid], s_sc[3][tid]));
}

// ======================================================= test (re)start
template <typename T>
__global__ __launch_bounds__(kBlock) void ftp_init_kernel(PassArgs a, InitParams p, int problem) {
  DevState *st = a.st;
  const int d = (int)a.d;
  const int tid = threadIdx.x;
  for (int c = tid; c < d; c += kBlock) {
    double y0 = 0.0;
    if (problem == kSES) y0 = to_f64(reinterpret_cast<const T *>(a.X)[a.v1 * a.ld + c]);
    a.vec[kVecS * d + c] = 0.0;
    a.vec[kVecMean * d + c] = y0;  // SES: ubar(0) = v1 (only distances of pass 1 use it)
    a.vec[kVecBest * d + c] = y0;
    a.vec[kVecLast * d + c] = 0.0;
  }
  if (tid == 0) {
    DevState s = {};
    s.alpha = p.alpha;
    s.eta = p.eta;
    s.kscale = p.kscale;
    s.delta = p.delta;
    s.tau = p.tau;
    s.D = p.D;
    s.gamma1 = p.gamma1;
    s.T = p.T;
    s.t = 0;
    s.t_end = 0;
    s.t_best = 0;
    s.status = kRunning;
    s.cnt = 0;
    s.patience = p.patience;
    s.early = p.early;
    s.f_prev = -1.0;
    s.f_best = problem == kSES ? INFINITY : -INFINITY;
    s.f_last = NAN;
    s.shift_bound = 0.0;
    s.bound = problem == kSES ? 0.0 : INFINITY;
    *st = s;
  }
}

// ============================================================== dispatch
template <typename T, int EPL, int VEC>
hipError_t launch_pass_t(int problem, bool cert, int grid, const PassArgs &a, hipStream_t s) {
  if (problem == kSES) {
    if (cert)
      hipLaunchKernelGGL((ses_pass_kernel<T, EPL, VEC, true>), dim3(grid), dim3(kPassBlock), 0, s, a);
    else
      hipLaunchKernelGGL((ses_pass_kernel<T, EPL, VEC, false>), dim3(grid), dim3(kPassBlock), 0, s, a);
  } else {
    hipLaunchKernelGGL((svm_pass_kernel<T, EPL, VEC>), dim3(grid), dim3(kPassBlock), 0, s, a);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_epilogue_typed(int problem, bool cert, int grid, const PassArgs &a, hipStream_t s) {
  if (problem == kSES) {
    if (cert)
      hipLaunchKernelGGL((epilogue_kernel<T, kSES, true>), dim3(1), dim3(kCombBlock), 0, s, a, grid);
    else
      hipLaunchKernelGGL((epilogue_kernel<T, kSES, false>), dim3(1), dim3(kCombBlock), 0, s, a, grid);
  } else {
    hipLaunchKernelGGL((epilogue_kernel<T, kSVM, false>), dim3(1), dim3(kCombBlock), 0, s, a, grid);
  }
  return hipGetLastError();
}

template <typename T, int EPL>
hipError_t launch_pass_v(int problem, const LaunchCfg &c, const PassArgs &a, hipStream_t s) {
  constexpr int VF = (16 / (int)sizeof(T)) < EPL ? (16 / (int)sizeof(T)) : EPL;
  if (c.vec == VF) return launch_pass_t<T, EPL, VF>(problem, c.cert, c.grid, a, s);
  if constexpr (VF >= 4) {
    if (c.vec == VF / 2) return launch_pass_t<T, EPL, VF / 2>(problem, c.cert, c.grid, a, s);
  }
  if constexpr (VF > 1) {
    if (c.vec == 1) return launch_pass_t<T, EPL, 1>(problem, c.cert, c.grid, a, s);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_pass_typed(int problem, const LaunchCfg &c, const PassArgs &a, hipStream_t s) {
  switch (c.epl) {
    case 1: return launch_pass_v<T, 1>(problem, c, a, s);
    case 2: return launch_pass_v<T, 2>(problem, c, a, s);
    case 4: return launch_pass_v<T, 4>(problem, c, a, s);
    case 8: return launch_pass_v<T, 8>(problem, c, a, s);
    case 16: return launch_pass_v<T, 16>(problem, c, a, s);
    case 32: return launch_pass_v<T, 32>(problem, c, a, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_monitor_typed(int grid, const PassArgs &a, const double *center, int64_t exclude,
                                int mode, double *out, hipStream_t s) {
  hipLaunchKernelGGL((monitor_kernel<T>), dim3(grid), dim3(kBlock), 0, s, a, center, exclude, mode, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_init_typed(const PassArgs &a, const InitParams &p, int problem, hipStream_t s) {
  hipLaunchKernelGGL((ftp_init_kernel<T>), dim3(1), dim3(kBlock), 0, s, a, p, problem);
  return hipGetLastError();
}

}  // namespace scpmwu
