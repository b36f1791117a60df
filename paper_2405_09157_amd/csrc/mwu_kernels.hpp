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
// Each workgroup writes one record of partial sums and maxima; the pass has
// no inter-workgroup synchronisation.  The one-workgroup kernel launched
// after it (preceded, when the records are large, by a kernel that sums
// groups of 16) sums the records in a fixed order, and one wave runs the FP64
// epilogue: ORACLE closed form, the separation test, the running mean and the
// early-exit rules.  All arithmetic on point data is binary64; results are
// bitwise reproducible for a fixed grid.
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
// FP8 E4M3 code (the low byte of c) -> its value, exactly (hardware decode;
// the scale of the row is applied separately)
__device__ __forceinline__ float fp8_value(uint32_t c) { return __builtin_amdgcn_cvt_f32_fp8(c, 0); }
template <>
__device__ __forceinline__ double to_f64<uint8_t>(uint8_t c) {
  return (double)fp8_value(c);
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
template <>
__device__ __forceinline__ float to_reg<uint8_t>(uint8_t c) {
  return fp8_value(c);
}

// Occupancy target of the streaming pass (waves per SIMD): caps the
// register budget at 512 / target VGPRs so that enough waves are resident
// to keep loads in flight.
#ifndef SCPMWU_PASS_WAVES
#define SCPMWU_PASS_WAVES 2
#endif

// Register image of one batch: SB load steps x EPL elements of the lane.
// F32 and F64 elements are held in their own type (binary32 holds F32 and
// BF16 values exactly at half the registers of binary64); with PACK, BF16
// keeps its raw pairs, two elements per 32-bit register, widened on use.
template <typename T, int SB, int EPL, bool PACK>
struct Batch {
  using R = typename RegT<T>::type;
  R x[SB][EPL];
  double gi;  // SES: radius of the batch row of this lane (lanes < B)
  float sc;   // FP8: scale of the batch row of this lane (lanes < B)
  __device__ __forceinline__ double get(int s, int k) const { return (double)x[s][k]; }
  __device__ __forceinline__ float getf(int s, int k) const { return (float)x[s][k]; }
  template <int VEC>
  __device__ __forceinline__ void put(int s, int q, const VecT<T, VEC> &raw) {
#pragma unroll
    for (int e = 0; e < VEC; ++e) x[s][q * VEC + e] = to_reg(raw.v[e]);
  }
  // keeps the elements in their narrow type across the per-row phase
  // instead of caching binary64 conversions (which would double the live
  // registers)
  __device__ __forceinline__ void pin() {
#pragma unroll
    for (int s = 0; s < SB; ++s)
#pragma unroll
      for (int k = 0; k < EPL; ++k) asm volatile("" : "+v"(x[s][k]));
  }
};
template <int SB, int EPL>
struct Batch<uint16_t, SB, EPL, true> {
  static_assert(EPL % 2 == 0, "packed BF16 needs an even number of columns per lane");
  uint32_t w[SB][EPL / 2];
  double gi;
  float sc;
  __device__ __forceinline__ float getf(int s, int k) const {
    const uint32_t u = w[s][k >> 1];
    return __uint_as_float((k & 1) ? (u & 0xffff0000u) : (u << 16));
  }
  __device__ __forceinline__ double get(int s, int k) const { return (double)getf(s, k); }
  template <int VEC>
  __device__ __forceinline__ void put(int s, int q, const VecT<uint16_t, VEC> &raw) {
    if constexpr (VEC >= 2) {
      __builtin_memcpy(&w[s][q * VEC / 2], &raw, VEC * 2);
    } else {
      const uint32_t h = raw.v[0];
      w[s][q >> 1] = (q & 1) ? (w[s][q >> 1] | (h << 16)) : h;
    }
  }
  __device__ __forceinline__ void pin() {
#pragma unroll
    for (int s = 0; s < SB; ++s)
#pragma unroll
      for (int k = 0; k < EPL / 2; ++k) asm volatile("" : "+v"(w[s][k]));
  }
};

// BF16 and FP8 with one column per lane: one raw code per 32-bit register,
// widened on use.  (Widening at load time let the compiler route every narrow
// load of a batch through one temporary register and wait for each in turn.)
template <int SB>
struct Batch<uint8_t, SB, 1, false> {
  uint32_t w[SB];
  double gi;
  float sc;
  __device__ __forceinline__ float getf(int s, int) const { return __builtin_amdgcn_cvt_f32_fp8(w[s], 0); }
  __device__ __forceinline__ double get(int s, int k) const { return (double)getf(s, k); }
  template <int VEC>
  __device__ __forceinline__ void put(int s, int, const VecT<uint8_t, VEC> &raw) {
    static_assert(VEC == 1, "one column per lane");
    w[s] = raw.v[0];
  }
  __device__ __forceinline__ void pin() {
#pragma unroll
    for (int s = 0; s < SB; ++s) asm volatile("" : "+v"(w[s]));
  }
};
template <int SB>
struct Batch<uint16_t, SB, 1, false> {
  uint32_t w[SB];
  double gi;
  float sc;
  __device__ __forceinline__ float getf(int s, int) const { return __uint_as_float(w[s] << 16); }
  __device__ __forceinline__ double get(int s, int k) const { return (double)getf(s, k); }
  template <int VEC>
  __device__ __forceinline__ void put(int s, int, const VecT<uint16_t, VEC> &raw) {
    static_assert(VEC == 1, "one column per lane");
    w[s] = raw.v[0];
  }
  __device__ __forceinline__ void pin() {
#pragma unroll
    for (int s = 0; s < SB; ++s) asm volatile("" : "+v"(w[s]));
  }
};

// FP8 E4M3 codes kept packed, four per 32-bit register, decoded on use.
template <int SB, int EPL>
struct Batch<uint8_t, SB, EPL, true> {
  static_assert(EPL % 4 == 0, "packed FP8 needs a multiple of 4 columns per lane");
  uint32_t w[SB][EPL / 4];
  double gi;
  float sc;
  __device__ __forceinline__ float getf(int s, int k) const {
    // the pair conversion decodes the low two bytes of its operand; the high
    // pair is shifted down (k is a constant once unrolled, and the two
    // elements of a pair share one conversion)
    const uint32_t u = w[s][k >> 2];
    const auto p = __builtin_amdgcn_cvt_pk_f32_fp8((int)((k & 2) ? (u >> 16) : u), false);
    return (k & 1) ? p[1] : p[0];
  }
  __device__ __forceinline__ double get(int s, int k) const { return (double)getf(s, k); }
  template <int VEC>
  __device__ __forceinline__ void put(int s, int q, const VecT<uint8_t, VEC> &raw) {
    if constexpr (VEC % 4 == 0) {
      __builtin_memcpy(&w[s][q * VEC / 4], &raw, VEC);
    } else {
      uint32_t bits = 0;
      __builtin_memcpy(&bits, &raw, VEC);
      const int byte = (q * VEC) & 3;
      w[s][(q * VEC) >> 2] = byte == 0 ? bits : (w[s][(q * VEC) >> 2] | (bits << (8 * byte)));
    }
  }
  __device__ __forceinline__ void pin() {
#pragma unroll
    for (int s = 0; s < SB; ++s)
#pragma unroll
      for (int k = 0; k < EPL / 4; ++k) asm volatile("" : "+v"(w[s][k]));
  }
};

// Batch shape of the streaming pass (pass_steps): SB load steps of 4 rows.
// k-way slots (KS <= 3) keep KS sets of accumulators in registers beside the
// batch.
template <typename T, int EPL, int PROB, int PFM, int KS = 1>
struct PassShape {
  static constexpr bool PACK = pass_packed((int)sizeof(T), EPL, PROB);
  static constexpr int SB = pass_steps((int)sizeof(T), EPL, PROB, PFM);
  static constexpr int B = SB * kRowsPerStep;
  static_assert(B <= kWave, "the per-row phase holds one row per lane");
  using Regs = Batch<T, SB, EPL, PACK>;
};

// Lanes of one wavefront exchange data through LDS only: DS instructions of a
// wave execute in order, so a compiler barrier is all that is needed.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wave reductions without LDS round trips: DPP moves within each 16-lane row
// (pairs, quads, then rotations by 4 and 8 lanes), then the four row values
// read from lanes 0, 16, 32, 48 and combined in that fixed order.  Every lane
// returns the same value; the order is fixed, so results are reproducible.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double readlane_f64(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l), __builtin_amdgcn_readlane(__double2loint(v), l));
}
constexpr int kDppPairs = 0xB1;  // quad_perm [1,0,3,2]
constexpr int kDppQuads = 0x4E;  // quad_perm [2,3,0,1]
constexpr int kDppRor4 = 0x124;  // row_ror:4
constexpr int kDppRor8 = 0x128;  // row_ror:8

__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<kDppPairs>(v);
  v += dpp_f64<kDppQuads>(v);
  v += dpp_f64<kDppRor4>(v);
  v += dpp_f64<kDppRor8>(v);
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}
// Several wave sums, independent so that their latencies overlap.
__device__ __forceinline__ void wave_sum2(double &a, double &b) {
  a = wave_sum(a);
  b = wave_sum(b);
}
__device__ __forceinline__ void wave_sum3(double &a, double &b, double &c) {
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
}
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_f64<kDppPairs>(v));
  v = fmax(v, dpp_f64<kDppQuads>(v));
  v = fmax(v, dpp_f64<kDppRor4>(v));
  v = fmax(v, dpp_f64<kDppRor8>(v));
  return fmax(fmax(readlane_f64(v, 0), readlane_f64(v, 16)), fmax(readlane_f64(v, 32), readlane_f64(v, 48)));
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

// ------------------------------------------------------------ buffer loads
// Rows [r0, r0 + rows) of X as a raw buffer resource: bytes past the last
// valid element of the last valid row read as zero (hardware range check),
// so a batch needs no per-row branch or zero fill.  The range check covers
// the lane (VGPR) offset and the immediate offset but not the SGPR offset,
// so the whole offset of a load (row step and column) goes in the lane
// offset.
constexpr int32_t kBufWord3 = 0x00020000;  // raw buffer, gfx9 family
constexpr int32_t kOffInvalid = 0x40000000;  // a lane offset beyond any batch

// A raw buffer resource over [base, base + num bytes) built from the first
// lane's values (the caller guarantees they are wave-uniform), so that it
// lives in scalar registers: a resource the compiler cannot prove uniform
// makes it loop over lanes around every load.  readfirstlane returns a signed
// int: both address halves go through uint32_t so that the low half is
// zero-extended.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t uniform_rsrc(const void *base, int32_t num) {
  const uint64_t a = reinterpret_cast<uint64_t>(base);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void *>(((uint64_t)hi << 32) | (uint64_t)lo), (short)0,
                                           __builtin_amdgcn_readfirstlane(num), kBufWord3);
}

// Rows [r0, r0 + rows) of X (r0, rows wave-uniform).
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rows_rsrc(const T *X, int64_t r0, int64_t rows, int64_t ld,
                                                          int d) {
  const int32_t num = rows > 0 ? (int32_t)(((rows - 1) * ld + d) * (int64_t)sizeof(T)) : 0;
  return uniform_rsrc(X + r0 * ld, num);
}

// Radii of rows [r0, r0 + rows) (none: an empty resource, every load reads 0).
__device__ __forceinline__ double radius_load(const double *radii, int64_t r0, int64_t rows, int lane) {
  const int32_t num = (radii != nullptr && rows > 0) ? (int32_t)(rows * 8) : 0;
  const __amdgpu_buffer_rsrc_t r = uniform_rsrc(radii != nullptr ? radii + r0 : nullptr, num);
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, lane * 8, 0, 0);
  double g;
  __builtin_memcpy(&g, &v, 8);
  return g;
}

// FP8 scales of rows [r0, r0 + rows) (none: every load reads 0).
__device__ __forceinline__ float scale_load(const float *scales, int64_t r0, int64_t rows, int lane) {
  const int32_t num = (scales != nullptr && rows > 0) ? (int32_t)(rows * 4) : 0;
  const __amdgpu_buffer_rsrc_t r = uniform_rsrc(scales != nullptr ? scales + r0 : nullptr, num);
  const auto v = __builtin_amdgcn_raw_buffer_load_b32(r, lane * 4, 0, 0);
  float f;
  __builtin_memcpy(&f, &v, 4);
  return f;
}

// Element (row, c) of the stored points as the value the method works on:
// FP8 codes times their row's scale (exact in binary64).
template <typename T>
__device__ __forceinline__ double row_value(const PassArgs &a, int64_t row, int64_t c) {
  const double v = to_f64(reinterpret_cast<const T *>(a.X)[row * a.ld + c]);
  if constexpr (sizeof(T) == 1) return v * (double)a.scales[row];
  return v;
}

template <typename T, int VEC>
__device__ __forceinline__ VecT<T, VEC> buf_load(__amdgpu_buffer_rsrc_t r, int32_t voff, int32_t soff) {
  VecT<T, VEC> v;
  constexpr int BYTES = VEC * (int)sizeof(T);
  if constexpr (BYTES == 16) {
    const auto x = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    __builtin_memcpy(&v, &x, 16);
  } else if constexpr (BYTES == 8) {
    const auto x = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    __builtin_memcpy(&v, &x, 8);
  } else if constexpr (BYTES == 4) {
    const auto x = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
    __builtin_memcpy(&v, &x, 4);
  } else if constexpr (BYTES == 2) {
    const auto x = __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
    __builtin_memcpy(&v, &x, 2);
  } else {
    static_assert(BYTES == 1, "load width");
    const auto x = __builtin_amdgcn_raw_buffer_load_b8(r, voff, soff, 0);
    __builtin_memcpy(&v, &x, 1);
  }
  return v;
}

// ------------------------------------------------------- workgroup records
// Layout of a workgroup record (binary64): [vec0: d] [8 scalars] [vec1: d],
// the scalar block starting at the even offset dp = d rounded up to even.
//   SES: vec0 = sum a_i x_i, scalars = (B, E, G, sum b_i d_i^2, A | gmax, fmax),
//        vec1 = sum b_i x_i (certificate passes only; not read otherwise)
//   SVM: vec0 = sum_P e_i x_i, scalars = (T1, T2, 0, 0 | -min_P x.w, max_Q x.w,
//        -min slack), vec1 = sum_Q e_i x_i
__host__ __device__ inline int rec_dp(int d) { return (d + 1) & ~1; }
__host__ __device__ inline int rec_width(int d) { return partial_width(d); }

// =========================================================== SES pass
// Column of element k (chunk k / VEC) of lane cl: chunk q of the 16 lanes of
// a row covers VEC * 16 contiguous columns, so every load instruction reads
// whole lines.
template <int VEC>
__device__ __forceinline__ int lane_col(int cl, int k) {
  return ((k / VEC) * kG + cl) * VEC + (k % VEC);
}

// The SES pass of one problem, run by workgroup vb of the vg workgroups
// assigned to it (its batches are b = vb * 8 + wave, strided by vg * 8; its
// record goes to partials[vb]).
// What a pass needs from the state of its test: the status, the exponent
// scale kappa = kscale * t, the carried shift bound, the candidate mean, and
// where the workgroup records go.
struct PassIn {
  int32_t status;
  double kappa, Gb;
  const double *ybar;
  double *rec;   // records (one per workgroup), or the global sum (gsum)
  bool gsum;     // add the workgroup's sums into rec with atomics
};

// Maxima kept in a global sum are combined by an unsigned integer atomic max
// on an order-preserving key: non-negative doubles with the sign bit set,
// negative ones complemented, so that the key order is the numeric order;
// the zero key (never produced by a number) stands for "no value" (-inf).
__device__ __forceinline__ unsigned long long max_key(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double from_max_key(unsigned long long k) {
  if (k == 0ull) return -INFINITY;
  const unsigned long long b = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
  return __longlong_as_double((long long)b);
}
__device__ __forceinline__ void gsum_add(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void gsum_max(double *p, double v) {
  if (v == -INFINITY) return;  // the identity
  __hip_atomic_fetch_max(reinterpret_cast<unsigned long long *>(p), max_key(v), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
}

// The pass reads its inputs through a prologue object: pre() runs before the
// workgroup's first batch of rows is requested, post() once it is in flight
// and returns the inputs (the fused kernel issues the previous pass's record
// loads in pre() and runs that pass's epilogue in post()); the plain form
// reads the state as it is.
__device__ __forceinline__ PassIn state_pass_in(const PassArgs &a) {
  const DevState *st = a.st;
  return PassIn{st->status, st->kscale * (double)st->t, st->shift_bound, a.vec + kVecMean * a.d,
                a.gsum != nullptr ? a.gsum : a.partials, a.gsum != nullptr};
}
struct StatePrologue {
  const PassArgs &a;
  __device__ __forceinline__ void pre() {}
  __device__ __forceinline__ PassIn post() { return state_pass_in(a); }
};

// KS > 1: the k-way search's tests over one point set (a: the set; slot j's
// inputs from prologue.slot(j), j >= 1): each batch of rows is loaded once and
// phases 1-3 run once per slot, each slot with its own mean, exponent scale,
// sums and record.  KS = 1 is the single test.
template <typename T, int EPL, int VEC, bool CERT, int PFM, typename Pro, int KS = 1>
__device__ __forceinline__ void ses_pass_body(const PassArgs &a, int vb, int vg, Pro &prologue) {
  static_assert(KS >= 1 && (KS == 1 || (!CERT && PFM == kPrefetchNone)), "k-way slots: no certificate, no prefetch");
  using Sh = PassShape<T, EPL, kSES, PFM, KS>;
  constexpr int SB = Sh::SB, B = Sh::B;
  using Regs = typename Sh::Regs;
  // BF16 storage: per-element arithmetic in binary32 (the row distance
  // partials and the batch's weighted sums), everything per row and across
  // batches in binary64; F32 and F64 storage: binary64 throughout
  constexpr bool M32 = sizeof(T) <= 2;
  // FP8 storage: codes times one binary32 scale per row
  constexpr bool FP8 = sizeof(T) == 1;
  __shared__ double s_part[kPassWaves][B][kG + 1];
  __shared__ double s_wa[kPassWaves][B];
  __shared__ double s_wb[kPassWaves][CERT ? B : 1];
  __shared__ float s_scl[kPassWaves][FP8 ? B : 1];
  __shared__ double s_vec[kPassWaves][kG * EPL];
  __shared__ double s_sc[kPassWaves][8];
  __shared__ double s_ctr[KS][kG * EPL];  // each slot's candidate (ubar), zero-padded

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, cl = lane & 15;
  const int64_t n = a.n, ld = a.ld;
  const int d = (int)a.d;
  const T *__restrict__ X = reinterpret_cast<const T *>(a.X);
  const double *__restrict__ radii = a.radii;
  const int64_t v1 = a.v1;
  // set by the prologue (grid-uniform per slot), read by the phases below
  int32_t status[KS];
  double kappa[KS], Gb[KS];
  double *rec_base[KS];
  bool to_gsum = false, any_running = false;
  auto start = [&]() {
#pragma unroll
    for (int j = 0; j < KS; ++j) {
      PassIn in;
      if constexpr (KS == 1)
        in = prologue.post();
      else
        in = j == 0 ? prologue.post() : prologue.slot(j);
      status[j] = __builtin_amdgcn_readfirstlane(in.status);
      kappa[j] = in.kappa;
      Gb[j] = in.Gb;
      rec_base[j] = in.rec;
      to_gsum = in.gsum;
      any_running = any_running || status[j] == kRunning;
      for (int c = tid; c < kG * EPL; c += kPassBlock) s_ctr[j][c] = c < d ? in.ybar[c] : 0.0;
    }
    // each status is the same for the whole grid: either every wave returns
    // after this barrier or none does
    __syncthreads();
  };
  double wacc[KS][EPL], cacc[CERT ? EPL : 1];
#pragma unroll
  for (int j = 0; j < KS; ++j)
#pragma unroll
    for (int k = 0; k < EPL; ++k) wacc[j][k] = 0.0;
#pragma unroll
  for (int k = 0; k < (CERT ? EPL : 1); ++k) cacc[k] = 0.0;
  double asum[KS], bsum[KS], esum[KS], gsum[KS], gmax[KS], fall[KS], bd2 = 0.0;
#pragma unroll
  for (int j = 0; j < KS; ++j) {
    asum[j] = bsum[j] = esum[j] = gsum[j] = 0.0;
    gmax[j] = fall[j] = -INFINITY;
  }

  const int64_t nb = (n + B - 1) / B;
  const int64_t GW = (int64_t)vg * kPassWaves;
  // lane offsets (bytes) of the lane's column chunks within its row of a
  // load step; chunks past column d get an offset beyond the buffer range
  int32_t voff[EPL / VEC];
#pragma unroll
  for (int q = 0; q < EPL / VEC; ++q) {
    const int c0 = lane_col<VEC>(cl, q * VEC);
    voff[q] = c0 < d ? (int32_t)(((int64_t)g * ld + c0) * (int64_t)sizeof(T)) : kOffInvalid;
  }
  const int32_t step_bytes = (int32_t)(kRowsPerStep * ld * (int64_t)sizeof(T));
  // rows [r0, r0 + rows) (rows <= B) into registers; the batch's other
  // rows read as zeros without touching memory
  auto load_rows = [&](Regs &xs, int64_t r0, int64_t rows) {
    const __amdgpu_buffer_rsrc_t rs = rows_rsrc<T>(X, r0, rows, ld, d);
#pragma unroll
    for (int s = 0; s < SB; ++s)
#pragma unroll
      for (int q = 0; q < EPL / VEC; ++q)
        xs.template put<VEC>(s, q, buf_load<T, VEC>(rs, voff[q] + s * step_bytes, 0));
    xs.gi = radius_load(radii, r0, rows, lane);
    if constexpr (FP8) xs.sc = scale_load(a.scales, r0, rows, lane);
  };
  auto load_batch = [&](Regs &xs, int64_t b) {
    const int64_t r0 = b * B;
    load_rows(xs, r0, n - r0 < B ? n - r0 : B);
  };
  // phases 1-3 on the rows [r0, r0 + rows) held in xs, for slot j
  auto process_slot = [&](Regs &xs, int64_t r0, int64_t rows, int j) {
    // re-read the candidate each batch: it stays out of registers in phases 2-3
    asm volatile("" ::: "memory");
    // binary32 storage types: the mean rounded to binary32, used by phases 1 and 3
    float ub32[M32 ? EPL : 1];
    if constexpr (M32) {
      if constexpr (FP8) {
        if (lane < B) s_scl[wave][lane] = xs.sc;
        wave_lds_sync();
      }
      float *ub = ub32;
#pragma unroll
      for (int k = 0; k < EPL; ++k) ub[k] = (float)s_ctr[j][lane_col<VEC>(cl, k)];
#pragma unroll
      for (int s = 0; s < SB; ++s) {
        const float sr = FP8 ? s_scl[wave][s * kRowsPerStep + g] : 1.f;
        float dsq = 0.f;
#pragma unroll
        for (int k = 0; k < EPL; ++k) {
          const float df = FP8 ? fmaf(sr, xs.getf(s, k), -ub[k]) : xs.getf(s, k) - ub[k];
          dsq = fmaf(df, df, dsq);
        }
        s_part[wave][s * kRowsPerStep + g][cl] = (double)dsq;
      }
    } else {
      double ub[EPL];
#pragma unroll
      for (int k = 0; k < EPL; ++k) ub[k] = s_ctr[j][lane_col<VEC>(cl, k)];
#pragma unroll
      for (int s = 0; s < SB; ++s) {
        double dsq = 0.0;
#pragma unroll
        for (int k = 0; k < EPL; ++k) {
          const double df = xs.get(s, k) - ub[k];
          dsq = fma(df, df, dsq);
        }
        s_part[wave][s * kRowsPerStep + g][cl] = dsq;
      }
    }
    wave_lds_sync();
    if (lane < B) {
      double dsq = 0.0;
#pragma unroll
      for (int c = 0; c < kG; ++c) dsq += s_part[wave][lane][c];
      const int64_t row = r0 + lane;
      const bool valid = lane < rows;
      const bool incl = valid && row != v1;
      const double di = sqrt(dsq);
      const double gi = xs.gi;  // 0 past n or without radii
      const double h = di + gi;
      // shifted lambda_+ = kappa (h - alpha) - kappa (G - alpha) <= ~0
      const double kap = kappa[j];
      const double ep = exp(kap * (h - Gb[j]));
      const double om = -expm1(-2.0 * kap * di);  // 1 - e^{lambda_- - lambda_+}
      double aw = di > 0.0 ? ep * om / di : 2.0 * kap * ep;
      double bw = ep * (2.0 - om);
      double ew = ep * om * di;
      if (!incl) aw = bw = ew = 0.0;
      asum[j] += aw;
      bsum[j] += bw;
      esum[j] += ew;
      gsum[j] += gi * bw;
      if (CERT) bd2 += bw * dsq;
      if (incl) gmax[j] = fmax(gmax[j], h);
      if (valid) fall[j] = fmax(fall[j], h);
      s_wa[wave][lane] = aw;
      if (CERT) s_wb[wave][lane] = bw;
    }
    wave_lds_sync();
    xs.pin();
    if constexpr (M32) {
      // sum_i a_i (x_i - ubar32) (and the b_i sum): the batch's rows in
      // binary32 on the differences, so that no offset of the points from the
      // origin cancels in binary32; added to the binary64 sums per batch (the
      // epilogue adds (sum a_i)(ubar32 - ubar))
      float w32[EPL], c32[CERT ? EPL : 1];
#pragma unroll
      for (int k = 0; k < EPL; ++k) w32[k] = 0.f;
#pragma unroll
      for (int k = 0; k < (CERT ? EPL : 1); ++k) c32[k] = 0.f;
#pragma unroll
      for (int s = 0; s < SB; ++s) {
        const float ar = (float)s_wa[wave][s * kRowsPerStep + g];
        const float sr = FP8 ? s_scl[wave][s * kRowsPerStep + g] : 1.f;
        const float br = CERT ? (float)s_wb[wave][s * kRowsPerStep + g] : 0.f;
#pragma unroll
        for (int k = 0; k < EPL; ++k) {
          const float df = FP8 ? fmaf(sr, xs.getf(s, k), -ub32[k]) : xs.getf(s, k) - ub32[k];
          w32[k] = fmaf(ar, df, w32[k]);
          if (CERT) c32[k] = fmaf(br, df, c32[k]);
        }
      }
#pragma unroll
      for (int k = 0; k < EPL; ++k) wacc[j][k] += (double)w32[k];
      if (CERT)
#pragma unroll
        for (int k = 0; k < EPL; ++k) cacc[k] += (double)c32[k];
    } else {
      // sum_i a_i x_i (and sum_i b_i x_i); the epilogue subtracts (sum a_i) ubar
#pragma unroll
      for (int s = 0; s < SB; ++s) {
        const double ar = s_wa[wave][s * kRowsPerStep + g];
#pragma unroll
        for (int k = 0; k < EPL; ++k) wacc[j][k] = fma(ar, xs.get(s, k), wacc[j][k]);
        if (CERT) {
          const double br = s_wb[wave][s * kRowsPerStep + g];
#pragma unroll
          for (int k = 0; k < EPL; ++k) cacc[k] = fma(br, xs.get(s, k), cacc[k]);
        }
      }
    }
    wave_lds_sync();
  };
  auto process_rows = [&](Regs &xs, int64_t r0, int64_t rows) {
#pragma unroll
    for (int j = 0; j < KS; ++j)
      if (KS == 1 || status[j] == kRunning) process_slot(xs, r0, rows, j);
  };
  auto process = [&](Regs &xs, int64_t b) {
    const int64_t r0 = b * B;
    process_rows(xs, r0, n - r0 < B ? n - r0 : B);
  };
  const int64_t b0 = (int64_t)vb * kPassWaves + wave;
  if constexpr (PFM == kPrefetchRegs) {
    // two register batches, unrolled by two so that neither is copied: the
    // loads of the next batch are in flight while the current one is
    // processed.  The loads are unconditional (a batch past the end has an
    // empty resource and reads zeros without touching memory), so that the
    // waits for the current batch never include the next one's loads.
    Regs xa, xb;
    int64_t b = b0;
    prologue.pre();
    load_batch(xa, b);
    start();
    if (!any_running) return;
    while (b < nb) {
      const int64_t b1 = b + GW;
      load_batch(xb, b1);
      process(xa, b);
      if (b1 >= nb) break;
      const int64_t b2 = b1 + GW;
      load_batch(xa, b2);
      process(xb, b1);
      b = b2;
    }
  } else {
    // the first batch's loads go out before the prologue (a batch past the
    // end reads zeros without touching memory)
    Regs xs;
    prologue.pre();
    load_batch(xs, b0);
    start();
    if (!any_running) return;
    for (int64_t b = b0; b < nb; b += GW) {
      if (b != b0) load_batch(xs, b);
      process(xs, b);
    }
  }
  if (!any_running) return;
  const int pw = rec_width(d);
  const int dp = rec_dp(d);

  // ---- workgroup record of each running slot: W, C(cert), sums, maxima
#pragma unroll
  for (int j = 0; j < KS; ++j) {
  if (KS > 1 && status[j] != kRunning) continue;
  if (KS > 1 && j > 0) __syncthreads();  // the previous slot's record is read from LDS
#pragma unroll
  for (int k = 0; k < EPL; ++k) {
    wacc[j][k] += __shfl_xor(wacc[j][k], 16);
    wacc[j][k] += __shfl_xor(wacc[j][k], 32);
  }
  if (g == 0)
#pragma unroll
    for (int k = 0; k < EPL; ++k) s_vec[wave][lane_col<VEC>(cl, k)] = wacc[j][k];
  const double w_asum = wave_sum(asum[j]);
  const double w_bsum = wave_sum(bsum[j]);
  const double w_esum = wave_sum(esum[j]);
  const double w_gsum = wave_sum(gsum[j]);
  const double w_bd2 = wave_sum(bd2);
  const double w_gmax = wave_max(gmax[j]);
  const double w_fall = wave_max(fall[j]);
  if (lane == 0) {
    s_sc[wave][0] = w_bsum;
    s_sc[wave][1] = w_esum;
    s_sc[wave][2] = w_gsum;
    s_sc[wave][3] = w_bd2;
    s_sc[wave][4] = w_asum;
    s_sc[wave][5] = w_gmax;
    s_sc[wave][6] = w_fall;
  }
  __syncthreads();
  // the workgroup's record, or its sums added into the global sum
  double *rec = to_gsum ? rec_base[j] : rec_base[j] + (int64_t)vb * pw;
  for (int c = tid; c < d; c += kPassBlock) {
    const double v = sum_waves(s_vec, c);
    if (to_gsum)
      gsum_add(rec + c, v);
    else
      rec[c] = v;
  }
  __syncthreads();
  if (CERT) {
#pragma unroll
    for (int k = 0; k < EPL; ++k) {
      cacc[k] += __shfl_xor(cacc[k], 16);
      cacc[k] += __shfl_xor(cacc[k], 32);
    }
    if (g == 0)
#pragma unroll
      for (int k = 0; k < EPL; ++k) s_vec[wave][lane_col<VEC>(cl, k)] = cacc[k];
    __syncthreads();
    for (int c = tid; c < d; c += kPassBlock) {
      const double v = sum_waves(s_vec, c);
      if (to_gsum)
        gsum_add(rec + dp + 8 + c, v);
      else
        rec[dp + 8 + c] = v;
    }
  }
  if (tid < 8) {
    double v;
    if (tid < 5)
      v = sum_waves(s_sc, tid);
    else if (tid < 7)
      v = max_waves(s_sc, tid);
    else
      v = -INFINITY;
    if (!to_gsum)
      rec[dp + tid] = v;
    else if (tid < 5)
      gsum_add(rec + dp + tid, v);
    else if (tid < 7)
      gsum_max(rec + dp + tid, v);
  }
  }
}

template <typename T, int EPL, int VEC, bool CERT, int PFM>
__device__ __forceinline__ void ses_pass_body(const PassArgs &a, int vb, int vg) {
  StatePrologue pro{a};
  ses_pass_body<T, EPL, VEC, CERT, PFM>(a, vb, vg, pro);
}

template <typename T, int EPL, int VEC, bool CERT, int PFM>
__global__ __launch_bounds__(kPassBlock) __attribute__((amdgpu_waves_per_eu(SCPMWU_PASS_WAVES)))
void ses_pass_kernel(PassArgs a) {
  ses_pass_body<T, EPL, VEC, CERT, PFM>(a, (int)blockIdx.x, (int)gridDim.x);
}

// =========================================================== SVM pass
template <typename T, int EPL, int VEC, int PFM>
__global__ __launch_bounds__(kPassBlock) __attribute__((amdgpu_waves_per_eu(SCPMWU_PASS_WAVES)))
void svm_pass_kernel(PassArgs a) {
  using Sh = PassShape<T, EPL, kSVM, PFM>;
  constexpr int SB = Sh::SB, B = Sh::B;
  using Regs = typename Sh::Regs;
  __shared__ double s_part[kPassWaves][B][kG + 1];
  __shared__ double s_wa[kPassWaves][B];
  __shared__ double s_vec[kPassWaves][kG * EPL];
  __shared__ double s_sc[kPassWaves][8];
  __shared__ double s_ctr[kG * EPL];  // the candidate (ubar or wbar), zero-padded

  DevState *st = a.st;
  const int32_t status0 = __builtin_amdgcn_readfirstlane(st->status);  // grid-uniform

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, cl = lane & 15;
  const int64_t n = a.n, ld = a.ld, n_pos = a.n_pos;
  const int d = (int)a.d;
  const T *__restrict__ X = reinterpret_cast<const T *>(a.X);
  const double kappa = st->kscale * (double)st->t;
  const double slb = st->shift_bound;
  const double s1b = st->s1bar, s2b = st->s2bar;
  const double *wbar = a.vec + kVecMean * d;

  for (int c = tid; c < kG * EPL; c += kPassBlock) s_ctr[c] = c < d ? wbar[c] : 0.0;
  double accP[EPL], accQ[EPL];
#pragma unroll
  for (int k = 0; k < EPL; ++k) accP[k] = accQ[k] = 0.0;
  double t1 = 0.0, t2 = 0.0, nminP = -INFINITY, maxQ = -INFINITY, nslmin = -INFINITY;

  const int64_t nb = (n + B - 1) / B;
  const int64_t GW = (int64_t)gridDim.x * kPassWaves;
  // lane offsets (bytes) of the lane's column chunks within its row of a
  // load step; chunks past column d get an offset beyond the buffer range
  int32_t voff[EPL / VEC];
#pragma unroll
  for (int q = 0; q < EPL / VEC; ++q) {
    const int c0 = cl * EPL + q * VEC;
    voff[q] = c0 < d ? (int32_t)(((int64_t)g * ld + c0) * (int64_t)sizeof(T)) : kOffInvalid;
  }
  const int32_t step_bytes = (int32_t)(kRowsPerStep * ld * (int64_t)sizeof(T));
  // rows of batch b into registers (rows >= n read as zeros)
  auto load_batch = [&](Regs &xv, int64_t b) {
    const int64_t r0 = b * B;
    const int64_t rows = n - r0 < B ? n - r0 : B;
    const __amdgpu_buffer_rsrc_t rs = rows_rsrc<T>(X, r0, rows, ld, d);
#pragma unroll
    for (int s = 0; s < SB; ++s)
#pragma unroll
      for (int q = 0; q < EPL / VEC; ++q)
        xv.template put<VEC>(s, q, buf_load<T, VEC>(rs, voff[q] + s * step_bytes, 0));
    if constexpr (sizeof(T) == 1) xv.sc = scale_load(a.scales, r0, rows, lane);
  };
  // phases 1-3 on the batch b held in xv
  auto process = [&](Regs &xv, int64_t b) {
    const int64_t r0 = b * B;
    // re-read the candidate each batch: it stays out of registers in phases 2-3
    asm volatile("" ::: "memory");
    // binary64 for every storage type: the binary32 per-element variant of
    // the SES pass is slower here, where a BF16 batch at d = 256 holds 8 rows
    // and its flush to binary64 costs as much as the batch's FMAs
    double ub[EPL];
#pragma unroll
    for (int k = 0; k < EPL; ++k) ub[k] = s_ctr[cl * EPL + k];
#pragma unroll
    for (int s = 0; s < SB; ++s) {
      double dot = 0.0;
#pragma unroll
      for (int k = 0; k < EPL; ++k) dot = fma(xv.get(s, k), ub[k], dot);
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
      if constexpr (sizeof(T) == 1) dot *= (double)xv.sc;  // FP8: x_i = s_i q_i
      const double sl = (isP ? dot : -dot) - (isP ? s1b : s2b);
      // weight exp(-kappa' slack) shifted by the lower bound on the slack
      const double e = valid ? exp(-kappa * (sl - slb)) : 0.0;
      if (isP) t1 += e; else t2 += e;
      if (valid) {
        if (isP) nminP = fmax(nminP, -dot); else maxQ = fmax(maxQ, dot);
        nslmin = fmax(nslmin, -sl);
      }
      s_wa[wave][lane] = sizeof(T) == 1 ? e * (double)xv.sc : e;  // weight of the stored codes
    }
    wave_lds_sync();
    xv.pin();
    if (r0 + B <= n_pos) {
#pragma unroll
      for (int s = 0; s < SB; ++s) {
        const double er = s_wa[wave][s * kRowsPerStep + g];
#pragma unroll
        for (int k = 0; k < EPL; ++k) accP[k] = fma(er, xv.get(s, k), accP[k]);
      }
    } else if (r0 >= n_pos) {
#pragma unroll
      for (int s = 0; s < SB; ++s) {
        const double er = s_wa[wave][s * kRowsPerStep + g];
#pragma unroll
        for (int k = 0; k < EPL; ++k) accQ[k] = fma(er, xv.get(s, k), accQ[k]);
      }
    } else {
#pragma unroll
      for (int s = 0; s < SB; ++s) {
        const double er = s_wa[wave][s * kRowsPerStep + g];
        const bool rp = (r0 + s * kRowsPerStep + g) < n_pos;
        const double eP = rp ? er : 0.0, eQ = rp ? 0.0 : er;
#pragma unroll
        for (int k = 0; k < EPL; ++k) {
          accP[k] = fma(eP, xv.get(s, k), accP[k]);
          accQ[k] = fma(eQ, xv.get(s, k), accQ[k]);
        }
      }
    }
    wave_lds_sync();
  };
  const int64_t b0 = (int64_t)blockIdx.x * kPassWaves + wave;
  // status0 is the same for the whole grid: either every wave returns below
  // (after this barrier) or none does
  __syncthreads();
  if constexpr (PFM == kPrefetchRegs) {
    Regs xa, xb;
    int64_t b = b0;
    load_batch(xa, b);
    if (status0 != kRunning) return;
    while (b < nb) {
      const int64_t b1 = b + GW;
      load_batch(xb, b1);
      process(xa, b);
      if (b1 >= nb) break;
      const int64_t b2 = b1 + GW;
      load_batch(xa, b2);
      process(xb, b1);
      b = b2;
    }
  } else {
    Regs xv;
    for (int64_t b = b0; b < nb; b += GW) {
      load_batch(xv, b);
      // the first batch's loads go out before the state word is waited on
      if (b == b0 && status0 != kRunning) return;
      process(xv, b);
    }
  }
  if (status0 != kRunning) return;

#pragma unroll
  for (int k = 0; k < EPL; ++k) {
    accP[k] += __shfl_xor(accP[k], 16);
    accP[k] += __shfl_xor(accP[k], 32);
    accQ[k] += __shfl_xor(accQ[k], 16);
    accQ[k] += __shfl_xor(accQ[k], 32);
  }
  const int pw = rec_width(d);
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
  // the workgroup's record, or its sums added into the global sum
  const bool to_gsum = a.gsum != nullptr;
  double *rec = to_gsum ? a.gsum : a.partials + (int64_t)blockIdx.x * pw;
  const int dp = rec_dp(d);
  for (int c = tid; c < d; c += kPassBlock) {
    const double v = sum_waves(s_vec, c);
    if (to_gsum)
      gsum_add(rec + c, v);
    else
      rec[c] = v;
  }
  __syncthreads();
  if (g == 0)
#pragma unroll
    for (int k = 0; k < EPL; ++k) s_vec[wave][cl * EPL + k] = accQ[k];
  __syncthreads();
  for (int c = tid; c < d; c += kPassBlock) {
    const double v = sum_waves(s_vec, c);
    if (to_gsum)
      gsum_add(rec + dp + 8 + c, v);
    else
      rec[dp + 8 + c] = v;
  }
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
    if (!to_gsum)
      rec[dp + tid] = v;
    else if (tid < 2)
      gsum_add(rec + dp + tid, v);
    else if (tid >= 4 && tid < 7)
      gsum_max(rec + dp + tid, v);
  }
}

// ===================================================== combine + epilogue
// Section 5 monitor for the mean evaluated by pass k (iteration k-1 >= 1),
// on the LDS copy of the state; one lane.  Returns the new status.
__device__ inline int monitor_rules(DevState &S, int64_t k, double f, bool better, bool beat,
                                    int *copy_best) {
  int status = kRunning;
  S.f_last = f;
  if (!isfinite(f)) return kNumeric;
  if (better) {
    S.f_best = f;
    S.t_best = k - 1;
    *copy_best = 1;
  }
  if (S.early) {
    if (beat) {
      status = kBeat;
    } else {
      if (S.f_prev >= 0.0) {  // a previous monitored iteration exists
        if (S.f_prev > 0.0 && fabs(f - S.f_prev) / S.f_prev < S.delta)
          S.cnt += 1;
        else
          S.cnt = 0;
      }
      S.f_prev = f;
      if (S.cnt >= S.patience) status = kStabilized;
    }
  }
  if (status == kRunning && k - 1 >= S.T) status = kTReached;
  return status;
}

// Columns per lane in the one-wave epilogue: PL = DMAX / 64 for records of
// at most DMAX columns.

// SES epilogue of pass k, one wave: ORACLE of eq.(ses_oracle), separation
// test, running mean and the bound for the next pass's exponent shift.
// S (state), vout (the test's vectors, kNumVec x d) and v1 are LDS copies,
// updated in place (a lane reads and writes only its own columns).
template <int PL>
__device__ inline void ses_epilogue(const PassArgs &a, DevState &S, double *vout, const double *v1,
                                    const double *comb, bool cert, bool centred) {
  const int d = (int)a.d, lane = threadIdx.x & 63;
  const double *y = vout + kVecMean * d, *Sv = vout + kVecS * d;
  const double *sc = comb + rec_dp(d);
  const int64_t k = S.t + 1;
  const double Bsum = sc[0], Esum = sc[1], Gsum = sc[2], BD2 = sc[3], Asum = sc[4];
  const double gmax = sc[5], fall = sc[6];
  int status = kRunning, copy = 0;
  if (lane == 0 && k >= 2) status = monitor_rules(S, k, fall, fall < S.f_best, fall < S.alpha, &copy);
  status = __builtin_amdgcn_readfirstlane(status);  // lane 0's decision
  copy = __builtin_amdgcn_readfirstlane(copy);
  wave_lds_sync();
  if (copy)
    for (int c = lane; c < d; c += kWave) vout[kVecBest * d + c] = y[c];
  if (status != kRunning) {
    if (lane == 0) {
      S.status = status;
      S.t_end = k - 1;
    }
    return;
  }
  // W = sum_i a_i (v_i - ubar) = sum a_i v_i - (sum a_i) ubar.  One
  // butterfly sums ||W||^2, (v1 - ubar).W and, with a certificate,
  // ||sum_i b_i (v_i - ubar)||^2.
  double Wr[PL], u[PL];
  double p = 0.0, r = 0.0, cc = 0.0;
#pragma unroll
  for (int j = 0; j < PL; ++j) {
    const int c = lane + j * kWave;
    // the record holds sum a_i x_i, or (centred) sum a_i (x_i - fl32(ubar))
    Wr[j] = c < d ? comb[c] - Asum * (centred ? y[c] - (double)(float)y[c] : y[c]) : 0.0;
    p += Wr[j] * Wr[j];
    if (c < d) r += (v1[c] - y[c]) * Wr[j];
  }
  if (cert) {
    const double *cx = comb + rec_dp(d) + 8;
    for (int c = lane; c < d; c += kWave) {
      const double cv = cx[c] - Bsum * (centred ? y[c] - (double)(float)y[c] : y[c]);
      cc += cv * cv;
    }
    wave_sum3(p, r, cc);
  } else {
    wave_sum2(p, r);
  }
  const double nW = sqrt(p);
  const double alpha = S.alpha, g1 = S.gamma1;
#pragma unroll
  for (int j = 0; j < PL; ++j) {
    const int c = lane + j * kWave;
    u[j] = 0.0;
    if (c < d) u[j] = nW > 0.0 ? v1[c] + (alpha - g1) * (Wr[j] / nW) : v1[c];
  }
  // sum_i (u - v_i).w_i + (alpha - gamma_i) s_i, scaled by sqrt2 C e^{-M}:
  // (u - ubar).W - sum (e+ - e-) d_i + alpha sum b_i - sum gamma_i b_i, where
  // (u - ubar).W = (v1 - ubar).W + (alpha - gamma1) ||W||.
  const double q = nW > 0.0 ? r + (alpha - g1) * nW : r;
  const double obj = q - Esum + alpha * Bsum - Gsum;
  const double scale = alpha * (nW + Bsum);
  const double lb2 = cert ? BD2 / Bsum - cc / (Bsum * Bsum) : 0.0;
  const bool bad = !isfinite(obj) || !(Bsum > 0.0) || !isfinite(nW);
  const bool separated = obj < -S.tau * scale;
#pragma unroll
  for (int j = 0; j < PL; ++j) {
    const int c = lane + j * kWave;
    if (c < d) vout[kVecLast * d + c] = u[j];
  }
  double dl = 0.0;
  if (!bad && !separated) {
#pragma unroll
    for (int j = 0; j < PL; ++j) {
      const int c = lane + j * kWave;
      if (c < d) {
        const double sm = Sv[c] + u[j];
        const double yn = sm / (double)k;
        const double dd = yn - y[c];
        dl += dd * dd;
        vout[kVecS * d + c] = sm;
        vout[kVecMean * d + c] = yn;
      }
    }
  }
  const double Delta = sqrt(wave_sum(dl));
  if (lane == 0) {
    const double M = S.kscale * (double)S.t * (S.shift_bound - alpha);
    S.value = obj / (M_SQRT2 * Bsum);
    S.scale = scale / (M_SQRT2 * Bsum);
    S.log_trace = M + log(Bsum);
    S.degenerate = !(nW > 0.0);
    S.cert = cert ? 1 : 0;
    if (cert && a.radii == nullptr) S.bound = fmax(S.bound, sqrt(fmax(lb2, 0.0)));
    if (bad || separated) {
      S.status = bad ? kNumeric : kSeparated;
      S.t_end = k;
    } else {
      // ||v_i - ubar(k)|| <= ||v_i - ubar(k-1)|| + ||ubar(k) - ubar(k-1)||
      S.shift_bound = gmax + Delta;
      S.t = k;
    }
  }
}

// SVM epilogue of pass k, one wave: ORACLE of eq.(svm_oracle), separation
// test, the polytope-distance certificate, running means, next slack bound.
template <int PL>
__device__ inline void svm_epilogue(const PassArgs &a, DevState &S, double *vout, const double *comb) {
  const int d = (int)a.d, lane = threadIdx.x & 63;
  const double *wb = vout + kVecMean * d, *Sv = vout + kVecS * d;
  const double *sc = comb + rec_dp(d);
  const double *AP = comb, *AQ = comb + rec_dp(d) + 8;
  const int64_t k = S.t + 1;
  const double T1 = sc[0], T2 = sc[1];
  const double minP = -sc[4], maxQ = sc[5], slmin = -sc[6];
  int status = kRunning, copy = 0;
  if (lane == 0 && k >= 2) {
    const double nw = S.wbar_norm;
    const double f = nw > 0.0 ? fmax((minP - maxQ) / nw, 0.0) : 0.0;
    status = monitor_rules(S, k, f, f > S.f_best, f > S.alpha, &copy);
  }
  status = __builtin_amdgcn_readfirstlane(status);  // lane 0's decision
  copy = __builtin_amdgcn_readfirstlane(copy);
  wave_lds_sync();
  if (copy)
    for (int c = lane; c < d; c += kWave) vout[kVecBest * d + c] = wb[c];
  if (status != kRunning) {
    if (lane == 0) {
      S.status = status;
      S.t_end = k - 1;
    }
    return;
  }
  const bool both = T1 > 0.0 && T2 > 0.0;
  double p = 0.0, pu = 0.0;
  for (int c = lane; c < d; c += kWave) {
    const double V = AP[c] - AQ[c];
    p += V * V;
    if (both) {
      const double U = AP[c] / T1 - AQ[c] / T2;
      pu += U * U;
    }
  }
  wave_sum2(p, pu);
  const double nV = sqrt(p);
  const double ub = both ? sqrt(pu) : INFINITY;
  const double alpha = S.alpha, D = S.D;
  const double s1 = (T1 <= T2) ? D : alpha - D;
  const double s2 = alpha - s1;
  const double obj = nV - T1 * s1 - T2 * s2;
  const double scale = nV + T1 * fabs(s1) + T2 * fabs(s2);
  const bool bad = !isfinite(obj) || !(T1 + T2 > 0.0);
  const bool separated = obj < -S.tau * scale;
  double w[PL];
#pragma unroll
  for (int j = 0; j < PL; ++j) {
    const int c = lane + j * kWave;
    w[j] = 0.0;
    if (c < d) {
      w[j] = nV > 0.0 ? (AP[c] - AQ[c]) / nV : 0.0;
      vout[kVecLast * d + c] = w[j];
    }
  }
  double dl = 0.0, wn = 0.0;
  if (!bad && !separated) {
#pragma unroll
    for (int j = 0; j < PL; ++j) {
      const int c = lane + j * kWave;
      if (c < d) {
        const double sm = Sv[c] + w[j];
        const double yn = sm / (double)k;
        const double dd = yn - wb[c];
        dl += dd * dd;
        wn += yn * yn;
        vout[kVecS * d + c] = sm;
        vout[kVecMean * d + c] = yn;
      }
    }
  }
  wave_sum2(dl, wn);
  const double Dw = sqrt(dl);
  const double nwb = sqrt(wn);
  if (lane == 0) {
    const double M = -S.kscale * (double)S.t * S.shift_bound;
    S.value = obj / (T1 + T2);
    S.scale = scale / (T1 + T2);
    S.log_trace = M + log(T1 + T2);
    S.degenerate = !(nV > 0.0);
    S.bound = fmin(S.bound, ub);
    S.s1_last = s1;
    S.s2_last = s2;
    if (bad || separated) {
      S.status = bad ? kNumeric : kSeparated;
      S.t_end = k;
    } else {
      S.S1 += s1;
      S.S2 += s2;
      const double n1 = S.S1 / (double)k, n2 = S.S2 / (double)k;
      const double ds = fmax(fabs(n1 - S.s1bar), fabs(n2 - S.s2bar));
      S.s1bar = n1;
      S.s2bar = n2;
      S.wbar_norm = nwb;
      // slack_i(k) >= slack_i(k-1) - ||x_i|| ||dwbar|| - |dsbar_c|, ||x_i|| <= D
      S.shift_bound = slmin - D * Dw - ds;
      S.t = k;
    }
  }
}

// Columns of a record the epilogue reads: SES without a certificate skips the
// second vector.
template <int PROB, bool CERT>
__host__ __device__ inline int rec_read_cols(int d) {
  return (PROB == kSES && !CERT) ? rec_dp(d) + 8 : rec_width(d);
}

// First level of the record combine (large records only): workgroup g sums
// records [g * kRecGroup, (g + 1) * kRecGroup) column by column in record
// order (the maximum slots by max) into record g of `out`.
template <int PROB, bool CERT>
__global__ __launch_bounds__(kBlock) void record_combine_kernel(const double *__restrict__ in, int P, int d,
                                                                double *__restrict__ out) {
  const int dp = rec_dp(d), pw = rec_width(d);
  const int ncols = rec_read_cols<PROB, CERT>(d);
  const int nsc = PROB == kSES ? 5 : 4;
  const int b0 = blockIdx.x * kRecGroup;
  const int b1 = b0 + kRecGroup < P ? b0 + kRecGroup : P;
  for (int c = threadIdx.x; c < ncols; c += kBlock) {
    const bool mx = c >= dp + nsc && c < dp + 8;
    double acc = mx ? -INFINITY : 0.0;
#pragma unroll 16
    for (int b = b0; b < b1; ++b) {
      const double v = in[(int64_t)b * pw + c];
      acc = mx ? fmax(acc, v) : acc + v;
    }
    out[(int64_t)blockIdx.x * pw + c] = acc;
  }
}

static_assert(sizeof(DevState) % 8 == 0, "DevState is copied as 8-byte words");
constexpr int kStateWords = (int)(sizeof(DevState) / 8);

// Record groups of the fixed-order combine: column pairs are summed over
// `groups` interleaved record subsets (record b in subset b mod groups, each
// in increasing order), then the subset sums in subset order.  The order
// depends on the record width only, so every kernel that combines a set of
// records (the epilogue kernel, every workgroup of the fused pass) gets the
// same bits.
__host__ __device__ inline int comb_groups(int npairs) {
  const int g = 1024 / (npairs > 0 ? npairs : 1);
  return g < 1 ? 1 : (g > 8 ? 8 : g);
}
constexpr int kCombAcc = 2048;  // >= comb_groups(p) * 2p for every p

// LDS image of one epilogue: the state, the test's vectors (S, mean, best,
// last), row v1 and the combined record.
template <int DMAX>
struct EpiLDS {
  DevState st;
  double vout[kNumVec * DMAX];
  double v1[DMAX];
  double comb[2 * DMAX + 8];
  double acc[kCombAcc];
};

// Fixed-order sum of P records (the maximum slots by max) into L.comb; all NT
// threads call it.
template <int PROB, bool CERT, int NT, int DMAX>
__device__ __forceinline__ void combine_records(const double *__restrict__ rec, int P, int d, EpiLDS<DMAX> &L) {
  const int dp = rec_dp(d), pw = rec_width(d);
  const int ncols = rec_read_cols<PROB, CERT>(d);
  const int nsc = PROB == kSES ? 5 : 4;  // summed scalars; the rest are maxima
  const int npairs = ncols / 2;
  const int groups = comb_groups(npairs);
  for (int jp = threadIdx.x; jp < npairs * groups; jp += NT) {
    const int j = jp % npairs, grp = jp / npairs;
    const int c0 = 2 * j;
    const bool m0 = c0 >= dp + nsc && c0 < dp + 8, m1 = c0 + 1 >= dp + nsc && c0 + 1 < dp + 8;
    double acc0 = m0 ? -INFINITY : 0.0, acc1 = m1 ? -INFINITY : 0.0;
#pragma unroll 8
    for (int b = grp; b < P; b += groups) {
      const double2 v = *reinterpret_cast<const double2 *>(rec + (int64_t)b * pw + c0);
      acc0 = m0 ? fmax(acc0, v.x) : acc0 + v.x;
      acc1 = m1 ? fmax(acc1, v.y) : acc1 + v.y;
    }
    L.acc[grp * ncols + c0] = acc0;
    L.acc[grp * ncols + c0 + 1] = acc1;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < ncols; c += NT) {
    const bool mx = c >= dp + nsc && c < dp + 8;
    double r = mx ? -INFINITY : 0.0;
    for (int g = 0; g < groups; ++g) r = mx ? fmax(r, L.acc[g * ncols + c]) : r + L.acc[g * ncols + c];
    L.comb[c] = r;
  }
  __syncthreads();
}

// The epilogue of the records `rec` (P of them) on the state st_in and the
// vectors vec_in, into LDS: every read is issued at once, the records are
// combined in the fixed order, and one wave runs the FP64 epilogue.  It runs
// when the test is running and records are pending (`force`: the caller knows
// they are, i.e. a pass kernel just ran; otherwise DevState::pending says so).
// All NT threads call it; afterwards L.st and L.vout hold the new state and
// vectors (unchanged when nothing ran).
template <typename T, int PROB, bool CERT, int NT, int DMAX>
__device__ __forceinline__ void epilogue_load(const PassArgs &a, const DevState *st_in, const double *vec_in,
                                              EpiLDS<DMAX> &L) {
  const int d = (int)a.d, tid = threadIdx.x;
  if (tid < kStateWords) reinterpret_cast<double *>(&L.st)[tid] = reinterpret_cast<const double *>(st_in)[tid];
  for (int c = tid; c < kNumVec * d; c += NT) L.vout[c] = vec_in[c];
  if (PROB == kSES)
    for (int c = tid; c < d; c += NT) L.v1[c] = row_value<T>(a, a.v1, c);
}

template <typename T, int PROB, bool CERT, int NT, int DMAX>
__device__ __forceinline__ void epilogue_tail(const PassArgs &a, EpiLDS<DMAX> &L) {
  if (threadIdx.x < kWave) {
    if (PROB == kSES)
      ses_epilogue<DMAX / kWave>(a, L.st, L.vout, L.v1, L.comb, CERT, sizeof(T) <= 2);
    else
      svm_epilogue<DMAX / kWave>(a, L.st, L.vout, L.comb);
  }
  __syncthreads();
}

// gmode: rec is one global sum of a fused pass (SES), its maxima as keys.
template <typename T, int PROB, bool CERT, int NT, int DMAX>
__device__ __forceinline__ void epilogue_stage(const PassArgs &a, const DevState *st_in, const double *vec_in,
                                               const double *rec, int P, bool force, EpiLDS<DMAX> &L,
                                               bool gmode = false) {
  epilogue_load<T, PROB, CERT, NT, DMAX>(a, st_in, vec_in, L);
  __syncthreads();
  if (L.st.status != kRunning || !(force || L.st.pending)) return;  // uniform: read from LDS
  if (gmode) {
    const int dp = rec_dp((int)a.d), ncols = rec_read_cols<PROB, CERT>((int)a.d);
    const int nsc = PROB == kSES ? 5 : 4;  // summed scalars; then the maxima up to slot 6
    for (int c = threadIdx.x; c < ncols; c += NT)
      L.comb[c] = (c >= dp + nsc && c <= dp + 6)
                      ? from_max_key((unsigned long long)__double_as_longlong(rec[c])) : rec[c];
    __syncthreads();
  } else {
    combine_records<PROB, CERT, NT, DMAX>(rec, P, (int)a.d, L);
  }
  epilogue_tail<T, PROB, CERT, NT, DMAX>(a, L);
}

// Write L's state (with the given pending flag) and vectors to global memory.
template <int NT, int DMAX>
__device__ __forceinline__ void epilogue_store(EpiLDS<DMAX> &L, int d, int32_t pending, DevState *st_out,
                                               double *vec_out) {
  if (threadIdx.x == 0) L.st.pending = pending;
  __syncthreads();
  if (threadIdx.x < kStateWords)
    reinterpret_cast<double *>(st_out)[threadIdx.x] = reinterpret_cast<const double *>(&L.st)[threadIdx.x];
  for (int c = threadIdx.x; c < kNumVec * d; c += NT) vec_out[c] = L.vout[c];
}

// One workgroup per iteration (the batched epilogue: one per instance), in
// place on a.st / a.vec.  The kernel boundary after the pass makes every
// record visible: no fences.  force: records of a pass that just ran are
// there (the unfused iteration); otherwise only pending records are applied
// (the flush after fused passes).
// gmode: a.partials is one global sum; it is cleared after it is read (the
// next unfused pass adds into it).
template <typename T, int PROB, bool CERT, int NT = kCombBlock>
__device__ __forceinline__ void epilogue_body(const PassArgs &a, int P, bool force = true, bool gmode = false) {
  __shared__ EpiLDS<kMaxD> L;
  epilogue_stage<T, PROB, CERT, NT, kMaxD>(a, a.st, a.vec, a.partials, P, force, L, gmode);
  epilogue_store<NT, kMaxD>(L, (int)a.d, 0, a.st, a.vec);
  if (gmode)
    for (int c = threadIdx.x; c < rec_width((int)a.d); c += NT) a.partials[c] = 0.0;
}

template <typename T, int PROB, bool CERT>
__global__ __launch_bounds__(kCombBlock) void epilogue_kernel(PassArgs a, int P, int force, int gmode) {
  epilogue_body<T, PROB, CERT>(a, P, force != 0, gmode != 0);
}

// ============================================== fused epilogue + SES pass
// One MWU iteration in one launch: every workgroup first runs the epilogue of
// the previous pass (its records, state and vectors in slot `cur` of two)
// on its own, redundantly and in the same fixed order, so all workgroups
// agree bit for bit on the new mean, shift bound and status; workgroup 0
// writes the new state and vectors to slot 1 - cur, and the pass writes its
// records to slot 1 - cur.  The previous kernel's boundary makes its records
// visible; nobody writes what this launch reads.  Records are small
// (d <= 128, a few hundred KB over all workgroups), so each workgroup reads
// them from L2.
//
// Loads return in order, so the records are requested first (pre()): a
// thread's first (column pair, record subset) item has all of its loads in
// flight before the first batch of rows is requested, and the combine and
// the FP64 tail run while those rows arrive from HBM.  Stale records (none
// pending) are read harmlessly and ignored.  The item is summed in the order
// combine_records uses, so the result is bitwise that of the epilogue kernel.
constexpr int kFuseMaxD = 128;
constexpr int kRecInFlight = 32;

// With global sums (GS) the previous pass left one sum in g_in instead of P
// records: each thread loads one of its columns, the pass adds into g_out,
// and workgroup 0 clears g_zero (the slot the pass after next adds into, last
// read by the previous pass) -- three slots in rotation.  GS is a template
// parameter so that the global-sum kernel does not hold the record loads'
// registers across its first batch of rows.
template <typename T, int NT, int DMAX, bool GS>
struct FusedPrologue {
  const PassArgs &a;
  int cur, P;
  int64_t rec_stride;
  double *g_in, *g_out, *g_zero;
  EpiLDS<DMAX> &L;
  double2 rv[GS ? 1 : kRecInFlight];
  double gv;           // gmode: a column of the global sum
  double sv, vv, v1v;  // a state word, a vector element, an element of row v1

  static_assert(NT >= kNumVec * DMAX && NT >= kStateWords, "one thread per vector element and state word");

  __device__ __forceinline__ int npairs() const { return rec_read_cols<kSES, false>((int)a.d) / 2; }

  __device__ __forceinline__ void pre() {
    const int d = (int)a.d, tid = threadIdx.x;
    const int pw = rec_width(d), np = npairs(), groups = comb_groups(np);
    const double *rec = a.partials + cur * rec_stride;
    if constexpr (GS) gv = tid < 2 * np ? g_in[tid] : 0.0;
    // state, vectors and row v1 into registers (written to LDS in post())
    sv = tid < kStateWords ? reinterpret_cast<const double *>(a.st + cur)[tid] : 0.0;
    vv = tid < kNumVec * d ? a.vec[cur * (int64_t)kNumVec * d + tid] : 0.0;
    v1v = tid < d ? row_value<T>(a, a.v1, tid) : 0.0;
    if constexpr (!GS) {
      if (tid < np * groups) {
        const int c0 = 2 * (tid % np), g0 = tid / np;
#pragma unroll
        for (int r = 0; r < kRecInFlight; ++r) {
          const int b = g0 + r * groups;
          rv[r] = b < P ? *reinterpret_cast<const double2 *>(rec + (int64_t)b * pw + c0) : make_double2(0.0, 0.0);
        }
      }
    }
  }

  __device__ __forceinline__ PassIn post() {
    const int d = (int)a.d, tid = threadIdx.x;
    const int64_t vs = (int64_t)kNumVec * d;
    const int dp = rec_dp(d), pw = rec_width(d);
    const int np = npairs(), ncols = 2 * np, groups = comb_groups(np), items = np * groups;
    constexpr int nsc = 5;
    const double *rec = a.partials + cur * rec_stride;
    if (tid < kStateWords) reinterpret_cast<double *>(&L.st)[tid] = sv;
    if (tid < kNumVec * d) L.vout[tid] = vv;
    if (tid < d) L.v1[tid] = v1v;
    if (GS && tid < ncols)
      L.comb[tid] = (tid == dp + 5 || tid == dp + 6) ? from_max_key((unsigned long long)__double_as_longlong(gv)) : gv;
    if (blockIdx.x == 0 && g_zero != nullptr)
      for (int c = tid; c < pw; c += NT) g_zero[c] = 0.0;
    __syncthreads();
    if constexpr (GS) {
      if (L.st.status == kRunning && L.st.pending) epilogue_tail<T, kSES, false, NT, DMAX>(a, L);
    } else if (L.st.status == kRunning && L.st.pending) {  // uniform: read from LDS
      for (int jp = tid; jp < items; jp += NT) {
        const int j = jp % np, grp = jp / np;
        const int c = 2 * j;
        const bool m0 = c >= dp + nsc && c < dp + 8, m1 = c + 1 >= dp + nsc && c + 1 < dp + 8;
        double acc0 = m0 ? -INFINITY : 0.0, acc1 = m1 ? -INFINITY : 0.0;
        int b = grp;
        if (jp == tid) {  // the item whose loads are in flight
#pragma unroll
          for (int r = 0; r < (GS ? 1 : kRecInFlight); ++r) {
            if (b < P) {
              acc0 = m0 ? fmax(acc0, rv[r].x) : acc0 + rv[r].x;
              acc1 = m1 ? fmax(acc1, rv[r].y) : acc1 + rv[r].y;
            }
            b += groups;
          }
        }
        for (; b < P; b += groups) {
          const double2 v = *reinterpret_cast<const double2 *>(rec + (int64_t)b * pw + c);
          acc0 = m0 ? fmax(acc0, v.x) : acc0 + v.x;
          acc1 = m1 ? fmax(acc1, v.y) : acc1 + v.y;
        }
        L.acc[grp * ncols + c] = acc0;
        L.acc[grp * ncols + c + 1] = acc1;
      }
      __syncthreads();
      for (int c = tid; c < ncols; c += NT) {
        const bool mx = c >= dp + nsc && c < dp + 8;
        double r = mx ? -INFINITY : 0.0;
        for (int g = 0; g < groups; ++g) r = mx ? fmax(r, L.acc[g * ncols + c]) : r + L.acc[g * ncols + c];
        L.comb[c] = r;
      }
      __syncthreads();
      epilogue_tail<T, kSES, false, NT, DMAX>(a, L);
    }
    if (blockIdx.x == 0)
      epilogue_store<NT, DMAX>(L, d, L.st.status == kRunning ? 1 : 0, a.st + (1 - cur), a.vec + (1 - cur) * vs);
    if constexpr (GS)
      return PassIn{L.st.status, L.st.kscale * (double)L.st.t, L.st.shift_bound, L.vout + kVecMean * d, g_out, true};
    return PassIn{L.st.status, L.st.kscale * (double)L.st.t, L.st.shift_bound, L.vout + kVecMean * d,
                  a.partials + (1 - cur) * rec_stride, false};
  }
};

template <typename T, int EPL, int VEC, bool CERT, int PFM, bool GS>
__global__ __launch_bounds__(kPassBlock) __attribute__((amdgpu_waves_per_eu(SCPMWU_PASS_WAVES)))
void ses_fused_kernel(PassArgs a, int cur, int P, int64_t rec_stride, double *g_in, double *g_out,
                      double *g_zero) {
  static_assert(kG * EPL <= kFuseMaxD, "fused pass: d <= 128");
  __shared__ EpiLDS<kFuseMaxD> L;
  FusedPrologue<T, kPassBlock, kFuseMaxD, GS> pro{a, cur, P, rec_stride, g_in, g_out, g_zero, L};
  ses_pass_body<T, EPL, VEC, CERT, PFM>(a, (int)blockIdx.x, (int)gridDim.x, pro);
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
        const double x = row_value<T>(a, row, c);
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
      // a non-finite input value must not vanish in fmax (which drops NaN):
      // it turns the maxima into +inf, which the host rejects
      if (mode == 0) {
        double h = sqrt(acc) + (a.radii ? a.radii[row] : 0.0);
        if (!isfinite(h)) h = INFINITY;
        if (row != exclude) r0 = fmax(r0, h);
        r1 = fmax(r1, h);
      } else {
        const double v = isfinite(acc) ? acc : INFINITY;
        if (row < a.n_pos) r2 = fmax(r2, isfinite(acc) ? -acc : INFINITY); else r3 = fmax(r3, v);
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
__device__ __forceinline__ void ftp_init_body(const PassArgs &a, const InitParams &p, int problem) {
  DevState *st = a.st;
  const int d = (int)a.d;
  const int tid = threadIdx.x;
  for (int c = tid; c < d; c += kBlock) {
    double y0 = 0.0;
    if (problem == kSES) y0 = row_value<T>(a, a.v1, c);
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

template <typename T>
__global__ __launch_bounds__(kBlock) void ftp_init_kernel(PassArgs a, InitParams p, int problem) {
  ftp_init_body<T>(a, p, problem);
}

// ============================================================== dispatch
template <typename T, int EPL, int VEC, int PFM>
hipError_t launch_pass_p(int problem, bool cert, int grid, const PassArgs &a, hipStream_t s) {
  if (problem == kSES) {
    if (cert)
      hipLaunchKernelGGL((ses_pass_kernel<T, EPL, VEC, true, PFM>), dim3(grid), dim3(kPassBlock), 0, s, a);
    else
      hipLaunchKernelGGL((ses_pass_kernel<T, EPL, VEC, false, PFM>), dim3(grid), dim3(kPassBlock), 0, s, a);
  } else {
    hipLaunchKernelGGL((svm_pass_kernel<T, EPL, VEC, PFM>), dim3(grid), dim3(kPassBlock), 0, s, a);
  }
  return hipGetLastError();
}

template <typename T, int EPL, int VEC>
hipError_t launch_pass_t(int problem, const LaunchCfg &c, const PassArgs &a, hipStream_t s) {
  return c.pfm == kPrefetchRegs ? launch_pass_p<T, EPL, VEC, kPrefetchRegs>(problem, c.cert, c.grid, a, s)
                                : launch_pass_p<T, EPL, VEC, kPrefetchNone>(problem, c.cert, c.grid, a, s);
}

template <typename T, int PROB, bool CERT>
hipError_t launch_epilogue_p(int grid, const PassArgs &a, hipStream_t s) {
  if (a.gsum != nullptr) {  // the pass added into one global sum
    PassArgs e = a;
    e.partials = a.gsum;
    hipLaunchKernelGGL((epilogue_kernel<T, PROB, CERT>), dim3(1), dim3(kCombBlock), 0, s, e, 1, 1, 1);
    return hipGetLastError();
  }
  // records of the pass: a.partials[0 .. grid); group sums after them
  PassArgs e = a;
  int P = grid;
  const int d = (int)a.d;
  if (rec_two_level(grid, rec_read_cols<PROB, CERT>(d))) {
    double *l1 = a.partials + (int64_t)grid * rec_width(d);
    hipLaunchKernelGGL((record_combine_kernel<PROB, CERT>), dim3(rec_groups(grid)), dim3(kBlock), 0, s, a.partials,
                       grid, d, l1);
    e.partials = l1;
    P = rec_groups(grid);
  }
  hipLaunchKernelGGL((epilogue_kernel<T, PROB, CERT>), dim3(1), dim3(kCombBlock), 0, s, e, P, 1, 0);
  return hipGetLastError();
}

// The flush after fused passes: the pending records (or global sum, gmode)
// in a.partials applied in place on a.st / a.vec.
template <typename T>
hipError_t launch_flush_typed(bool cert, int P, bool gmode, const PassArgs &a, hipStream_t s) {
  if (cert)
    hipLaunchKernelGGL((epilogue_kernel<T, kSES, true>), dim3(1), dim3(kCombBlock), 0, s, a, P, 0, gmode ? 1 : 0);
  else
    hipLaunchKernelGGL((epilogue_kernel<T, kSES, false>), dim3(1), dim3(kCombBlock), 0, s, a, P, 0, gmode ? 1 : 0);
  return hipGetLastError();
}

template <typename T, int EPL, int VEC, int PFM, bool GS>
hipError_t launch_fused_g(bool cert, int grid, const PassArgs &a, const FusedSlots &f, hipStream_t s) {
  if (cert)
    hipLaunchKernelGGL((ses_fused_kernel<T, EPL, VEC, true, PFM, GS>), dim3(grid), dim3(kPassBlock), 0, s, a, f.cur,
                       grid, f.rec_stride, f.g_in, f.g_out, f.g_zero);
  else
    hipLaunchKernelGGL((ses_fused_kernel<T, EPL, VEC, false, PFM, GS>), dim3(grid), dim3(kPassBlock), 0, s, a, f.cur,
                       grid, f.rec_stride, f.g_in, f.g_out, f.g_zero);
  return hipGetLastError();
}

template <typename T, int EPL, int VEC, int PFM>
hipError_t launch_fused_p(bool cert, int grid, const PassArgs &a, const FusedSlots &f, hipStream_t s) {
  if constexpr (kG * EPL <= kFuseMaxD) {
    return f.g_in != nullptr ? launch_fused_g<T, EPL, VEC, PFM, true>(cert, grid, a, f, s)
                             : launch_fused_g<T, EPL, VEC, PFM, false>(cert, grid, a, f, s);
  } else {
    return hipErrorInvalidValue;
  }
}

template <typename T, int EPL, int VEC>
hipError_t launch_fused_t(const LaunchCfg &c, const PassArgs &a, const FusedSlots &f, hipStream_t s) {
  return c.pfm == kPrefetchRegs ? launch_fused_p<T, EPL, VEC, kPrefetchRegs>(c.cert, c.grid, a, f, s)
                                : launch_fused_p<T, EPL, VEC, kPrefetchNone>(c.cert, c.grid, a, f, s);
}

template <typename T, int EPL>
hipError_t launch_fused_v(const LaunchCfg &c, const PassArgs &a, const FusedSlots &f, hipStream_t s) {
  constexpr int VF = (16 / (int)sizeof(T)) < EPL ? (16 / (int)sizeof(T)) : EPL;
  if (c.vec == VF) return launch_fused_t<T, EPL, VF>(c, a, f, s);
  if constexpr (VF >= 4) {
    if (c.vec == VF / 2) return launch_fused_t<T, EPL, VF / 2>(c, a, f, s);
  }
  if constexpr (VF > 1) {
    if (c.vec == 1) return launch_fused_t<T, EPL, 1>(c, a, f, s);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_fused_typed(const LaunchCfg &c, const PassArgs &a, const FusedSlots &f, hipStream_t s) {
  switch (c.epl) {
    case 1: return launch_fused_v<T, 1>(c, a, f, s);
    case 2: return launch_fused_v<T, 2>(c, a, f, s);
    case 4: return launch_fused_v<T, 4>(c, a, f, s);
    case 8: return launch_fused_v<T, 8>(c, a, f, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_epilogue_typed(int problem, bool cert, int grid, const PassArgs &a, hipStream_t s) {
  if (problem == kSES)
    return cert ? launch_epilogue_p<T, kSES, true>(grid, a, s) : launch_epilogue_p<T, kSES, false>(grid, a, s);
  return launch_epilogue_p<T, kSVM, false>(grid, a, s);
}

template <typename T, int EPL>
hipError_t launch_pass_v(int problem, const LaunchCfg &c, const PassArgs &a, hipStream_t s) {
  constexpr int VF = (16 / (int)sizeof(T)) < EPL ? (16 / (int)sizeof(T)) : EPL;
  if (c.vec == VF) return launch_pass_t<T, EPL, VF>(problem, c, a, s);
  if constexpr (VF >= 4) {
    if (c.vec == VF / 2) return launch_pass_t<T, EPL, VF / 2>(problem, c, a, s);
  }
  if constexpr (VF > 1) {
    if (c.vec == 1) return launch_pass_t<T, EPL, 1>(problem, c, a, s);
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
