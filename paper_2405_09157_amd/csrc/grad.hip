// Reverse pass of the SES radius after T fixed-alpha iterations: the adjoint
// recursion through the unrolled iterations (Section 4.1 split, eq.(ses_oracle),
// Section 2.1 SOC exponential), with the running sum stored every K <= 50
// iterations and each segment recomputed forward before it is reversed, or
// with the whole tape (O(d) numbers per iteration) kept from one forward run.
//
// Per iteration t (reverse order), with lambda the adjoint of S_t:
//   lambda_W = alpha (I - What What^T) lambda / ||W_t||
//   row i != v1: delta_i = v_i - c_t, a_i, a_i' = da/dd, beta_i = a_i' (delta_i . lambda_W) / d_i;
//                grad_i += a_i lambda_W + beta_i delta_i
//   lambda <- lambda - (sum_i a_i lambda_W + beta_i delta_i) / (t - 1)
//   (the rows' own terms are kept as the two coefficients a_i, beta_i per
//   iteration and contracted once per segment)
//   v1 collects lambda (u(t) = v1 + ...); D collects -kappa_t/D sum_i (da_i/dkappa)(delta_i . lambda_W)
// and finally R's own term at its active row and D's at v1 and its far row.
//
// Lanes run over the columns of a row (16 lanes per row for d <= 64, else 64
// lanes with PER <= 8 columns each); each wave takes rows kRB at a time (all
// loads issued before the arithmetic) and reduces a row's sums with a
// butterfly.  The per-iteration passes run one workgroup per CU, so that
// their one-workgroup epilogues sum one partial row per CU; the per-segment
// contraction of the rows' coefficients is a binary64 MFMA product.  All
// arithmetic is binary64 on the stored values (FP32, FP64 or BF16 points,
// widened exactly); the gradient is accumulated in a binary64 workspace and
// rounded once to the caller's FP32 buffer.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "../../include/scp_mwu.h"
#include "grad.hpp"

namespace scpmwu {
namespace grad {

constexpr int kBlk = 256, kW = 64, kNW = kBlk / kW, kMaxPer = 8, kRB = 4;
constexpr int kEpi = 1024;  // threads of the one-workgroup epilogues
constexpr int kMaxCols = kMaxPer * kW;
// The per-iteration passes run one workgroup per CU (grid `pgrid`), so that
// their epilogues sum one partial row per CU: 16 waves for the forward pass,
// 12 for the reverse pass (whose registers allow three waves per SIMD).
constexpr int kFwdBlk = 1024, kBwdBlk = 768;

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kW);
  return v;
}

// Lanes of one wave exchange values through LDS: a wave's DS instructions
// run in order, so a compiler barrier is all that is needed.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum over the NT threads of one workgroup (every thread gets the result).
template <int NT>
__device__ __forceinline__ double bsum(double v, double *s_r) {
  v = wsum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s_r[w] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int q = 0; q < NT / kW; ++q) r += s_r[q];
  return r;
}

template <typename P>
__device__ __forceinline__ double xval(const Buffers &b, int64_t i, int col) {
  return (double)((const P *)b.X)[i * b.ld + col];
}
// BF16 storage: the stored value, exactly (the upper half of a binary32)
template <>
__device__ __forceinline__ double xval<uint16_t>(const Buffers &b, int64_t i, int col) {
  const uint16_t h = ((const uint16_t *)b.X)[i * b.ld + col];
  return (double)__uint_as_float((uint32_t)h << 16);
}

// dst[c] = sum over the grid's partial rows of column c, c < ncol, by the NT
// threads of one workgroup (fixed order).  Rows are part_stride(ncol - 2)
// apart; each thread sums one pair of adjacent columns (16-byte loads, four
// in flight), which halves the load instructions of the one compute unit
// that runs the epilogue.  tmp holds 2 NT doubles.
template <int NT>
__device__ void reduce_parts(const double *part, int G, int ncol, double *dst, double *tmp) {
  const int tid = threadIdx.x, np = (ncol + 1) / 2;
  const int64_t ps = part_stride(ncol - 2);
  for (int p0 = 0; p0 < np; p0 += NT) {
    const int span = np - p0 < NT ? np - p0 : NT;
    const int groups = NT / span;
    const int grp = tid / span, c = 2 * (p0 + tid - grp * span);
    double2 a0 = make_double2(0.0, 0.0), a1 = a0, a2 = a0, a3 = a0;
    if (grp < groups) {
      const double *col = part + c;
      int g = grp;
      for (; g + 3 * groups < G; g += 4 * groups) {
        const double2 v0 = *reinterpret_cast<const double2 *>(col + (int64_t)g * ps);
        const double2 v1 = *reinterpret_cast<const double2 *>(col + (int64_t)(g + groups) * ps);
        const double2 v2 = *reinterpret_cast<const double2 *>(col + (int64_t)(g + 2 * groups) * ps);
        const double2 v3 = *reinterpret_cast<const double2 *>(col + (int64_t)(g + 3 * groups) * ps);
        a0.x += v0.x, a0.y += v0.y, a1.x += v1.x, a1.y += v1.y;
        a2.x += v2.x, a2.y += v2.y, a3.x += v3.x, a3.y += v3.y;
      }
      for (; g < G; g += groups) {
        const double2 v = *reinterpret_cast<const double2 *>(col + (int64_t)g * ps);
        a0.x += v.x, a0.y += v.y;
      }
    }
    tmp[2 * tid] = (a0.x + a1.x) + (a2.x + a3.x);
    tmp[2 * tid + 1] = (a0.y + a1.y) + (a2.y + a3.y);
    __syncthreads();
    for (int e = tid; e < 2 * span; e += NT) {  // column 2 p0 + e
      const int k = e >> 1, h = e & 1;
      double r = 0.0;
      for (int q = 0; q < groups; ++q) r += tmp[2 * (q * span + k) + h];
      if (2 * p0 + e < ncol) dst[2 * p0 + e] = r;
    }
    __syncthreads();
  }
}

// ---- forward iteration t = t0 + 1 + slot: partial sums of W_t
template <typename P, int PER>
__global__ __launch_bounds__(kFwdBlk) void fwd_pass(Buffers b, int slot) {
  constexpr int RB = PER >= 8 ? 2 : kRB;  // rows in flight per wave (registers)
  constexpr int NW = kFwdBlk / kW;
  __shared__ double red[NW][kMaxCols];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, d = (int)b.d;
  const double *c = b.tc + (int64_t)slot * d;
  const double kap = b.ts[slot * 4 + 0], sh = b.ts[slot * 4 + 1];
  double cr[PER], acc[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int col = lane + j * kW;
    cr[j] = col < d ? c[col] : 0.0;
    acc[j] = 0.0;
  }
  if (kap > 0.0) {
    const int64_t stride = (int64_t)gridDim.x * NW;
    for (int64_t base = (int64_t)blockIdx.x * NW + w; base < b.n; base += RB * stride) {
      double x[RB][PER];
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int64_t i = base + r * stride;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
          const int col = lane + j * kW;
          x[r][j] = (i < b.n && col < d) ? xval<P>(b, i, col) : cr[j];
        }
      }
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int64_t i = base + r * stride;
        if (i >= b.n || i == b.v1) continue;
        double dl[PER], s2 = 0.0;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
          dl[j] = x[r][j] - cr[j];
          s2 += dl[j] * dl[j];
        }
        const double di = sqrt(wsum(s2));
        if (!(di > 0.0)) continue;  // a row at the centre adds a_i * 0
        const double ep = exp(kap * di - sh), em = exp(-kap * di - sh);
        const double a = (ep - em) / di;
#pragma unroll
        for (int j = 0; j < PER; ++j) acc[j] += a * dl[j];
      }
    }
  }
#pragma unroll
  for (int j = 0; j < PER; ++j) red[w][lane + j * kW] = acc[j];
  __syncthreads();
  double *p = b.part + (int64_t)blockIdx.x * part_stride(d);
  for (int col = threadIdx.x; col < part_stride(d); col += kFwdBlk) {
    double v = 0.0;
    if (col < d)
#pragma unroll
      for (int q = 0; q < NW; ++q) v += red[q][col];
    p[col] = v;
  }
}

// ---- forward epilogue of iteration t: u(t), S_t, the tape of slot and the
// centre, kappa and shift of the next iteration (slot + 1).  The shift bound:
// c_t - v1 is alpha times a mean of unit vectors (u(1) = v1), so d_i <=
// ||v_i - v1|| + ||v1 - c_t|| <= D + alpha and kappa (D + alpha) caps every
// exponent at 0, while the largest stays above -2 kappa alpha (the row at
// distance D from v1 lies at least D - ||v1 - c_t|| from c_t); the map does
// not depend on the shift.
template <typename P>
__global__ __launch_bounds__(kEpi) void fwd_epi(Buffers b, int slot, int64_t t, int write_ck) {
  static_assert(kMaxCols <= kEpi, "one column per thread");
  __shared__ double s_W[kMaxCols + 2], tmp[2 * kEpi], s_r[kEpi / kW];
  const int tid = threadIdx.x, d = (int)b.d;
  // this thread's column of S and of row v1, and the slot's kappa and D,
  // requested together with the partial sums
  const int col = tid;
  const double S0 = col < d ? b.S[col] : 0.0;
  const double v1c = col < d ? xval<P>(b, b.v1, col) : 0.0;
  const double kap = b.ts[slot * 4 + 0], D = b.misc[2];
  reduce_parts<kEpi>(b.part, b.pgrid, d + 2, s_W, tmp);
  const double p = col < d ? s_W[col] * s_W[col] : 0.0;
  const double nW = sqrt(bsum<kEpi>(p, s_r));
  const bool ok = kap > 0.0 && nW > 0.0;
  const double tt = (double)t;
  if (col < d) {
    const double wh = ok ? s_W[col] / nW : 0.0;
    const double S = S0 + (v1c + b.alpha * wh);
    b.S[col] = S;
    b.tw[(int64_t)slot * d + col] = wh;
    b.tc[(int64_t)(slot + 1) * d + col] = S / tt;
    if (write_ck && t % b.seg == 0) b.ck[(t / b.seg) * d + col] = S;
  }
  if (tid == 0) {
    b.ts[slot * 4 + 2] = ok ? nW : 0.0;
    const double kn = b.eta * tt / (3.0 * D);
    b.ts[(slot + 1) * 4 + 0] = kn;
    b.ts[(slot + 1) * 4 + 1] = kn * (D + b.alpha);  // the shift bound
  }
}

// ---- start of the segment whose first iteration is t0 + 1: S = S_{t0}.
template <typename P>
__global__ __launch_bounds__(kBlk) void seg_init(Buffers b, int64_t t0) {
  const int tid = threadIdx.x, d = (int)b.d;
  for (int col = tid; col < d; col += kBlk) {
    const double S = b.ck[(t0 / b.seg) * d + col];
    b.S[col] = S;
    b.tc[col] = t0 > 0 ? S / (double)t0 : xval<P>(b, b.v1, col);
  }
  if (tid == 0) {
    const double k0 = b.eta * (double)t0 / (3.0 * b.misc[2]);
    b.ts[0] = k0;
    b.ts[1] = k0 * (b.misc[2] + b.alpha);  // the shift bound of the forward epilogue
  }
}

// lambda_W of slot from lambda, computed by every workgroup of the reverse
// pass; workgroup 0 also stores it for the epilogue.
template <int NT>
__device__ __forceinline__ void lambda_w(const Buffers &b, int slot, double *s_lw, double *s_r) {
  const int tid = threadIdx.x, d = (int)b.d;
  const double *Wh = b.tw + (int64_t)slot * d;
  const double nW = b.ts[slot * 4 + 2];
  double p = 0.0;
  for (int col = tid; col < d; col += NT) p += Wh[col] * b.lam[col];
  p = bsum<NT>(p, s_r);
  for (int col = tid; col < d; col += NT) {
    const double v = nW > 0.0 ? b.alpha * (b.lam[col] - Wh[col] * p) / nW : 0.0;
    s_lw[col] = v;
    if (blockIdx.x == 0) b.lw[(int64_t)slot * d + col] = v;
  }
  __syncthreads();
}

// ---- reverse iteration t = t0 + 1 + slot (t >= 2)
template <typename P, int PER>
__global__ __launch_bounds__(kBwdBlk) void bwd_pass(Buffers b, int slot) {
  constexpr int RB = PER >= 8 ? 2 : kRB;  // rows in flight per wave (registers)
  constexpr int NW = kBwdBlk / kW;
  __shared__ double red[NW][kMaxCols];
  __shared__ double s_lw[kMaxCols], s_r[NW], s_a[NW], s_k[NW];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, d = (int)b.d;
  lambda_w<kBwdBlk>(b, slot, s_lw, s_r);
  const double *c = b.tc + (int64_t)slot * d;
  const double kap = b.ts[slot * 4 + 0], sh = b.ts[slot * 4 + 1], nW = b.ts[slot * 4 + 2];
  double cr[PER], lw[PER], accB[PER];
  double accA = 0.0, accK = 0.0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int col = lane + j * kW;
    cr[j] = col < d ? c[col] : 0.0;
    lw[j] = col < d ? s_lw[col] : 0.0;
    accB[j] = 0.0;
  }
  const bool live = kap > 0.0 && nW > 0.0;
  double *sa = b.sa + (int64_t)slot * b.n, *sb = b.sb + (int64_t)slot * b.n;
  {
    const int64_t stride = (int64_t)gridDim.x * NW;
    for (int64_t base = (int64_t)blockIdx.x * NW + w; base < b.n; base += RB * stride) {
      double x[RB][PER];
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int64_t i = base + r * stride;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
          const int col = lane + j * kW;
          x[r][j] = (i < b.n && col < d) ? xval<P>(b, i, col) : cr[j];
        }
      }
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int64_t i = base + r * stride;
        if (i >= b.n) continue;
        double dl[PER], s2 = 0.0, q = 0.0;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
          dl[j] = x[r][j] - cr[j];
          s2 += dl[j] * dl[j];
          q += dl[j] * lw[j];
        }
        s2 = wsum(s2);
        q = wsum(q);
        const double di = sqrt(s2);
        const bool valid = live && i != b.v1 && di > 0.0;
        double a = 0.0, beta = 0.0, ep = 0.0, em = 0.0;
        if (valid) {
          ep = exp(kap * di - sh);
          em = exp(-kap * di - sh);
          a = (ep - em) / di;
          const double a1 = (kap * (ep + em) * di - (ep - em)) / (di * di);
          beta = a1 * q / di;
        }
        if (lane == 0) {  // the row's coefficients, contracted after the segment
          sa[i] = a;
          sb[i] = beta;
        }
        if (!valid) continue;
#pragma unroll
        for (int j = 0; j < PER; ++j) accB[j] += beta * dl[j];
        accA += a;
        accK += (ep + em) * q;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < PER; ++j) red[w][lane + j * kW] = accB[j];
  if (lane == 0) {
    s_a[w] = accA;
    s_k[w] = accK;
  }
  __syncthreads();
  double *p = b.part + (int64_t)blockIdx.x * part_stride(d);
  for (int col = threadIdx.x; col < part_stride(d); col += kBwdBlk) {
    const double *src = col < d ? &red[0][col] : (col == d ? s_a : s_k);
    const int step = col < d ? kMaxCols : 1;
    double v = 0.0;
    if (col < d + 2)
#pragma unroll
      for (int q = 0; q < NW; ++q) v += src[q * step];
    p[col] = v;
  }
}

// ---- the same two passes for d <= 64 with 16 lanes per row (4 rows per
// wave at a time, CPL <= 4 adjacent columns per lane): the row sums take a
// 4-step butterfly inside the 16 lanes and serve 4 rows at once.
constexpr int kLPR = 16, kRPW = kW / kLPR;
constexpr int kRBR = 8;                    // row steps of one wave per loop
constexpr int kRowsPerLoop = kRBR * kRPW;  // rows of one wave per loop (32)

__device__ __forceinline__ double gsum16(double v) {
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o, kLPR);
  return v;
}

// The CPL columns of row i a lane holds (its centre values for a row past n
// or a column past d).  V4: float points, CPL = 4, d and the row stride
// multiples of 4 and a 16-byte aligned base, so one 16-byte load per row.
template <typename P, int CPL, bool V4>
__device__ __forceinline__ void load_cols(const Buffers &b, int64_t i, int cl, const double *cr, double *x) {
  const int d = (int)b.d;
  if constexpr (V4) {
    if (i < b.n && cl * 4 < d) {
      const float4 v = *(const float4 *)((const float *)b.X + i * b.ld + cl * 4);
      x[0] = v.x;
      x[1] = v.y;
      x[2] = v.z;
      x[3] = v.w;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) x[j] = cr[j];
    }
  } else {
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
      const int col = cl * CPL + j;
      x[j] = (i < b.n && col < d) ? xval<P>(b, i, col) : cr[j];
    }
  }
}

// A wave's four row groups (lanes cl, cl + 16, cl + 32, cl + 48) summed in a
// fixed order; lane cl of group 0 holds the result.
__device__ __forceinline__ double rowgroup_sum(double v) {
  v += __shfl_xor(v, 16, kW);
  return v + __shfl_xor(v, 32, kW);
}

template <typename P, int CPL, bool V4>
__global__ __launch_bounds__(kFwdBlk) void fwd_rows(Buffers b, int slot) {
  constexpr int NW = kFwdBlk / kW;
  __shared__ double red[NW][kLPR * CPL];
  __shared__ double s_row[NW][kRowsPerLoop];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, d = (int)b.d;
  const int rg = lane >> 4, cl = lane & 15;
  const double *c = b.tc + (int64_t)slot * d;
  const double kap = b.ts[slot * 4 + 0], sh = b.ts[slot * 4 + 1];
  double cr[CPL], acc[CPL];
  const double zero[CPL] = {};
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    const int col = cl * CPL + j;
    cr[j] = col < d ? c[col] : 0.0;
    acc[j] = 0.0;
  }
  // kappa = 0 (the first iteration) leaves every a_i zero; the rows' loads
  // do not wait for kappa or the centre (zeros stand in past n and d)
  {
    const int64_t wstride = (int64_t)gridDim.x * NW * kRPW;
    for (int64_t wb = ((int64_t)blockIdx.x * NW + w) * kRPW; wb < b.n; wb += kRBR * wstride) {
      double x[kRBR][CPL];
#pragma unroll
      for (int r = 0; r < kRBR; ++r) load_cols<P, CPL, V4>(b, wb + r * wstride + rg, cl, zero, x[r]);
      // squared distances of the loop's 32 rows (row r, group rg at r * 4 + rg)
#pragma unroll
      for (int r = 0; r < kRBR; ++r) {
        double s2 = 0.0;
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
          const double dl = x[r][j] - cr[j];
          s2 += dl * dl;
        }
        s2 = gsum16(s2);
        if (cl == 0) s_row[w][r * kRPW + rg] = s2;
      }
      wave_lds_sync();
      // the cone exponentials: one row per lane (lanes 0 .. 31)
      if (lane < kRowsPerLoop) {
        const int64_t i = wb + (lane / kRPW) * wstride + lane % kRPW;
        const double di = sqrt(s_row[w][lane]);
        const bool valid = kap > 0.0 && i < b.n && i != b.v1 && di > 0.0;
        const double ep = exp(kap * di - sh), em = exp(-kap * di - sh);
        s_row[w][lane] = valid ? (ep - em) / di : 0.0;
      }
      wave_lds_sync();
#pragma unroll
      for (int r = 0; r < kRBR; ++r) {
        const double a = s_row[w][r * kRPW + rg];
#pragma unroll
        for (int j = 0; j < CPL; ++j) acc[j] += a * (x[r][j] - cr[j]);
      }
      wave_lds_sync();
    }
  }
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    const double v = rowgroup_sum(acc[j]);
    if (rg == 0) red[w][cl * CPL + j] = v;
  }
  __syncthreads();
  double *p = b.part + (int64_t)blockIdx.x * part_stride(d);
  for (int col = threadIdx.x; col < part_stride(d); col += kFwdBlk) {
    double v = 0.0;
    if (col < d)
#pragma unroll
      for (int q = 0; q < NW; ++q) v += red[q][col];
    p[col] = v;
  }
}

template <typename P, int CPL, bool V4>
__global__ __launch_bounds__(kBwdBlk) void bwd_rows(Buffers b, int slot) {
  constexpr int NW = kBwdBlk / kW;
  __shared__ double red[NW][kLPR * CPL];
  __shared__ double s_lw[kMaxCols], s_r[NW], s_a[NW], s_k[NW];
  __shared__ double s_row[NW][kRowsPerLoop], s_q[NW][kRowsPerLoop];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, d = (int)b.d;
  const int rg = lane >> 4, cl = lane & 15;
  // the slot's centre and scalars are requested with lambda_W's inputs
  const double *c = b.tc + (int64_t)slot * d;
  const double kap = b.ts[slot * 4 + 0], sh = b.ts[slot * 4 + 1], nW = b.ts[slot * 4 + 2];
  double cr[CPL], lw[CPL], accB[CPL];
  double accA = 0.0, accK = 0.0;
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    const int col = cl * CPL + j;
    cr[j] = col < d ? c[col] : 0.0;
    accB[j] = 0.0;
  }
  lambda_w<kBwdBlk>(b, slot, s_lw, s_r);
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    const int col = cl * CPL + j;
    lw[j] = col < d ? s_lw[col] : 0.0;
  }
  const bool live = kap > 0.0 && nW > 0.0;
  double *sa = b.sa + (int64_t)slot * b.n, *sb = b.sb + (int64_t)slot * b.n;
  {
    const int64_t wstride = (int64_t)gridDim.x * NW * kRPW;
    for (int64_t wb = ((int64_t)blockIdx.x * NW + w) * kRPW; wb < b.n; wb += kRBR * wstride) {
      double x[kRBR][CPL];
#pragma unroll
      for (int r = 0; r < kRBR; ++r) load_cols<P, CPL, V4>(b, wb + r * wstride + rg, cl, cr, x[r]);
      // squared distances and projections on lambda_W of the loop's 32 rows
#pragma unroll
      for (int r = 0; r < kRBR; ++r) {
        double s2 = 0.0, q = 0.0;
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
          const double dl = x[r][j] - cr[j];
          s2 += dl * dl;
          q += dl * lw[j];
        }
        s2 = gsum16(s2);
        q = gsum16(q);
        if (cl == 0) {
          s_row[w][r * kRPW + rg] = s2;
          s_q[w][r * kRPW + rg] = q;
        }
      }
      wave_lds_sync();
      // a_i and beta_i: one row per lane (lanes 0 .. 31); the row's
      // coefficients are kept for the contraction after the segment
      if (lane < kRowsPerLoop) {
        const int64_t i = wb + (lane / kRPW) * wstride + lane % kRPW;
        const double di = sqrt(s_row[w][lane]), q = s_q[w][lane];
        const bool valid = live && i < b.n && i != b.v1 && di > 0.0;
        double a = 0.0, beta = 0.0;
        if (valid) {
          const double ep = exp(kap * di - sh), em = exp(-kap * di - sh);
          a = (ep - em) / di;
          const double a1 = (kap * (ep + em) * di - (ep - em)) / (di * di);
          beta = a1 * q / di;
          accA += a;
          accK += (ep + em) * q;
        }
        if (i < b.n) {
          sa[i] = a;
          sb[i] = beta;
        }
        s_row[w][lane] = beta;
      }
      wave_lds_sync();
#pragma unroll
      for (int r = 0; r < kRBR; ++r) {
        const double beta = s_row[w][r * kRPW + rg];
#pragma unroll
        for (int j = 0; j < CPL; ++j) accB[j] += beta * (x[r][j] - cr[j]);
      }
      wave_lds_sync();
    }
  }
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    const double v = rowgroup_sum(accB[j]);
    if (rg == 0) red[w][cl * CPL + j] = v;
  }
  accA = wsum(accA);
  accK = wsum(accK);
  if (lane == 0) {
    s_a[w] = accA;
    s_k[w] = accK;
  }
  __syncthreads();
  double *p = b.part + (int64_t)blockIdx.x * part_stride(d);
  for (int col = threadIdx.x; col < part_stride(d); col += kBwdBlk) {
    double v = 0.0;
    if (col < d) {
#pragma unroll
      for (int q = 0; q < NW; ++q) v += red[q][col];
    } else if (col < d + 2) {
      const double *src = col == d ? s_a : s_k;
#pragma unroll
      for (int q = 0; q < NW; ++q) v += src[q];
    }
    p[col] = v;
  }
}

// ---- the rows' share of a walked-back segment, slots [jlo, jhi), as one
// product on the binary64 matrix cores.  With m = jhi - jlo slots, for row i
// and column c
//   g_ic += sum_j a_{j,i} lambda_W(j)_c - beta_{j,i} c(j)_c + x_ic sum_j beta_{j,i},
// i.e. the (rows x 2m) matrix [a | -beta] times the (2m x columns) matrix
// [lambda_W ; c], plus x_ic times the row's beta sum.  A wave takes 16 rows
// and a 64-column tile as four 16 x 16 tiles of v_mfma_f64_16x16x4 (A
// operand: lane l holds row l % 16 at k = 4 s + l / 16; B operand: column
// l % 16 at the same k; result r = 0 .. 3 of lane l is row 4 r + l / 16 of
// column l % 16).  [lambda_W ; c] of the column tile sits in
// LDS; each lane loads its own row's coefficients (16 adjacent rows per k).
constexpr int kMK = 2 * kSegment;  // the longest k extent
constexpr int kCS = 5;             // k steps whose operands are loaded together
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename P>
__global__ __launch_bounds__(kBlk) void seg_contract_mfma(Buffers b, int jlo, int jhi) {
  __shared__ double s_B[kMK][kW];
  __shared__ double s_bs[kNW][16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, d = (int)b.d;
  const int m = jhi - jlo, K2 = 2 * m, KS = (K2 + 3) / 4;  // k steps of 4
  const int c0 = blockIdx.y * kW;
  for (int k = threadIdx.x; k < 4 * KS * kW; k += kBlk) {
    const int kk = k / kW, cc = c0 + k % kW;
    double v = 0.0;
    if (cc < d) {
      if (kk < m)
        v = b.lw[(int64_t)(jlo + kk) * d + cc];
      else if (kk < K2)
        v = b.tc[(int64_t)(jlo + kk - m) * d + cc];
    }
    s_B[kk][k % kW] = v;
  }
  __syncthreads();
  const int mr = lane & 15, kq = lane >> 4;
  const int64_t rstride = (int64_t)gridDim.x * kNW * 16;
  for (int64_t i0 = ((int64_t)blockIdx.x * kNW + w) * 16; i0 < b.n; i0 += rstride) {
    const int64_t i = i0 + mr;
    // this lane's A operands (k = 4 st + kq: a_{k,i} for k < m, beta_{k-m,i}
    // after), kCS k steps at a time, the next group's loads issued before
    // this group's products
    const bool live = i < b.n;
    const int64_t ia = (int64_t)(jlo + kq) * b.n + (live ? i : 0), ib = ia - (int64_t)m * b.n;
    const int64_t step = 4 * b.n;
    double bs = 0.0;
    auto load_group = [&](int s0, double *av) {
#pragma unroll
      for (int u = 0; u < kCS; ++u) {
        const int st = s0 + u, k = 4 * st + kq;
        double a = 0.0;
        if (st < KS && live) {
          if (k < m) {
            a = b.sa[ia + st * step];
          } else if (k < K2) {
            const double be = b.sb[ib + st * step];
            a = -be;
            bs += be;
          }
        }
        av[u] = a;
      }
    };
    f64x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
    double av[kCS], an[kCS];
    load_group(0, av);
    for (int s0 = 0; s0 < KS; s0 += kCS) {
      if (s0 + kCS < KS) load_group(s0 + kCS, an);  // uniform
#pragma unroll
      for (int u = 0; u < kCS; ++u) {
        if (s0 + u < KS) {  // uniform
          const int k = 4 * (s0 + u) + kq;
#pragma unroll
          for (int t = 0; t < 4; ++t)
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], s_B[k][16 * t + mr], acc[t], 0, 0, 0);
        }
      }
#pragma unroll
      for (int u = 0; u < kCS; ++u) av[u] = an[u];
    }
    // the row's beta sum over its four k groups, then handed to the lanes
    // that hold the row's results
    bs += __shfl_xor(bs, 16, kW);
    bs += __shfl_xor(bs, 32, kW);
    if (kq == 0) s_bs[w][mr] = bs;
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = i0 + 4 * r + kq;
      const double brow = s_bs[w][4 * r + kq];
      if (row < b.n) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int col = c0 + 16 * t + mr;
          if (col < d) b.gacc[row * b.d + col] += acc[t][r] + xval<P>(b, row, col) * brow;
        }
      }
    }
    wave_lds_sync();  // s_bs is rewritten by the next rows
  }
}

// ---- reverse epilogue of iteration t: v1's share, the D share, lambda_{t-1}.
__global__ __launch_bounds__(kEpi) void bwd_epi(Buffers b, int slot, int64_t t) {
  static_assert(kMaxCols <= kEpi, "one column per thread");
  __shared__ double s_P[kMaxCols + 2], tmp[2 * kEpi];
  const int tid = threadIdx.x, d = (int)b.d;
  // this thread's column of lambda, v1's accumulator and lambda_W, and the
  // slot's kappa and D, requested together with the partial sums
  const int col = tid;
  const double lam = col < d ? b.lam[col] : 0.0;
  const double g1 = col < d ? b.gv1[col] : 0.0;
  const double lwc = col < d && t >= 2 ? b.lw[(int64_t)slot * d + col] : 0.0;
  const double kap = b.ts[slot * 4 + 0], D = b.misc[2];
  if (t >= 2) reduce_parts<kEpi>(b.part, b.pgrid, d + 2, s_P, tmp);
  if (col < d) {
    b.gv1[col] = g1 + lam;
    if (t >= 2) {
      const double lc = -s_P[d] * lwc - s_P[col];
      b.lam[col] = lam + lc / (double)(t - 1);
    }
  }
  if (tid == 0 && t >= 2) b.misc[0] += -(kap / D) * s_P[d + 1];
}

// ---- farthest row from a centre (ties: smallest index), per workgroup
template <typename P, int PER>
__global__ __launch_bounds__(kBlk) void far_pass(Buffers b, const double *center, int64_t exclude) {
  __shared__ double s_d[kNW];
  __shared__ int64_t s_i[kNW];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, d = (int)b.d;
  double cr[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int col = lane + j * kW;
    cr[j] = col < d ? center[col] : 0.0;
  }
  double best = -1.0;
  int64_t bi = -1;
  const int64_t stride = (int64_t)gridDim.x * kNW;
  for (int64_t i = (int64_t)blockIdx.x * kNW + w; i < b.n; i += stride) {
    if (i == exclude) continue;
    double s2 = 0.0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int col = lane + j * kW;
      const double dl = col < d ? xval<P>(b, i, col) - cr[j] : 0.0;
      s2 += dl * dl;
    }
    s2 = wsum(s2);
    if (s2 > best) {  // rows ascend within a wave: the first maximum stays
      best = s2;
      bi = i;
    }
  }
  if (lane == 0) {
    s_d[w] = best;
    s_i[w] = bi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < kNW; ++q)
      if (s_d[q] > best || (s_d[q] == best && s_i[q] >= 0 && (bi < 0 || s_i[q] < bi))) {
        best = s_d[q];
        bi = s_i[q];
      }
    b.part[2 * blockIdx.x] = best;
    b.part[2 * blockIdx.x + 1] = (double)bi;
  }
}

__global__ __launch_bounds__(kW) void far_final(Buffers b, int which) {
  __shared__ double s_v[kW];
  __shared__ int64_t s_i[kW];
  double best = -1.0;
  int64_t bi = -1;
  for (int g = threadIdx.x; g < b.grid; g += kW) {  // each lane a strided share of the partials
    const double v = b.part[2 * g];
    const int64_t i = (int64_t)b.part[2 * g + 1];
    if (i >= 0 && (v > best || (v == best && i < bi))) {
      best = v;
      bi = i;
    }
  }
  s_v[threadIdx.x] = best;
  s_i[threadIdx.x] = bi;
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int q = 1; q < kW; ++q)  // the largest distance, ties to the smallest row
    if (s_i[q] >= 0 && (s_v[q] > best || (s_v[q] == best && (bi < 0 || s_i[q] < bi)))) {
      best = s_v[q];
      bi = s_i[q];
    }
  b.misc[which == 0 ? 1 : 2] = sqrt(best);
  b.idx[which] = bi;
}

// v1 as a centre, zero checkpoint, zero accumulators.
template <typename P>
__global__ __launch_bounds__(kBlk) void init_kernel(Buffers b) {
  const int d = (int)b.d;
  for (int col = threadIdx.x; col < d; col += kBlk) {
    b.ubar[col] = xval<P>(b, b.v1, col);
    b.ck[col] = 0.0;
    b.gv1[col] = 0.0;
  }
  if (threadIdx.x == 0) b.misc[0] = 0.0;
}

__global__ __launch_bounds__(kBlk) void mean_kernel(Buffers b) {
  for (int col = threadIdx.x; col < (int)b.d; col += kBlk) b.ubar[col] = b.S[col] / (double)b.T;
}

// lambda_T = g (ubar_T - v_i*) / (R T)
template <typename P>
__global__ __launch_bounds__(kBlk) void lambda_init(Buffers b, double gv) {
  const int64_t is = b.idx[0];
  const double R = b.misc[1];
  if (is < 0) return;  // no finite distance: the result stays zero
  for (int col = threadIdx.x; col < (int)b.d; col += kBlk)
    b.lam[col] = R > 0.0 ? gv * (b.ubar[col] - xval<P>(b, is, col)) / (R * (double)b.T) : 0.0;
}

// The rows of v1 (its share of every u(t) and of D), of D's far row j* and of
// R's active row i*, added in that order by one thread per column.
template <typename P>
__global__ __launch_bounds__(kBlk) void final_kernel(Buffers b, double gv) {
  const int64_t v1 = b.v1, js = b.idx[1], is = b.idx[0];
  const double lD = b.misc[0], R = b.misc[1], D = b.misc[2];
  if (is < 0 || js < 0) return;
  for (int col = threadIdx.x; col < (int)b.d; col += kBlk) {
    const double e = (xval<P>(b, v1, col) - xval<P>(b, js, col)) / D;
    double *g = b.gacc;
    g[v1 * b.d + col] += b.gv1[col] + lD * e;
    g[js * b.d + col] += -lD * e;
    if (R > 0.0) g[is * b.d + col] += gv * (xval<P>(b, is, col) - b.ubar[col]) / R;
  }
}

// zero fill by a kernel (not a memset node, which a caller's graph capture
// would record)
__global__ __launch_bounds__(kBlk) void zero_kernel(double *dst, int64_t count) {
  for (int64_t k = (int64_t)blockIdx.x * kBlk + threadIdx.x; k < count; k += (int64_t)gridDim.x * kBlk)
    dst[k] = 0.0;
}

__global__ __launch_bounds__(kBlk) void round_kernel(const double *src, float *dst, int64_t count) {
  for (int64_t k = (int64_t)blockIdx.x * kBlk + threadIdx.x; k < count; k += (int64_t)gridDim.x * kBlk)
    dst[k] = (float)src[k];
}

template <typename P, int PER, bool ROWS, bool V4 = false>
hipError_t run_typed(const Buffers &b, double gv, hipStream_t s) {
  const int G = b.grid, PG = b.pgrid;
  const int64_t T = b.T;
  if (b.grad) zero_kernel<<<G, kBlk, 0, s>>>(b.gacc, b.n * b.d);
  init_kernel<P><<<1, kBlk, 0, s>>>(b);
  far_pass<P, ROWS ? 1 : PER><<<G, kBlk, 0, s>>>(b, b.ubar, b.v1);
  far_final<<<1, kW, 0, s>>>(b, 1);
  const int64_t K = b.seg, nseg = (T + K - 1) / K;
  // the tape of the segment starting after iteration t0: with the whole tape
  // kept, slot j of that segment is iteration t0 + 1 + j of one long tape
  auto at = [&](int64_t t0) {
    Buffers x = b;
    if (b.full) {
      x.tc = b.tc + t0 * b.d;
      x.tw = b.tw + t0 * b.d;
      x.ts = b.ts + t0 * 4;
    }
    return x;
  };
  // forward, storing S every K iterations (and, with the whole tape, every slot)
  for (int64_t sg = 0; sg < nseg; ++sg) {
    const int64_t t0 = sg * K, t1 = std::min<int64_t>(t0 + K, T);
    const Buffers bx = at(t0);
    if (!b.full || sg == 0) seg_init<P><<<1, kBlk, 0, s>>>(bx, t0);
    for (int64_t t = t0 + 1; t <= t1; ++t) {
      const int slot = (int)(t - t0 - 1);
      if constexpr (ROWS)
        fwd_rows<P, PER, V4><<<PG, kFwdBlk, 0, s>>>(bx, slot);
      else
        fwd_pass<P, PER><<<PG, kFwdBlk, 0, s>>>(bx, slot);
      fwd_epi<P><<<1, kEpi, 0, s>>>(bx, slot, t, 1);
    }
  }
  mean_kernel<<<1, kBlk, 0, s>>>(b);
  far_pass<P, ROWS ? 1 : PER><<<G, kBlk, 0, s>>>(b, b.ubar, -1);
  far_final<<<1, kW, 0, s>>>(b, 0);
  if (!b.grad) return hipGetLastError();  // the map's value only
  lambda_init<P><<<1, kBlk, 0, s>>>(b, gv);
  // reverse, one segment at a time: recompute its tape (unless kept), then walk it back
  for (int64_t sg = nseg - 1; sg >= 0; --sg) {
    const int64_t t0 = sg * K, t1 = std::min<int64_t>(t0 + K, T);
    const Buffers bx = at(t0);
    if (!b.full) {
      seg_init<P><<<1, kBlk, 0, s>>>(bx, t0);
      for (int64_t t = t0 + 1; t <= t1; ++t) {
        const int slot = (int)(t - t0 - 1);
        if constexpr (ROWS)
          fwd_rows<P, PER, V4><<<PG, kFwdBlk, 0, s>>>(bx, slot);
        else
          fwd_pass<P, PER><<<PG, kFwdBlk, 0, s>>>(bx, slot);
        fwd_epi<P><<<1, kEpi, 0, s>>>(bx, slot, t, 0);
      }
    }
    for (int64_t t = t1; t > t0; --t) {
      const int slot = (int)(t - t0 - 1);
      if (t >= 2) {
        if constexpr (ROWS)
          bwd_rows<P, PER, V4><<<PG, kBwdBlk, 0, s>>>(bx, slot);
        else
          bwd_pass<P, PER><<<PG, kBwdBlk, 0, s>>>(bx, slot);
      }
      bwd_epi<<<1, kEpi, 0, s>>>(bx, slot, t);
    }
    const int jlo = t0 == 0 ? 1 : 0, jhi = (int)(t1 - t0);  // slots of t >= 2
    if (jhi > jlo)
      seg_contract_mfma<P><<<dim3(G, (unsigned)((b.d + kW - 1) / kW)), kBlk, 0, s>>>(bx, jlo, jhi);
  }
  final_kernel<P><<<1, kBlk, 0, s>>>(b, gv);
  round_kernel<<<G, kBlk, 0, s>>>(b.gacc, b.grad, b.n * b.d);
  return hipGetLastError();
}

template <typename P>
hipError_t run_per(const Buffers &b, double gv, hipStream_t s) {
  // d <= 64: 16 lanes per row with 1, 2 or 4 columns each; else 64 lanes per row
  if (b.d <= 16) return run_typed<P, 1, true>(b, gv, s);
  if (b.d <= 32) return run_typed<P, 2, true>(b, gv, s);
  if (b.d <= 64) {
    if constexpr (sizeof(P) == 4)
      if (b.d % 4 == 0 && b.ld % 4 == 0 && ((uintptr_t)b.X & 15) == 0) return run_typed<P, 4, true, true>(b, gv, s);
    return run_typed<P, 4, true>(b, gv, s);
  }
  const int64_t per = (b.d + kW - 1) / kW;
  if (per <= 2) return run_typed<P, 2, false>(b, gv, s);
  if (per <= 4) return run_typed<P, 4, false>(b, gv, s);
  return run_typed<P, 8, false>(b, gv, s);
}

hipError_t run_backward(const Buffers &b, double gv, hipStream_t s) {
  if (b.d < 1 || b.d > kMaxCols || b.n < 2 || b.T < 1 || b.grid < 1 || b.pgrid < 1 || b.pgrid > b.grid || b.seg < 1 ||
      b.seg > kSegment)
    return hipErrorInvalidValue;
  if (b.dtype == 1) return run_per<double>(b, gv, s);
  if (b.dtype == 2) return run_per<uint16_t>(b, gv, s);
  return run_per<float>(b, gv, s);
}

}  // namespace grad
}  // namespace scpmwu

// ====================================================== no-alloc reverse pass
// scp_mwu_backward for callers that may not allocate device memory: the same
// kernels on a workspace held in this library's static device memory,
// `scratch` (kScratchBytes on every GPU the library runs on, for the life of
// the process).  In host code the array's name stands for the symbol, not a
// device address: its address is looked up once per device, with that device
// current, and only that pointer is handed to the kernels.  Every call on a
// GPU shares its array, so calls that overlap on one GPU race; a call leaves
// its contents behind, and the reverse pass clears what it accumulates into
// (the gradient accumulator) before use.
namespace {

constexpr size_t kScratchBytes = size_t(128) << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

extern "C" int scp_mwu_backward_noalloc(scp_mwu_ctx *ctx, double grad_value, float *grad_points, double *value,
                                        int32_t checkpoint_every) {
  if (!ctx) return SCP_MWU_E_INVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SCP_MWU_E_HIP;
  void *ptr = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void *p = nullptr;
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SCP_MWU_E_HIP;
      g_scratch_ptr[dev] = p;
    }
    ptr = g_scratch_ptr[dev];
  }
  return scpmwu::backward_with_workspace(ctx, grad_value, grad_points, value, checkpoint_every, ptr, kScratchBytes);
}
