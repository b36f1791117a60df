// Gradient of the SES radius after T fixed-alpha iterations (point sets): the
// map, its adjoint recursion and the device buffers of the reverse pass.
//
// The map (Section 4.1 split, eq.(ses_oracle) ORACLE, Section 2.1 SOC
// exponential, Section 5 monitor): u(t) = v1 + alpha W_t/||W_t|| with
// W_t = sum_{i != v1} a_i (v_i - c_t), c_t the mean of u(1..t-1),
// a_i = (e^{kappa_t d_i - s_t} - e^{-kappa_t d_i - s_t}) / d_i,
// d_i = ||v_i - c_t||, kappa_t = eta (t-1) / (3D) and s_t any shift common to
// all rows; R = max_i ||v_i - ubar_T||.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

struct scp_mwu_ctx;

namespace scpmwu {
namespace grad {

constexpr int kSegment = 50;  // the longest segment (iterations between stored running sums)

// Device buffers of one reverse pass (allocated by the host for one call).
struct Buffers {
  int64_t n, d, ld, v1, T;
  int dtype;         // 0: float points, 1: double points, 2: BF16 points
  const void *X;
  double alpha, eta;     // kappa_t = eta (t - 1) / (3D), D recomputed on the device
  int grid;          // workgroups of the 256-thread kernels
  int pgrid;         // workgroups of the per-iteration passes (<= grid)
  int seg;           // segment length K (1 .. kSegment)
  int full;          // 1: the tape holds all T iterations (no recomputation)
  // running sum and its checkpoints S_{j K}
  double *S, *ck;
  // tape of one segment (K slots; all T with `full`), slot j = iteration t0 + 1 + j:
  //   tc: c_t (one slot more), tw: W_t/||W_t||, ts: {kappa_t, s_t, ||W_t||, 0} (one slot more)
  double *tc, *tw, *ts;
  double *part;      // per-workgroup partial sums: pgrid x part_stride(d), or 2 grid (far rows)
  double *lam;       // adjoint of S_t
  double *lw;        // lambda_W of each slot of the segment (K x d)
  double *sa, *sb;   // a_i and beta_i of each slot and row (K x n each)
  double *gv1;       // accumulated adjoint of v1 from u(t) = v1 + ...
  double *ubar;      // ubar_T
  double *misc;      // [0] adjoint of D, [1] R, [2] D (recomputed), [3..4] scratch
  int64_t *idx;      // [0] i* (argmax of R), [1] j* (argmax of D)
  double *gacc;      // n x d accumulator of the gradient (row stride d)
  float *grad;       // caller's n x d output (row stride d)
};

// Sizes of the buffers (in doubles) for given d, T.
inline int64_t ck_count(int64_t T, int64_t K) { return T / K + 2; }
// Row stride (doubles) of the per-workgroup partial sums: d + 2 columns
// rounded up to even, so that column pairs are 16-byte aligned.
__host__ __device__ inline int64_t part_stride(int64_t d) { return (d + 3) & ~int64_t(1); }

// Launch the whole reverse pass (forward with checkpoints, reverse segments,
// the terms of R and D) on stream s.  grad_value scales the result.
hipError_t run_backward(const Buffers &b, double grad_value, hipStream_t s);

}  // namespace grad

// scp_mwu_backward on a workspace: allocated for the call when ws is nullptr,
// else the caller's ws_bytes at ws (a call that needs more fails with
// SCP_MWU_E_INVAL before any launch).  Defined with the C ABI's host code.
int backward_with_workspace(scp_mwu_ctx *c, double grad_value, float *grad_points, double *value,
                            int32_t checkpoint_every, void *ws, size_t ws_bytes);
}  // namespace scpmwu
