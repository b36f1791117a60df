// SCMWU iterate over a product cone R^{n0}_+ (+) Q^{d_1+1} (+) ... (+) Q^{d_k+1}
// (eq.(SCMWU); Section 2.1: the Loewner exponential and the trace of a direct
// sum act blockwise): p = exp(-eta m) / Tr(exp(-eta m)).
//
// Three launches, all binary64: (1) the largest eigenvalue per workgroup
// (orthant coordinates x_i = -eta m_i; a Lorentz block's
// (x0 + ||xbar||)/sqrt2), (2) the exponentials about the common maximum and
// per-workgroup traces, (3) the trace summed in a fixed order and the
// normalisation.  Orthant coordinates are spread over all threads; a Lorentz
// block belongs to one wave, its lanes striding over its vector part.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/scp_mwu.h"

namespace scpmwu {
namespace cone {

constexpr int kBlk = 256, kW = 64, kNW = kBlk / kW;

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kW);
  return v;
}
__device__ __forceinline__ double wmax(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kW));
  return v;
}

struct Args {
  const double *m;
  double *p;
  const int64_t *off;  // device: k + 1 block offsets, off[0] = n0
  int64_t n0, k;
  double eta;
  double *part_max, *part_tr, *out;  // out[0] = shift, out[1] = ln C
};

// ||xbar|| of block b (every lane of the wave gets it)
__device__ __forceinline__ double block_norm(const Args &a, int64_t b, int lane, double *x0) {
  const int64_t lo = a.off[b], hi = a.off[b + 1] - 1;  // vector part [lo, hi), scalar at hi
  double s = 0.0;
  for (int64_t i = lo + lane; i < hi; i += kW) {
    const double x = -a.eta * a.m[i];
    s += x * x;
  }
  *x0 = -a.eta * a.m[hi];
  return sqrt(wsum(s));
}

__global__ __launch_bounds__(kBlk) void max_kernel(Args a) {
  __shared__ double s_m[kNW];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double mx = -INFINITY;
  for (int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x; i < a.n0; i += (int64_t)gridDim.x * kBlk)
    mx = fmax(mx, -a.eta * a.m[i]);
  for (int64_t b = (int64_t)blockIdx.x * kNW + w; b < a.k; b += (int64_t)gridDim.x * kNW) {
    double x0;
    const double nu = block_norm(a, b, lane, &x0);
    mx = fmax(mx, (x0 + nu) * M_SQRT1_2);
  }
  mx = wmax(mx);
  if (lane == 0) s_m[w] = mx;
  __syncthreads();
  if (threadIdx.x == 0) a.part_max[blockIdx.x] = fmax(fmax(s_m[0], s_m[1]), fmax(s_m[2], s_m[3]));
}

__global__ __launch_bounds__(kBlk) void exp_kernel(Args a) {
  __shared__ double s_r[kNW];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double sh = -INFINITY;
  for (int g = 0; g < (int)gridDim.x; ++g) sh = fmax(sh, a.part_max[g]);
  double tr = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x; i < a.n0; i += (int64_t)gridDim.x * kBlk) {
    const double e = exp(-a.eta * a.m[i] - sh);
    a.p[i] = e;
    tr += e;
  }
  double trb = 0.0;  // Lorentz blocks: one value per wave (lane 0 adds it)
  for (int64_t b = (int64_t)blockIdx.x * kNW + w; b < a.k; b += (int64_t)gridDim.x * kNW) {
    double x0;
    const double nu = block_norm(a, b, lane, &x0);
    const double e1 = exp((x0 + nu) * M_SQRT1_2 - sh), e2 = exp((x0 - nu) * M_SQRT1_2 - sh);
    // vector part (e1 - e2)/sqrt2 * xbar/||xbar|| (zero when xbar = 0), scalar (e1 + e2)/sqrt2
    const double f = nu > 0.0 ? (e1 - e2) * M_SQRT1_2 / nu : 0.0;
    const int64_t lo = a.off[b], hi = a.off[b + 1] - 1;
    for (int64_t i = lo + lane; i < hi; i += kW) a.p[i] = f * (-a.eta * a.m[i]);
    if (lane == 0) {
      a.p[hi] = (e1 + e2) * M_SQRT1_2;
      trb += e1 + e2;  // trace of the block: sqrt2 times its scalar part
    }
  }
  tr = wsum(tr + trb);
  if (lane == 0) s_r[w] = tr;
  __syncthreads();
  if (threadIdx.x == 0) {
    a.part_tr[blockIdx.x] = (s_r[0] + s_r[1]) + (s_r[2] + s_r[3]);
    if (blockIdx.x == 0) a.out[0] = sh;
  }
}

__global__ __launch_bounds__(kBlk) void norm_kernel(Args a, int64_t total) {
  double C = 0.0;
  for (int g = 0; g < (int)gridDim.x; ++g) C += a.part_tr[g];  // same order in every workgroup
  const double inv = 1.0 / C;
  for (int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlk)
    a.p[i] *= inv;
  if (blockIdx.x == 0 && threadIdx.x == 0) a.out[1] = a.out[0] + log(C);
}

}  // namespace cone
}  // namespace scpmwu

// A product-cone layout validated once: its block offsets resident on the
// device, the workspace of the three launches, the stream they go on.
struct scp_mwu_product {
  int64_t n0 = 0, k = 0, len = 0;
  int G = 0;
  hipStream_t stream = nullptr;
  void *mem = nullptr;  // 2G + 2 doubles (partials, shift, ln C), then k + 1 offsets
};

extern "C" int scp_mwu_product_init(int64_t n_orth, const int64_t *offsets, int64_t nblocks, int64_t len,
                                    void *stream, scp_mwu_product **out) {
  using namespace scpmwu::cone;
  if (!out) return SCP_MWU_E_INVAL;
  *out = nullptr;
  if (n_orth < 0 || nblocks < 0 || n_orth + nblocks == 0 || len < 1) return SCP_MWU_E_INVAL;
  if (nblocks > 0) {
    if (!offsets || offsets[0] != n_orth) return SCP_MWU_E_INVAL;
    for (int64_t b = 0; b < nblocks; ++b)
      if (offsets[b + 1] - offsets[b] < 2) return SCP_MWU_E_INVAL;
    if (offsets[nblocks] != len) return SCP_MWU_E_INVAL;
  } else if (n_orth != len) {
    return SCP_MWU_E_INVAL;
  }
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return SCP_MWU_E_HIP;
  auto *pc = new scp_mwu_product();
  pc->n0 = n_orth;
  pc->k = nblocks;
  pc->len = len;
  pc->stream = (hipStream_t)stream;
  const int64_t want = std::max<int64_t>((n_orth + kBlk - 1) / kBlk, (nblocks + kNW - 1) / kNW);
  pc->G = (int)std::max<int64_t>(1, std::min<int64_t>(want, 4 * (int64_t)std::max(cus, 1)));
  const size_t nbytes = sizeof(double) * (2 * (size_t)pc->G + 2) + sizeof(int64_t) * (size_t)(nblocks + 1);
  if (hipMalloc(&pc->mem, nbytes) != hipSuccess) {
    delete pc;
    return SCP_MWU_E_NOMEM;
  }
  if (nblocks > 0) {
    int64_t *doff = (int64_t *)((double *)pc->mem + 2 * (size_t)pc->G + 2);
    if (hipMemcpy(doff, offsets, sizeof(int64_t) * (size_t)(nblocks + 1), hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(pc->mem);
      delete pc;
      return SCP_MWU_E_HIP;
    }
  }
  *out = pc;
  return SCP_MWU_OK;
}

extern "C" int scp_mwu_product_exp(scp_mwu_product *pc, const double *m, double eta, double *p, double *log_trace) {
  using namespace scpmwu::cone;
  if (!pc || !m || !p || m == p || !(eta > 0.0) || !std::isfinite(eta)) return SCP_MWU_E_INVAL;
  const hipStream_t s = pc->stream;
  Args a{};
  a.m = m;
  a.p = p;
  a.n0 = pc->n0;
  a.k = pc->k;
  a.eta = eta;
  a.part_max = (double *)pc->mem;
  a.part_tr = a.part_max + pc->G;
  a.out = a.part_tr + pc->G;
  a.off = pc->k > 0 ? (const int64_t *)(a.out + 2) : nullptr;
  max_kernel<<<pc->G, kBlk, 0, s>>>(a);
  exp_kernel<<<pc->G, kBlk, 0, s>>>(a);
  norm_kernel<<<pc->G, kBlk, 0, s>>>(a, pc->len);
  if (hipGetLastError() != hipSuccess) return SCP_MWU_E_HIP;
  if (!log_trace) return SCP_MWU_OK;
  double lt = 0.0;
  if (hipMemcpyAsync(&lt, a.out + 1, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return SCP_MWU_E_HIP;
  *log_trace = lt;
  return SCP_MWU_OK;
}

extern "C" void scp_mwu_product_destroy(scp_mwu_product *pc) {
  if (!pc) return;
  (void)hipStreamSynchronize(pc->stream);
  (void)hipFree(pc->mem);
  delete pc;
}
