// Host side of the C ABI declared in include/scp_mwu.h: descriptor
// validation, workspace ownership, the alpha-feasibility test state machine
// driven through captured HIP graphs of the streaming pass, and the adaptive
// alpha search of Section 3 ("From feasibility to optimization"), mirrored
// for the SVM min form.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <string>
#include <cstdlib>
#include <vector>

#include "../../include/scp_mwu.h"
#include "grad.hpp"
#include "mwu_common.hpp"


using namespace scpmwu;

namespace {

thread_local std::string g_init_error;

constexpr double kTau = 1e-12;  // relative tie tolerance of the separation test
// Largest record set the fused pass reads in every workgroup (256 records of
// d = 128 are 278 KB).
constexpr int64_t kFuseRecBytes = 288 * 1024;

size_t elem_size(int dt) { return dt == kFP8 ? 1 : (dt == kBF16 ? 2 : (dt == kF32 ? 4 : 8)); }

}  // namespace

struct scp_mwu_ctx {
  // problem
  int problem = 0, dtype = 0;  // dtype: storage type streamed by the kernels
  int64_t n = 0, d = 0, ld = 0, n_pos = 0, v1 = 0;
  const void *X = nullptr;
  void *owned = nullptr;
  float *owned_scales = nullptr;  // FP8 storage: one scale per row
  const double *radii = nullptr;
  double eps = 1e-3, delta = 1e-4;
  int32_t patience = 10, flags = 0, chunk = 32;
  int64_t t_cap = 0, max_iters = 0;
  hipStream_t stream = nullptr, cap_stream = nullptr;
  // constants of the split
  double D = 0, gamma1 = 0, rho = 0, R = 0;
  int64_t r = 0;
  // device workspace: state, vectors and records in two slots (the fused
  // pass reads one slot and writes the other); st, vec, partials and args
  // view the current slot `cur`
  DevState *st_base = nullptr, *st = nullptr;
  double *vec_base = nullptr, *vec = nullptr, *part_base = nullptr, *partials = nullptr, *mon = nullptr;
  int64_t rec_stride = 0;  // doubles per record slot
  int cur = 0;
  bool fused = false;      // SES with small records: epilogue fused into the next pass
  // fused passes without SCP_MWU_FLAG_DETERMINISTIC add their sums into one
  // of three global sums (atomics) instead of writing per-workgroup records
  bool gmode = false;
  double *g_base = nullptr;
  int64_t g_stride = 0;    // doubles per global-sum slot
  int g_cur = 0;           // the slot holding the last pass's sums
  DevState *host_st = nullptr;  // pinned readback
  int grid = 0;
  LaunchCfg cfg{}, cfg_cert{};
  PassArgs args{}, base{};
  // current test
  bool active = false;
  double alpha = 0, eta = 0;
  int64_t T = 0;
  // graphs: `chunk` passes, the last one optionally with certificates (and
  // the flush), one per starting slot; gend: the slot a graph ends in
  hipGraphExec_t gexec[2][3] = {};
  int gend[2][3] = {}, gend_g[2][3] = {};
  std::string err;

  int fail(int code, const std::string &msg) {
    err = msg;
    return code;
  }
  int hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return SCP_MWU_OK;
    err = std::string(what) + ": " + hipGetErrorString(e);
    return SCP_MWU_E_HIP;
  }
};

namespace {

// Make slot p current.
void set_cur(scp_mwu_ctx *c, int p) {
  c->cur = p;
  c->st = c->st_base + p;
  c->vec = c->vec_base + (int64_t)p * kNumVec * c->d;
  c->partials = c->part_base + (int64_t)p * c->rec_stride;
  c->args.st = c->st;
  c->args.vec = c->vec;
  c->args.partials = c->partials;
}

// The streaming pass kernel of one MWU iteration (no epilogue).
hipError_t pass_kernel(scp_mwu_ctx *c, bool cert, hipStream_t s) {
  const LaunchCfg &cfg = cert ? c->cfg_cert : c->cfg;
  switch (c->dtype) {
    case kF32: return launch_pass_f32(c->problem, cfg, c->args, s);
    case kBF16: return launch_pass_bf16(c->problem, cfg, c->args, s);
    case kFP8: return launch_pass_fp8(c->problem, cfg, c->args, s);
    default: return launch_pass_f64(c->problem, cfg, c->args, s);
  }
}

// The combine + FP64 epilogue kernel of one MWU iteration.
hipError_t epilogue_kernel(scp_mwu_ctx *c, bool cert, hipStream_t s) {
  const LaunchCfg &cfg = cert ? c->cfg_cert : c->cfg;
  switch (c->dtype) {
    case kF32: return launch_epilogue_f32(c->problem, cfg, c->args, s);
    case kBF16: return launch_epilogue_bf16(c->problem, cfg, c->args, s);
    case kFP8: return launch_epilogue_fp8(c->problem, cfg, c->args, s);
    default: return launch_epilogue_f64(c->problem, cfg, c->args, s);
  }
}

// The fused kernel: the epilogue of the pending records of slot cur, then
// the pass, whose records and new state go to the other slot.
double *gslot(const scp_mwu_ctx *c, int k) { return c->g_base + (int64_t)(k % 3) * c->g_stride; }

hipError_t fused_kernel(scp_mwu_ctx *c, bool cert, hipStream_t s) {
  const LaunchCfg &cfg = cert ? c->cfg_cert : c->cfg;
  FusedSlots f{c->cur, c->rec_stride, nullptr, nullptr, nullptr};
  if (c->gmode) {
    f.g_in = gslot(c, c->g_cur);
    f.g_out = gslot(c, c->g_cur + 1);
    f.g_zero = gslot(c, c->g_cur + 2);
  }
  hipError_t e;
  switch (c->dtype) {
    case kF32: e = launch_fused_f32(cfg, c->base, f, s); break;
    case kBF16: e = launch_fused_bf16(cfg, c->base, f, s); break;
    case kFP8: e = launch_fused_fp8(cfg, c->base, f, s); break;
    default: e = launch_fused_f64(cfg, c->base, f, s); break;
  }
  if (e == hipSuccess) {
    set_cur(c, 1 - c->cur);
    if (c->gmode) c->g_cur = (c->g_cur + 1) % 3;
  }
  return e;
}

// The pending records of the current slot applied (fused mode; the records
// of a certificate pass need cert).
hipError_t flush(scp_mwu_ctx *c, bool cert, hipStream_t s) {
  if (!c->fused) return hipSuccess;
  PassArgs a = c->args;
  int P = c->grid;
  if (c->gmode) {
    a.partials = gslot(c, c->g_cur);
    P = 1;
  }
  switch (c->dtype) {
    case kF32: return launch_flush_f32(cert, P, c->gmode, a, s);
    case kBF16: return launch_flush_bf16(cert, P, c->gmode, a, s);
    case kFP8: return launch_flush_fp8(cert, P, c->gmode, a, s);
    default: return launch_flush_f64(cert, P, c->gmode, a, s);
  }
}

// One MWU iteration: streaming pass, then combine + epilogue (in fused mode
// the epilogue runs at the start of the next pass or in the flush).
hipError_t pass(scp_mwu_ctx *c, bool cert, hipStream_t s) {
  if (c->fused) return fused_kernel(c, cert, s);
  hipError_t e = pass_kernel(c, cert, s);
  if (e != hipSuccess) return e;
  return epilogue_kernel(c, cert, s);
}

hipError_t monitor(scp_mwu_ctx *c, const double *center, int64_t exclude, int mode) {
  switch (c->dtype) {
    case kF32: return launch_monitor_f32(c->grid, c->args, center, exclude, mode, c->mon, c->stream);
    case kBF16: return launch_monitor_bf16(c->grid, c->args, center, exclude, mode, c->mon, c->stream);
    case kFP8: return launch_monitor_fp8(c->grid, c->args, center, exclude, mode, c->mon, c->stream);
    default: return launch_monitor_f64(c->grid, c->args, center, exclude, mode, c->mon, c->stream);
  }
}

// Read the per-workgroup monitor records and max-combine them.
int monitor_result(scp_mwu_ctx *c, double out[4]) {
  std::vector<double> h((size_t)c->grid * 4);
  int rc = c->hip(hipMemcpyAsync(h.data(), c->mon, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                                 c->stream), "monitor readback");
  if (rc) return rc;
  rc = c->hip(hipStreamSynchronize(c->stream), "monitor sync");
  if (rc) return rc;
  for (int k = 0; k < 4; ++k) out[k] = -INFINITY;
  for (int b = 0; b < c->grid; ++b)
    for (int k = 0; k < 4; ++k) out[k] = std::max(out[k], h[(size_t)b * 4 + k]);
  return SCP_MWU_OK;
}

int read_state(scp_mwu_ctx *c) {
  int rc = c->hip(hipMemcpyAsync(c->host_st, c->st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream),
                  "state readback");
  if (rc) return rc;
  return c->hip(hipStreamSynchronize(c->stream), "state sync");
}

int start_test(scp_mwu_ctx *c, double alpha, int64_t T, bool early) {
  InitParams p{};
  p.alpha = alpha;
  p.T = T;
  p.eta = std::sqrt(std::log((double)c->r) / (double)T);
  p.kscale = c->problem == kSES ? p.eta / (c->rho * std::sqrt(2.0)) : p.eta / c->rho;
  p.delta = c->delta;
  p.tau = kTau;
  p.D = c->D;
  p.gamma1 = c->gamma1;
  p.patience = c->patience;
  p.early = early ? 1 : 0;
  set_cur(c, 0);
  if (c->gmode) {  // every global sum starts cleared (not in a captured graph)
    int rc = c->hip(hipMemsetAsync(c->g_base, 0, sizeof(double) * 3 * (size_t)c->g_stride, c->stream), "sum clear");
    if (rc) return rc;
    c->g_cur = 0;
  }
  hipError_t e;
  switch (c->dtype) {
    case kF32: e = launch_init_f32(c->args, p, c->problem, c->stream); break;
    case kBF16: e = launch_init_bf16(c->args, p, c->problem, c->stream); break;
    case kFP8: e = launch_init_fp8(c->args, p, c->problem, c->stream); break;
    default: e = launch_init_f64(c->args, p, c->problem, c->stream); break;
  }
  int rc = c->hip(e, "test init");
  if (rc) return rc;
  c->active = true;
  c->alpha = alpha;
  c->T = T;
  c->eta = p.eta;
  return SCP_MWU_OK;
}

// The graph of `chunk` passes starting in the current slot (then the flush
// of the last pass's records); capture launches nothing, so the slot is
// restored afterwards and the graph's end slot kept.
int build_graph(scp_mwu_ctx *c) {
  const int p0 = c->cur, g0 = c->g_cur;
  if (c->gexec[p0][g0]) return SCP_MWU_OK;
  hipGraph_t g = nullptr;
  int rc = c->hip(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
  if (rc) return rc;
  const bool cert = (c->flags & SCP_MWU_FLAG_CERTIFICATES) && c->problem == kSES;
  hipError_t e = hipSuccess;
  for (int k = 0; k < c->chunk && e == hipSuccess; ++k)
    e = pass(c, cert && k == c->chunk - 1, c->cap_stream);
  if (e == hipSuccess) e = flush(c, cert, c->cap_stream);
  c->gend[p0][g0] = c->cur;
  c->gend_g[p0][g0] = c->g_cur;
  set_cur(c, p0);
  c->g_cur = g0;
  hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
  if (e != hipSuccess) return c->hip(e, "capture pass");
  rc = c->hip(e2, "end capture");
  if (rc) return rc;
  e = hipGraphInstantiate(&c->gexec[p0][g0], g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  return c->hip(e, "graph instantiate");
}

// Run up to k passes of the current test; stop early once it has ended.
// Whole chunks replay the captured graph and the state is read after each
// (a test that ended stops the loop); fewer than `chunk` passes are enqueued
// back to back and the state is read once: a pass whose test has ended does
// nothing, so passes past the end cost only their launch.
int run_iters(scp_mwu_ctx *c, int64_t k) {
  int rc;
  const bool cert = (c->flags & SCP_MWU_FLAG_CERTIFICATES) && c->problem == kSES;
  while (k > 0) {
    if (k >= c->chunk && c->chunk > 1) {
      rc = build_graph(c);
      if (rc) return rc;
      rc = c->hip(hipGraphLaunch(c->gexec[c->cur][c->g_cur], c->stream), "graph launch");
      if (rc) return rc;
      const int p1 = c->gend[c->cur][c->g_cur], g1 = c->gend_g[c->cur][c->g_cur];
      set_cur(c, p1);
      c->g_cur = g1;
      k -= c->chunk;
    } else {
      for (; k > 0; --k) {
        rc = c->hip(pass(c, cert && k == 1, c->stream), "pass launch");
        if (rc) return rc;
      }
      rc = c->hip(flush(c, cert, c->stream), "flush launch");
      if (rc) return rc;
    }
    rc = read_state(c);
    if (rc) return rc;
    if (c->host_st->status != kRunning) break;
  }
  return SCP_MWU_OK;
}

void fill_info(const scp_mwu_ctx *c, scp_mwu_stepinfo *info) {
  const DevState &s = *c->host_st;
  info->t = s.t;
  info->t_end = s.status == kRunning ? 0 : s.t_end;
  info->T = s.T;
  info->outcome = s.status;
  info->degenerate = s.degenerate;
  info->alpha = s.alpha;
  info->eta = s.eta;
  info->f_last = s.f_last;
  info->f_best = s.f_best;
  info->t_best = s.t_best;
  info->value = s.value;
  info->scale = s.scale;
  info->log_trace = s.log_trace;
  info->bound = s.bound;
}

int64_t theory_T(const scp_mwu_ctx *c, double eps, double alpha) {
  const double v = 4.0 * (c->R * c->R) * (c->rho * c->rho) * std::log((double)c->r) /
                   ((eps * eps) * (alpha * alpha));
  if (!(v < 9.0e18)) return INT64_MAX / 2;
  return (int64_t)std::ceil(v);
}

int64_t min_T(const scp_mwu_ctx *c) {
  return std::max<int64_t>(1, (int64_t)std::ceil(std::log((double)c->r)));
}

// Run one whole alpha-feasibility test; the final device state is in host_st.
int run_test(scp_mwu_ctx *c, double alpha, int64_t T, bool early, int64_t budget) {
  int rc = start_test(c, alpha, T, early);
  if (rc) return rc;
  // T + 1 passes evaluate f(T); the test can only end earlier
  int64_t left = budget > 0 ? std::min<int64_t>(budget + 1, T + 1) : T + 1;
  while (true) {
    const int64_t k = std::min<int64_t>(left, c->chunk);
    rc = run_iters(c, k);
    if (rc) return rc;
    left -= k;
    if (c->host_st->status != kRunning || left <= 0) break;
  }
  return SCP_MWU_OK;
}

int read_vec(scp_mwu_ctx *c, int which, double *out) {
  int rc = c->hip(hipMemcpyAsync(out, c->vec + (size_t)which * c->d, (size_t)c->d * sizeof(double),
                                 hipMemcpyDeviceToHost, c->stream), "vector readback");
  if (rc) return rc;
  return c->hip(hipStreamSynchronize(c->stream), "vector sync");
}

}  // namespace

// The reverse pass of scp_mwu_backward on a workspace: allocated here for
// the call (ws == nullptr) or the caller's (ws_bytes long; too small is an
// error and nothing is launched).
int scpmwu::backward_with_workspace(scp_mwu_ctx *c, double grad_value, float *grad_points, double *value,
                                    int32_t checkpoint_every, void *ws, size_t ws_bytes) {
  if (!c) return SCP_MWU_E_INVAL;
  if (!grad_points && !value) return c->fail(SCP_MWU_E_INVAL, "grad_points and value are both NULL");
  if (!std::isfinite(grad_value)) return c->fail(SCP_MWU_E_INVAL, "grad_value is not finite");
  if (checkpoint_every < 0 || checkpoint_every > grad::kSegment)
    return c->fail(SCP_MWU_E_INVAL, "checkpoint_every must be 0 (keep the whole tape) or 1 .. 50");
  if (c->problem != kSES || c->radii)
    return c->fail(SCP_MWU_E_UNSUPPORTED, "backward: SES on point sets only");
  if (c->dtype != kF32 && c->dtype != kF64 && c->dtype != kBF16)
    return c->fail(SCP_MWU_E_UNSUPPORTED, "backward: points streamed as F32, F64 or BF16 only (no FP8 storage)");
  if (c->d > 512) return c->fail(SCP_MWU_E_UNSUPPORTED, "backward: d > 512");
  if (!c->active) return c->fail(SCP_MWU_E_STATE, "backward before any test");
  int rc = SCP_MWU_OK;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return c->fail(SCP_MWU_E_HIP, "device query failed");
  grad::Buffers b{};
  b.n = c->n;
  b.d = c->d;
  b.ld = c->ld;
  b.v1 = c->v1;
  b.T = c->T;
  b.dtype = c->dtype == kF64 ? 1 : (c->dtype == kBF16 ? 2 : 0);
  b.X = c->X;
  b.alpha = c->alpha;
  b.eta = c->eta;
  // four 256-thread workgroups per CU, at least 64 rows per workgroup; the
  // per-iteration passes one workgroup per CU
  b.grid = (int)std::max<int64_t>(1, std::min<int64_t>(4 * (int64_t)std::max(cus, 1), (c->n + 63) / 64));
  b.pgrid = (int)std::max<int64_t>(1, std::min<int64_t>(std::max(cus, 1), (c->n + 63) / 64));
  const bool full = checkpoint_every == 0;
  b.full = full ? 1 : 0;
  b.seg = full ? grad::kSegment : checkpoint_every;
  const int64_t d = c->d, K = b.seg, L = full ? c->T : K;  // tape slots
  // the value alone needs neither the per-row coefficients nor the accumulator
  const int64_t rows = grad_points ? c->n : 0;
  const int64_t sizes[] = {d, grad::ck_count(c->T, K) * d, (L + 1) * d, L * d, (L + 1) * 4,
                           (int64_t)b.grid * grad::part_stride(d), d, K * d, d, d, 8, K * rows, K * rows, 2, rows * d};
  int64_t total = 0;
  for (int64_t v : sizes) total += (v + 31) / 32 * 32;
  const size_t need = (size_t)total * sizeof(double);
  void *mem = ws;
  if (ws) {
    if (need > ws_bytes)
      return c->fail(SCP_MWU_E_INVAL, "backward: the call needs " + std::to_string(need) +
                                           " bytes of workspace, more than the " + std::to_string(ws_bytes) +
                                           " available (fewer rows, a smaller d or checkpoint_every)");
  } else if (hipMalloc(&mem, need) != hipSuccess) {
    return c->fail(SCP_MWU_E_NOMEM, "backward workspace");
  }
  double *p = (double *)mem;
  double **dst[] = {&b.S, &b.ck, &b.tc, &b.tw, &b.ts, &b.part, &b.lam, &b.lw, &b.gv1, &b.ubar, &b.misc, &b.sa, &b.sb};
  for (int k = 0; k < 13; ++k) {
    *dst[k] = p;
    p += (sizes[k] + 31) / 32 * 32;
  }
  b.idx = (int64_t *)p;
  p += 32;
  b.gacc = p;
  b.grad = grad_points;
  rc = c->hip(grad::run_backward(b, grad_value, c->stream), "backward");
  double misc[3] = {0, 0, 0};
  if (!rc) rc = c->hip(hipMemcpyAsync(misc, b.misc, sizeof(misc), hipMemcpyDeviceToHost, c->stream), "backward readback");
  const hipError_t es = hipStreamSynchronize(c->stream);  // the workspace is freed (or reusable) only when idle
  if (!rc) rc = c->hip(es, "backward sync");
  if (!ws) hipFree(mem);
  if (!rc && value) *value = misc[1];
  return rc;
}

// ============================================================== C ABI
extern "C" {

const char *scp_mwu_strerror(int code) {
  switch (code) {
    case SCP_MWU_OK: return "ok";
    case SCP_MWU_STOPPED: return "stopped: iteration budget spent before the stop rule";
    case SCP_MWU_E_INVAL: return "invalid argument";
    case SCP_MWU_E_NOMEM: return "out of memory";
    case SCP_MWU_E_HIP: return "HIP runtime error";
    case SCP_MWU_E_STATE: return "call not valid in the current state";
    case SCP_MWU_E_NUMERIC: return "non-finite value in the input or the iteration";
    case SCP_MWU_E_INFEASIBLE: return "classes certified not separable";
    case SCP_MWU_E_UNSUPPORTED: return "not supported by this version";
    default: return "unknown error code";
  }
}

const char *scp_mwu_last_error(const scp_mwu_ctx *ctx) {
  return ctx ? ctx->err.c_str() : g_init_error.c_str();
}

void scp_mwu_destroy(scp_mwu_ctx *c) {
  if (!c) return;
  hipStreamSynchronize(c->stream);
  for (auto &row : c->gexec)
    for (auto &g : row)
      if (g) hipGraphExecDestroy(g);
  if (c->cap_stream) hipStreamDestroy(c->cap_stream);
  hipFree(c->st_base);
  hipFree(c->vec_base);
  hipFree(c->part_base);
  hipFree(c->g_base);
  hipFree(c->mon);
  hipFree(c->owned);
  hipFree(c->owned_scales);
  if (c->host_st) hipHostFree(c->host_st);
  delete c;
}

int scp_mwu_init(const scp_mwu_desc *desc, scp_mwu_ctx **out) {
  g_init_error.clear();
  auto bad = [&](const char *m) {
    g_init_error = m;
    return SCP_MWU_E_INVAL;
  };
  if (!out) return bad("out is NULL");
  *out = nullptr;
  if (!desc) return bad("desc is NULL");
  if (desc->struct_size < sizeof(scp_mwu_desc)) return bad("desc->struct_size too small");
  if (desc->problem != SCP_MWU_PROBLEM_SES && desc->problem != SCP_MWU_PROBLEM_SVM)
    return bad("unknown problem");
  if (desc->dtype < SCP_MWU_F32 || desc->dtype > SCP_MWU_F64) return bad("unknown dtype");
  const int storage = desc->storage ? desc->storage : desc->dtype;
  if (storage < SCP_MWU_F32 || storage > SCP_MWU_FP8) return bad("unknown storage type");
  if (storage != desc->dtype &&
      !(desc->dtype == SCP_MWU_F32 && (storage == SCP_MWU_BF16 || storage == SCP_MWU_FP8)))
    return bad("storage conversion other than F32 -> BF16 or F32 -> FP8");
  if (!desc->points) return bad("points is NULL");
  if (desc->n < 2) return bad("n < 2");
  if (desc->d < 1 || desc->d > kMaxD) return bad("d outside [1, 512]");
  const int64_t ld = desc->ld ? desc->ld : desc->d;
  if (ld < desc->d) return bad("ld < d");
  if ((uintptr_t)desc->points % elem_size(desc->dtype)) return bad("points misaligned");
  // a batch of up to 64 rows is addressed with 32-bit lane byte offsets, and a
  // column past d gets the offset 2^30 (plus up to 60 rows of steps): both the
  // batch's byte range and that offset stay below 2^31, and the range stays
  // below 2^30 so that the invalid offset always falls outside it
  if (ld * (int64_t)elem_size(desc->dtype) * 64 >= (int64_t)1 << 30) return bad("row stride too large");
  if (desc->problem == SCP_MWU_PROBLEM_SVM) {
    if (desc->n_pos < 1 || desc->n_pos > desc->n - 1) return bad("n_pos outside [1, n-1]");
    if (desc->radii) return bad("radii given for SVM");
  } else {
    if (desc->v1_index < 0 || desc->v1_index >= desc->n) return bad("v1_index outside [0, n)");
  }
  if (desc->eps < 0 || desc->delta < 0 || desc->patience < 0 || desc->t_cap < 0 || desc->max_iters < 0 ||
      desc->chunk < 0 || desc->grid < 0)
    return bad("negative parameter");

  auto *c = new scp_mwu_ctx();
  c->problem = desc->problem;
  c->n = desc->n;
  c->d = desc->d;
  c->ld = ld;
  c->n_pos = desc->n_pos;
  c->v1 = desc->problem == SCP_MWU_PROBLEM_SES ? desc->v1_index : 0;
  c->radii = desc->radii;
  c->eps = desc->eps > 0 ? desc->eps : 1e-3;
  c->delta = desc->delta > 0 ? desc->delta : 1e-4;
  c->patience = desc->patience > 0 ? desc->patience : 10;
  c->flags = desc->flags;
  c->max_iters = desc->max_iters;
  c->chunk = desc->chunk > 0 ? desc->chunk : 32;
  c->stream = (hipStream_t)desc->stream;
  c->t_cap = desc->t_cap > 0 ? desc->t_cap
                             : std::min<int64_t>((int64_t)std::ceil(std::log((double)c->n) / (c->eps * c->eps)),
                                                 20000);
  auto fail = [&](int code, const std::string &m) {
    g_init_error = m;
    scp_mwu_destroy(c);
    return code;
  };
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return fail(SCP_MWU_E_HIP, "no HIP device");

  // storage: borrowed, or a library-owned BF16 copy or FP8 codes and scales
  c->dtype = storage;
  c->X = desc->points;
  if (storage == kBF16 && desc->dtype != kBF16) {
    const int64_t ldb = desc->d;
    if (hipMalloc(&c->owned, (size_t)c->n * ldb * 2) != hipSuccess) return fail(SCP_MWU_E_NOMEM, "BF16 copy");
    if (launch_cast((const float *)desc->points, (uint16_t *)c->owned, c->n, c->d, ld, ldb, c->stream) != hipSuccess)
      return fail(SCP_MWU_E_HIP, "BF16 cast launch");
    c->X = c->owned;
    c->ld = ldb;
  } else if (storage == kFP8) {
    if (hipMalloc(&c->owned, (size_t)c->n * c->d) != hipSuccess ||
        hipMalloc(&c->owned_scales, sizeof(float) * (size_t)c->n) != hipSuccess)
      return fail(SCP_MWU_E_NOMEM, "FP8 codes and scales");
    if (launch_quantize_fp8((const float *)desc->points, c->n, c->d, ld, (uint8_t *)c->owned, c->owned_scales,
                            c->stream) != hipSuccess)
      return fail(SCP_MWU_E_HIP, "FP8 quantize launch");
    c->X = c->owned;
    c->ld = c->d;
  }

  // launch shape
  int epl = 1;
  while (kG * epl < c->d) epl *= 2;
  const int es = (int)elem_size(c->dtype);
  const int vf = std::min(epl, 16 / es);
  int vec = 1;
  for (int v : {vf, vf >= 4 ? vf / 2 : 1, 1}) {
    if (c->d % v == 0 && c->ld % v == 0 && ((uintptr_t)c->X % (size_t)(v * es)) == 0) {
      vec = v;
      break;
    }
  }
  // prefetch mode: none (measured fastest); SCPMWU_PASS_PREFETCH=1 selects two
  // register batches
  int pfm = kPrefetchNone;
  if (const char *pfe = getenv("SCPMWU_PASS_PREFETCH"))
    if (pfe[0] == '1') pfm = kPrefetchRegs;
  const int B = pass_steps(es, epl, c->problem, pfm) * kRowsPerStep;
  const int64_t nb = (c->n + B - 1) / B;
  int grid = desc->grid > 0 ? desc->grid : cus;
  grid = (int)std::max<int64_t>(1, std::min<int64_t>(grid, (nb + kPassWaves - 1) / kPassWaves));
  c->grid = grid;
  c->cfg = LaunchCfg{grid, epl, vec, false, pfm};
  c->cfg_cert = LaunchCfg{grid, epl, vec, true, pfm};

  const int pw = partial_width((int)c->d);
  // fused epilogue for SES when every workgroup can read all records from
  // L2 cheaply: d <= 128 and at most kFuseRecBytes of records
  c->fused = c->problem == kSES && kG * epl <= 128 &&
             (int64_t)grid * (((c->d + 1) & ~1) + 8) * 8 <= kFuseRecBytes;
  if (const char *fe = getenv("SCPMWU_FUSED"))
    if (fe[0] == '0') c->fused = false;
  c->rec_stride = (int64_t)(grid + rec_groups(grid)) * pw;
  c->gmode = c->fused && !(c->flags & SCP_MWU_FLAG_DETERMINISTIC);
  // unfused passes (SVM, SES with large records) add into one global sum
  // that their epilogue reads and clears
  const bool gsum_unfused = !c->fused && !(c->flags & SCP_MWU_FLAG_DETERMINISTIC);
  c->g_stride = (pw + 31) / 32 * 32;
  if (hipMalloc(&c->st_base, 2 * sizeof(DevState)) != hipSuccess ||
      hipMalloc(&c->vec_base, 2 * sizeof(double) * kNumVec * c->d) != hipSuccess ||
      hipMalloc(&c->part_base, 2 * sizeof(double) * (size_t)c->rec_stride) != hipSuccess ||
      hipMalloc(&c->g_base, 3 * sizeof(double) * (size_t)c->g_stride) != hipSuccess ||
      hipMalloc(&c->mon, sizeof(double) * (size_t)grid * 4) != hipSuccess ||
      hipHostMalloc((void **)&c->host_st, sizeof(DevState), hipHostMallocDefault) != hipSuccess)
    return fail(SCP_MWU_E_NOMEM, "workspace allocation");
  if (hipStreamCreate(&c->cap_stream) != hipSuccess) return fail(SCP_MWU_E_HIP, "capture stream");

  PassArgs &a = c->args;
  a.X = c->X;
  a.n = c->n;
  a.d = c->d;
  a.ld = c->ld;
  a.radii = c->radii;
  a.v1 = c->v1;
  a.n_pos = c->n_pos;
  a.scales = c->owned_scales;
  if (gsum_unfused) {
    if (hipMemsetAsync(c->g_base, 0, sizeof(double) * (size_t)c->g_stride, c->stream) != hipSuccess)
      return fail(SCP_MWU_E_HIP, "sum clear");
    a.gsum = c->g_base;
  }
  a.st = c->st_base;
  a.vec = c->vec_base;
  a.partials = c->part_base;
  c->base = a;
  set_cur(c, 0);

  // D (one streaming pass): SES distance from v1, SVM largest norm.
  c->r = c->problem == kSES ? 2 * (c->n - 1) : c->n;
  c->rho = 1.0;  // placeholder until D is known
  int rc = start_test(c, 1.0, 1, false);  // ubar = v1 (SES) / 0 (SVM)
  if (rc) return fail(rc, c->err);
  c->active = false;
  if (c->problem == kSES && c->radii) {
    if (hipMemcpyAsync(&c->gamma1, c->radii + c->v1, sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
      return fail(SCP_MWU_E_HIP, "radius readback");
  }
  if (monitor(c, c->vec + kVecMean * c->d, c->problem == kSES ? c->v1 : -1, 0) != hipSuccess)
    return fail(SCP_MWU_E_HIP, "D pass launch");
  double m[4];
  rc = monitor_result(c, m);
  if (rc) return fail(rc, c->err);
  if (c->problem == kSES) {
    c->D = m[0] + c->gamma1;
    c->R = std::sqrt(2.0);
    c->rho = 3.0 * c->D / std::sqrt(2.0);
    if (!std::isfinite(c->D) || !std::isfinite(m[1])) return fail(SCP_MWU_E_NUMERIC, "non-finite input");
    if (!(c->D > 0)) return fail(SCP_MWU_E_INVAL, "all spheres coincide (D = 0)");
    if (c->gamma1 > c->D / 2) return fail(SCP_MWU_E_INVAL, "radius of sphere v1 exceeds D/2");
  } else {
    c->D = m[1];
    c->R = 2.0;
    c->rho = 2.0 * c->D;
    if (!std::isfinite(c->D)) return fail(SCP_MWU_E_NUMERIC, "non-finite input");
    if (!(c->D > 0)) return fail(SCP_MWU_E_INVAL, "all points are zero");
  }
  *out = c;
  return SCP_MWU_OK;
}

int scp_mwu_time_passes(scp_mwu_ctx *c, int32_t k, double *ms_pass, double *ms_iter) {
  if (!c) return SCP_MWU_E_INVAL;
  if (!ms_pass || !ms_iter || k < 1)
    return c->fail(SCP_MWU_E_INVAL, "time_passes: k >= 1 and both outputs required");
  if (!c->active) return c->fail(SCP_MWU_E_STATE, "no test started");
  // three events per iteration: before the pass, between pass and epilogue,
  // after.  Fused mode: one kernel is the whole iteration (its epilogue part
  // being the previous pass's), timed as both; the flush follows, untimed.
  std::vector<hipEvent_t> ev(3 * (size_t)k, nullptr);
  int rc = SCP_MWU_OK;
  for (auto &e : ev)
    if (!rc) rc = c->hip(hipEventCreate(&e), "event create");
  for (int32_t i = 0; i < k && !rc; ++i) {
    rc = c->hip(hipEventRecord(ev[3 * i], c->stream), "event record");
    if (c->fused) {
      if (!rc) rc = c->hip(fused_kernel(c, false, c->stream), "pass launch");
      if (!rc) rc = c->hip(hipEventRecord(ev[3 * i + 1], c->stream), "event record");
    } else {
      if (!rc) rc = c->hip(pass_kernel(c, false, c->stream), "pass launch");
      if (!rc) rc = c->hip(hipEventRecord(ev[3 * i + 1], c->stream), "event record");
      if (!rc) rc = c->hip(epilogue_kernel(c, false, c->stream), "epilogue launch");
    }
    if (!rc) rc = c->hip(hipEventRecord(ev[3 * i + 2], c->stream), "event record");
  }
  if (!rc) rc = c->hip(flush(c, false, c->stream), "flush launch");
  if (!rc) rc = c->hip(hipEventSynchronize(ev.back()), "event sync");
  double tp = 0.0, ti = 0.0;
  for (int32_t i = 0; i < k && !rc; ++i) {
    float a = 0.f, b = 0.f;
    rc = c->hip(hipEventElapsedTime(&a, ev[3 * i], ev[3 * i + 1]), "event elapsed");
    if (!rc) rc = c->hip(hipEventElapsedTime(&b, ev[3 * i], ev[3 * i + 2]), "event elapsed");
    tp += a;
    ti += b;
  }
  for (auto &e : ev)
    if (e) (void)hipEventDestroy(e);
  if (rc) return rc;
  *ms_pass = tp / k;
  *ms_iter = ti / k;
  return read_state(c);
}

int scp_mwu_get_D(const scp_mwu_ctx *c, double *D) {
  if (!c || !D) return SCP_MWU_E_INVAL;
  *D = c->D;
  return SCP_MWU_OK;
}

int scp_mwu_step(scp_mwu_ctx *c, double alpha, int64_t T, int32_t k, int32_t reset, scp_mwu_stepinfo *info) {
  if (!c) return SCP_MWU_E_INVAL;
  if (!info || !(alpha > 0) || !std::isfinite(alpha) || T < 1 || k < 0)
    return c->fail(SCP_MWU_E_INVAL, "step: alpha > 0, T >= 1, k >= 0 and info required");
  int rc;
  if (reset || !c->active || alpha != c->alpha || T != c->T) {
    const bool early = !(c->flags & (SCP_MWU_FLAG_NO_EARLY_STOP | SCP_MWU_FLAG_THEORY));
    rc = start_test(c, alpha, T, early);
    if (rc) return rc;
  }
  rc = run_iters(c, k);
  if (rc) return rc;
  if (k == 0 && (rc = read_state(c))) return rc;
  fill_info(c, info);
  if (c->host_st->status == kNumeric) return c->fail(SCP_MWU_E_NUMERIC, "non-finite value in the iteration");
  return SCP_MWU_OK;
}

int scp_mwu_get_state(scp_mwu_ctx *c, double *sums, int64_t *t) {
  if (!c) return SCP_MWU_E_INVAL;
  if (!sums || !t) return c->fail(SCP_MWU_E_INVAL, "NULL output");
  if (!c->active) return c->fail(SCP_MWU_E_STATE, "no test started");
  int rc = read_state(c);
  if (rc) return rc;
  rc = read_vec(c, kVecS, sums);
  if (rc) return rc;
  if (c->problem == kSVM) {
    sums[c->d] = c->host_st->S1;
    sums[c->d + 1] = c->host_st->S2;
  }
  *t = c->host_st->t;
  return SCP_MWU_OK;
}

int scp_mwu_set_state(scp_mwu_ctx *c, double alpha, int64_t T, int64_t t, const double *sums) {
  if (!c) return SCP_MWU_E_INVAL;
  if (!(alpha > 0) || !std::isfinite(alpha) || T < 1 || t < 0 || (t > 0 && !sums))
    return c->fail(SCP_MWU_E_INVAL, "set_state: alpha > 0, T >= 1, t >= 0, sums");
  const bool early = !(c->flags & (SCP_MWU_FLAG_NO_EARLY_STOP | SCP_MWU_FLAG_THEORY));
  int rc = start_test(c, alpha, T, early);
  if (rc) return rc;
  if (t == 0) return read_state(c);
  for (int64_t j = 0; j < c->d + (c->problem == kSVM ? 2 : 0); ++j)
    if (!std::isfinite(sums[j])) return c->fail(SCP_MWU_E_INVAL, "set_state: non-finite sums");
  rc = c->hip(hipMemcpyAsync(c->vec + kVecS * c->d, sums, sizeof(double) * c->d, hipMemcpyHostToDevice, c->stream),
              "state upload");
  if (rc) return rc;
  const double S1 = c->problem == kSVM ? sums[c->d] : 0.0, S2 = c->problem == kSVM ? sums[c->d + 1] : 0.0;
  rc = c->hip(launch_set_state_k(c->args, c->problem, t, S1, S2, c->stream), "set_state launch");
  if (rc) return rc;
  // bound on the next pass's largest exponent, measured exactly
  double m[4];
  double sb;
  if (c->problem == kSES) {
    rc = c->hip(monitor(c, c->vec + kVecMean * c->d, c->v1, 0), "bound pass");
    if (rc) return rc;
    if ((rc = monitor_result(c, m))) return rc;
    sb = m[0];
  } else {
    rc = c->hip(monitor(c, c->vec + kVecMean * c->d, -1, 1), "bound pass");
    if (rc) return rc;
    if ((rc = monitor_result(c, m))) return rc;
    const double s1b = S1 / (double)t, s2b = S2 / (double)t;
    sb = std::min(-m[2] - s1b, -m[3] - s2b);
  }
  rc = c->hip(hipMemcpyAsync((char *)c->st + offsetof(DevState, shift_bound), &sb, sizeof(double),
                             hipMemcpyHostToDevice, c->stream), "bound upload");
  if (rc) return rc;
  return read_state(c);
}

int scp_mwu_get_vector(scp_mwu_ctx *c, int32_t which, double *y) {
  if (!c) return SCP_MWU_E_INVAL;
  if (!y || which < 0 || which > 2) return c->fail(SCP_MWU_E_INVAL, "get_vector: which in {0,1,2}, y");
  if (!c->active) return c->fail(SCP_MWU_E_STATE, "no test started");
  const int slot = which == 0 ? kVecMean : (which == 1 ? kVecBest : kVecLast);
  int rc = read_vec(c, slot, y);
  if (rc) return rc;
  if ((rc = read_state(c))) return rc;
  if (c->problem == kSVM) {
    const DevState &s = *c->host_st;
    y[c->d] = which == 0 ? s.s1bar : (which == 2 ? s.s1_last : NAN);
    y[c->d + 1] = which == 0 ? s.s2bar : (which == 2 ? s.s2_last : NAN);
  }
  return SCP_MWU_OK;
}

int scp_mwu_backward(scp_mwu_ctx *c, double grad_value, float *grad_points, double *value,
                     int32_t checkpoint_every) {
  return scpmwu::backward_with_workspace(c, grad_value, grad_points, value, checkpoint_every, nullptr, 0);
}

int scp_mwu_solve(scp_mwu_ctx *c, scp_mwu_result *res, double *y) {
  if (!c) return SCP_MWU_E_INVAL;
  if (!res) return c->fail(SCP_MWU_E_INVAL, "res is NULL");
  const bool theory = (c->flags & SCP_MWU_FLAG_THEORY) != 0;
  const bool early = !(c->flags & (SCP_MWU_FLAG_NO_EARLY_STOP | SCP_MWU_FLAG_THEORY));
  const bool ses = c->problem == kSES;
  const int64_t d = c->d;
  std::vector<double> best((size_t)d + 2, 0.0);
  double L, U, Lc, Uc;
  if (ses) {
    L = c->D / 2.0;
    U = c->D;
    // the sphere at v1 of radius D encloses every input: start from v1
    int rc = start_test(c, 1.0, 1, false);
    if (rc) return rc;
    if ((rc = read_vec(c, kVecMean, best.data()))) return rc;
  } else {
    L = 0.0;
    U = 2.0 * c->D;
  }
  Lc = L;
  Uc = U;
  double lb_cert = 0.0;
  bool have_w = false;
  int64_t iters = 0;
  int tests = 0;
  bool converged = false;
  int rc;
  for (int step = 0; step < (ses ? 200 : 400); ++step) {
    if (U - L <= c->eps * (ses ? L : U)) {
      converged = true;
      break;
    }
    if (c->max_iters > 0 && iters >= c->max_iters) break;
    const double alpha = ses ? L + (U - L) / 3.0 : U - (U - L) / 3.0;
    const double eps_k = (U - L) / (3.0 * alpha);
    int64_t T = theory ? theory_T(c, eps_k, alpha) : std::min(theory_T(c, eps_k, alpha), c->t_cap);
    T = std::max(T, min_T(c));
    const int64_t budget = c->max_iters > 0 ? c->max_iters - iters : 0;
    if ((rc = run_test(c, alpha, T, early, budget))) return rc;
    const DevState s = *c->host_st;
    ++tests;
    if (s.status == kNumeric) return c->fail(SCP_MWU_E_NUMERIC, "non-finite value in the iteration");
    if (s.status == kRunning) {  // budget spent inside the test
      iters += s.t;
      break;
    }
    iters += s.t_end;
    if (ses) {
      if (s.f_best < Uc) {
        Uc = s.f_best;
        if ((rc = read_vec(c, kVecBest, best.data()))) return rc;
      }
      if ((c->flags & SCP_MWU_FLAG_CERTIFICATES) && !c->radii) lb_cert = std::max(lb_cert, s.bound);
      if (s.status == kSeparated) {
        L = alpha;
        Lc = std::max(Lc, alpha);
      } else if (s.status == kBeat) {
        U = s.f_best;
      } else {
        U = std::min(U, L + 2.0 * (U - L) / 3.0);
      }
      U = std::min(U, Uc);
    } else {
      Uc = std::min(Uc, s.bound);
      if (s.t_best > 0 && s.f_best > Lc) {
        Lc = s.f_best;
        if ((rc = read_vec(c, kVecBest, best.data()))) return rc;
        have_w = true;
      }
      if (s.status == kSeparated)
        U = alpha;
      else if (s.status == kBeat)
        L = std::max(L, s.f_best);
      else
        L = std::max(L, std::max(s.f_best, L + (U - L) / 3.0));
      U = std::min(U, Uc);
      L = std::max(L, Lc);
    }
  }
  if (!converged) converged = (U - L <= c->eps * (ses ? L : U));
  res->D = c->D;
  res->iters = iters;
  res->passes = iters;
  res->tests = tests;
  res->converged = converged ? 1 : 0;
  res->search_lo = L;
  res->search_hi = U;
  if (ses) {
    res->value = Uc;
    res->lower = std::max(Lc, lb_cert);
    res->upper = Uc;
    if (y) {
      std::memcpy(y, best.data(), sizeof(double) * d);
      y[d] = Uc;
    }
  } else {
    if (!(Uc > 0)) return c->fail(SCP_MWU_E_INFEASIBLE, "certified margin upper bound <= 0");
    res->value = Lc;
    res->lower = Lc;
    res->upper = Uc;
    if (y) {
      double nw = 0;
      for (int64_t j = 0; j < d; ++j) nw += best[j] * best[j];
      nw = std::sqrt(nw);
      for (int64_t j = 0; j < d; ++j) y[j] = have_w && nw > 0 ? best[j] / nw : 0.0;
      double s1 = 0, s2 = 0;
      if (have_w && nw > 0) {
        // s1 = min_P x.w, s2 = -max_Q x.w for the returned unit normal
        if ((rc = c->hip(hipMemcpyAsync(c->vec + kVecLast * d, y, sizeof(double) * d, hipMemcpyHostToDevice, c->stream),
                         "normal upload")))
          return rc;
        if ((rc = c->hip(monitor(c, c->vec + kVecLast * d, -1, 1), "margin pass"))) return rc;
        double m[4];
        if ((rc = monitor_result(c, m))) return rc;
        s1 = -m[2];
        s2 = -m[3];
      }
      y[d] = s1;
      y[d + 1] = s2;
    }
  }
  c->active = false;
  return converged ? SCP_MWU_OK : SCP_MWU_STOPPED;
}

int scp_mwu_read_reference(const void *buf, int64_t bytes, int32_t reps, void *stream, double *ms) {
  if (!buf || !ms || bytes <= 0 || reps < 1 || (reinterpret_cast<uintptr_t>(buf) & 15u) != 0)
    return SCP_MWU_E_INVAL;
  const hipStream_t s = (hipStream_t)stream;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    return SCP_MWU_E_HIP;
  float *sink = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = SCP_MWU_OK;
  if (hipMalloc(&sink, 64) != hipSuccess) return SCP_MWU_E_NOMEM;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = SCP_MWU_E_HIP;
  // one launch to warm up, then reps timed launches
  if (!rc && launch_read_reference(buf, bytes, cus, sink, s) != hipSuccess) rc = SCP_MWU_E_HIP;
  if (!rc && hipEventRecord(e0, s) != hipSuccess) rc = SCP_MWU_E_HIP;
  for (int32_t i = 0; i < reps && !rc; ++i)
    if (launch_read_reference(buf, bytes, cus, sink, s) != hipSuccess) rc = SCP_MWU_E_HIP;
  if (!rc && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)) rc = SCP_MWU_E_HIP;
  float t = 0.f;
  if (!rc && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = SCP_MWU_E_HIP;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(sink);
  if (!rc) *ms = (double)t / reps;
  return rc;
}

int scp_mwu_quantize_fp8(const float *src, int64_t n, int64_t d, int64_t ld, uint8_t *codes, float *scales,
                         void *stream) {
  if (!src || !codes || !scales || n < 0 || d < 1 || ld < d) return SCP_MWU_E_INVAL;
  if (n == 0) return SCP_MWU_OK;
  const hipError_t e = launch_quantize_fp8(src, n, d, ld, codes, scales, (hipStream_t)stream);
  return e == hipSuccess ? SCP_MWU_OK : SCP_MWU_E_HIP;
}

int scp_mwu_cast_bf16(const float *src, uint16_t *dst, int64_t n, void *stream) {
  if (!src || !dst || n < 0) return SCP_MWU_E_INVAL;
  if (n == 0) return SCP_MWU_OK;
  hipError_t e = launch_cast(src, dst, 1, n, n, n, (hipStream_t)stream);
  return e == hipSuccess ? SCP_MWU_OK : SCP_MWU_E_HIP;
}

}  // extern "C"
