// Host side of the batched smallest-enclosing-sphere entry points declared in
// include/scp_mwu.h: instance layout (column layouts, workgroup shares,
// record blocks), graph-captured iterations of the whole batch, and the
// adaptive alpha search of Section 3 run for every instance at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/scp_mwu.h"
#include "mwu_common.hpp"

using namespace scpmwu;

namespace {

thread_local std::string g_batch_init_error;

constexpr double kTauB = 1e-12;  // relative tie tolerance of the separation test

// Alpha search of one SES instance (Section 3, "From feasibility to
// optimization", max form): the interval [L, U] starts at [D/2, D]; a test at
// alpha = L + (U - L)/3 either separates (OPT > alpha: L = alpha) or not
// (U shrinks to the best f seen, or by the paper's conclusion to
// L + 2(U - L)/3); the certified radius is the best f over all tests.  The
// same rules as scp_mwu_solve for a point set.
struct SesSearch {
  double L = 0, U = 0, Lc = 0, Uc = 0;
  int64_t iters = 0;
  int tests = 0, steps = 0;
  bool converged = false, done = false;

  void start(double D) {
    L = Lc = D / 2.0;
    U = Uc = D;
  }
  // the next test's alpha and eps_k, or false when the search is over
  bool next(double eps, int64_t max_iters, double *alpha, double *eps_k) {
    if (U - L <= eps * L) {
      converged = true;
      return false;
    }
    if (steps >= 200 || (max_iters > 0 && iters >= max_iters)) {
      converged = U - L <= eps * L;
      return false;
    }
    ++steps;
    *alpha = L + (U - L) / 3.0;
    *eps_k = (U - L) / (3.0 * *alpha);
    return true;
  }
  // outcome of a finished test; true when its best mean improves the radius
  bool apply(const DevState &s, double alpha) {
    ++tests;
    iters += s.t_end;
    bool improved = false;
    if (s.f_best < Uc) {
      Uc = s.f_best;
      improved = true;
    }
    if (s.status == kSeparated) {
      L = alpha;
      Lc = std::max(Lc, alpha);
    } else if (s.status == kBeat) {
      U = s.f_best;
    } else {
      U = std::min(U, L + 2.0 * (U - L) / 3.0);
    }
    U = std::min(U, Uc);
    return improved;
  }
};

struct Inst {
  int64_t n = 0, d = 0, offset = 0;
  int rows = 0;  // 1: row-per-lane layout (d <= 16), epl = columns held per lane
  int epl = 1, vec = 1, vg = 1;
  int64_t rec_off = 0, vec_off = 0;
  double D = 0, rho = 0, R = 0;
  int64_t r = 0, t_cap = 0;
  // current test
  bool active = false;
  double alpha = 0;
  int64_t T = 0;
};

struct Layout {
  int rows, epl, vec;
  BatchTile *tiles;  // device
  int ntiles;
  std::vector<BatchTile> htiles;  // host copy of tiles
  BatchTile *act = nullptr;       // device: the tiles of the instances listed as running
  int nact = 0;
};

}  // namespace

struct scp_mwu_batch {
  int m = 0, dtype = 0;  // dtype: storage streamed by the kernels (F32 or BF16)
  double eps = 1e-3, delta = 1e-4;
  int32_t patience = 10, flags = 0, chunk = 32, rows_per_group = 16384;
  int64_t t_cap = 0, max_iters = 0;
  hipStream_t stream = nullptr, cap_stream = nullptr;
  const void *X = nullptr;
  void *owned = nullptr;
  std::vector<Inst> inst;
  std::vector<Layout> layouts;
  int64_t vec_total = 0, d_total = 0;
  // device workspace
  PassArgs *args = nullptr;
  DevState *st = nullptr;
  double *vec = nullptr, *partials = nullptr, *Dd = nullptr;
  int32_t *nrec = nullptr, *list = nullptr;
  InitParams *params = nullptr;
  // pinned host staging
  DevState *h_st = nullptr;
  int32_t *h_list = nullptr;
  InitParams *h_params = nullptr;
  double *h_vec = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool any_test = false;
  // the solve's running instances: their tiles (Layout::act) and their
  // PassArgs and record counts back to back, so that the launches of an
  // iteration cover only them; rebuilt as instances finish
  std::vector<PassArgs> h_args;
  std::vector<int32_t> h_nrec;
  PassArgs *act_args = nullptr;
  int32_t *act_nrec = nullptr;
  int nact = 0;
  bool use_act = false;
  // 2 .. 4 instances over one point set (the k-way search): one pass loads
  // each batch of rows once for all of them (column layout kw_epl, kw_vec,
  // kw_grid workgroups = every instance's share count)
  int kway = 0, kw_epl = 1, kw_vec = 1, kw_grid = 1;
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

hipError_t pass_launch(scp_mwu_batch *b, const Layout &l, hipStream_t s) {
  const int nt = b->use_act ? l.nact : l.ntiles;
  const BatchTile *tl = b->use_act ? l.act : l.tiles;
  if (nt == 0) return hipSuccess;
  if (l.rows)
    return b->dtype == kBF16 ? launch_rows_batch_bf16(l.epl, l.vec, nt, b->args, tl, s)
                             : launch_rows_batch_f32(l.epl, l.vec, nt, b->args, tl, s);
  return b->dtype == kBF16 ? launch_pass_batch_bf16(l.epl, l.vec, nt, b->args, tl, s)
                           : launch_pass_batch_f32(l.epl, l.vec, nt, b->args, tl, s);
}

hipError_t epilogue_launch(scp_mwu_batch *b, hipStream_t s) {
  const int m = b->use_act ? b->nact : b->m;
  const PassArgs *args = b->use_act ? b->act_args : b->args;
  const int32_t *nrec = b->use_act ? b->act_nrec : b->nrec;
  if (m == 0) return hipSuccess;
  return b->dtype == kBF16 ? launch_epilogue_batch_bf16(m, args, nrec, s)
                           : launch_epilogue_batch_f32(m, args, nrec, s);
}

void drop_graph(scp_mwu_batch *b) {
  if (b->gexec) hipGraphExecDestroy(b->gexec);
  b->gexec = nullptr;
}

// List the instances marked active as the only running ones: their tiles per
// layout and their PassArgs / record counts, uploaded once; the captured
// graph is dropped so that the next chunk is captured with the new counts.
// An instance left out must stay out of every launch until the next call,
// so this runs only between chunks and only over the instances that will
// run (every other instance's state says its test has ended).
int set_active(scp_mwu_batch *b, bool on) {
  drop_graph(b);
  b->use_act = on;
  if (!on) return SCP_MWU_OK;
  std::vector<PassArgs> aa;
  std::vector<int32_t> an;
  for (int k = 0; k < b->m; ++k)
    if (b->inst[k].active) {
      aa.push_back(b->h_args[k]);
      an.push_back(b->h_nrec[k]);
    }
  b->nact = (int)aa.size();
  if (b->nact && (hipMemcpy(b->act_args, aa.data(), sizeof(PassArgs) * aa.size(), hipMemcpyHostToDevice) != hipSuccess ||
                  hipMemcpy(b->act_nrec, an.data(), sizeof(int32_t) * an.size(), hipMemcpyHostToDevice) != hipSuccess))
    return b->fail(SCP_MWU_E_HIP, "running-instance upload");
  for (Layout &l : b->layouts) {
    std::vector<BatchTile> t;
    for (const BatchTile &x : l.htiles)
      if (b->inst[x.inst].active) t.push_back(x);
    l.nact = (int)t.size();
    if (l.nact && hipMemcpy(l.act, t.data(), sizeof(BatchTile) * t.size(), hipMemcpyHostToDevice) != hipSuccess)
      return b->fail(SCP_MWU_E_HIP, "running-tile upload");
  }
  return SCP_MWU_OK;
}

// The streaming pass of every running instance (one launch per layout, or
// the shared-read pass of a k-way batch).
hipError_t passes(scp_mwu_batch *b, hipStream_t s) {
  if (b->kway) {
    // 2 or 3 tests: one shared pass; 4 tests: two shared passes of two
    const int ks = b->kway == 4 ? 2 : b->kway;
    for (int j0 = 0; j0 < b->kway; j0 += ks) {
      const hipError_t e =
          b->dtype == kBF16 ? launch_kway_batch_bf16(b->kw_epl, b->kw_vec, ks, b->kw_grid, b->args + j0, s)
                            : launch_kway_batch_f32(b->kw_epl, b->kw_vec, ks, b->kw_grid, b->args + j0, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  for (const Layout &l : b->layouts) {
    const hipError_t e = pass_launch(b, l, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// One iteration of every running instance.
hipError_t iteration(scp_mwu_batch *b, hipStream_t s) {
  const hipError_t e = passes(b, s);
  if (e != hipSuccess) return e;
  return epilogue_launch(b, s);
}

int build_graph(scp_mwu_batch *b) {
  if (b->gexec) return SCP_MWU_OK;
  hipGraph_t g = nullptr;
  int rc = b->hip(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
  if (rc) return rc;
  hipError_t e = hipSuccess;
  for (int k = 0; k < b->chunk && e == hipSuccess; ++k) e = iteration(b, b->cap_stream);
  const hipError_t e2 = hipStreamEndCapture(b->cap_stream, &g);
  if (e != hipSuccess) return b->hip(e, "capture iteration");
  if ((rc = b->hip(e2, "end capture"))) return rc;
  e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  return b->hip(e, "graph instantiate");
}

int read_states(scp_mwu_batch *b) {
  int rc = b->hip(hipMemcpyAsync(b->h_st, b->st, sizeof(DevState) * (size_t)b->m, hipMemcpyDeviceToHost, b->stream),
                  "state readback");
  if (rc) return rc;
  return b->hip(hipStreamSynchronize(b->stream), "state sync");
}

int read_vectors(scp_mwu_batch *b) {
  int rc = b->hip(hipMemcpyAsync(b->h_vec, b->vec, sizeof(double) * (size_t)b->vec_total, hipMemcpyDeviceToHost,
                                 b->stream),
                  "vector readback");
  if (rc) return rc;
  return b->hip(hipStreamSynchronize(b->stream), "vector sync");
}

bool any_running(const scp_mwu_batch *b) {
  for (int k = 0; k < b->m; ++k)
    if (b->inst[k].active && b->h_st[k].status == kRunning) return true;
  return false;
}

// Up to k iterations of the batch; stops early once no test is running.
int run_iters(scp_mwu_batch *b, int64_t k) {
  int rc;
  while (k > 0) {
    if (k >= b->chunk && b->chunk > 1) {
      if ((rc = build_graph(b))) return rc;
      if ((rc = b->hip(hipGraphLaunch(b->gexec, b->stream), "graph launch"))) return rc;
      k -= b->chunk;
    } else {
      if ((rc = b->hip(iteration(b, b->stream), "iteration launch"))) return rc;
      k -= 1;
    }
    if ((rc = read_states(b))) return rc;
    if (!any_running(b)) break;
  }
  return SCP_MWU_OK;
}

InitParams test_params(const scp_mwu_batch *b, const Inst &I, double alpha, int64_t T, bool early) {
  InitParams p{};
  p.alpha = alpha;
  p.T = T;
  p.eta = std::sqrt(std::log((double)I.r) / (double)T);
  p.kscale = p.eta / (I.rho * std::sqrt(2.0));
  p.delta = b->delta;
  p.tau = kTauB;
  p.D = I.D;
  p.gamma1 = 0.0;
  p.patience = b->patience;
  p.early = early ? 1 : 0;
  return p;
}

// Start the tests staged in h_list / h_params[0 .. count).  The staging
// buffers are reused only after a later stream synchronisation.
int start_tests(scp_mwu_batch *b, int count) {
  if (count == 0) return SCP_MWU_OK;
  int rc = b->hip(hipMemcpyAsync(b->list, b->h_list, sizeof(int32_t) * count, hipMemcpyHostToDevice, b->stream),
                  "test list upload");
  if (rc) return rc;
  if ((rc = b->hip(hipMemcpyAsync(b->params, b->h_params, sizeof(InitParams) * count, hipMemcpyHostToDevice,
                                  b->stream),
                   "test parameter upload")))
    return rc;
  const hipError_t e = b->dtype == kBF16 ? launch_init_batch_bf16(count, b->args, b->list, b->params, b->stream)
                                         : launch_init_batch_f32(count, b->args, b->list, b->params, b->stream);
  if ((rc = b->hip(e, "test init"))) return rc;
  for (int j = 0; j < count; ++j) {
    Inst &I = b->inst[b->h_list[j]];
    I.active = true;
    I.alpha = b->h_params[j].alpha;
    I.T = b->h_params[j].T;
  }
  b->any_test = true;
  return SCP_MWU_OK;
}

int64_t theory_T(const Inst &I, double eps, double alpha) {
  const double v = 4.0 * (I.R * I.R) * (I.rho * I.rho) * std::log((double)I.r) / ((eps * eps) * (alpha * alpha));
  if (!(v < 9.0e18)) return INT64_MAX / 2;
  return (int64_t)std::ceil(v);
}

void fill_info(const DevState &s, scp_mwu_stepinfo *info) {
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

}  // namespace

extern "C" {

const char *scp_mwu_batch_last_error(const scp_mwu_batch *b) {
  return b ? b->err.c_str() : g_batch_init_error.c_str();
}

void scp_mwu_batch_destroy(scp_mwu_batch *b) {
  if (!b) return;
  if (b->gexec) hipGraphExecDestroy(b->gexec);
  if (b->cap_stream) hipStreamDestroy(b->cap_stream);
  for (Layout &l : b->layouts) {
    hipFree(l.tiles);
    hipFree(l.act);
  }
  hipFree(b->act_args);
  hipFree(b->act_nrec);
  hipFree(b->args);
  hipFree(b->st);
  hipFree(b->vec);
  hipFree(b->partials);
  hipFree(b->Dd);
  hipFree(b->nrec);
  hipFree(b->list);
  hipFree(b->params);
  hipFree(b->owned);
  hipHostFree(b->h_st);
  hipHostFree(b->h_list);
  hipHostFree(b->h_params);
  hipHostFree(b->h_vec);
  delete b;
}

int scp_mwu_batch_init(const scp_mwu_batch_desc *desc, scp_mwu_batch **out) {
  g_batch_init_error.clear();
  auto bad = [&](const std::string &m) {
    g_batch_init_error = m;
    return SCP_MWU_E_INVAL;
  };
  if (!out) return bad("out is NULL");
  *out = nullptr;
  if (!desc) return bad("desc is NULL");
  if (desc->struct_size < sizeof(scp_mwu_batch_desc)) return bad("desc->struct_size too small");
  if (desc->dtype != SCP_MWU_F32) return bad("batched dtype must be F32");
  const int storage = desc->storage ? desc->storage : desc->dtype;
  if (storage != SCP_MWU_F32 && storage != SCP_MWU_BF16) return bad("batched storage must be F32 or BF16");
  if (desc->count < 1) return bad("count < 1");
  if (!desc->n || !desc->d || !desc->offset || !desc->points) return bad("NULL array or points");
  if ((uintptr_t)desc->points % 4) return bad("points misaligned");
  if (desc->eps < 0 || desc->delta < 0 || desc->patience < 0 || desc->t_cap < 0 || desc->max_iters < 0 ||
      desc->chunk < 0 || desc->rows_per_group < 0)
    return bad("negative parameter");
  const int m = desc->count;
  int64_t total = 0;
  for (int k = 0; k < m; ++k) {
    if (desc->n[k] < 2) return bad("instance " + std::to_string(k) + ": n < 2");
    if (desc->d[k] < 1 || desc->d[k] > kMaxD) return bad("instance " + std::to_string(k) + ": d outside [1, 512]");
    if (desc->offset[k] < 0) return bad("instance " + std::to_string(k) + ": negative offset");
    if (desc->d[k] * 4 * 64 >= (int64_t)1 << 30) return bad("row too long");
    total = std::max(total, desc->offset[k] + desc->n[k] * desc->d[k]);
  }

  auto *b = new scp_mwu_batch();
  auto fail = [&](int code, const std::string &msg) {
    g_batch_init_error = msg;
    scp_mwu_batch_destroy(b);
    return code;
  };
  b->m = m;
  b->dtype = storage;
  b->eps = desc->eps > 0 ? desc->eps : 1e-3;
  b->delta = desc->delta > 0 ? desc->delta : 1e-4;
  b->patience = desc->patience > 0 ? desc->patience : 10;
  b->flags = desc->flags;
  b->chunk = desc->chunk > 0 ? desc->chunk : 32;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return fail(SCP_MWU_E_HIP, "no HIP device");
  if (desc->rows_per_group > 0) {
    b->rows_per_group = desc->rows_per_group;
  } else {
    // about two workgroups per compute unit over all instances, within
    // [1024, 16384] rows per workgroup share
    int64_t rows = 0;
    for (int k = 0; k < m; ++k) rows += desc->n[k];
    const int64_t want = (rows + 2 * (int64_t)cus - 1) / (2 * (int64_t)cus);
    b->rows_per_group = (int32_t)std::min<int64_t>(16384, std::max<int64_t>(1024, want));
  }
  b->t_cap = desc->t_cap;
  b->max_iters = desc->max_iters;
  b->stream = (hipStream_t)desc->stream;
  b->X = desc->points;
  const int64_t es = storage == kBF16 ? 2 : 4;
  if (storage == kBF16) {
    if (hipMalloc(&b->owned, (size_t)total * 2) != hipSuccess) return fail(SCP_MWU_E_NOMEM, "BF16 copy");
    if (launch_cast((const float *)desc->points, (uint16_t *)b->owned, 1, total, total, total, b->stream) !=
        hipSuccess)
      return fail(SCP_MWU_E_HIP, "BF16 cast launch");
    b->X = b->owned;
  }

  // instance layout: column layout, workgroup shares, record and vector blocks
  b->inst.resize(m);
  std::map<std::tuple<int, int, int>, std::vector<int>> groups;
  int64_t rec_total = 0;
  for (int k = 0; k < m; ++k) {
    Inst &I = b->inst[k];
    I.n = desc->n[k];
    I.d = desc->d[k];
    I.offset = desc->offset[k];
    // d <= 16: one lane per row, epl = columns held per lane (2, 3, 4, 8, 16;
    // d = 3 exactly, loaded one value at a time); otherwise 16 lanes per row
    // with epl columns each
    I.rows = I.d <= 16 ? 1 : 0;
    if (I.rows) {
      I.epl = 2;
      while (I.epl < I.d) I.epl *= 2;
      if (I.d == 3) I.epl = 3;
    } else {
      while (kG * I.epl < I.d) I.epl *= 2;
    }
    const int vf = I.epl == 3 ? 1 : std::min<int>(I.epl, (int)(16 / es));
    const uintptr_t base = (uintptr_t)b->X + (uintptr_t)(I.offset * es);
    for (int v : {vf, vf >= 4 ? vf / 2 : 1, 1}) {
      if (I.d % v == 0 && base % (uintptr_t)(v * es) == 0) {
        I.vec = v;
        break;
      }
    }
    I.vg = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (I.n + b->rows_per_group - 1) / b->rows_per_group));
    I.rec_off = rec_total;
    rec_total += (int64_t)I.vg * partial_width((int)I.d);
    I.vec_off = b->vec_total;
    b->vec_total += kNumVec * I.d;
    b->d_total += I.d;
    I.r = 2 * (I.n - 1);
    I.t_cap = b->t_cap > 0 ? b->t_cap
                           : std::min<int64_t>((int64_t)std::ceil(std::log((double)I.n) / (b->eps * b->eps)), 20000);
    groups[{I.rows, I.epl, I.vec}].push_back(k);
  }
  if (hipMalloc(&b->args, sizeof(PassArgs) * m) != hipSuccess ||
      hipMalloc(&b->st, sizeof(DevState) * m) != hipSuccess ||
      hipMalloc(&b->vec, sizeof(double) * (size_t)b->vec_total) != hipSuccess ||
      hipMalloc(&b->partials, sizeof(double) * (size_t)rec_total) != hipSuccess ||
      hipMalloc(&b->Dd, sizeof(double) * m) != hipSuccess || hipMalloc(&b->nrec, sizeof(int32_t) * m) != hipSuccess ||
      hipMalloc(&b->list, sizeof(int32_t) * m) != hipSuccess ||
      hipMalloc(&b->act_args, sizeof(PassArgs) * m) != hipSuccess ||
      hipMalloc(&b->act_nrec, sizeof(int32_t) * m) != hipSuccess ||
      hipMalloc(&b->params, sizeof(InitParams) * m) != hipSuccess ||
      hipHostMalloc((void **)&b->h_st, sizeof(DevState) * m, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&b->h_list, sizeof(int32_t) * m, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&b->h_params, sizeof(InitParams) * m, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&b->h_vec, sizeof(double) * (size_t)b->vec_total, hipHostMallocDefault) != hipSuccess)
    return fail(SCP_MWU_E_NOMEM, "batch workspace");
  if (hipStreamCreate(&b->cap_stream) != hipSuccess) return fail(SCP_MWU_E_HIP, "capture stream");

  std::vector<PassArgs> hargs(m);
  std::vector<int32_t> hn(m);
  for (int k = 0; k < m; ++k) {
    const Inst &I = b->inst[k];
    PassArgs &a = hargs[k];
    a = PassArgs{};
    a.X = (const char *)b->X + I.offset * es;
    a.n = I.n;
    a.d = I.d;
    a.ld = I.d;
    a.radii = nullptr;
    a.v1 = 0;
    a.n_pos = 0;
    a.st = b->st + k;
    a.vec = b->vec + I.vec_off;
    a.partials = b->partials + I.rec_off;
    a.scales = nullptr;
    hn[k] = I.vg;
  }
  if (hipMemcpy(b->args, hargs.data(), sizeof(PassArgs) * m, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->nrec, hn.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice) != hipSuccess)
    return fail(SCP_MWU_E_HIP, "instance table upload");
  b->h_args = hargs;
  b->h_nrec = hn;
  for (auto &kv : groups) {
    // tiles interleaved by share index: share v of every instance of the
    // layout, then share v + 1, ...  Instances over the same rows (the
    // k-way search) then read each row block at about the same time.
    std::vector<BatchTile> tiles;
    int vmax = 0;
    for (int k : kv.second) vmax = std::max(vmax, b->inst[k].vg);
    for (int v = 0; v < vmax; ++v)
      for (int k : kv.second)
        if (v < b->inst[k].vg) tiles.push_back(BatchTile{k, v, b->inst[k].vg, 0});
    Layout l{std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), nullptr, (int)tiles.size()};
    if (hipMalloc(&l.tiles, sizeof(BatchTile) * tiles.size()) != hipSuccess ||
        hipMalloc(&l.act, sizeof(BatchTile) * tiles.size()) != hipSuccess) {
      hipFree(l.tiles);
      return fail(SCP_MWU_E_NOMEM, "tiles");
    }
    l.htiles = tiles;
    b->layouts.push_back(l);
    if (hipMemcpy(l.tiles, tiles.data(), sizeof(BatchTile) * tiles.size(), hipMemcpyHostToDevice) != hipSuccess)
      return fail(SCP_MWU_E_HIP, "tile upload");
  }
  // a k-way batch: 2 or 3 instances over the same rows with d <= 128 share
  // each load; 4 instances share it in pairs (the per-test work makes a
  // shared pass of four tests slower than four passes; SCPMWU_KWAY_SHARED=0
  // keeps one pass per instance)
  bool same = m >= 2 && m <= 4 && b->inst[0].d <= kG * 8;
  if (const char *ke = getenv("SCPMWU_KWAY_SHARED"))
    if (ke[0] == '0') same = false;
  for (int k = 1; k < m && same; ++k)
    same = b->inst[k].n == b->inst[0].n && b->inst[k].d == b->inst[0].d && b->inst[k].offset == b->inst[0].offset;
  if (same) {
    const Inst &I0 = b->inst[0];
    int ce = 1;
    while (kG * ce < I0.d) ce *= 2;
    const int vf = std::min<int>(ce, (int)(16 / es));
    const uintptr_t base = (uintptr_t)b->X + (uintptr_t)(I0.offset * es);
    int cv = 1;
    for (int v : {vf, vf >= 4 ? vf / 2 : 1, 1}) {
      if (I0.d % v == 0 && base % (uintptr_t)(v * es) == 0) {
        cv = v;
        break;
      }
    }
    b->kway = m;
    b->kw_epl = ce;
    b->kw_vec = cv;
    b->kw_grid = I0.vg;
  }
  // the state words start as "not running", so that a pass before any test
  // does nothing
  if (hipMemsetAsync(b->st, 0xFF, sizeof(DevState) * m, b->stream) != hipSuccess)
    return fail(SCP_MWU_E_HIP, "state clear");

  // D of every instance
  const hipError_t e = storage == kBF16 ? launch_diameter_batch_bf16(m, b->args, b->Dd, b->stream)
                                        : launch_diameter_batch_f32(m, b->args, b->Dd, b->stream);
  if (e != hipSuccess) return fail(SCP_MWU_E_HIP, "D launch");
  std::vector<double> hD(m);
  if (hipMemcpyAsync(hD.data(), b->Dd, sizeof(double) * m, hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
      hipStreamSynchronize(b->stream) != hipSuccess)
    return fail(SCP_MWU_E_HIP, "D readback");
  for (int k = 0; k < m; ++k) {
    Inst &I = b->inst[k];
    I.D = hD[k];
    if (!std::isfinite(I.D)) return fail(SCP_MWU_E_NUMERIC, "instance " + std::to_string(k) + ": non-finite input");
    if (!(I.D > 0)) return fail(SCP_MWU_E_INVAL, "instance " + std::to_string(k) + ": all points coincide (D = 0)");
    I.R = std::sqrt(2.0);
    I.rho = 3.0 * I.D / std::sqrt(2.0);
  }
  *out = b;
  return SCP_MWU_OK;
}

int scp_mwu_batch_get_D(const scp_mwu_batch *b, double *D) {
  if (!b || !D) return SCP_MWU_E_INVAL;
  for (int k = 0; k < b->m; ++k) D[k] = b->inst[k].D;
  return SCP_MWU_OK;
}

int scp_mwu_batch_step(scp_mwu_batch *b, const double *alpha, const int64_t *T, int32_t k, int32_t reset,
                       scp_mwu_stepinfo *info) {
  if (!b) return SCP_MWU_E_INVAL;
  if (!alpha || !T || !info || k < 0) return b->fail(SCP_MWU_E_INVAL, "batch step: alpha, T, info and k >= 0 required");
  for (int j = 0; j < b->m; ++j)
    if (!(alpha[j] > 0) || !std::isfinite(alpha[j]) || T[j] < 1)
      return b->fail(SCP_MWU_E_INVAL, "batch step: alpha > 0 and T >= 1 required for every instance");
  const bool early = !(b->flags & (SCP_MWU_FLAG_NO_EARLY_STOP | SCP_MWU_FLAG_THEORY));
  int count = 0;
  for (int j = 0; j < b->m; ++j) {
    const Inst &I = b->inst[j];
    if (reset || !I.active || alpha[j] != I.alpha || T[j] != I.T) {
      b->h_list[count] = j;
      b->h_params[count] = test_params(b, I, alpha[j], T[j], early);
      ++count;
    }
  }
  int rc = start_tests(b, count);
  if (rc) return rc;
  if ((rc = run_iters(b, k))) return rc;
  if (k == 0 && (rc = read_states(b))) return rc;
  bool numeric = false;
  for (int j = 0; j < b->m; ++j) {
    fill_info(b->h_st[j], info + j);
    numeric = numeric || b->h_st[j].status == kNumeric;
  }
  if (numeric) return b->fail(SCP_MWU_E_NUMERIC, "non-finite value in the iteration");
  return SCP_MWU_OK;
}

int scp_mwu_batch_get_vector(scp_mwu_batch *b, int32_t which, double *y) {
  if (!b) return SCP_MWU_E_INVAL;
  if (!y || which < 0 || which > 2) return b->fail(SCP_MWU_E_INVAL, "get_vector: which in [0, 2], y required");
  if (!b->any_test) return b->fail(SCP_MWU_E_STATE, "no test started");
  const int slot = which == 0 ? kVecMean : (which == 1 ? kVecBest : kVecLast);
  int rc = read_vectors(b);
  if (rc) return rc;
  int64_t o = 0;
  for (const Inst &I : b->inst) {
    std::memcpy(y + o, b->h_vec + I.vec_off + slot * I.d, sizeof(double) * I.d);
    o += I.d;
  }
  return SCP_MWU_OK;
}

int scp_mwu_batch_time_iters(scp_mwu_batch *b, int32_t k, double *ms_pass, double *ms_iter) {
  if (!b) return SCP_MWU_E_INVAL;
  if (k < 1 || !ms_pass || !ms_iter) return b->fail(SCP_MWU_E_INVAL, "time_iters: k >= 1 and outputs required");
  if (!b->any_test) return b->fail(SCP_MWU_E_STATE, "no test started");
  std::vector<hipEvent_t> ev(3 * (size_t)k, nullptr);
  int rc = SCP_MWU_OK;
  for (auto &e : ev)
    if (!rc) rc = b->hip(hipEventCreate(&e), "event create");
  for (int i = 0; i < k && !rc; ++i) {
    rc = b->hip(hipEventRecord(ev[3 * i], b->stream), "event record");
    if (!rc) rc = b->hip(passes(b, b->stream), "pass launch");
    if (!rc) rc = b->hip(hipEventRecord(ev[3 * i + 1], b->stream), "event record");
    if (!rc) rc = b->hip(epilogue_launch(b, b->stream), "epilogue launch");
    if (!rc) rc = b->hip(hipEventRecord(ev[3 * i + 2], b->stream), "event record");
  }
  if (!rc) rc = b->hip(hipStreamSynchronize(b->stream), "timing sync");
  double tp = 0, ti = 0;
  for (int i = 0; i < k && !rc; ++i) {
    float a = 0, c = 0;
    rc = b->hip(hipEventElapsedTime(&a, ev[3 * i], ev[3 * i + 1]), "elapsed");
    if (!rc) rc = b->hip(hipEventElapsedTime(&c, ev[3 * i], ev[3 * i + 2]), "elapsed");
    tp += a;
    ti += c;
  }
  for (auto &e : ev)
    if (e) hipEventDestroy(e);
  if (rc) return rc;
  *ms_pass = tp / k;
  *ms_iter = ti / k;
  return read_states(b);
}

int scp_mwu_batch_solve(scp_mwu_batch *b, scp_mwu_result *res, double *y) {
  if (!b) return SCP_MWU_E_INVAL;
  if (!res) return b->fail(SCP_MWU_E_INVAL, "res is NULL");
  const bool theory = (b->flags & SCP_MWU_FLAG_THEORY) != 0;
  const bool early = !(b->flags & (SCP_MWU_FLAG_NO_EARLY_STOP | SCP_MWU_FLAG_THEORY));
  const int m = b->m;
  std::vector<SesSearch> S(m);
  std::vector<double> best((size_t)b->d_total);
  std::vector<int64_t> doff(m);
  int64_t o = 0;
  for (int k = 0; k < m; ++k) {
    S[k].start(b->inst[k].D);
    doff[k] = o;
    o += b->inst[k].d;
  }
  int rc;
  // every search starts from the sphere at v1 of radius D: a test staged for
  // every instance sets ubar = v1, read back as the initial centres; the
  // state words are then cleared to "not running"
  for (int k = 0; k < m; ++k) {
    b->h_list[k] = k;
    b->h_params[k] = test_params(b, b->inst[k], 1.0, 1, false);
  }
  if ((rc = start_tests(b, m)) || (rc = read_vectors(b))) return rc;
  for (int k = 0; k < m; ++k) {
    std::memcpy(best.data() + doff[k], b->h_vec + b->inst[k].vec_off + kVecBest * b->inst[k].d,
                sizeof(double) * b->inst[k].d);
    b->inst[k].active = false;
  }
  if ((rc = b->hip(hipMemsetAsync(b->st, 0xFF, sizeof(DevState) * m, b->stream), "state clear"))) return rc;
  // as instances finish their searches, the launches shrink to the running
  // ones (relisted whenever a quarter of the listed instances has finished);
  // the full lists are restored when the solve returns
  struct FullLists {
    scp_mwu_batch *b;
    ~FullLists() { set_active(b, false); }
  } full_lists{b};
  int listed = m;
  while (true) {
    // start the next test of every instance without one
    int count = 0;
    for (int k = 0; k < m; ++k) {
      Inst &I = b->inst[k];
      if (S[k].done || I.active) continue;
      double alpha, eps_k;
      if (!S[k].next(b->eps, b->max_iters, &alpha, &eps_k)) {
        S[k].done = true;
        continue;
      }
      int64_t T = theory ? theory_T(I, eps_k, alpha) : std::min(theory_T(I, eps_k, alpha), I.t_cap);
      T = std::max<int64_t>(T, std::max<int64_t>(1, (int64_t)std::ceil(std::log((double)I.r))));
      b->h_list[count] = k;
      b->h_params[count] = test_params(b, I, alpha, T, early);
      ++count;
    }
    if ((rc = start_tests(b, count))) return rc;
    int nrun = 0;
    for (int k = 0; k < m; ++k) nrun += b->inst[k].active ? 1 : 0;
    if (nrun == 0) break;
    if (4 * nrun <= 3 * listed) {
      if ((rc = set_active(b, true))) return rc;
      listed = nrun;
    }
    if ((rc = run_iters(b, b->chunk))) return rc;
    // finished tests: outcome, best centre
    bool need_vec = false;
    for (int k = 0; k < m; ++k) {
      const DevState &s = b->h_st[k];
      if (!b->inst[k].active || s.status == kRunning) continue;
      if (s.status == kNumeric) return b->fail(SCP_MWU_E_NUMERIC, "instance " + std::to_string(k) + ": non-finite value");
      need_vec = need_vec || s.f_best < S[k].Uc;
    }
    if (need_vec && (rc = read_vectors(b))) return rc;
    for (int k = 0; k < m; ++k) {
      Inst &I = b->inst[k];
      const DevState &s = b->h_st[k];
      if (!I.active || s.status == kRunning) continue;
      if (S[k].apply(s, I.alpha))
        std::memcpy(best.data() + doff[k], b->h_vec + I.vec_off + kVecBest * I.d, sizeof(double) * I.d);
      I.active = false;
    }
  }
  bool all = true;
  int64_t yo = 0;
  for (int k = 0; k < m; ++k) {
    const SesSearch &s = S[k];
    scp_mwu_result &r = res[k];
    r.value = s.Uc;
    r.lower = s.Lc;
    r.upper = s.Uc;
    r.search_lo = s.L;
    r.search_hi = s.U;
    r.D = b->inst[k].D;
    r.iters = s.iters;
    r.passes = s.iters;
    r.tests = s.tests;
    r.converged = s.converged ? 1 : 0;
    all = all && s.converged;
    if (y) {
      std::memcpy(y + yo, best.data() + doff[k], sizeof(double) * b->inst[k].d);
      y[yo + b->inst[k].d] = s.Uc;
      yo += b->inst[k].d + 1;
    }
  }
  return all ? SCP_MWU_OK : SCP_MWU_STOPPED;
}

int scp_mwu_batch_solve_kway(scp_mwu_batch *b, scp_mwu_result *res, double *y) {
  if (!b) return SCP_MWU_E_INVAL;
  if (!res) return b->fail(SCP_MWU_E_INVAL, "res is NULL");
  const int k = b->m;
  const Inst &I0 = b->inst[0];
  for (const Inst &I : b->inst)
    if (I.n != I0.n || I.d != I0.d || I.offset != I0.offset)
      return b->fail(SCP_MWU_E_INVAL, "k-way search: the instances must be one point set");
  const bool theory = (b->flags & SCP_MWU_FLAG_THEORY) != 0;
  const bool early = !(b->flags & (SCP_MWU_FLAG_NO_EARLY_STOP | SCP_MWU_FLAG_THEORY));
  const int64_t d = I0.d;
  const double D = I0.D;
  double L = D / 2.0, U = D, Lc = L, Uc = U;
  std::vector<double> best((size_t)d), alpha(k), concl(k);
  int64_t iters = 0, passes = 0;
  int tests = 0, rc;
  bool converged = false;
  // the search starts from the sphere at v1 of radius D
  for (int j = 0; j < k; ++j) {
    b->h_list[j] = j;
    b->h_params[j] = test_params(b, b->inst[j], 1.0, 1, false);
  }
  if ((rc = start_tests(b, k)) || (rc = read_vectors(b))) return rc;
  std::memcpy(best.data(), b->h_vec + I0.vec_off + kVecBest * d, sizeof(double) * d);
  int round = 0;
  for (; round < 200; ++round) {
    if (U - L <= b->eps * L) {
      converged = true;
      break;
    }
    if (b->max_iters > 0 && iters >= b->max_iters) break;
    const double g = 2.0 * k + 1.0;
    for (int i = 1; i <= k; ++i) {
      const Inst &I = b->inst[i - 1];
      alpha[i - 1] = L + (2.0 * i - 1.0) * (U - L) / g;
      concl[i - 1] = L + 2.0 * i * (U - L) / g;
      const double eps_i = (U - L) / (g * alpha[i - 1]);
      int64_t T = theory ? theory_T(I, eps_i, alpha[i - 1]) : std::min(theory_T(I, eps_i, alpha[i - 1]), I.t_cap);
      T = std::max<int64_t>(T, std::max<int64_t>(1, (int64_t)std::ceil(std::log((double)I.r))));
      b->h_list[i - 1] = i - 1;
      b->h_params[i - 1] = test_params(b, I, alpha[i - 1], T, early);
    }
    if ((rc = start_tests(b, k))) return rc;
    // the tests advance together; between chunks, the tests that ended are
    // taken in the order in which they ended (ties: the lower alpha first),
    // and each stops the tests its outcome makes moot: a separated test those
    // below it, any other test those above it.  A stopped test decides
    // nothing and counts the iterations it ran until it was stopped.
    std::vector<int64_t> stop(k, -1);  // the iteration at which a moot test was stopped
    std::vector<bool> seen(k, false);   // ended tests already taken
    while (true) {
      if ((rc = run_iters(b, b->chunk))) return rc;
      std::vector<int> ended;
      for (int j = 0; j < k; ++j)
        if (!seen[j] && stop[j] < 0 && b->h_st[j].status != kRunning) ended.push_back(j);
      std::sort(ended.begin(), ended.end(), [&](int x, int z) {
        return b->h_st[x].t_end != b->h_st[z].t_end ? b->h_st[x].t_end < b->h_st[z].t_end : x < z;
      });
      for (int i : ended) {
        if (stop[i] >= 0) continue;  // made moot by a test that ended before it
        seen[i] = true;
        const bool sep = b->h_st[i].status == kSeparated;
        for (int j = sep ? 0 : i + 1; j < (sep ? i : k); ++j) {
          if (seen[j] || stop[j] >= 0) continue;
          stop[j] = b->h_st[i].t_end;
          if (b->h_st[j].status == kRunning) {
            // end the test on the device (the stream is idle between chunks)
            const int32_t st = kTReached;
            if ((rc = b->hip(hipMemcpy((char *)(b->st + j) + offsetof(DevState, status), &st, sizeof(st),
                                       hipMemcpyHostToDevice),
                             "stop a moot test")))
              return rc;
            b->h_st[j].status = kTReached;
          }
        }
      }
      if (!any_running(b)) break;
    }
    bool need_vec = false;
    int64_t longest = 0;
    for (int j = 0; j < k; ++j) {
      const DevState &s = b->h_st[j];
      if (stop[j] < 0 && s.status == kNumeric) return b->fail(SCP_MWU_E_NUMERIC, "non-finite value in the iteration");
      // a moot test ended (or would have ended) no earlier than the test that
      // made it moot
      const int64_t ran = stop[j] >= 0 ? stop[j] : s.t_end;
      if (stop[j] < 0) need_vec = need_vec || s.f_best < Uc;
      iters += ran;
      longest = std::max<int64_t>(longest, ran);
      b->inst[j].active = false;
    }
    passes += longest;
    tests += k;
    if (need_vec && (rc = read_vectors(b))) return rc;
    for (int j = 0; j < k; ++j) {
      const DevState &s = b->h_st[j];
      if (stop[j] < 0 && s.f_best < Uc) {
        Uc = s.f_best;
        std::memcpy(best.data(), b->h_vec + b->inst[j].vec_off + kVecBest * d, sizeof(double) * d);
      }
    }
    double Ln = L;
    for (int j = 0; j < k; ++j)
      if (stop[j] < 0 && b->h_st[j].status == kSeparated) Ln = std::max(Ln, alpha[j]);
    Lc = std::max(Lc, Ln);
    double Un = std::min(U, Uc);
    for (int j = 0; j < k; ++j) {
      const DevState &s = b->h_st[j];
      if (stop[j] < 0 && s.status != kSeparated && alpha[j] >= Ln)
        Un = std::min(Un, s.status == kBeat ? s.f_best : concl[j]);
    }
    L = Ln;
    U = Un;
  }
  if (round == 200) converged = U - L <= b->eps * L;
  res->value = Uc;
  res->lower = Lc;
  res->upper = Uc;
  res->search_lo = L;
  res->search_hi = U;
  res->D = D;
  res->iters = iters;
  res->passes = passes;
  res->tests = tests;
  res->converged = converged ? 1 : 0;
  if (y) {
    std::memcpy(y, best.data(), sizeof(double) * d);
    y[d] = Uc;
  }
  return converged ? SCP_MWU_OK : SCP_MWU_STOPPED;
}

}  // extern "C"
