/*
 * scp_mwu.h -- C ABI of the MI355X (gfx950) primal-dual symmetric-cone MWU
 * library for the smallest enclosing sphere (SES) and hard-margin SVM
 * problems of Zheng, Varvitsiotis, Tan and Lin, "A Primal-Dual Framework for
 * Symmetric Cone Programming" (arXiv 2405.09157).
 *
 * The caller states its problem in the paper's natural form:
 *   SES  (problem SES, Section 4.1):  min gamma  s.t. ||u - v_i|| <= gamma - gamma_i
 *   SVM  (problem SVM, Section 4.2):  max s1 + s2 s.t. P^T w >= s1 1,
 *                                     -Q^T w >= s2 1, ||w|| <= 1
 * and the library forms the cones, a_j, c and b of the primal/dual pair
 * (LCP)/(SCP) of Sections 1 and 3 internally: for SES the hard cone is the
 * product over i != v1 of second-order cones Q^{d+1} (eq. dualses), for SVM
 * it is the orthant R^n_+ (eq. svm_dual_scp).  Results come back as the
 * paper's primal/dual pair, i.e. a dual point y (the centre / the normal and
 * offsets) with its objective, plus certified lower and upper bounds on OPT.
 *
 * One MWU iteration (the hot path) is one streaming pass over the n x d
 * point matrix in HBM fused with the SCMWU update (eq. SCMWU, eq. implement /
 * eq. min_implement): per-point loss, Jordan exponential of every cone block
 * from its spectral values, trace normalisation, and the weighted sum that
 * gives the ORACLE's next centre (eq. ses_oracle) or hyperplane
 * (eq. svm_oracle), followed by the FP64 epilogue of the meta-algorithm
 * (separation test, running mean, f(t) monitor and early stopping of
 * Section 5).
 *
 * Conventions
 *   - All pointers named "device" must point to memory on the GPU that the
 *     context's stream can access (e.g. the data_ptr() of a torch tensor).
 *     They are BORROWED: the caller keeps them alive until scp_mwu_destroy.
 *   - Pointers named "host" are ordinary CPU memory owned by the caller.
 *   - Every call enqueues device work on the context's stream and
 *     synchronises that stream only to read back small results.  A context
 *     may be used by one host thread at a time.
 *   - Return codes: SCP_MWU_OK (0), SCP_MWU_STOPPED (1: budget spent, outputs
 *     valid but the search interval is wider than requested), or a negative
 *     SCP_MWU_E_* code.  Output structures are written only on OK / STOPPED.
 *     The text of the last error of a context is given by
 *     scp_mwu_last_error().
 */
#ifndef SCP_MWU_H
#define SCP_MWU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SCP_MWU_ABI_VERSION 1

/* problem kinds */
enum {
  SCP_MWU_PROBLEM_SES = 1, /* smallest enclosing sphere of n points/spheres in R^d */
  SCP_MWU_PROBLEM_SVM = 2  /* hard-margin SVM of two point sets in R^d */
};

/* element types of the point matrix */
enum {
  SCP_MWU_F32 = 1,  /* IEEE binary32 */
  SCP_MWU_BF16 = 2, /* bfloat16 (upper half of a binary32), stored as uint16 */
  SCP_MWU_F64 = 3,  /* IEEE binary64 */
  SCP_MWU_FP8 = 4   /* storage only: FP8 E4M3 codes (uint8) with one binary32
                       scale per row, made by init from binary32 points */
};

/* return codes */
enum {
  SCP_MWU_OK = 0,
  SCP_MWU_STOPPED = 1,
  SCP_MWU_E_INVAL = -1,      /* bad argument or descriptor */
  SCP_MWU_E_NOMEM = -2,      /* device or host allocation failed */
  SCP_MWU_E_HIP = -3,        /* a HIP runtime call failed (text in last_error) */
  SCP_MWU_E_STATE = -4,      /* call not valid in the context's current state */
  SCP_MWU_E_NUMERIC = -5,    /* NaN/Inf in the input or in the iteration */
  SCP_MWU_E_INFEASIBLE = -6, /* SVM: classes certified not separable */
  SCP_MWU_E_UNSUPPORTED = -7 /* valid request the library does not implement */
};

/* outcome of an alpha-feasibility test (Section 3 meta-algorithm; Section 5
 * early exits) */
enum {
  SCP_MWU_OUT_RUNNING = 0,    /* test still in progress */
  SCP_MWU_OUT_SEPARATED = 1,  /* ORACLE value < 0: SES OPT > alpha, SVM OPT < alpha */
  SCP_MWU_OUT_BEAT = 2,       /* f(t) already better than alpha (Section 5) */
  SCP_MWU_OUT_STABILIZED = 3, /* |f(t)-f(t-1)|/f(t-1) < delta for `patience` runs */
  SCP_MWU_OUT_T_REACHED = 4,  /* T iterations without separation (meta theorem) */
  SCP_MWU_OUT_NUMERIC = 5     /* NaN/Inf met in the epilogue */
};

/* descriptor flags */
enum {
  SCP_MWU_FLAG_NO_EARLY_STOP = 1, /* disable the Section 5 exits (f better than
                                     alpha, stabilisation) in every test */
  SCP_MWU_FLAG_THEORY = 2,        /* solve with T = T_theory of the meta theorem
                                     (no cap) and no early exits: the certified
                                     (1 +- eps) guarantee, at its full cost */
  SCP_MWU_FLAG_CERTIFICATES = 4,  /* SES on points: also compute the weak-duality
                                     lower bound of eq.(ses_qp) from the MWU weights
                                     on the last pass of every launch chunk */
  SCP_MWU_FLAG_DETERMINISTIC = 8  /* results bitwise reproducible for a given grid:
                                     the per-workgroup partial sums of a pass are
                                     combined in a fixed order.  Without it, SES
                                     with d <= 128 adds them with atomics into one
                                     sum (faster; the sums then vary in their last
                                     bits from run to run) */
};

/*
 * Problem descriptor, read by scp_mwu_init (copied; may be freed afterwards).
 * Zero-valued optional fields take the documented default.
 */
typedef struct scp_mwu_desc {
  uint32_t struct_size; /* sizeof(scp_mwu_desc) as compiled by the caller */
  int32_t problem;      /* SCP_MWU_PROBLEM_SES or SCP_MWU_PROBLEM_SVM */
  int32_t dtype;        /* element type of `points` (SCP_MWU_F32/BF16/F64) */
  int32_t storage;      /* element type the iteration streams: 0 = dtype;
                           SCP_MWU_BF16 with dtype SCP_MWU_F32 makes init round
                           the points once (nearest, ties to even) into a
                           library-owned BF16 copy; SCP_MWU_FP8 with dtype
                           SCP_MWU_F32 makes init quantize them once into
                           library-owned per-row scaled FP8 codes (see
                           scp_mwu_quantize_fp8).  With BF16 or FP8 storage
                           the SES pass computes per element in binary32
                           (rows and all sums across rows in binary64). */
  int64_t n;            /* number of points (SES: >= 2; SVM: n_pos + n_neg) */
  int64_t d;            /* dimension, 1 <= d <= 512 */
  int64_t ld;           /* row stride of `points` in elements, >= d (0 = d) */
  const void *points;   /* device, row-major n x d; SVM: rows [0, n_pos) are
                           class +1 (the paper's P), rows [n_pos, n) class -1 (Q) */
  const double *radii;  /* SES: device, n sphere radii gamma_i >= 0, or NULL for
                           a point set; must be NULL for SVM */
  int64_t n_pos;        /* SVM: number of class +1 rows, 1 <= n_pos <= n-1 */
  int64_t v1_index;     /* SES: index of the sphere kept as the easy set C
                           (Section 4.1 keeps "the first one"); default 0 */
  double eps;           /* target accuracy of scp_mwu_solve; default 1e-3 */
  double delta;         /* stabilisation threshold of Section 5; default 1e-4 */
  int32_t patience;     /* consecutive stabilised iterations; default 10 */
  int32_t flags;        /* SCP_MWU_FLAG_* */
  int64_t t_cap;        /* cap on T per test; 0 = min(ceil(ln n / eps^2), 20000) */
  int64_t max_iters;    /* scp_mwu_solve iteration budget; 0 = unlimited */
  void *stream;         /* hipStream_t to enqueue on; NULL = the null stream */
  int32_t chunk;        /* iterations per graph launch; 0 = 32 */
  int32_t grid;         /* workgroups of the streaming pass; 0 = chosen from the
                           device's compute-unit count */
} scp_mwu_desc;

/* State of the current alpha-feasibility test after scp_mwu_step. */
typedef struct scp_mwu_stepinfo {
  int64_t t;          /* ORACLE outputs averaged so far (iterations done) */
  int64_t t_end;      /* iteration at which the test ended, 0 while running */
  int64_t T;          /* iteration cap of this test */
  int32_t outcome;    /* SCP_MWU_OUT_* */
  int32_t degenerate; /* 1 if the last ORACLE met W = 0 (SES) / V = 0 (SVM) */
  double alpha;       /* the guess of OPT under test */
  double eta;         /* SCMWU step size sqrt(ln r / T) */
  double f_last;      /* f of the newest evaluated mean: f(t-1) of the last pass,
                         NaN before any (Section 5 monitor) */
  double f_best;      /* best f in this test (SES: min, SVM: max), a certified
                         upper (SES) / lower (SVM) bound on OPT */
  int64_t t_best;     /* iteration whose mean gave f_best */
  double value;       /* ORACLE objective of the last iteration for the
                         trace-one p(t) (eq. ses_oracle / eq. svm_oracle) */
  double scale;       /* magnitude the separation test compares value with */
  double log_trace;   /* ln Tr exp(-eta sum_tau m(tau)) of the last iteration */
  double bound;       /* SES: certified lower bound from the MWU weights (0 if
                         not computed); SVM: best certified upper bound
                         ||P mu/Tr mu - Q gamma/Tr gamma|| of this test */
} scp_mwu_stepinfo;

/* Result of scp_mwu_solve. */
typedef struct scp_mwu_result {
  double value;        /* SES: radius of the returned sphere (max_i ||c - v_i|| +
                          gamma_i, exact for the returned centre); SVM: margin
                          s1 + s2 achieved by the returned unit normal */
  double lower;        /* certified lower bound on OPT */
  double upper;        /* certified upper bound on OPT */
  double search_lo;    /* final search interval [L, U] of the alpha search */
  double search_hi;
  double D;            /* SES: max_{i != v1} ||v1 - v_i|| + gamma1 + gamma_i;
                          SVM: max_i ||x_i|| */
  int64_t iters;       /* MWU iterations over all tests */
  int32_t tests;       /* alpha-feasibility tests run */
  int32_t converged;   /* 1 if the search met its stop rule */
  int64_t passes;      /* streaming passes over the points: iters, except for
                          the k-way search (scp_mwu_batch_solve_kway), whose k
                          tests of a round share passes (sum over rounds of
                          the round's length) */
} scp_mwu_result;

typedef struct scp_mwu_ctx scp_mwu_ctx;

/*
 * Validate the descriptor, allocate the context's workspace on the current
 * HIP device, make the BF16 copy if asked, and compute D with one streaming
 * pass (SES: Section 4.1 bounds [D/2, D]; SVM: Lemma svm_bound, range
 * (0, 2D]).  No MWU iteration runs.
 *
 * Errors: E_INVAL (NULL pointer, n < 2, d outside [1, 512], ld < d, unknown
 * dtype/storage/problem, misaligned points, n_pos outside [1, n-1], v1_index
 * outside [0, n), radii given for SVM, eps <= 0 or delta < 0),
 * E_NUMERIC (NaN/Inf in the points: D not finite), E_NOMEM, E_HIP.
 * *out is set to NULL on error.
 */
int scp_mwu_init(const scp_mwu_desc *desc, scp_mwu_ctx **out);

/*
 * Run up to k iterations (k >= 0) of the alpha-feasibility test with guess
 * `alpha` > 0 and iteration cap T >= 1 (step size eta = sqrt(ln r / T), r the
 * rank of the hard cone: 2(n-1) for SES, n for SVM).  A new test starts
 * (p(1) = e/r, running mean cleared) when `reset` is non-zero, when no test
 * has been started, or when alpha or T differ from the current test;
 * otherwise the current test continues.  Iterations stop early when the test
 * ends (info->outcome != RUNNING).  The state of the test is written to
 * *info (host).
 *
 * Errors: E_INVAL (alpha <= 0 or not finite, T < 1, k < 0, info NULL),
 * E_HIP, E_NUMERIC (outcome NUMERIC).
 */
int scp_mwu_step(scp_mwu_ctx *ctx, double alpha, int64_t T, int32_t k,
                 int32_t reset, scp_mwu_stepinfo *info);

/*
 * Solve to the descriptor's eps with the adaptive alpha search of Section 3
 * ("From feasibility to optimization"; mirrored for the SVM min form),
 * running one alpha-feasibility test per search step.
 * y (host, >= d + 2 doubles, may be NULL): SES receives the centre c (d
 * values) followed by the radius; SVM receives the unit normal w (d values)
 * followed by s1 and s2 with s1 + s2 = margin.
 * Returns OK when the search met its stop rule, STOPPED when max_iters ran
 * out first (outputs valid).
 * Errors: E_INVAL (res NULL), E_HIP, E_NUMERIC, E_INFEASIBLE (SVM with a
 * certified upper bound <= 0 on the margin).
 */
int scp_mwu_solve(scp_mwu_ctx *ctx, scp_mwu_result *res, double *y);

/*
 * Gradient of the radius after the current test with respect to the points:
 * the adjoint of the unrolled fixed-alpha, fixed-T iterations of the SES
 * split (Section 4.1; ORACLE eq.(ses_oracle); SOC exponential, Section 2.1).
 * The differentiated map runs T iterations at the test's alpha and
 * eta = sqrt(ln r / T) from an empty running sum, with the exponent scale
 * kappa_t = eta (t - 1) / (3D) and D = max_i ||v1 - v_i|| recomputed from the
 * points, and returns R = max_i ||v_i - ubar_T|| (the Section 5 monitor at the
 * final mean); R is differentiable where both maxima are attained once.
 * The call runs the forward iterations once, then walks them back segment by
 * segment.  checkpoint_every = K in 1 .. 50 keeps the running sum every K
 * iterations and recomputes each K-iteration segment before walking it back
 * (three streaming passes over the points per iteration; device workspace
 * about (T/K + 2K) d + 2 K n + n d binary64 values); checkpoint_every = 0
 * keeps the whole tape of the forward run, 2d + 4 numbers per iteration (two
 * passes per iteration; about 2 T d + 100 n + n d values).
 * Requires: an SES context on points without radii, streamed as F32, F64 or
 * BF16 (the gradient is then with respect to the stored BF16 values; no FP8
 * storage), d <= 512, and a current test (scp_mwu_step with
 * reset, any k >= 0): its alpha and T define the map, which always runs all
 * T iterations, also where the test itself stopped earlier (a separation
 * or a Section 5 exit).  The test's state is left unchanged.
 * grad_value: the upstream scalar dL/dR; the output is grad_value * dR/dV.
 * grad_points: device, n x d FP32, row stride d, owned by the caller;
 *   overwritten.  NULL: only the forward iterations run and only *value is
 *   written (the map's value without its gradient).
 * value (host, may be NULL): receives R as the recomputed forward found it.
 * Errors: E_INVAL (grad_points and value both NULL, non-finite grad_value,
 * checkpoint_every outside 0 .. 50), E_UNSUPPORTED
 * (SVM, radii, FP8 storage, d > 512), E_STATE (no test started),
 * E_NOMEM, E_HIP.  Blocks until the result is written.
 */
int scp_mwu_backward(scp_mwu_ctx *ctx, double grad_value, float *grad_points, double *value,
                     int32_t checkpoint_every);

/*
 * scp_mwu_backward for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
 * the same reverse pass, arguments and results, with its workspace in a
 * static device array of the library (128 MiB on every GPU the library runs
 * on, held until the process ends) instead of a per-call allocation.  No
 * hipMalloc, hipFree or allocating routine is called.  A call whose
 * workspace would exceed the array (about (T/K + 2K) d + 2 K n + n d
 * doubles with checkpoint_every = K; 2 T d + 100 n + n d for K = 0) fails
 * with SCP_MWU_E_INVAL before any launch, its text naming the bytes needed.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (two streams, two host threads) race.  Blocks until the result is
 * written, like scp_mwu_backward.
 */
int scp_mwu_backward_noalloc(scp_mwu_ctx *ctx, double grad_value, float *grad_points, double *value,
                             int32_t checkpoint_every);

/*
 * Inspect or replace the running sums of the current test (checkpoint /
 * resume, and step-level comparison with a reference).
 * sums (host): SES: d values sum_{tau<=t} u(tau); SVM: d + 2 values
 *   (sum w(tau), sum s1(tau), sum s2(tau)).
 * scp_mwu_set_state starts a test with (alpha, T) at iteration count t >= 0
 * with the given sums, then runs one streaming pass to bound the exponent
 * range of the next iteration (no MWU step).  E_INVAL on bad sizes/values,
 * E_STATE if get_state is called before any test.
 */
int scp_mwu_get_state(scp_mwu_ctx *ctx, double *sums, int64_t *t);
int scp_mwu_set_state(scp_mwu_ctx *ctx, double alpha, int64_t T, int64_t t,
                      const double *sums);

/*
 * Vectors of the current test (host outputs, d (+2 for SVM) doubles):
 * which = 0: mean ybar(t) of the ORACLE outputs; 1: the mean that gave
 * f_best; 2: the last ORACLE output y(t).  E_STATE before any test.
 */
int scp_mwu_get_vector(scp_mwu_ctx *ctx, int32_t which, double *y);

/*
 * Measurement helper: run k >= 1 further MWU iterations of the current test
 * with HIP events recorded on the context's stream before each streaming
 * pass, between the pass and its combine/epilogue kernel, and after it.
 * Returns (host outputs, milliseconds) the mean duration of the streaming
 * pass kernel (*ms_pass) and of the whole iteration (*ms_iter).  The
 * iterations advance the test exactly as scp_mwu_step does.
 * E_INVAL (k < 1, NULL), E_STATE (no test started), E_HIP.
 */
int scp_mwu_time_passes(scp_mwu_ctx *ctx, int32_t k, double *ms_pass, double *ms_iter);

/* D of the problem (see scp_mwu_result.D); E_INVAL on NULL. */
int scp_mwu_get_D(const scp_mwu_ctx *ctx, double *D);

/* Release the workspace and any library-owned copy.  NULL is a no-op. */
void scp_mwu_destroy(scp_mwu_ctx *ctx);

/* Text of the last error of ctx (never NULL; "" if none; ctx may be NULL,
 * then the last scp_mwu_init failure in this thread is described). */
const char *scp_mwu_last_error(const scp_mwu_ctx *ctx);

/* Static text for a return code. */
const char *scp_mwu_strerror(int code);

/*
 * Batched smallest enclosing sphere: m independent SES point sets (Section
 * 4.1 for each), advanced together.  Every MWU iteration of the batch is one
 * streaming pass per column layout over all instances (each instance split
 * into workgroup shares of about rows_per_group rows) and one epilogue launch
 * with one workgroup per instance; `chunk` iterations are captured in one HIP
 * graph.  Per instance the arithmetic, the alpha-feasibility test and the
 * alpha search are those of scp_mwu_step / scp_mwu_solve for a point set
 * (no radii, v1 = row 0, no certificates).
 */
typedef struct scp_mwu_batch_desc {
  uint32_t struct_size;  /* sizeof(scp_mwu_batch_desc) as compiled by the caller */
  int32_t dtype;         /* SCP_MWU_F32 */
  int32_t storage;       /* 0 = dtype, or SCP_MWU_BF16: init rounds the points
                            once into a library-owned BF16 copy (binary32
                            per-element arithmetic, as for one problem) */
  int32_t count;         /* number of instances m >= 1 */
  const int64_t *n;      /* host, m values: points of instance k, >= 2 */
  const int64_t *d;      /* host, m values: dimension of instance k, in [1, 512] */
  const int64_t *offset; /* host, m values: element offset of instance k's first
                            point in `points`; its n[k] rows are dense (stride
                            d[k]).  Instances may share rows (the points are
                            only read), as the k-way search's slots do */
  const void *points;    /* device, binary32 */
  double eps;            /* target accuracy of scp_mwu_batch_solve; default 1e-3 */
  double delta;          /* stabilisation threshold; default 1e-4 */
  int32_t patience;      /* default 10 */
  int32_t flags;         /* SCP_MWU_FLAG_NO_EARLY_STOP, SCP_MWU_FLAG_THEORY */
  int64_t t_cap;         /* cap on T per test; 0 = min(ceil(ln n_k / eps^2), 20000) */
  int64_t max_iters;     /* per-instance iteration budget of scp_mwu_batch_solve,
                            checked between tests; 0 = unlimited */
  void *stream;          /* hipStream_t; NULL = the null stream */
  int32_t chunk;         /* iterations per graph launch; default 32 */
  int32_t rows_per_group;/* rows per workgroup share of the pass; 0 = about two
                            workgroups per compute unit over all instances,
                            within [1024, 16384] */
} scp_mwu_batch_desc;

typedef struct scp_mwu_batch scp_mwu_batch;

/*
 * Validate, allocate the batch's workspace (state, vectors and records of
 * every instance, the tile tables, pinned readback), make the BF16 copy if
 * asked, and compute every instance's D (one workgroup per instance).
 * Errors: E_INVAL (NULL pointers, count < 1, n < 2, d outside [1, 512],
 * negative offset, misaligned points, dtype other than F32, storage other
 * than F32/BF16, an instance whose points all coincide), E_NUMERIC (NaN/Inf
 * in some instance's points), E_NOMEM, E_HIP.  *out is NULL on error.
 */
int scp_mwu_batch_init(const scp_mwu_batch_desc *desc, scp_mwu_batch **out);

/*
 * Run up to k >= 0 iterations of every instance's alpha-feasibility test.
 * alpha, T (host, m values each): instance j (re)starts its test when reset
 * is non-zero, when it has none, or when alpha[j] or T[j] differ from its
 * current test.  Instances whose test ends stop iterating.  info (host, m
 * entries) receives each instance's state.  Errors: E_INVAL (NULL, k < 0,
 * some alpha <= 0 or T < 1), E_HIP, E_NUMERIC (some outcome NUMERIC).
 */
int scp_mwu_batch_step(scp_mwu_batch *b, const double *alpha, const int64_t *T, int32_t k,
                       int32_t reset, scp_mwu_stepinfo *info);

/*
 * Solve every instance to eps with the alpha search of scp_mwu_solve; the
 * instances' searches run concurrently (a test that ends inside a graph chunk
 * waits for the chunk's end).  res (host, m entries); y (host, may be NULL):
 * instance k's centre (d_k values) then its radius, instances in order
 * (sum of d_k + 1 values).  OK when every search met its stop rule, STOPPED
 * when some budget ran out first (outputs valid).  Errors: E_INVAL, E_HIP,
 * E_NUMERIC.
 */
int scp_mwu_batch_solve(scp_mwu_batch *b, scp_mwu_result *res, double *y);

/*
 * k-way alpha search on one point set (Section 3 allows other searching
 * methods than the one it details).  The batch must hold k >= 1 instances
 * that are the same point set (equal n, d and offset); they serve as the k
 * test slots.  Each round cuts [L, U] into 2k + 1 equal parts and runs the k
 * alpha-feasibility tests at alpha_i = L + (2i - 1)(U - L)/(2k + 1) with
 * eps_i = (U - L)/((2k + 1) alpha_i) together (2 or 3 tests share each read
 * of the rows, 4 tests in pairs, with d <= 128; otherwise one pass per test,
 * their workgroups interleaved by rows so that the reads of a row block
 * coincide in the cache).  In the order in which the tests end (ties: the
 * lower alpha first), an ended test stops the tests its outcome makes moot:
 * a separated test those below it, any other test those above it; a stopped
 * test decides nothing.  After the round every deciding separation raises L
 * to its alpha, every other deciding test whose alpha is not below the new L
 * lowers U to f_best (f beat alpha) or to L + 2i(U - L)/(2k + 1), and every
 * deciding test's f tightens U and the certified radius.  k = 1 is the search
 * of scp_mwu_solve.  res (host, one entry): as scp_mwu_solve, with iters
 * counting a stopped test's iterations until it was stopped and passes = sum
 * over rounds of the round's length (its last deciding test's end); y (host,
 * d + 1 doubles, may be NULL): centre then radius.  OK / STOPPED as
 * scp_mwu_solve.  Errors: E_INVAL (instances not all the same point set,
 * res NULL), E_HIP, E_NUMERIC.
 */
int scp_mwu_batch_solve_kway(scp_mwu_batch *b, scp_mwu_result *res, double *y);

/*
 * Vectors of every instance's current test (host, sum of d_k doubles,
 * instances in order): which = 0 mean, 1 best mean, 2 last ORACLE output.
 * E_INVAL (NULL, which outside [0, 2]), E_STATE before any test, E_HIP.
 */
int scp_mwu_batch_get_vector(scp_mwu_batch *b, int32_t which, double *y);

/* D of every instance (host, m values); E_INVAL on NULL. */
int scp_mwu_batch_get_D(const scp_mwu_batch *b, double *D);

/*
 * Measurement helper: k >= 1 further iterations of the current tests with
 * HIP events around the streaming passes (all column layouts) and around the
 * whole iteration, on the batch's stream; mean milliseconds of each in
 * *ms_pass, *ms_iter (host).  E_INVAL, E_STATE (no test), E_HIP.
 */
int scp_mwu_batch_time_iters(scp_mwu_batch *b, int32_t k, double *ms_pass, double *ms_iter);

/* Release the batch's workspace; NULL is a no-op. */
void scp_mwu_batch_destroy(scp_mwu_batch *b);

/* Text of the batch's last error ("" if none; b NULL: the last failed
 * scp_mwu_batch_init in this thread). */
const char *scp_mwu_batch_last_error(const scp_mwu_batch *b);

/*
 * The SCMWU iterate over a general product cone (eq.(SCMWU); Section 2.1:
 * the Loewner exponential and the trace of a direct sum act blockwise):
 * p = exp(-eta m) / Tr(exp(-eta m)) on K = R^{n_orth}_+ (+) Q^{d_1+1} (+) ...
 * (+) Q^{d_k+1}, in the Jordan algebra whose identity is (0; sqrt2) on each
 * Lorentz block (eigenvalues (x0 +- ||xbar||)/sqrt2, trace sqrt2 x0).
 *
 * A vector of the cone has len binary64 values: the orthant coordinates
 * first, then block j in [offsets[j], offsets[j+1]) as its vector part (d_j
 * values) followed by its scalar part.
 *
 * scp_mwu_product_init validates a layout once and keeps it on the device:
 *   offsets (host, nblocks + 1 values; may be NULL when nblocks = 0):
 *   offsets[0] = n_orth, each block at least 2 long (d_j >= 1), and
 *   offsets[nblocks] = len (len = n_orth without blocks).  The layout's
 *   workspace (a few doubles per workgroup plus the offsets) is owned by
 *   the handle; its launches go on stream (a hipStream_t; NULL = default).
 *   E_INVAL (out NULL, n_orth < 0, nblocks < 0, an empty cone, len < 1,
 *   offsets inconsistent with n_orth or len), E_NOMEM, E_HIP.  Synchronous.
 * scp_mwu_product_exp enqueues the three launches of one iterate:
 *   m (device, len binary64): the cumulative loss;
 *   p (device, len binary64, caller-owned, not aliasing m): the normalised
 *   iterate, trace one;
 *   log_trace (host, may be NULL): ln Tr(exp(-eta m)); when given, the call
 *   waits for the stream to read it, otherwise it returns once the launches
 *   are enqueued.  E_INVAL (NULL handle, m or p, m == p, eta not a positive
 *   finite number), E_HIP.  Calls on one handle are ordered by its stream;
 *   overlapping calls on different streams may not share a handle.
 * scp_mwu_product_destroy waits for the handle's stream and frees it (NULL
 *   is a no-op).
 */
typedef struct scp_mwu_product scp_mwu_product;
int scp_mwu_product_init(int64_t n_orth, const int64_t *offsets, int64_t nblocks, int64_t len, void *stream,
                         scp_mwu_product **out);
int scp_mwu_product_exp(scp_mwu_product *pc, const double *m, double eta, double *p, double *log_trace);
void scp_mwu_product_destroy(scp_mwu_product *pc);

/*
 * Round n FP32 values to BF16 (nearest, ties to even; NaN stays NaN) on the
 * device: src (device, n floats) -> dst (device, n uint16).  The storage
 * conversion init uses; exported so callers can build BF16 inputs.
 * E_INVAL on NULL pointers or n < 0, E_HIP.
 */
int scp_mwu_cast_bf16(const float *src, uint16_t *dst, int64_t n, void *stream);

/*
 * Per-row scaled FP8 storage of an n x d binary32 matrix src (device, row
 * stride ld >= d elements): scales[r] = max_c |src[r][c]| / 448 (binary32
 * division; 1 for an all-zero row) and codes[r * d + c] = the FP8 E4M3 code
 * of src[r][c] / scales[r] (binary32 division), rounded to nearest with ties
 * to even and saturated at 448; E4M3 is sign, 4 exponent bits with bias 7,
 * 3 mantissa bits, no infinities.  The stored value is scales[r] times the
 * decoded code.  codes (device, n * d bytes) and scales (device, n floats)
 * are caller-owned; a NaN element gives a NaN code.  The conversion init uses
 * for SCP_MWU_FP8 storage; exported so callers can inspect it.  Enqueued on
 * stream (a hipStream_t; NULL = default).  E_INVAL (NULL pointers, n < 0,
 * d < 1, ld < d), E_HIP.
 */
int scp_mwu_quantize_fp8(const float *src, int64_t n, int64_t d, int64_t ld, uint8_t *codes, float *scales,
                         void *stream);

/*
 * Measurement helper: the achievable read bandwidth the streaming pass is
 * held to.  Times reps >= 1 launches of a plain streaming read of the bytes
 * bytes at buf (device, 16-byte aligned, only read; no arithmetic on the data)
 * on the stream (a hipStream_t; NULL = default), after one untimed launch,
 * and returns the mean milliseconds per launch in *ms (host).  Allocates and
 * frees a 64-byte device buffer.  E_INVAL (NULL, bytes <= 0, reps < 1,
 * misaligned buf), E_NOMEM, E_HIP.
 */
int scp_mwu_read_reference(const void *buf, int64_t bytes, int32_t reps, void *stream, double *ms);

#ifdef __cplusplus
}
#endif

#endif /* SCP_MWU_H */
