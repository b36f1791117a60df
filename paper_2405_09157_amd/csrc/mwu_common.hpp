// Internal definitions shared by the HIP kernels and the host driver of the
// primal-dual symmetric-cone MWU library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scpmwu {

// Launch geometry.  In the streaming pass a wavefront owns G = 16 lanes per
// point row (one DPP row), so a wave covers 4 rows per load step.  The small
// kernels (monitor, init, state, cast, record groups) use kBlock threads.
constexpr int kWave = 64;
constexpr int kG = 16;
constexpr int kRowsPerStep = kWave / kG;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
// The streaming pass runs 8 waves per workgroup, one workgroup per compute
// unit; its per-workgroup records are combined by one workgroup of
// kCombBlock threads.
constexpr int kPassWaves = 8;
constexpr int kPassBlock = kPassWaves * kWave;
constexpr int kCombBlock = 1024;
// Maximum dimension supported by the streaming pass (16 lanes x 32 columns).
constexpr int kMaxD = 512;
// Width of a workgroup's record: two d-vectors (each padded to an even
// length) around 8 scalars, so that pairs of entries are 16-byte aligned.
inline __host__ __device__ int partial_width(int d) { return 2 * ((d + 1) & ~1) + 8; }

// Records are summed by the one-workgroup epilogue kernel, whose loads are
// bound by one compute unit; when the records it would read exceed
// kRecSingleBytes, a first kernel of ceil(grid / kRecGroup) workgroups sums
// groups of kRecGroup records (the extra kernel boundary costs a few us, the
// single unit reads ~40 KB/us).  The record buffer holds grid + that many
// records.
constexpr int kRecGroup = 16;
constexpr int64_t kRecSingleBytes = 384 * 1024;
inline __host__ __device__ int rec_groups(int grid) { return (grid + kRecGroup - 1) / kRecGroup; }
inline __host__ __device__ bool rec_two_level(int grid, int read_cols) {
  return rec_groups(grid) > 1 && (int64_t)grid * read_cols * 8 > kRecSingleBytes;
}

enum Problem : int32_t { kSES = 1, kSVM = 2 };
enum DType : int32_t { kF32 = 1, kBF16 = 2, kF64 = 3, kFP8 = 4 };

// Load steps per batch of the streaming pass (B = 4 * steps rows, B <= 64),
// shared by the kernels and the host's grid sizing.  A batch's elements stay
// in registers through its three phases, within a budget of 64 VGPRs:
// binary32 registers for F32, BF16 and FP8 values, binary64 for F64.  Raw
// codes stay packed (widened on use) where the columns per lane allow it:
// BF16 pairs for SES with an even count (at most 16), FP8 quadruples for a
// count that is a multiple of 4 (at most 16); packing multiplies the rows per
// batch.  SVM keeps two binary64 class accumulators per column and halves the
// budget; with prefetch two batches share it.  At most 16 steps (64 rows,
// one per lane in the per-row phase).
inline __host__ __device__ constexpr bool pass_packed(int storage_size, int epl, int problem) {
  return (storage_size == 2 && epl % 2 == 0 && epl <= 16 && problem == kSES) ||
         (storage_size == 1 && epl % 4 == 0 && epl <= 16);
}
// Prefetch modes of the streaming pass: none, or two register batches (the
// next one loading while the current one is processed).
enum Prefetch : int32_t { kPrefetchNone = 0, kPrefetchRegs = 1 };
inline __host__ __device__ constexpr int pass_steps(int storage_size, int epl, int problem, int pfm) {
  const bool pack = pass_packed(storage_size, epl, problem);
  const int lim = (storage_size == 8 ? 32 : (pack ? 128 : 64)) /
                  (problem == kSVM ? 2 : 1) / (pfm == kPrefetchRegs ? 2 : 1);
  return lim / epl < 1 ? 1 : (lim / epl > 16 ? 16 : lim / epl);
}

enum Status : int32_t {
  kRunning = 0,
  kSeparated = 1,
  kBeat = 2,
  kStabilized = 3,
  kTReached = 4,
  kNumeric = 5
};

// State of the current alpha-feasibility test, resident in device memory and
// updated only by the epilogue of the streaming pass (and by the init/set
// kernels).  All floating-point members are binary64.
struct DevState {
  // parameters of the test
  double alpha;    // the guess of OPT
  double eta;      // SCMWU step size
  double kscale;   // SES: eta / (rho sqrt2); SVM: eta / rho  (kappa = kscale * t)
  double delta;    // stabilisation threshold
  double tau;      // relative tie tolerance of the separation test
  double D;        // problem bound D
  double gamma1;   // SES: radius of sphere v1
  int64_t T;       // iteration cap
  int64_t t;       // ORACLE outputs averaged so far
  int64_t t_end;   // iteration at which the test ended
  int64_t t_best;  // iteration of the best monitored mean
  int32_t status;  // Status
  int32_t cnt;     // consecutive stabilised iterations
  int32_t patience;
  int32_t early;   // Section 5 exits enabled
  int32_t degenerate;
  int32_t cert;    // a certificate was computed on the last pass
  int32_t pending; // records of a fused pass wait for their epilogue
  // monitor
  double f_prev;   // f of the previous monitored iteration (-1: none)
  double f_best;
  double f_last;
  // exponent bound for the next pass: SES an upper bound G on
  // max_{i != v1} ||v_i - ubar|| + gamma_i; SVM a lower bound on the slack
  double shift_bound;
  // last ORACLE
  double value, scale, log_trace;
  double bound;     // SES: best weight lower bound; SVM: best PD upper bound
  // SVM scalar parts of y = (w; s1; s2): running sums and means
  double S1, S2, s1bar, s2bar, s1_last, s2_last;
  double wbar_norm; // ||wbar|| of the current mean
};

// Device vectors of a test, each of length d (binary64):
//   vec + 0*d: S     running sum of ORACLE centres / normals
//   vec + 1*d: ybar  current mean (the pass's candidate)
//   vec + 2*d: best  mean that gave f_best
//   vec + 3*d: last  last ORACLE output
constexpr int kVecS = 0, kVecMean = 1, kVecBest = 2, kVecLast = 3, kNumVec = 4;

struct PassArgs {
  const void *X;          // row-major points (storage type)
  int64_t n, d, ld;
  const double *radii;    // SES radii or nullptr
  int64_t v1;             // SES easy-set row
  int64_t n_pos;          // SVM class boundary
  DevState *st;
  double *vec;            // kNumVec * d
  double *partials;       // gridDim.x * partial_width(d), 16-byte aligned
  const float *scales;    // FP8 storage: one binary32 scale per row; else nullptr
  double *gsum;           // unfused single-problem pass: add the workgroup sums
                          // into this one global sum (atomics) instead of
                          // writing records; nullptr: records
};

// Parameters of a new alpha-feasibility test (written by the init kernel).
struct InitParams {
  double alpha, eta, kscale, delta, tau, D, gamma1;
  int64_t T;
  int32_t patience, early;
};

// Host-side launchers (one translation unit per storage type).
struct LaunchCfg {
  int grid;
  int epl;     // columns per lane: 16 * epl >= d
  int vec;     // elements per vector load (1 = scalar loads)
  bool cert;   // SES weight certificate accumulators
  int pfm;     // Prefetch mode
};

// One workgroup's share of a batched pass: workgroup vb of the vg workgroups
// of instance inst.
struct BatchTile {
  int32_t inst, vb, vg, pad;
};

#define SCPMWU_DECLARE_BATCH(name)                                                                       \
  hipError_t launch_pass_batch_##name(int epl, int vec, int ntiles, const PassArgs *args,                \
                                      const BatchTile *tiles, hipStream_t s);                            \
  hipError_t launch_epilogue_batch_##name(int m, const PassArgs *args, const int32_t *nrec, hipStream_t s); \
  hipError_t launch_init_batch_##name(int count, const PassArgs *args, const int32_t *list,              \
                                      const InitParams *params, hipStream_t s);                          \
  hipError_t launch_diameter_batch_##name(int m, const PassArgs *args, double *D, hipStream_t s);         \
  hipError_t launch_rows_batch_##name(int dm, int vec, int ntiles, const PassArgs *args,                  \
                                      const BatchTile *tiles, hipStream_t s);                            \
  hipError_t launch_kway_batch_##name(int epl, int vec, int ks, int grid, const PassArgs *args, hipStream_t s);
SCPMWU_DECLARE_BATCH(f32)
SCPMWU_DECLARE_BATCH(bf16)
#undef SCPMWU_DECLARE_BATCH

hipError_t launch_read_reference(const void *buf, int64_t bytes, int grid, float *sink, hipStream_t s);
hipError_t launch_quantize_fp8(const float *src, int64_t n, int64_t d, int64_t ld, uint8_t *codes, float *scales,
                               hipStream_t s);

// Slots of a fused pass: state/vector/record slot `cur` is read and 1 - cur
// written (rec_stride doubles per record slot); with global sums the pass
// reads g_in, adds into g_out and clears g_zero (all nullptr: records).
struct FusedSlots {
  int cur;
  int64_t rec_stride;
  double *g_in, *g_out, *g_zero;
};

#define SCPMWU_DECLARE_TYPED(name)                                                              \
  hipError_t launch_pass_##name(int problem, const LaunchCfg &c, const PassArgs &a, hipStream_t s); \
  hipError_t launch_fused_##name(const LaunchCfg &c, const PassArgs &a, const FusedSlots &f, hipStream_t s); \
  hipError_t launch_flush_##name(bool cert, int P, bool gmode, const PassArgs &a, hipStream_t s);  \
  hipError_t launch_epilogue_##name(int problem, const LaunchCfg &c, const PassArgs &a, hipStream_t s); \
  hipError_t launch_monitor_##name(int grid, const PassArgs &a, const double *center,            \
                                   int64_t exclude, int mode, double *out, hipStream_t s);      \
  hipError_t launch_init_##name(const PassArgs &a, const InitParams &p, int problem, hipStream_t s);
SCPMWU_DECLARE_TYPED(f32)
SCPMWU_DECLARE_TYPED(bf16)
SCPMWU_DECLARE_TYPED(f64)
SCPMWU_DECLARE_TYPED(fp8)
#undef SCPMWU_DECLARE_TYPED
hipError_t launch_set_state_k(const PassArgs &a, int problem, int64_t t, double S1, double S2,
                              hipStream_t s);
hipError_t launch_cast(const float *src, uint16_t *dst, int64_t n, int64_t d, int64_t ld_src,
                       int64_t ld_dst, hipStream_t s);

}  // namespace scpmwu
