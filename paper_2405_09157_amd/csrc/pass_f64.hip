// Streaming-pass kernels instantiated for double point storage.
#include "mwu_kernels.hpp"

namespace scpmwu {

hipError_t launch_pass_f64(int problem, const LaunchCfg &c, const PassArgs &a, hipStream_t s) {
  return launch_pass_typed<double>(problem, c, a, s);
}
hipError_t launch_fused_f64(const LaunchCfg &c, const PassArgs &a, const FusedSlots &f, hipStream_t s) {
  return launch_fused_typed<double>(c, a, f, s);
}
hipError_t launch_flush_f64(bool cert, int P, bool gmode, const PassArgs &a, hipStream_t s) {
  return launch_flush_typed<double>(cert, P, gmode, a, s);
}
hipError_t launch_epilogue_f64(int problem, const LaunchCfg &c, const PassArgs &a, hipStream_t s) {
  return launch_epilogue_typed<double>(problem, c.cert, c.grid, a, s);
}
hipError_t launch_monitor_f64(int grid, const PassArgs &a, const double *center, int64_t exclude,
                               int mode, double *out, hipStream_t s) {
  return launch_monitor_typed<double>(grid, a, center, exclude, mode, out, s);
}
hipError_t launch_init_f64(const PassArgs &a, const InitParams &p, int problem, hipStream_t s) {
  return launch_init_typed<double>(a, p, problem, s);
}

}  // namespace scpmwu
