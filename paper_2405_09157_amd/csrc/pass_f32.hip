// Streaming-pass kernels instantiated for float point storage.
#include "mwu_kernels.hpp"

namespace scpmwu {

hipError_t launch_pass_f32(int problem, const LaunchCfg &c, const PassArgs &a, hipStream_t s) {
  return launch_pass_typed<float>(problem, c, a, s);
}
hipError_t launch_fused_f32(const LaunchCfg &c, const PassArgs &a, const FusedSlots &f, hipStream_t s) {
  return launch_fused_typed<float>(c, a, f, s);
}
hipError_t launch_flush_f32(bool cert, int P, bool gmode, const PassArgs &a, hipStream_t s) {
  return launch_flush_typed<float>(cert, P, gmode, a, s);
}
hipError_t launch_epilogue_f32(int problem, const LaunchCfg &c, const PassArgs &a, hipStream_t s) {
  return launch_epilogue_typed<float>(problem, c.cert, c.grid, a, s);
}
hipError_t launch_monitor_f32(int grid, const PassArgs &a, const double *center, int64_t exclude,
                               int mode, double *out, hipStream_t s) {
  return launch_monitor_typed<float>(grid, a, center, exclude, mode, out, s);
}
hipError_t launch_init_f32(const PassArgs &a, const InitParams &p, int problem, hipStream_t s) {
  return launch_init_typed<float>(a, p, problem, s);
}

}  // namespace scpmwu
