// Streaming-pass kernels instantiated for uint16_t point storage.
#include "mwu_kernels.hpp"

namespace scpmwu {

hipError_t launch_pass_bf16(int problem, const LaunchCfg &c, const PassArgs &a, hipStream_t s) {
  return launch_pass_typed<uint16_t>(problem, c, a, s);
}
hipError_t launch_fused_bf16(const LaunchCfg &c, const PassArgs &a, const FusedSlots &f, hipStream_t s) {
  return launch_fused_typed<uint16_t>(c, a, f, s);
}
hipError_t launch_flush_bf16(bool cert, int P, bool gmode, const PassArgs &a, hipStream_t s) {
  return launch_flush_typed<uint16_t>(cert, P, gmode, a, s);
}
hipError_t launch_epilogue_bf16(int problem, const LaunchCfg &c, const PassArgs &a, hipStream_t s) {
  return launch_epilogue_typed<uint16_t>(problem, c.cert, c.grid, a, s);
}
hipError_t launch_monitor_bf16(int grid, const PassArgs &a, const double *center, int64_t exclude,
                               int mode, double *out, hipStream_t s) {
  return launch_monitor_typed<uint16_t>(grid, a, center, exclude, mode, out, s);
}
hipError_t launch_init_bf16(const PassArgs &a, const InitParams &p, int problem, hipStream_t s) {
  return launch_init_typed<uint16_t>(a, p, problem, s);
}

}  // namespace scpmwu
