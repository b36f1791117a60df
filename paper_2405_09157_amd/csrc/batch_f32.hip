// Batched SES kernels instantiated for float point storage.
#include "batch_kernels.hpp"

namespace scpmwu {

hipError_t launch_pass_batch_f32(int epl, int vec, int ntiles, const PassArgs *args, const BatchTile *tiles,
                                hipStream_t s) {
  return launch_pass_batch_typed<float>(epl, vec, ntiles, args, tiles, s);
}
hipError_t launch_epilogue_batch_f32(int m, const PassArgs *args, const int32_t *nrec, hipStream_t s) {
  return launch_epilogue_batch_typed<float>(m, args, nrec, s);
}
hipError_t launch_init_batch_f32(int count, const PassArgs *args, const int32_t *list, const InitParams *params,
                                hipStream_t s) {
  return launch_init_batch_typed<float>(count, args, list, params, s);
}
hipError_t launch_rows_batch_f32(int dm, int vec, int ntiles, const PassArgs *args, const BatchTile *tiles,
                               hipStream_t s) {
  return launch_rows_batch_typed<float>(dm, vec, ntiles, args, tiles, s);
}
hipError_t launch_diameter_batch_f32(int m, const PassArgs *args, double *D, hipStream_t s) {
  return launch_diameter_batch_typed<float>(m, args, D, s);
}

}  // namespace scpmwu
