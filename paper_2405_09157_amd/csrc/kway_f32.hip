// The k-way search's shared-read pass instantiated for float point storage
// (its own unit so that it compiles beside the other kernels).
#include "batch_kernels.hpp"

namespace scpmwu {

hipError_t launch_kway_batch_f32(int epl, int vec, int ks, int grid, const PassArgs *args, hipStream_t s) {
  return launch_kway_batch_typed<float>(epl, vec, ks, grid, args, s);
}

}  // namespace scpmwu
