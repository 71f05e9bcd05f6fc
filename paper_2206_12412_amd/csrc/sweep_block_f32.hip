// The T-step sweep for F32S storage (one translation unit per storage, so
// that the instantiations compile in parallel).
#include "sweep_block.hpp"

namespace lbmk {

hipError_t launch_sweep_block_f32(const void *args, int rows, int waves, hipStream_t st,
                                  const SideStream &ss) {
  return blk::block_r<float, float, float, 4>(args, rows, waves, st, ss);
}

}  // namespace lbmk
