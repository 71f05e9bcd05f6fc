// The T-step sweep for BF16S storage (one translation unit per storage, so
// that the instantiations compile in parallel).
#include "sweep_block.hpp"

namespace lbmk {

hipError_t launch_sweep_block_bf16(const void *args, int rows, int waves, hipStream_t st,
                                  const SideStream &ss) {
  return blk::block_r<__bf16, float, float, 4>(args, rows, waves, st, ss);
}

}  // namespace lbmk
