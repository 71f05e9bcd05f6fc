// The T-step sweep for F16S storage (one translation unit per storage, so
// that the instantiations compile in parallel); eight steps per sweep in a
// unit of their own (sweep_block_f16_t8.hip).
#include "sweep_block.hpp"

namespace lbmk {

hipError_t launch_sweep_block_f16_t8(const void *args, int rows, int waves, hipStream_t st,
                                     const SideStream &ss);

hipError_t launch_sweep_block_f16(const void *args, int rows, int waves, hipStream_t st,
                                  const SideStream &ss) {
  if (static_cast<const BlockArgs<_Float16, float, float> *>(args)->steps == 8)
    return launch_sweep_block_f16_t8(args, rows, waves, st, ss);
  return blk::block_r<_Float16, float, float, 4, 2, 7>(args, rows, waves, st, ss);
}

}  // namespace lbmk
