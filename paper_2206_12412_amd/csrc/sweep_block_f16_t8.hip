// The T-step sweep for F16S storage at eight steps per sweep.  Built with a
// raised limit on the unrolled size of loops marked for full unrolling: at
// the default limit the 24-row march of eight levels stays a loop whose ring
// buffers are indexed at run time (87 KB of code, 182 us per step on the
// 16384 x 8192 plate); unrolled it is 45 KB and takes 51 us.  The other
// step counts keep the default limit, under which they are faster (with the
// raised one T = 6 takes 66.8 instead of 58.2 us per step).
#include "sweep_block.hpp"

namespace lbmk {

hipError_t launch_sweep_block_f16_t8(const void *args, int rows, int waves, hipStream_t st,
                                     const SideStream &ss) {
  return blk::block_r<_Float16, float, float, 4, 8, 8>(args, rows, waves, st, ss);
}

}  // namespace lbmk
