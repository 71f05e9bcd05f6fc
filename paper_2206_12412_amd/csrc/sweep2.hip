// Dispatch of the T-step sweep (sweep_block.hpp) to the translation unit of
// each storage.
#include "lbm_internal.hpp"

namespace lbmk {

hipError_t launch_sweep_block_f64(const void *args, int rows, int waves, hipStream_t st,
                                  const SideStream &ss);
hipError_t launch_sweep_block_f32(const void *args, int rows, int waves, hipStream_t st,
                                  const SideStream &ss);
hipError_t launch_sweep_block_f16(const void *args, int rows, int waves, hipStream_t st,
                                  const SideStream &ss);
hipError_t launch_sweep_block_bf16(const void *args, int rows, int waves, hipStream_t st,
                                   const SideStream &ss);

hipError_t launch_sweep_block(Store s, const void *args, int rows, int waves, hipStream_t st,
                              const SideStream &ss) {
  const bool rows_ok = rows == 4 || rows == 8 || rows == 16 || rows == 24 || rows == 32;
  if (!rows_ok || (waves != 1 && waves != 2 && waves != 4 && waves != 8)) return hipErrorInvalidValue;
  switch (s) {
    case Store::F64S: return launch_sweep_block_f64(args, rows, waves, st, ss);
    case Store::F32S: return launch_sweep_block_f32(args, rows, waves, st, ss);
    case Store::F16S: return launch_sweep_block_f16(args, rows, waves, st, ss);
    case Store::BF16S: return launch_sweep_block_bf16(args, rows, waves, st, ss);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lbmk
