// Single-plate sweep kernels and their launchers.  A step launches the
// interior kernel (interior rows, no bounce-back code) and the boundary-row
// kernel (edge rows and crack rows); both read the source buffers and write
// disjoint sites of the destination buffers.  The arithmetic lives in
// sweep_core.hpp.
#include "sweep_core.hpp"

namespace lbmk {
namespace {

template <typename S, typename W, typename C, int VEC, bool SHIFT>
__global__ void __launch_bounds__(512)
sweep_interior(const S *__restrict__ fin, S *__restrict__ fout, const W *__restrict__ win,
               W *__restrict__ wout, const SweepArgs<S, W, C> a, const core::InteriorMap m) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int task = blockIdx.x * a.waves + wave;
  const int strip = task % m.n_strips;
  const int chunk = task / m.n_strips;
  int jb, jlast;
  if (chunk < m.nc1) {
    jb = m.lo1 + chunk * m.rows;
    jlast = min(jb + m.rows - 1, m.hi1);
  } else {
    jb = m.lo2 + (chunk - m.nc1) * m.rows;
    jlast = min(jb + m.rows - 1, m.hi2);
  }
  if (jb > jlast) return;
  core::interior_rows<S, W, C, VEC, SHIFT>(fin, fout, win, wout, a, strip, jb, jlast);
}

template <typename S, typename W, typename C, int VEC, bool SHIFT>
__global__ void __launch_bounds__(256)
sweep_boundary(const S *__restrict__ fin, S *__restrict__ fout, const W *__restrict__ win,
               W *__restrict__ wout, const uint32_t *__restrict__ mV,
               const uint32_t *__restrict__ mH, const MaskRows *__restrict__ mrows,
               const SweepArgs<S, W, C> a, const core::BoundaryMap m) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int task = blockIdx.x * 4 + wave;
  if (task >= m.n_strips * m.nb) return;
  const int strip = task % m.n_strips;
  const int j = m.brow[task / m.n_strips];
  core::boundary_row<S, W, C, VEC, SHIFT>(fin, fout, win, wout, mV, mH, mrows, a, strip, j);
}

template <typename S, typename W, typename C, int VEC, bool SHIFT>
hipError_t launch_t(const void *args, int part, hipStream_t st) {
  const auto &a = *static_cast<const SweepArgs<S, W, C> *>(args);
  if (part == 0) {
    const core::InteriorMap m = core::interior_map(a.p.nx, a.p.ny, VEC, a.rows, a.skip_lo, a.skip_hi);
    const long tasks = core::interior_task_count(m);
    if (tasks > 0) {
      const unsigned blocks = (unsigned)((tasks + a.waves - 1) / a.waves);
      hipLaunchKernelGGL((sweep_interior<S, W, C, VEC, SHIFT>), dim3(blocks), dim3(64 * a.waves),
                         a.lds_bytes, st, a.fin, a.fout, a.win, a.wout, a, m);
    }
  } else {
    const core::BoundaryMap m = core::boundary_map(a.p.nx, a.p.ny, VEC, a.skip_lo, a.skip_hi);
    const long tasks = core::boundary_task_count(m);
    if (tasks > 0) {
      const unsigned blocks = (unsigned)((tasks + 3) / 4);
      hipLaunchKernelGGL((sweep_boundary<S, W, C, VEC, SHIFT>), dim3(blocks), dim3(256), 0, st,
                         a.fin, a.fout, a.win, a.wout, a.mV, a.mH, a.mrows, a, m);
    }
  }
  return hipGetLastError();
}

}  // namespace

int64_t interior_sites(const Plate &p, int skip_lo, int skip_hi) {
  int rows = p.ny - 2;
  for (int j = skip_lo; j <= skip_hi; ++j)
    if (j >= 1 && j <= p.ny - 2) --rows;
  return rows > 0 ? (int64_t)rows * p.nx : 0;
}

int sweep_vec(Store s) {
  switch (s) {
    case Store::F64: return 2;
    case Store::F32_PLAIN: return 4;
    case Store::F32S: return 4;
    case Store::F16S: return 4;
    case Store::BF16S: return 4;
  }
  return 0;
}

hipError_t launch_sweep(Store s, const void *args, int part, hipStream_t st) {
  switch (s) {
    case Store::F64: return launch_t<double, double, double, 2, false>(args, part, st);
    case Store::F32_PLAIN: return launch_t<float, float, float, 4, false>(args, part, st);
    case Store::F32S: return launch_t<float, float, float, 4, true>(args, part, st);
    case Store::F16S: return launch_t<_Float16, float, float, 4, true>(args, part, st);
    case Store::BF16S: return launch_t<__bf16, float, float, 4, true>(args, part, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace lbmk
