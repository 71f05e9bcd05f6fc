// Single-plate sweep kernels and their launchers.  A step launches the
// interior kernel (interior rows, no bounce-back code) and the boundary-row
// kernel (edge rows and crack rows); both read the source buffers and write
// disjoint sites of the destination buffers.  The arithmetic lives in
// sweep_core.hpp.
#include "sweep_core.hpp"

namespace lbmk {
namespace {

template <typename S, typename W, typename C, int VEC, bool SHIFT, bool SR>
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
  core::interior_rows<S, W, C, VEC, SHIFT, SR>(fin, fout, win, wout, a, strip, jb, jlast);
}

template <typename S, typename W, typename C, int VEC, bool SHIFT, bool SR>
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
  core::boundary_row<S, W, C, VEC, SHIFT, SR>(fin, fout, win, wout, mV, mH, mrows, a, strip, j);
}

template <typename S, typename W, typename C, int VEC, bool SHIFT, bool SR>
hipError_t launch_t(const SweepArgs<S, W, C> &a, int part, hipStream_t st) {
  if (part == 0) {
    const core::InteriorMap m = core::interior_map(a.p.nx, a.p.ny, VEC, a.rows, a.skip_lo, a.skip_hi);
    const long tasks = core::interior_task_count(m);
    if (tasks > 0) {
      const unsigned blocks = (unsigned)((tasks + a.waves - 1) / a.waves);
      hipLaunchKernelGGL((sweep_interior<S, W, C, VEC, SHIFT, SR>), dim3(blocks), dim3(64 * a.waves),
                         a.lds_bytes, st, a.fin, a.fout, a.win, a.wout, a, m);
    }
  } else {
    const core::BoundaryMap m = core::boundary_map(a.p.nx, a.p.ny, VEC, a.skip_lo, a.skip_hi);
    const long tasks = core::boundary_task_count(m);
    if (tasks > 0) {
      const unsigned blocks = (unsigned)((tasks + 3) / 4);
      hipLaunchKernelGGL((sweep_boundary<S, W, C, VEC, SHIFT, SR>), dim3(blocks), dim3(256), 0, st,
                         a.fin, a.fout, a.win, a.wout, a.mV, a.mH, a.mrows, a, m);
    }
  }
  return hipGetLastError();
}

// stochastic rounding exists for the 16-bit storages only
template <typename S, typename W, typename C, int VEC, bool SHIFT>
hipError_t launch_r(const void *args, int part, hipStream_t st) {
  const auto &a = *static_cast<const SweepArgs<S, W, C> *>(args);
  if constexpr (sizeof(S) == 2) {
    if (a.sr) return launch_t<S, W, C, VEC, SHIFT, true>(a, part, st);
  }
  return launch_t<S, W, C, VEC, SHIFT, false>(a, part, st);
}

// The store conversion of the sweep applied to an array: element i is the
// value x[i] stored at plate-local site i of plane `plane`.
template <typename S>
__global__ void round16_kernel(const float *__restrict__ x, S *__restrict__ out, int64_t n,
                               int plane, uint32_t rkey, int sr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (sr) {
    uint32_t r[5];
    core::sr_draws((uint32_t)i, rkey, r);
    out[i] = core::round_sr<S>(x[i], r[plane]);
  } else {
    out[i] = static_cast<S>(x[i]);
  }
}

}  // namespace

hipError_t launch_round16(Store s, int sr, const float *x, void *out, int64_t n, int plane,
                          uint32_t rkey, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (s == Store::F16S)
    hipLaunchKernelGGL(round16_kernel<_Float16>, dim3(blocks), dim3(256), 0, st, x,
                       static_cast<_Float16 *>(out), n, plane, rkey, sr);
  else if (s == Store::BF16S)
    hipLaunchKernelGGL(round16_kernel<__bf16>, dim3(blocks), dim3(256), 0, st, x,
                       static_cast<__bf16 *>(out), n, plane, rkey, sr);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

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
    case Store::F64: return launch_r<double, double, double, 2, false>(args, part, st);
    case Store::F32_PLAIN: return launch_r<float, float, float, 4, false>(args, part, st);
    case Store::F32S: return launch_r<float, float, float, 4, true>(args, part, st);
    case Store::F16S: return launch_r<_Float16, float, float, 4, true>(args, part, st);
    case Store::BF16S: return launch_r<__bf16, float, float, 4, true>(args, part, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace lbmk
