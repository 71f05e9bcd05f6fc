// Single-plate sweep kernel and its launcher.  The interior strips (no
// bounce-back code) and the boundary rows (edge rows and crack rows) of a step
// run in one launch; both read the source buffers and write disjoint sites of
// the destination buffers.  The arithmetic lives in sweep_core.hpp.
#include "crack_core.hpp"
#include "sweep_core.hpp"

namespace lbmk {
namespace {

// One launch per step: the first `nbb` workgroups take the boundary rows (the
// two edge rows and the crack rows, full treatment), the rest the interior
// strips.  The two parts write disjoint sites, so they run side by side; one
// launch saves the dispatch gap of a second kernel (measured 0.5 % of a step
// on 134M sites, 10 % on 2M sites).  The kernel's register count is the
// larger of the two parts'; the occupancy cap (reserved LDS) binds first.
//
// With fc set the boundary part also runs the crack step of the previous step
// (Alg. 1 appends it to that step): one wave after the boundary rows executes
// it on the source w, and the waves of the two crack rows take the columns it
// severs from the same decision, evaluated on the same state and field, so
// that this step's bounce-back follows the crack as it is after that crack
// step.  The crack wave writes the new cut bits (the ones the forecast adds)
// and the state after the step into the other slot; everything else it
// writes (traces, events) no other wave reads.  This saves the launch of a
// separate crack kernel between two sweeps.  The crack step's arguments come
// through a device pointer and are read by the crack-row waves only (as
// kernel arguments the entry block would load and keep them in every wave);
// the instance with that code (FUSED) runs only when a crack step is folded
// in, and its equilibrium-layout forms keep the occupancy of the plain ones.
template <typename S, typename W, typename C, int VEC, bool SHIFT, bool SR, bool EQ, bool FUSED>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu((FUSED && EQ) ? 8 : 1)))
sweep_step(const S *__restrict__ fin, S *__restrict__ fout, const W *__restrict__ win,
           W *__restrict__ wout, const uint32_t *mV, const uint32_t *__restrict__ mH,
           const MaskRows *mrows, const SweepArgs<S, W, C> a, const core::InteriorMap m,
           const core::BoundaryMap bm, const unsigned nbb, const CrackArgs *fc) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (blockIdx.x < nbb) {
    const int task = blockIdx.x * a.waves + wave;
    const int nbt = bm.n_strips * bm.nb;
    if (task >= nbt) {
      if constexpr (FUSED) {
        if (task == nbt) core::crack_step_wave<false>(*fc);
      }
      return;
    }
    const int j = core::boundary_row_of(bm, task / bm.n_strips);
    core::CutForecast cf;
    if (FUSED && (j == a.p.j0 || j == a.p.j0 + 1) && fc->c.crack) {
      cf.row = a.p.j0;
      core::crack_cut_columns(*fc, *fc->st, threadIdx.x & 63, &cf.lo_r, &cf.hi_r, &cf.lo_l,
                              &cf.hi_l);
    }
    core::boundary_row<S, W, C, VEC, SHIFT, SR, EQ>(fin, fout, win, wout, mV, mH, mrows, a,
                                                    task % bm.n_strips, j, cf);
    return;
  }
  const int task = (blockIdx.x - nbb) * a.waves + wave;
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
  if (jb > jlast) return;  // the tail of the last workgroup
  core::interior_rows<S, W, C, VEC, SHIFT, SR, EQ>(fin, fout, win, wout, a, strip, jb, jlast);
}

template <typename S, typename W, typename C, int VEC, bool SHIFT, bool SR, bool EQ>
hipError_t launch_t(const SweepArgs<S, W, C> &a, hipStream_t st, const CrackArgs *fc) {
  const core::InteriorMap m = core::interior_map(a.p.nx, a.p.ny, VEC, a.rows, a.skip_lo, a.skip_hi);
  const core::BoundaryMap bm = core::boundary_map(a.p.nx, a.p.ny, VEC, a.skip_lo, a.skip_hi);
  const long itasks = core::interior_task_count(m);
  const long btasks = core::boundary_task_count(bm) + (fc ? 1 : 0);
  const unsigned nbb = (unsigned)((btasks + a.waves - 1) / a.waves);
  const unsigned nib = (unsigned)((itasks + a.waves - 1) / a.waves);
  if (nbb + nib == 0) return hipSuccess;
  if (fc)
    hipLaunchKernelGGL((sweep_step<S, W, C, VEC, SHIFT, SR, EQ, true>), dim3(nbb + nib),
                       dim3(64 * a.waves), a.lds_bytes, st, a.fin, a.fout, a.win, a.wout, a.mV, a.mH,
                       a.mrows, a, m, bm, nbb, fc);
  else
    hipLaunchKernelGGL((sweep_step<S, W, C, VEC, SHIFT, SR, EQ, false>), dim3(nbb + nib),
                       dim3(64 * a.waves), a.lds_bytes, st, a.fin, a.fout, a.win, a.wout, a.mV, a.mH,
                       a.mrows, a, m, bm, nbb, fc);
  return hipGetLastError();
}

// stochastic rounding exists for the 16-bit storages only, the equilibrium
// layout for the shifted ones only
template <typename S, typename W, typename C, int VEC, bool SHIFT>
hipError_t launch_r(const void *args, bool eq, hipStream_t st, const CrackArgs *fc) {
  const auto &a = *static_cast<const SweepArgs<S, W, C> *>(args);
  if constexpr (SHIFT) {
    if (eq) {
      if constexpr (sizeof(S) == 2) {
        if (a.sr) return launch_t<S, W, C, VEC, SHIFT, true, true>(a, st, fc);
      }
      return launch_t<S, W, C, VEC, SHIFT, false, true>(a, st, fc);
    }
  } else {
    if (eq) return hipErrorInvalidValue;
  }
  if constexpr (sizeof(S) == 2) {
    if (a.sr) return launch_t<S, W, C, VEC, SHIFT, true, false>(a, st, fc);
  }
  return launch_t<S, W, C, VEC, SHIFT, false, false>(a, st, fc);
}

// The store conversion of the sweep applied to an array: element i is the
// value x[i] stored at site (i, 0) of plane `plane` of a plate n sites wide.
template <typename S>
__global__ void round16_kernel(const float *__restrict__ x, S *__restrict__ out, int64_t n,
                               int plane, uint32_t rkey, int sr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (sr) {
    uint32_t h = mix32(core::sr_pair(0u, (uint32_t)i, (uint32_t)n) ^ rkey);
    for (int a = 1; a <= plane; ++a) h = mix32(h ^ core::kPlaneSalt);
    out[i] = core::round_sr<S>(x[i], core::sr_half(h, (uint32_t)i & 1u));
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

int sweep_vec(Store s) {
  switch (s) {
    case Store::F64: return 2;
    case Store::F64S: return 2;
    case Store::F32_PLAIN: return 4;
    case Store::F32S: return 4;
    case Store::F16S: return 4;
    case Store::BF16S: return 4;
  }
  return 0;
}

hipError_t launch_sweep(Store s, bool eq, const void *args, hipStream_t st, const CrackArgs *fc) {
  switch (s) {
    case Store::F64: return launch_r<double, double, double, 2, false>(args, eq, st, fc);
    // shifted FP64 exists only in the equilibrium layout
    case Store::F64S:
      return eq ? launch_t<double, double, double, 2, true, false, true>(
                      *static_cast<const SweepArgs<double, double, double> *>(args), st, fc)
                : hipErrorInvalidValue;
    case Store::F32_PLAIN: return launch_r<float, float, float, 4, false>(args, eq, st, fc);
    case Store::F32S: return launch_r<float, float, float, 4, true>(args, eq, st, fc);
    case Store::F16S: return launch_r<_Float16, float, float, 4, true>(args, eq, st, fc);
    case Store::BF16S: return launch_r<__bf16, float, float, 4, true>(args, eq, st, fc);
  }
  return hipErrorInvalidValue;
}

}  // namespace lbmk
