// Batched plates: many independent plates of uneven sizes, loads and crack
// rules stepped together.  Each plate keeps its own state block and its own
// task map; a global task index runs over the interior tasks of all plates,
// then over their boundary tasks, and the plate of a task is found by a
// binary search over the plates' first task indices.  Per-site arithmetic is
// the single-plate code (sweep_core.hpp, crack_core.hpp), so a plate of a
// batch evolves bit for bit as it does alone.
//
// Two ways to run a step:
//   per-step launches: one batched sweep kernel (boundary and interior tasks
//     of all plates) and one batched crack kernel (one wavefront per plate),
//     or, when every plate's crack runs along +x, the crack step of step n
//     folded into the sweep of step n + 1 and one crack launch at the end;
//   persistent: one cooperative launch runs many steps; every wave walks the
//     task list with a grid stride, and two grid barriers per step separate
//     the sweep from the crack step and the crack step from the next sweep.
//     The barrier spins on a generation counter with a bounded number of
//     tries: on time-out it raises an error flag, after which no barrier
//     waits, so every wave always reaches the end of the kernel.
#include <mutex>

#include "crack_core.hpp"
#include "sweep_core.hpp"

namespace lbmk {

// Fixed device scratch for callers that cannot allocate: the synchronisation
// words of lbm_batch_run_persistent_static live here instead of in the
// batch's device block.  Each GPU holds its own copy of the array from the
// moment the library's code object is loaded on it until the process ends.
// In host code `scratch` names a host-side stand-in, not a device address:
// only the address that static_scratch() looks up may be passed to kernels
// or copies.
constexpr size_t kStaticScratchBytes = 64 * 1024;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

hipError_t static_scratch(void **ptr, size_t *bytes) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void *addr[kMaxDevices] = {};
  *ptr = nullptr;
  *bytes = 0;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {  // once per device, with that device current
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  *bytes = kStaticScratchBytes;
  return hipSuccess;
}

size_t persistent_sync_bytes(int n_plates) {
  (void)n_plates;
  return 512;  // counter, generation and time-out flag on their own 128-byte lines
}

namespace {

__device__ __forceinline__ int plate_of(const BatchPlate *__restrict__ d, int n, int64_t task,
                                        bool interior) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {  // last plate whose first task is <= task
    const int mid = (lo + hi + 1) >> 1;
    const int64_t first = interior ? d[mid].itask0 : d[mid].btask0;
    if (first <= task) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename S, typename W, typename C>
__device__ __forceinline__ SweepArgs<S, W, C> args_of(const BatchPlate &d, int cur, int64_t step) {
  SweepArgs<S, W, C> a;
  a.fin = static_cast<const S *>(d.f[cur]);
  a.fout = static_cast<S *>(const_cast<void *>(d.f[1 - cur]));
  a.win = static_cast<const W *>(d.w[cur]);
  a.wout = static_cast<W *>(const_cast<void *>(d.w[1 - cur]));
  a.mV = d.mV;
  a.mH = d.mH;
  a.mrows = d.mrows;
  a.p = d.p;
  a.omega = (C)d.omega;
  a.dt = (C)d.dt;
  a.A0 = (C)d.A0;
  a.Ak = (C)d.Ak;
  const double tau = d.n_hist > 0 ? d.tau[step < d.n_hist ? step : d.n_hist - 1] : 0.0;
  a.t_top = d.p.periodic ? C(0) : (C)(d.coef * tau);
  a.t_bot = d.p.periodic ? C(0) : (C)(d.coef * -tau);
  a.t_up = d.p.periodic ? C(0) : (C)(d.coef * d.face);
  a.t_lo = d.p.periodic ? C(0) : (C)(d.coef * -d.face);
  a.rows = d.im.rows;
  a.waves = 4;
  a.lds_bytes = 0;
  a.skip_lo = d.skip_lo;
  a.skip_hi = d.skip_hi;
  a.sr = 0;  // the kernel's SR template argument decides
  a.rkey = step_key(d.seed, step);
  a.dmask = d.dmask;
  if (d.dmask) {
    const double *r = d.wD + 4 * (step < d.n_wD ? step : d.n_wD - 1);
    a.wD_bot = (C)r[0];
    a.wD_top = (C)r[1];
    a.wD_left = (C)r[2];
    a.wD_right = (C)r[3];
  } else {
    a.wD_bot = a.wD_top = a.wD_left = a.wD_right = C(0);
  }
  return a;
}

template <typename S, typename W, typename C, int VEC, bool SHIFT, bool SR, bool EQ>
__device__ __forceinline__ void interior_task(const BatchPlate *__restrict__ d, int n, int64_t task,
                                              int cur, int64_t step) {
  const int k = plate_of(d, n, task, true);
  const BatchPlate &q = d[k];
  const int64_t local = task - q.itask0;
  const core::InteriorMap &m = q.im;
  const int strip = (int)(local % m.n_strips);
  const int chunk = (int)(local / m.n_strips);
  int jb, jlast;
  if (chunk < m.nc1) {
    jb = m.lo1 + chunk * m.rows;
    jlast = min(jb + m.rows - 1, m.hi1);
  } else {
    jb = m.lo2 + (chunk - m.nc1) * m.rows;
    jlast = min(jb + m.rows - 1, m.hi2);
  }
  if (jb > jlast) return;
  const SweepArgs<S, W, C> a = args_of<S, W, C>(q, cur, step);
  core::interior_rows<S, W, C, VEC, SHIFT, SR, EQ>(a.fin, a.fout, a.win, a.wout, a, strip, jb, jlast);
}

// crack state slot k of plate q
__device__ __forceinline__ DevCrack *crack_slot(const BatchPlate &q, int k) {
  return k ? q.st2 : q.crack.st;
}

template <typename S, typename W, typename C, int VEC, bool SHIFT, bool SR, bool EQ, bool FUSED>
__device__ __forceinline__ void boundary_task(const BatchPlate *__restrict__ d, int n, int64_t task,
                                              int cur, int64_t step, int slot) {
  const int k = plate_of(d, n, task, false);
  const BatchPlate &q = d[k];
  const int64_t local = task - q.btask0;
  const int strip = (int)(local % q.bm.n_strips);
  const int r = (int)(local / q.bm.n_strips);
  const int j = core::boundary_row_of(q.bm, r);
  const SweepArgs<S, W, C> a = args_of<S, W, C>(q, cur, step);
  core::CutForecast cf;
  if (FUSED && (j == q.p.j0 || j == q.p.j0 + 1) && q.crack.c.crack) {
    // the links the folded crack step severs (it runs on the source w)
    const CrackArgs &fc = *q.fargs[2 * cur + slot];
    cf.row = q.p.j0;
    core::crack_cut_columns(fc, *fc.st, threadIdx.x & 63, &cf.lo_r, &cf.hi_r, &cf.lo_l, &cf.hi_l);
  }
  core::boundary_row<S, W, C, VEC, SHIFT, SR, EQ>(a.fin, a.fout, a.win, a.wout, a.mV, a.mH, a.mrows, a,
                                                  strip, j, cf);
}

// The crack step of plate k on w buffer wbuf, from the state in slot `in`
// into slot `out`.
__device__ __forceinline__ void crack_task(const BatchPlate *__restrict__ d, int k, int wbuf, int in,
                                           int out) {
  if (!d[k].has_crack && d[k].crack.n_sens == 0) return;
  CrackArgs c = d[k].crack;
  c.w = d[k].w[wbuf];
  c.st = crack_slot(d[k], in);
  c.st_out = out == in ? nullptr : crack_slot(d[k], out);
  core::crack_step_wave(c);
}

// One launch per step for the sweep of every plate: the first `nbb`
// workgroups take the boundary tasks, the rest the interior tasks.  FUSED:
// after the boundary tasks one wave per plate runs the crack step of the
// previous step (on the source w, state slot `slot` into the other slot),
// and the crack-row tasks forecast the links it severs, as the single-plate
// sweep does; its equilibrium-layout forms keep the occupancy of the plain
// ones (eight waves per SIMD).
template <typename S, typename W, typename C, int VEC, bool SHIFT, bool SR, bool EQ, bool FUSED>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu((FUSED && EQ) ? 8 : 1)))
batch_step(const BatchPlate *__restrict__ d, int n, int64_t n_int, int64_t n_bnd, unsigned nbb,
           int cur, int64_t step, int waves, int slot) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (blockIdx.x < nbb) {
    const int64_t task = (int64_t)blockIdx.x * waves + wave;
    if (task < n_bnd) {
      boundary_task<S, W, C, VEC, SHIFT, SR, EQ, FUSED>(d, n, task, cur, step, slot);
    } else if constexpr (FUSED) {
      if (task < n_bnd + n) {  // a crack along +x, or none
        const BatchPlate &q = d[task - n_bnd];
        if (q.has_crack || q.crack.n_sens > 0) core::crack_step_wave<false>(*q.fargs[2 * cur + slot]);
      }
    }
    return;
  }
  const int64_t task = (int64_t)(blockIdx.x - nbb) * waves + wave;
  if (task >= n_int) return;
  interior_task<S, W, C, VEC, SHIFT, SR, EQ>(d, n, task, cur, step);
}

__global__ void __launch_bounds__(256) batch_crack(const BatchPlate *__restrict__ d, int n, int wbuf,
                                                   int slot) {
  const int k = (int)(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (k >= n) return;
  crack_task(d, k, wbuf, slot, 0);
}

// Grid-wide barrier on three words, each on its own 128-byte line so that the
// pollers of the generation do not queue the arrivals' atomics behind them:
// sync[kCount] counts arrivals, sync[kGen] is the generation, sync[kErr] the
// time-out flag.
constexpr int kCount = 0, kGen = 32, kErr = 64;

__device__ __forceinline__ void grid_barrier(unsigned *sync, unsigned nblocks) {
  __syncthreads();
  if (threadIdx.x == 0) {
    if (__hip_atomic_load(&sync[kErr], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
      const unsigned gen = __hip_atomic_load(&sync[kGen], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
      __threadfence();
      const unsigned arrived = atomicAdd(&sync[kCount], 1u);
      if (arrived == nblocks - 1) {
        __hip_atomic_store(&sync[kCount], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&sync[kGen], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        unsigned tries = 0;
        while (__hip_atomic_load(&sync[kGen], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
          __builtin_amdgcn_s_sleep(4);
          ++tries;
          // bounded wait (~1 s): on time-out raise the flag; every later
          // barrier then falls through, so all waves reach the kernel's end
          if ((tries & 63u) == 0u &&
              (tries > (1u << 23) ||
               __hip_atomic_load(&sync[kErr], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u)) {
            atomicExch(&sync[kErr], 1u);
            break;
          }
        }
      }
      __threadfence();
    }
  }
  __syncthreads();
}

// Workgroups of the persistent kernel: WPB waves each, one workgroup per CU,
// because every grid barrier costs one agent-scope release / acquire (L2
// write-back and invalidation across the XCDs) per workgroup.
template <typename S, typename W, typename C, int VEC, bool SHIFT, bool SR, bool EQ, int WPB>
__global__ void __launch_bounds__(64 * WPB)
batch_persistent(const BatchPlate *__restrict__ d, int n, int64_t n_int, int64_t n_bnd, int cur0,
                 int64_t step0, int64_t nsteps, unsigned *sync) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t gw = (int64_t)blockIdx.x * WPB + wave;
  const int64_t nw = (int64_t)gridDim.x * WPB;
  for (int64_t s = 0; s < nsteps; ++s) {
    const int cur = (int)((cur0 + s) & 1);
    const int64_t step = step0 + s;
    for (int64_t t = gw; t < n_int + n_bnd; t += nw) {
      if (t < n_int) interior_task<S, W, C, VEC, SHIFT, SR, EQ>(d, n, t, cur, step);
      else boundary_task<S, W, C, VEC, SHIFT, SR, EQ, false>(d, n, t - n_int, cur, step, 0);
    }
    grid_barrier(sync, gridDim.x);
    for (int64_t k = gw; k < n; k += nw) crack_task(d, (int)k, 1 - cur, 0, 0);
    grid_barrier(sync, gridDim.x);
  }
}

template <typename S, typename W, typename C, int VEC, bool SHIFT, bool SR, bool EQ>
hipError_t step_t(const BatchPlate *d, int n, int64_t n_int, int64_t n_bnd, int cur, int64_t step,
                  int waves, int lds, int slot, hipStream_t st) {
  const int64_t btasks = n_bnd + (slot >= 0 ? n : 0);
  const unsigned nbb = (unsigned)((btasks + waves - 1) / waves);
  const unsigned nib = (unsigned)((n_int + waves - 1) / waves);
  if (nbb + nib == 0) return hipSuccess;
  if (slot >= 0)
    hipLaunchKernelGGL((batch_step<S, W, C, VEC, SHIFT, SR, EQ, true>), dim3(nbb + nib),
                       dim3(64 * waves), lds, st, d, n, n_int, n_bnd, nbb, cur, step, waves, slot);
  else
    hipLaunchKernelGGL((batch_step<S, W, C, VEC, SHIFT, SR, EQ, false>), dim3(nbb + nib),
                       dim3(64 * waves), lds, st, d, n, n_int, n_bnd, nbb, cur, step, waves, 0);
  return hipGetLastError();
}

template <typename S, typename W, typename C, int VEC, bool SHIFT, bool SR, bool EQ, int WPB>
hipError_t persistent_w(const BatchPlate *d, int n, int64_t n_int, int64_t n_bnd, int cur,
                        int64_t step, int64_t nsteps, unsigned *sync, int *blocks_used,
                        hipStream_t st) {
  auto kernel = batch_persistent<S, W, C, VEC, SHIFT, SR, EQ, WPB>;
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(kernel),
                                                   64 * WPB, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorCooperativeLaunchTooLarge;
  const int64_t want = (n_int + n_bnd + WPB - 1) / WPB;
  int blocks = cus;  // one workgroup per CU
  if (want < blocks) blocks = (int)(want > 0 ? want : 1);
  *blocks_used = blocks;
  void *args[] = {(void *)&d, (void *)&n, (void *)&n_int, (void *)&n_bnd, (void *)&cur,
                  (void *)&step, (void *)&nsteps, (void *)&sync};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(kernel), dim3(blocks),
                                    dim3(64 * WPB), args, 0, st);
}

template <typename S, typename W, typename C, int VEC, bool SHIFT, bool SR, bool EQ>
hipError_t persistent_t(const BatchPlate *d, int n, int64_t n_int, int64_t n_bnd, int cur,
                        int64_t step, int64_t nsteps, unsigned *sync, int *blocks_used,
                        hipStream_t st) {
  // one workgroup per CU (more workgroups pay for more barrier releases /
  // acquires), of 16 waves in the equilibrium layout and 8 with five planes:
  // measured on MI355X for the 64-plate FP32 batch against 4, 8 and 16 waves
  // (equilibrium layout 114 / 183 / 256 GLUPS, five planes 84 / 103 / 87)
  constexpr int kWaves = EQ ? 16 : 8;
  return persistent_w<S, W, C, VEC, SHIFT, SR, EQ, kWaves>(d, n, n_int, n_bnd, cur, step, nsteps,
                                                           sync, blocks_used, st);
}

// stochastic rounding exists for the 16-bit storages only, the equilibrium
// layout (eq) for the shifted storages only
template <typename S, typename W, typename C, int VEC, bool SHIFT, bool EQ>
hipError_t step_e(int sr, const BatchPlate *d, int n, int64_t n_int, int64_t n_bnd, int cur,
                  int64_t step, int waves, int lds, int slot, hipStream_t st) {
  if constexpr (sizeof(S) == 2) {
    if (sr) return step_t<S, W, C, VEC, SHIFT, true, EQ>(d, n, n_int, n_bnd, cur, step, waves, lds, slot, st);
  }
  return step_t<S, W, C, VEC, SHIFT, false, EQ>(d, n, n_int, n_bnd, cur, step, waves, lds, slot, st);
}

template <typename S, typename W, typename C, int VEC, bool SHIFT>
hipError_t step_r(int sr, bool eq, const BatchPlate *d, int n, int64_t n_int, int64_t n_bnd,
                  int cur, int64_t step, int waves, int lds, int slot, hipStream_t st) {
  if constexpr (SHIFT) {
    if (eq) return step_e<S, W, C, VEC, SHIFT, true>(sr, d, n, n_int, n_bnd, cur, step, waves, lds, slot, st);
  } else {
    if (eq) return hipErrorInvalidValue;
  }
  return step_e<S, W, C, VEC, SHIFT, false>(sr, d, n, n_int, n_bnd, cur, step, waves, lds, slot, st);
}

template <typename S, typename W, typename C, int VEC, bool SHIFT, bool EQ>
hipError_t persistent_e(int sr, const BatchPlate *d, int n, int64_t n_int, int64_t n_bnd, int cur,
                        int64_t step, int64_t nsteps, unsigned *sync, int *blocks_used,
                        hipStream_t st) {
  if constexpr (sizeof(S) == 2) {
    if (sr)
      return persistent_t<S, W, C, VEC, SHIFT, true, EQ>(d, n, n_int, n_bnd, cur, step, nsteps,
                                                         sync, blocks_used, st);
  }
  return persistent_t<S, W, C, VEC, SHIFT, false, EQ>(d, n, n_int, n_bnd, cur, step, nsteps, sync,
                                                      blocks_used, st);
}

template <typename S, typename W, typename C, int VEC, bool SHIFT>
hipError_t persistent_r(int sr, bool eq, const BatchPlate *d, int n, int64_t n_int, int64_t n_bnd,
                        int cur, int64_t step, int64_t nsteps, unsigned *sync, int *blocks_used,
                        hipStream_t st) {
  if constexpr (SHIFT) {
    if (eq)
      return persistent_e<S, W, C, VEC, SHIFT, true>(sr, d, n, n_int, n_bnd, cur, step, nsteps,
                                                     sync, blocks_used, st);
  } else {
    if (eq) return hipErrorInvalidValue;
  }
  return persistent_e<S, W, C, VEC, SHIFT, false>(sr, d, n, n_int, n_bnd, cur, step, nsteps, sync,
                                                  blocks_used, st);
}

}  // namespace

hipError_t launch_batch_sweep(Store s, int sr, bool eq, const BatchPlate *d, int n_plates,
                              int64_t n_int_tasks, int64_t n_bnd_tasks, int cur, int64_t step,
                              int waves, int lds_bytes, int fused_slot, hipStream_t st) {
  const int n = n_plates;
  const int64_t ni = n_int_tasks, nb = n_bnd_tasks;
  const int fs = fused_slot < 0 ? -1 : (fused_slot & 1);
  switch (s) {
    // shifted FP64 exists only in the equilibrium layout
    case Store::F64S: return eq ? step_e<double, double, double, 2, true, true>(sr, d, n, ni, nb, cur, step, waves, lds_bytes, fs, st) : hipErrorInvalidValue;
    case Store::F64: return step_r<double, double, double, 2, false>(sr, eq, d, n, ni, nb, cur, step, waves, lds_bytes, fs, st);
    case Store::F32_PLAIN: return step_r<float, float, float, 4, false>(sr, eq, d, n, ni, nb, cur, step, waves, lds_bytes, fs, st);
    case Store::F32S: return step_r<float, float, float, 4, true>(sr, eq, d, n, ni, nb, cur, step, waves, lds_bytes, fs, st);
    case Store::F16S: return step_r<_Float16, float, float, 4, true>(sr, eq, d, n, ni, nb, cur, step, waves, lds_bytes, fs, st);
    case Store::BF16S: return step_r<__bf16, float, float, 4, true>(sr, eq, d, n, ni, nb, cur, step, waves, lds_bytes, fs, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_batch_crack(const BatchPlate *d, int n_plates, int wbuf, int slot, hipStream_t st) {
  if (n_plates < 1) return hipSuccess;
  hipLaunchKernelGGL(batch_crack, dim3((unsigned)((n_plates + 3) / 4)), dim3(256), 0, st, d, n_plates,
                     wbuf & 1, slot & 1);
  return hipGetLastError();
}

hipError_t launch_batch_persistent(Store s, int sr, bool eq, const BatchPlate *d, int n_plates,
                                   int64_t n_int_tasks, int64_t n_bnd_tasks, int cur, int64_t step,
                                   int64_t nsteps, unsigned *sync, int *blocks_used,
                                   hipStream_t st) {
  switch (s) {
    case Store::F64S: return eq ? persistent_e<double, double, double, 2, true, true>(sr, d, n_plates, n_int_tasks, n_bnd_tasks, cur, step, nsteps, sync, blocks_used, st) : hipErrorInvalidValue;
    case Store::F64: return persistent_r<double, double, double, 2, false>(sr, eq, d, n_plates, n_int_tasks, n_bnd_tasks, cur, step, nsteps, sync, blocks_used, st);
    case Store::F32_PLAIN: return persistent_r<float, float, float, 4, false>(sr, eq, d, n_plates, n_int_tasks, n_bnd_tasks, cur, step, nsteps, sync, blocks_used, st);
    case Store::F32S: return persistent_r<float, float, float, 4, true>(sr, eq, d, n_plates, n_int_tasks, n_bnd_tasks, cur, step, nsteps, sync, blocks_used, st);
    case Store::F16S: return persistent_r<_Float16, float, float, 4, true>(sr, eq, d, n_plates, n_int_tasks, n_bnd_tasks, cur, step, nsteps, sync, blocks_used, st);
    case Store::BF16S: return persistent_r<__bf16, float, float, 4, true>(sr, eq, d, n_plates, n_int_tasks, n_bnd_tasks, cur, step, nsteps, sync, blocks_used, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace lbmk
