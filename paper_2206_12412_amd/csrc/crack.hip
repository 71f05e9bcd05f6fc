// Single-plate crack kernel and the initial cut mask; the crack step itself
// lives in crack_core.hpp.
#include <cmath>

#include "crack_core.hpp"

namespace lbmk {
namespace {

__global__ void __launch_bounds__(64) crack_kernel(const CrackArgs a) { core::crack_step_wave(a); }

// The crack steps of the n time steps one T-step sweep advanced, in order, by
// one wavefront: step m reads w from w[m] (rows from w_row0[m] on); the
// barrier makes each step's state, mask and trace writes visible to the next.
// Speculative sweeps (s.spec set): the sweep severed the links of its later
// steps as if each tip kept the speed of its last step.  The state at the
// start is kept; when crack step m < n - 1 leaves a tip in another column
// than that prediction (the links the sweep of steps m + 2 .. n used differ
// from the real ones), the state of the start is put back and valid = m + 1
// tells the host to run the sweep again for m + 1 steps; with a gate (several
// sweeps in flight) it also closes the gate, so that the sweeps and crack
// sequences queued after this one return at once and leave the state alone.
__global__ void __launch_bounds__(64) crack_seq_kernel(const CrackSeq s) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x & 63;
  if (s.gate && *s.gate == 0) return;
  const Plate p = s.a.p;
  const CrackParams q = s.a.c;
  uint32_t *row = s.a.mV + (size_t)p.j0 * p.mw;
  // the predicted tips (the sweep's own recurrence)
  double pR = 0.0, pL = 0.0, daR = 0.0, daL = 0.0;
  bool wR = true, wL = true;
  if (s.spec) {
    const DevCrack c0 = *s.a.st;
    pR = c0.tip;
    pL = c0.tipL;
    daR = (c0.v * q.cs) * q.dt;
    daL = (c0.vL * q.cs) * q.dt;
    wR = (c0.flags & core::kFlagWall) != 0;
    wL = (c0.flagsL & core::kFlagWall) != 0;
    for (int k = lane; k < p.mw; k += 64) s.spec_mask[k] = row[k];
    if (lane == 0) {
      s.spec->st = c0;
      s.spec->mr = *s.a.mrows;
    }
  }
  for (int m = 0; m < s.n; ++m) {
    CrackArgs a = s.a;
    a.w = s.w[m];
    a.w_row0 = s.w_row0[m];
    core::crack_step_wave(a);
    __syncthreads();
    if (!s.spec || m + 1 == s.n) continue;
    if (!wR) {
      pR = pR + daR;
      if (pR >= q.a_hi) {
        pR = q.a_hi;
        wR = true;
      }
    }
    if (q.both && !wL) {
      pL = pL - daL;
      if (pL <= q.a_lo) {
        pL = q.a_lo;
        wL = true;
      }
    }
    const DevCrack c = *s.a.st;
    if (floor(c.tip) != floor(pR) || (q.both && ceil(c.tipL) != ceil(pL))) {
      for (int k = lane; k < p.mw; k += 64) row[k] = s.spec_mask[k];
      if (lane == 0) {
        *s.a.st = s.spec->st;
        *s.a.mrows = s.spec->mr;
        s.spec_out->valid = m + 1;
        if (s.gate) *s.gate = 0;
      }
      return;
    }
  }
  if (s.spec && lane == 0) s.spec_out->valid = s.n;
}

// Mask words of every row: all links intact except the vertical links of the
// crack row at the columns lo..hi (the initial crack segment x0 .. a0 touches
// exactly those; Sec. 4.1 treats the initial crack's links like those of a
// grown segment).  With a crack the
// mask-row range names the crack row from the start (growth cuts only there).
__global__ void init_mask_kernel(uint32_t *mV, uint32_t *mH, MaskRows *mrows, Plate p, int lo,
                                 int hi, int has_crack) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t words = (size_t)p.ny * p.mw;
  if (t < words) {
    const int j = (int)(t / p.mw);
    const int wi = (int)(t % p.mw);
    uint32_t v = 0u;
    if (j == p.j0) {
      for (int b = 0; b < 32; ++b) {
        const int i = wi * 32 + b;
        if (i >= lo && i <= hi) v |= 1u << b;
      }
    }
    mV[t] = v;
    mH[t] = 0u;
  }
  if (t == 0) *mrows = has_crack ? MaskRows{p.j0, p.j0, 1, 0} : MaskRows{1, 0, 1, 0};
}

__global__ void set_flag_kernel(int32_t *p, int32_t v) { *p = v; }

}  // namespace

hipError_t launch_set_flag(int32_t *p, int32_t v, hipStream_t st) {
  hipLaunchKernelGGL(set_flag_kernel, dim3(1), dim3(1), 0, st, p, v);
  return hipGetLastError();
}

hipError_t launch_crack(const CrackArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(crack_kernel, dim3(1), dim3(64), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_crack_seq(const CrackSeq &s, hipStream_t st) {
  if (s.n < 1 || s.n > kMaxTimeBlock) return hipErrorInvalidValue;
  hipLaunchKernelGGL(crack_seq_kernel, dim3(1), dim3(64), 0, st, s);
  return hipGetLastError();
}

hipError_t launch_init_mask(uint32_t *mV, uint32_t *mH, MaskRows *mrows, const Plate &p,
                            int has_crack, double x0, double a0, hipStream_t st) {
  int lo = 1, hi = 0;  // empty
  if (has_crack) {
    lo = (int)std::ceil(x0);
    if (lo < 0) lo = 0;
    hi = (int)std::floor(a0);
    if (hi > p.nx - 1) hi = p.nx - 1;
  }
  const size_t words = (size_t)p.ny * p.mw;
  const unsigned blocks = (unsigned)((words + 255) / 256);
  hipLaunchKernelGGL(init_mask_kernel, dim3(blocks), dim3(256), 0, st, mV, mH, mrows, p, lo, hi,
                     has_crack);
  return hipGetLastError();
}

}  // namespace lbmk
