// Crack step of Alg. 1 (CrackGrowth), appended after the sweep of every step.
//
// One wavefront per plate.  It evaluates K_III from the displacement jump
// across the crack faces at the column i_K = floor(a - r_min), r = a - i_K
// (eq. sif; evaluation points of Sec. 4.2 with r_min = r0 / (1 - v), eq. r(v)),
// optionally fitted over a band of columns with a wavefront reduction; then
// the criterion (prescribed growth, or K > K_C with the tanh speed law,
// eq. sifCriterion and eq. v-tanh), the FP64 tip advance a += (v c_s) dt,
// and CheckLinks / ProcessPoints for the straight crack on the mid-line: the
// new segment (a_prev, a] touches exactly the vertical links of the crack row
// at the integer columns in that interval (the closed segment also touches
// column a_prev when a_prev is an integer, which was severed already).
// Each newly severed link is recorded as a cut event (step, column).
#include <cmath>

#include "lbm_internal.hpp"

namespace lbmk {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kGrowPrescribed = 1;
constexpr int kGrowSif = 2;
constexpr int kFlagGrew = 1, kFlagWall = 2, kFlagKUndef = 4;

__device__ __forceinline__ double w_at(const CrackArgs &a, int i, int j) {
  const size_t x = (size_t)j * a.p.pitch + i;
  return a.w_is_double ? static_cast<const double *>(a.w)[x]
                       : (double)static_cast<const float *>(a.w)[x];
}

__device__ __forceinline__ double wave_sum(double x) {
  // butterfly over the 64 lanes; every lane ends with the same value
  for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
  return x;
}

__global__ void __launch_bounds__(64) crack_kernel(const CrackArgs a) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x;
  const Plate p = a.p;
  const CrackParams q = a.c;
  DevCrack c = *a.st;
  const int64_t n = c.step;
  const int band = q.band;

  // --- K at the current tip (eq. sif) ---
  const double vK = (q.growth == kGrowPrescribed) ? q.v_rel : c.v;
  const double rmin = q.r0 / (1.0 - vK);
  const double iKf = floor(c.tip - rmin);
  const bool defined = (iKf - (band - 1) >= 0.0) && (iKf <= (double)(p.nx - 1)) &&
                       (iKf - (band - 1) >= q.x0);
  double K = __builtin_nan(""), r = __builtin_nan("");
  int iK = -1;
  if (defined) {
    iK = (int)iKf;
    r = c.tip - iK;
    if (band == 1) {
      const double delta = fabs(w_at(a, iK, p.j0 + 1) - w_at(a, iK, p.j0));
      K = delta * (q.mu / 4.0) * sqrt(2.0 * kPi / r);
    } else {
      double num = 0.0, den = 0.0;
      if (lane < band) {
        const int i = iK - lane;
        const double ri = c.tip - i;
        const double sq = sqrt(ri / (2.0 * kPi));
        const double delta = fabs(w_at(a, i, p.j0 + 1) - w_at(a, i, p.j0));
        num = delta * sq;
        den = sq * sq;
      }
      num = wave_sum(num);
      den = wave_sum(den);
      K = (q.mu / 4.0) * num / den;
    }
  }
  if (lane != 0) return;

  // --- EvaluateCriterion ---
  int flags = c.flags & kFlagWall;
  if (!defined) flags |= kFlagKUndef;
  bool grow = false;
  double v = 0.0;
  if (!(c.flags & kFlagWall)) {
    if (q.growth == kGrowPrescribed) {
      grow = true;
      v = q.v_rel;
    } else if (q.growth == kGrowSif && K > q.K_C) {
      const double qq = K / q.K_C;
      const double q2 = qq * qq;
      v = q.v_max * tanh(sqrt(q2 * q2 - 1.0));
      grow = true;
    }
  }
  // --- tip advance, CheckLinks, ProcessPoints ---
  if (grow) {
    const double a_prev = c.tip;
    double a_new = a_prev + (v * q.cs) * q.dt;
    if (a_new >= p.nx - 0.5) {
      a_new = p.nx - 0.5;
      flags |= kFlagWall;
    }
    const int i_lo = (int)floor(a_prev) + 1;
    const int i_hi = min((int)floor(a_new), p.nx - 1);
    uint32_t *row = a.mV + (size_t)p.j0 * p.mw;
    bool any = false;
    for (int i = max(i_lo, 0); i <= i_hi; ++i) {
      const uint32_t bit = 1u << (i & 31);
      const uint32_t word = row[i >> 5];
      if (!(word & bit)) {
        row[i >> 5] = word | bit;
        if (c.n_events < q.event_cap) {
          a.evStep[c.n_events] = n;
          a.evCol[c.n_events] = i;
        }
        c.n_events++;
        c.n_cut++;
        any = true;
      }
    }
    if (any) {
      MaskRows mr = *a.mrows;
      if (p.j0 < mr.vlo || mr.vlo > mr.vhi) mr.vlo = p.j0;
      if (p.j0 > mr.vhi) mr.vhi = p.j0;
      *a.mrows = mr;
    }
    c.tip = a_new;
    flags |= kFlagGrew;
  }
  c.v = v;
  c.K = K;
  c.r = r;
  c.col_K = iK;
  c.flags = flags;
  if (n < q.trace_cap) {
    a.trK[n] = K;
    a.trA[n] = c.tip;
    a.trV[n] = v;
    a.trF[n] = flags;
  }
  c.step = n + 1;
  *a.st = c;
}

// Mask words of every row: all links intact except the vertical links of the
// crack row at the columns lo..hi (the initial crack segment x0 .. a0 touches
// exactly those, Alg. 1 "as for the initial crack").  With a crack the
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

}  // namespace

hipError_t launch_crack(const CrackArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(crack_kernel, dim3(1), dim3(64), 0, st, a);
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
