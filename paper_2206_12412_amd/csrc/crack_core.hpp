// Crack step of Alg. 1 (CrackGrowth), appended after the sweep of every step;
// device code shared by the single-plate crack kernel (crack.hip) and the
// batched kernels (batch.hip).
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
// Each newly severed link is recorded as a cut event (step, column).  The
// same wavefront records w at the sensor sites (also on plates without a
// crack, where it does nothing else).
#pragma once

#include <cmath>

#include "lbm_internal.hpp"

namespace lbmk {
namespace core {

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

// The crack step of one plate, executed by one wavefront (lanes 0..63).
__device__ __forceinline__ void crack_step_wave(const CrackArgs &a) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x & 63;
  const Plate p = a.p;
  const CrackParams q = a.c;
  DevCrack c = *a.st;
  const int64_t n = c.step;
  const int band = q.band;

  // --- sensor traces: w after this step's sweep ---
  if (a.n_sens > 0 && n < q.trace_cap) {
    for (int s = lane; s < a.n_sens; s += 64)
      a.trS[n * a.n_sens + s] = w_at(a, a.sens[2 * s], a.sens[2 * s + 1]);
  }
  if (!q.crack) {
    if (lane == 0) a.st->step = n + 1;
    return;
  }

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

}  // namespace core
}  // namespace lbmk
