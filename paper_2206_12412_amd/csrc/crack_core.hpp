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
// Each newly severed link is recorded as a cut event (step, column).  With two
// tips the left end grows in -x by the same rule, mirrored (K at
// ceil(a + r_min), new columns in [a_new, a_prev)).  The same wavefront records
// w at the sensor sites (also on plates without a crack, where it does nothing
// else).
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

// K_III at one tip (eq. sif) from the current field, by all lanes of the
// wavefront (the band fit reduces over the lanes).  dir = +1: the right tip,
// evaluated at i_K = floor(a - r_min) (band: i_K, i_K - 1, ...); dir = -1: the
// left tip, at the mirrored i_K = ceil(a + r_min) (band: i_K, i_K + 1, ...).
// The columns must lie on the crack, between the tip and the other end.
__device__ __forceinline__ double tip_K(const CrackArgs &a, int dir, double tip, double vK,
                                       double other, int lane, double *r_out, int *iK_out,
                                       bool *defined_out) {
#pragma clang fp contract(off)
  const Plate p = a.p;
  const CrackParams q = a.c;
  const int band = q.band;
  const double rmin = q.r0 / (1.0 - vK);
  double iKf;
  bool defined;
  if (dir > 0) {
    iKf = floor(tip - rmin);
    defined = (iKf - (band - 1) >= 0.0) && (iKf <= (double)(p.nx - 1)) &&
              (iKf - (band - 1) >= other);
  } else {
    iKf = ceil(tip + rmin);
    defined = (iKf >= 0.0) && (iKf + (band - 1) <= (double)(p.nx - 1)) &&
              (iKf + (band - 1) <= other);
  }
  double K = __builtin_nan(""), r = __builtin_nan("");
  int iK = -1;
  if (defined) {
    iK = (int)iKf;
    r = dir > 0 ? tip - iK : iK - tip;
    if (band == 1) {
      const double delta = fabs(w_at(a, iK, p.j0 + 1) - w_at(a, iK, p.j0));
      K = delta * (q.mu / 4.0) * sqrt(2.0 * kPi / r);
    } else {
      double num = 0.0, den = 0.0;
      if (lane < band) {
        const int i = iK - dir * lane;
        const double ri = dir > 0 ? tip - i : i - tip;
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
  *r_out = r;
  *iK_out = iK;
  *defined_out = defined;
  return K;
}

// EvaluateCriterion for one tip: grow or not, and the speed / c_s.
__device__ __forceinline__ bool tip_criterion(const CrackParams &q, bool at_wall, double K,
                                              double *v) {
#pragma clang fp contract(off)
  *v = 0.0;
  if (at_wall) return false;
  if (q.growth == kGrowPrescribed) {
    *v = q.v_rel;
    return true;
  }
  if (q.growth == kGrowSif && K > q.K_C) {
    const double qq = K / q.K_C;
    const double q2 = qq * qq;
    *v = q.v_max * tanh(sqrt(q2 * q2 - 1.0));
    return true;
  }
  return false;
}

// Sever the crack-row links of columns lo..hi (those not yet severed) and
// record them as cut events of step n.
__device__ __forceinline__ bool cut_columns(const CrackArgs &a, DevCrack &c, int lo, int hi,
                                            int64_t n) {
  const Plate p = a.p;
  uint32_t *row = a.mV + (size_t)p.j0 * p.mw;
  bool any = false;
  for (int i = max(lo, 0); i <= min(hi, p.nx - 1); ++i) {
    const uint32_t bit = 1u << (i & 31);
    const uint32_t word = row[i >> 5];
    if (!(word & bit)) {
      row[i >> 5] = word | bit;
      if (c.n_events < a.c.event_cap) {
        a.evStep[c.n_events] = n;
        a.evCol[c.n_events] = i;
      }
      c.n_events++;
      c.n_cut++;
      any = true;
    }
  }
  return any;
}

// The crack step of one plate, executed by one wavefront (lanes 0..63): K and
// the criterion of each growing tip on the same field, then the tips advance
// (the right tip's cuts are recorded first).
__device__ __forceinline__ void crack_step_wave(const CrackArgs &a) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x & 63;
  const Plate p = a.p;
  const CrackParams q = a.c;
  DevCrack c = *a.st;
  const int64_t n = c.step;

  // --- sensor traces: w after this step's sweep ---
  if (a.n_sens > 0 && n < q.trace_cap) {
    for (int s = lane; s < a.n_sens; s += 64)
      a.trS[n * a.n_sens + s] = w_at(a, a.sens[2 * s], a.sens[2 * s + 1]);
  }
  if (!q.crack) {
    if (lane == 0) a.st->step = n + 1;
    return;
  }

  // --- K at the tips (eq. sif) ---
  double rR, rL = __builtin_nan("");
  int iKR, iKL = -1;
  bool defR, defL = true;
  const double KR = tip_K(a, 1, c.tip, (q.growth == kGrowPrescribed) ? q.v_rel : c.v, c.tipL,
                          lane, &rR, &iKR, &defR);
  double KL = __builtin_nan("");
  if (q.both)
    KL = tip_K(a, -1, c.tipL, (q.growth == kGrowPrescribed) ? q.v_rel : c.vL, c.tip, lane, &rL,
               &iKL, &defL);
  if (lane != 0) return;

  // --- EvaluateCriterion ---
  int flagsR = c.flags & kFlagWall, flagsL = c.flagsL & kFlagWall;
  if (!defR) flagsR |= kFlagKUndef;
  if (q.both && !defL) flagsL |= kFlagKUndef;
  double vR = 0.0, vL = 0.0;
  const bool growR = tip_criterion(q, c.flags & kFlagWall, KR, &vR);
  const bool growL = q.both && tip_criterion(q, c.flagsL & kFlagWall, KL, &vL);

  // --- tip advance, CheckLinks, ProcessPoints ---
  bool any = false;
  if (growR) {
    const double a_prev = c.tip;
    double a_new = a_prev + (vR * q.cs) * q.dt;
    if (a_new >= p.nx - 0.5) {
      a_new = p.nx - 0.5;
      flagsR |= kFlagWall;
    }
    // the new segment (a_prev, a_new] touches the columns in that interval
    any |= cut_columns(a, c, (int)floor(a_prev) + 1, (int)floor(a_new), n);
    c.tip = a_new;
    flagsR |= kFlagGrew;
  }
  if (growL) {
    const double a_prev = c.tipL;
    double a_new = a_prev - (vL * q.cs) * q.dt;
    if (a_new <= -0.5) {
      a_new = -0.5;
      flagsL |= kFlagWall;
    }
    // [a_new, a_prev) holds the newly touched columns
    any |= cut_columns(a, c, (int)ceil(a_new), (int)ceil(a_prev) - 1, n);
    c.tipL = a_new;
    flagsL |= kFlagGrew;
  }
  if (any) {
    MaskRows mr = *a.mrows;
    if (p.j0 < mr.vlo || mr.vlo > mr.vhi) mr.vlo = p.j0;
    if (p.j0 > mr.vhi) mr.vhi = p.j0;
    *a.mrows = mr;
  }
  c.v = vR;
  c.K = KR;
  c.r = rR;
  c.col_K = iKR;
  c.flags = flagsR;
  if (q.both) {
    c.vL = vL;
    c.KL = KL;
    c.rL = rL;
    c.col_KL = iKL;
    c.flagsL = flagsL;
  }
  if (n < q.trace_cap) {
    a.trK[n] = KR;
    a.trA[n] = c.tip;
    a.trV[n] = vR;
    a.trF[n] = flagsR;
    if (q.both) {
      a.trKL[n] = KL;
      a.trAL[n] = c.tipL;
      a.trVL[n] = vL;
      a.trFL[n] = flagsL;
    }
  }
  c.step = n + 1;
  *a.st = c;
}

}  // namespace core
}  // namespace lbmk
