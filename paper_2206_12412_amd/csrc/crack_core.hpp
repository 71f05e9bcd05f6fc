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
//
// A crack along another prescribed direction (crack_geom.hpp) takes K from the
// first link that crosses its line at or beyond r_min behind the tip (r to the
// projection of the two sites' midpoint), and severs every vertical or
// horizontal link that the new segment touches, found by testing the links
// around it (the segment is at most dh / kappa long).
#pragma once

#include <cmath>

#include "crack_geom.hpp"
#include "lbm_internal.hpp"

namespace lbmk {
namespace core {

constexpr double kPi = 3.14159265358979323846;
constexpr int kGrowPrescribed = 1;
constexpr int kGrowSif = 2;
constexpr int kFlagGrew = 1, kFlagWall = 2, kFlagKUndef = 4;

__device__ __forceinline__ double w_at(const CrackArgs &a, int i, int j) {
  const size_t x = (size_t)(j - a.w_row0) * a.p.pitch + i;
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
// K at one tip of a crack along another direction than +x: the first link
// crossing the line at or beyond r_min behind the tip (vertical links cross it
// at integer x, horizontal ones at integer y), delta the jump of w across it,
// r the distance along the line from the tip to the projection of the link's
// midpoint.  Undefined (NaN) when the crossing goes through a lattice site,
// lies off the crack or off the plate.  *iK_out is the link's column.
__device__ __forceinline__ double tip_K_line(const CrackArgs &a, int dir, double tip, double vK,
                                            double other, double *r_out, int *iK_out,
                                            bool *defined_out) {
#pragma clang fp contract(off)
  const Plate p = a.p;
  const CrackParams q = a.c;
  const double rmin = q.r0 / (1.0 - vK);
  const double st = tip - q.x0;
  const double so = other - q.x0;
  const double target = dir > 0 ? st - rmin : st + rmin;
  *r_out = __builtin_nan("");
  *iK_out = -1;
  *defined_out = false;
  bool have_v = false, have_h = false;
  double sv = 0.0, sh = 0.0, iv = 0.0, jh = 0.0;
  if (q.ux != 0.0) {
    const double xt = q.x0 + target * q.ux;
    iv = ((dir > 0) == (q.ux > 0)) ? floor(xt) : ceil(xt);
    sv = (iv - q.x0) / q.ux;
    have_v = true;
  }
  if (q.uy != 0.0) {
    const double yt = q.yc + target * q.uy;
    jh = ((dir > 0) == (q.uy > 0)) ? floor(yt) : ceil(yt);
    sh = (jh - q.yc) / q.uy;
    have_h = true;
  }
  const bool vertical = (have_v && have_h) ? (dir > 0 ? sv >= sh : sv <= sh) : have_v;
  const double sc = vertical ? sv : sh;
  if (dir > 0 ? sc < so : sc > so) return __builtin_nan("");
  int i0, j0, i1, j1;
  if (vertical) {
    const double y = q.yc + sc * q.uy;
    if (y == floor(y)) return __builtin_nan("");
    i0 = i1 = (int)iv;
    j0 = (int)floor(y);
    j1 = j0 + 1;
  } else {
    const double x = q.x0 + sc * q.ux;
    if (x == floor(x)) return __builtin_nan("");
    j0 = j1 = (int)jh;
    i0 = (int)floor(x);
    i1 = i0 + 1;
  }
  if (i0 < 0 || i1 > p.nx - 1 || j0 < 0 || j1 > p.ny - 1) return __builtin_nan("");
  const double delta = fabs(w_at(a, i1, j1) - w_at(a, i0, j0));
  const double mx = 0.5 * (double)(i0 + i1), my = 0.5 * (double)(j0 + j1);
  const double sm = (mx - q.x0) * q.ux + (my - q.yc) * q.uy;
  const double r = dir > 0 ? st - sm : sm - st;
  *r_out = r;
  *iK_out = i0;
  *defined_out = true;
  return delta * (q.mu / 4.0) * sqrt(2.0 * kPi / r);
}

// ANY_LINE false: the crack grows along +x (code for other lines left out).
template <bool ANY_LINE = true>
__device__ __forceinline__ double tip_K(const CrackArgs &a, int dir, double tip, double vK,
                                       double other, int lane, double *r_out, int *iK_out,
                                       bool *defined_out) {
#pragma clang fp contract(off)
  const Plate p = a.p;
  const CrackParams q = a.c;
  if constexpr (ANY_LINE) {
    if (!q.aligned) return tip_K_line(a, dir, tip, vK, other, r_out, iK_out, defined_out);
  }
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
        a.evRow[c.n_events] = p.j0;
        a.evOri[c.n_events] = 0;
      }
      c.n_events++;
      c.n_cut++;
      any = true;
    }
  }
  return any;
}

// Sever the links that the crack between line coordinates a0 and a1 touches
// (a crack along another direction than +x), recording them as cut events
// of step n and widening the mask-row range.  The segment is short, so the
// candidates are the links within its bounding box: vertical links at the
// integer x inside it, horizontal links at the integer y inside it.
__device__ __forceinline__ bool cut_segment(const CrackArgs &a, DevCrack &c, MaskRows &mr,
                                            double a0, double a1, int64_t n) {
  const Plate p = a.p;
  const geom::Line L{a.c.aligned, a.c.x0, a.c.yc, a.c.ux, a.c.uy};
  double x0, y0, x1, y1;
  geom::point_at(L, a0, &x0, &y0);
  geom::point_at(L, a1, &x1, &y1);
  const double xlo = fmin(x0, x1), xhi = fmax(x0, x1), ylo = fmin(y0, y1), yhi = fmax(y0, y1);
  bool any = false;
  auto cut = [&](int i, int j, int o) {
    uint32_t *m = (o == 0 ? a.mV : a.mH) + (size_t)j * p.mw;
    const uint32_t bit = 1u << (i & 31);
    const uint32_t word = m[i >> 5];
    if (word & bit) return;
    m[i >> 5] = word | bit;
    if (c.n_events < a.c.event_cap) {
      a.evStep[c.n_events] = n;
      a.evCol[c.n_events] = i;
      a.evRow[c.n_events] = j;
      a.evOri[c.n_events] = o;
    }
    c.n_events++;
    c.n_cut++;
    any = true;
    if (o == 0) {
      if (mr.vlo > mr.vhi) mr.vlo = mr.vhi = j;
      mr.vlo = min(mr.vlo, j);
      mr.vhi = max(mr.vhi, j);
    } else {
      if (mr.hlo > mr.hhi) mr.hlo = mr.hhi = j;
      mr.hlo = min(mr.hlo, j);
      mr.hhi = max(mr.hhi, j);
    }
  };
  // vertical links (i, j)-(i, j + 1): x = i in [xlo, xhi], [j, j + 1] meeting [ylo, yhi]
  for (int i = max((int)ceil(xlo), 0); i <= min((int)floor(xhi), p.nx - 1); ++i)
    for (int j = max((int)ceil(ylo) - 1, 0); j <= min((int)floor(yhi), p.ny - 2); ++j)
      if (geom::touches_link(L, a0, a1, i, j, 0, 1)) cut(i, j, 0);
  // horizontal links (i, j)-(i + 1, j): y = j in [ylo, yhi], [i, i + 1] meeting [xlo, xhi]
  for (int j = max((int)ceil(ylo), 0); j <= min((int)floor(yhi), p.ny - 1); ++j)
    for (int i = max((int)ceil(xlo) - 1, 0); i <= min((int)floor(xhi), p.nx - 2); ++i)
      if (geom::touches_link(L, a0, a1, i, j, 1, 0)) cut(i, j, 1);
  return any;
}

// The decision of one crack step (Alg. 1: K at each tip, EvaluateCriterion,
// the tip advance with the wall clamp) from the crack state c before it, by
// all lanes of a wavefront (the band fit reduces over the lanes).  WITH_K
// false: only the new tip positions, for a prescribed speed, where they do
// not depend on K.
struct CrackDecision {
  double KR, KL, rR, rL;
  int iKR, iKL;
  bool growR, growL;
  double vR, vL;
  double aR, aL;       // the tips after the step
  int flagsR, flagsL;  // the step's flags
};

template <bool WITH_K, bool ANY_LINE = true>
__device__ __forceinline__ CrackDecision crack_decide(const CrackArgs &a, const DevCrack &c,
                                                      int lane) {
#pragma clang fp contract(off)
  const CrackParams q = a.c;
  CrackDecision d;
  d.KR = d.KL = d.rR = d.rL = __builtin_nan("");
  d.iKR = d.iKL = -1;
  bool defR = true, defL = true;
  if constexpr (WITH_K) {
    d.KR = tip_K<ANY_LINE>(a, 1, c.tip, (q.growth == kGrowPrescribed) ? q.v_rel : c.v, c.tipL, lane, &d.rR,
                 &d.iKR, &defR);
    if (q.both)
      d.KL = tip_K<ANY_LINE>(a, -1, c.tipL, (q.growth == kGrowPrescribed) ? q.v_rel : c.vL, c.tip, lane,
                   &d.rL, &d.iKL, &defL);
  }
  d.flagsR = c.flags & kFlagWall;
  d.flagsL = c.flagsL & kFlagWall;
  if (!defR) d.flagsR |= kFlagKUndef;
  if (q.both && !defL) d.flagsL |= kFlagKUndef;
  d.vR = d.vL = 0.0;
  d.growR = tip_criterion(q, c.flags & kFlagWall, d.KR, &d.vR);
  d.growL = q.both && tip_criterion(q, c.flagsL & kFlagWall, d.KL, &d.vL);
  d.aR = c.tip;
  d.aL = c.tipL;
  if (d.growR) {
    double a_new = c.tip + (d.vR * q.cs) * q.dt;
    if (a_new >= q.a_hi) {
      a_new = q.a_hi;
      d.flagsR |= kFlagWall;
    }
    d.aR = a_new;
    d.flagsR |= kFlagGrew;
  }
  if (d.growL) {
    double a_new = c.tipL - (d.vL * q.cs) * q.dt;
    if (a_new <= q.a_lo) {
      a_new = q.a_lo;
      d.flagsL |= kFlagWall;
    }
    d.aL = a_new;
    d.flagsL |= kFlagGrew;
  }
  return d;
}

// The columns of the crack row (a crack along +x) whose vertical links the
// crack step from state c severs (those not severed yet among them are new):
// the right tip's [*lo_r, *hi_r] and the left tip's [*lo_l, *hi_l] (lo > hi:
// none), by all lanes of a wavefront.  The sweep of the next step uses this
// to run that crack step's cuts itself (see crack_step_wave).
__device__ __forceinline__ void crack_cut_columns(const CrackArgs &a, const DevCrack &c, int lane,
                                                  int *lo_r, int *hi_r, int *lo_l, int *hi_l) {
  const CrackDecision d = a.c.growth == kGrowSif ? crack_decide<true, false>(a, c, lane)
                                                 : crack_decide<false, false>(a, c, lane);
  *lo_r = 1;
  *hi_r = 0;
  *lo_l = 1;
  *hi_l = 0;
  if (d.growR) {
    *lo_r = (int)floor(c.tip) + 1;
    *hi_r = (int)floor(d.aR);
  }
  if (d.growL) {
    *lo_l = (int)ceil(d.aL);
    *hi_l = (int)ceil(c.tipL) - 1;
  }
}

// The crack step of one plate, executed by one wavefront (lanes 0..63): K and
// the criterion of each growing tip on the same field, then the tips advance
// (the right tip's cuts are recorded first).  It reads the crack state from
// a.st and writes the state after the step to a.st_out (a.st if null).
// ANY_LINE false: only for a crack along +x (fewer registers).
template <bool ANY_LINE = true>
__device__ __forceinline__ void crack_step_wave(const CrackArgs &a) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x & 63;
  const Plate p = a.p;
  const CrackParams q = a.c;
  DevCrack c = *a.st;
  DevCrack *out = a.st_out ? a.st_out : a.st;
  const int64_t n = c.step;

  // --- sensor traces: w after this step's sweep ---
  if (a.n_sens > 0 && n < q.trace_cap) {
    for (int s = lane; s < a.n_sens; s += 64)
      a.trS[n * a.n_sens + s] = w_at(a, a.sens[2 * s], a.sens[2 * s + 1]);
  }
  if (!q.crack) {
    if (lane == 0) {
      c.step = n + 1;
      *out = c;
    }
    return;
  }

  // --- K at the tips (eq. sif), EvaluateCriterion, tip advance ---
  const CrackDecision d = crack_decide<true, ANY_LINE>(a, c, lane);
  const bool aligned = !ANY_LINE || q.aligned;
  if (lane != 0) return;

  // --- CheckLinks, ProcessPoints ---
  bool any = false;
  MaskRows mr = *a.mrows;
  if (d.growR) {
    if (aligned) {
      // the new segment (a_prev, a_new] touches the columns in that interval
      any |= cut_columns(a, c, (int)floor(c.tip) + 1, (int)floor(d.aR), n);
    } else if constexpr (ANY_LINE) {
      any |= cut_segment(a, c, mr, c.tip, d.aR, n);
    }
    c.tip = d.aR;
  }
  if (d.growL) {
    if (aligned) {
      // [a_new, a_prev) holds the newly touched columns
      any |= cut_columns(a, c, (int)ceil(d.aL), (int)ceil(c.tipL) - 1, n);
    } else if constexpr (ANY_LINE) {
      any |= cut_segment(a, c, mr, d.aL, c.tipL, n);
    }
    c.tipL = d.aL;
  }
  if (any) {
    if (aligned) {
      if (p.j0 < mr.vlo || mr.vlo > mr.vhi) mr.vlo = p.j0;
      if (p.j0 > mr.vhi) mr.vhi = p.j0;
    }
    *a.mrows = mr;
  }
  c.v = d.vR;
  c.K = d.KR;
  c.r = d.rR;
  c.col_K = d.iKR;
  c.flags = d.flagsR;
  if (q.both) {
    c.vL = d.vL;
    c.KL = d.KL;
    c.rL = d.rL;
    c.col_KL = d.iKL;
    c.flagsL = d.flagsL;
  }
  if (n < q.trace_cap) {
    a.trK[n] = d.KR;
    a.trA[n] = c.tip;
    a.trV[n] = d.vR;
    a.trF[n] = d.flagsR;
    if (q.both) {
      a.trKL[n] = d.KL;
      a.trAL[n] = c.tipL;
      a.trVL[n] = d.vL;
      a.trFL[n] = d.flagsL;
    }
  }
  c.step = n + 1;
  *out = c;
}

}  // namespace core
}  // namespace lbmk
