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

__device__ __forceinline__ double tip_K(const CrackArgs &a, int dir, double tip, double vK,
                                       double other, int lane, double *r_out, int *iK_out,
                                       bool *defined_out) {
#pragma clang fp contract(off)
  const Plate p = a.p;
  const CrackParams q = a.c;
  if (!q.aligned) return tip_K_line(a, dir, tip, vK, other, r_out, iK_out, defined_out);
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
  MaskRows mr = *a.mrows;
  if (growR) {
    const double a_prev = c.tip;
    double a_new = a_prev + (vR * q.cs) * q.dt;
    if (a_new >= q.a_hi) {
      a_new = q.a_hi;
      flagsR |= kFlagWall;
    }
    if (q.aligned) {
      // the new segment (a_prev, a_new] touches the columns in that interval
      any |= cut_columns(a, c, (int)floor(a_prev) + 1, (int)floor(a_new), n);
    } else {
      any |= cut_segment(a, c, mr, a_prev, a_new, n);
    }
    c.tip = a_new;
    flagsR |= kFlagGrew;
  }
  if (growL) {
    const double a_prev = c.tipL;
    double a_new = a_prev - (vL * q.cs) * q.dt;
    if (a_new <= q.a_lo) {
      a_new = q.a_lo;
      flagsL |= kFlagWall;
    }
    if (q.aligned) {
      // [a_new, a_prev) holds the newly touched columns
      any |= cut_columns(a, c, (int)ceil(a_new), (int)ceil(a_prev) - 1, n);
    } else {
      any |= cut_segment(a, c, mr, a_new, a_prev, n);
    }
    c.tipL = a_new;
    flagsL |= kFlagGrew;
  }
  if (any) {
    if (q.aligned) {
      if (p.j0 < mr.vlo || mr.vlo > mr.vhi) mr.vlo = p.j0;
      if (p.j0 > mr.vhi) mr.vhi = p.j0;
    }
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
