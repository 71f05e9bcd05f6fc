// Two time steps in one sweep (time blocking) for the equilibrium layout:
// each wave loads the rest population and w of its rows once, computes step
// n for them and their neighbours in registers, then step n + 1, and stores
// once, so a step moves half the bytes of the one-step sweep.  The per-site
// arithmetic is that of the one-step sweep (site_update, sweep_core.hpp) with
// the same arguments, so FP32 and FP64 results are bit for bit those of two
// one-step sweeps; 16-bit storages round only after the second step (the
// intermediate stays in FP32), which is more accurate than two roundings.
//
// Scope: walls (no periodic wrap), no crack or a crack along +x on its row
// with prescribed or no growth.  The links step n + 1 sees severed are those
// of step n plus the ones step n's crack step will sever; with a prescribed
// speed they follow from the tips alone, computed here with the crack step's
// own FP64 expressions.  The crack steps of n and n + 1 run afterwards (K of
// step n from the w of the crack rows after step n, which this kernel also
// writes out).
//
// Geometry: a wave owns the columns of a strip of 62 * VEC sites and loads one
// extra lane of VEC sites on either side (the values there are wrong after a
// step by one site per step at the outer end, so two steps leave the owned
// columns exact); it marches rows jb - 2 .. jb + R + 1 to finish rows
// jb .. jb + R - 1 (R = 4, 8 or 16).  x-neighbours move between lanes with DPP; the plate edges
// and the severed links are handled per site as in the one-step sweep.
#include "crack_core.hpp"
#include "sweep_core.hpp"

namespace lbmk {
namespace {

using core::lane_next;
using core::lane_prev;

constexpr int kOwnLanes = 62;  // lanes 1 .. 62 own their columns

// Workgroups go to the 8 XCDs round robin (workgroup b to XCD b mod 8), each
// XCD with its own L2.  Renumbering so that XCD x takes a contiguous range of
// the task order puts vertically adjacent row chunks, which read each other's
// two halo rows, on the same XCD shortly after one another, so those re-reads
// hit its L2 instead of HBM.
__device__ __forceinline__ unsigned xcd_contiguous_block() {
  const unsigned nb = gridDim.x, b = blockIdx.x;
  const unsigned x = b % 8u, s = b / 8u;
  const unsigned q = nb / 8u, r = nb % 8u;
  return x * q + min(x, r) + s;
}

// Per-step values of one time level.
template <typename C>
struct Level {
  C t_top, t_bot, t_up, t_lo;
  C wD_bot, wD_top, wD_left, wD_right;
};

template <typename S, typename W, typename C>
__device__ __forceinline__ Level<C> level_of(const SweepArgs<S, W, C> &a) {
  return Level<C>{a.t_top, a.t_bot, a.t_up, a.t_lo, a.wD_bot, a.wD_top, a.wD_left, a.wD_right};
}

// One step for the VEC sites of a lane on row j: w of rows j - 1, j, j + 1
// (those outside the plate are not read), the rest population g of row j;
// cut_up / cut_dn: bit k set if the vertical link above / below site i0 + k
// is severed.  The boundary values are those the one-step sweep passes.
//
// edge_row (wave-uniform): the row is an edge row or next to the crack line;
// edge_strip (wave-uniform): the wave's columns include a plate edge.  The
// other rows take the arguments of the one-step sweep's interior rows (no
// bounce, no traction) without the per-site selects.
template <typename S, typename W, typename C, int VEC>
__device__ __forceinline__ void step_row(const SweepArgs<S, W, C> &a, const Level<C> &L, int j,
                                         int i0, const C (&wm)[VEC], const C (&wc)[VEC],
                                         const C (&wp)[VEC], const C (&g)[VEC], uint32_t cut_up,
                                         uint32_t cut_dn, bool edge_row, bool edge_strip,
                                         C (&g_out)[VEC], C (&w_out)[VEC]) {
  const Plate p = a.p;
  const int last = p.nx - 1;
  const C wL = lane_prev(wc[VEC - 1]);
  const C wR = lane_next(wc[0]);
  if (!edge_row && !edge_strip) {
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
      const C wl = (k == 0) ? wL : wc[k - 1];
      const C wr = (k == VEC - 1) ? wR : wc[k + 1];
      C o1, o2, o3, o4;
      core::site_update<C, true, true>(a, g[k], C(0), C(0), C(0), C(0), wc[k], wl, wr, wm[k], wp[k],
                                       false, false, C(0), C(0), g_out[k], o1, o2, o3, o4, w_out[k]);
    }
    return;
  }
  const bool jm_out = j == 0, jp_out = j == p.ny - 1;
  const bool db = jm_out && (a.dmask & core::kEdgeBottom);
  const bool dt_ = jp_out && (a.dmask & core::kEdgeTop);
#pragma unroll
  for (int k = 0; k < VEC; ++k) {
    const int i = i0 + k;
    const C w0 = wc[k];
    C wl = (k == 0) ? wL : wc[k - 1];
    C wr = (k == VEC - 1) ? wR : wc[k + 1];
    if (i == 0) wl = (a.dmask & core::kEdgeLeft) ? C(2) * L.wD_left - w0 : w0;
    if (i == last) wr = (a.dmask & core::kEdgeRight) ? C(2) * L.wD_right - w0 : w0;
    const bool bd = jm_out || ((cut_dn >> k) & 1u);
    const bool bu = jp_out || ((cut_up >> k) & 1u);
    const C td = db ? C(0) : (jm_out ? L.t_bot : (bd ? L.t_up : C(0)));
    const C wdn = db ? C(2) * L.wD_bot - w0 : (bd ? w0 : wm[k]);
    const C tu = dt_ ? C(0) : (jp_out ? L.t_top : (bu ? L.t_lo : C(0)));
    const C wup = dt_ ? C(2) * L.wD_top - w0 : (bu ? w0 : wp[k]);
    C o1, o2, o3, o4;
    core::site_update<C, true, true>(a, g[k], C(0), C(0), C(0), C(0), w0, wl, wr, wdn, wup, bd, bu,
                                     td, tu, g_out[k], o1, o2, o3, o4, w_out[k]);
  }
}

template <typename C, int VEC>
__device__ __forceinline__ void copy_row(C (&d)[VEC], const C (&s)[VEC]) {
#pragma unroll
  for (int k = 0; k < VEC; ++k) d[k] = s[k];
}

// Columns lo .. hi as bits of the lane's sites i0 .. i0 + VEC - 1.
template <int VEC>
__device__ __forceinline__ uint32_t range_bits(int i0, int lo, int hi) {
  uint32_t b = 0u;
#pragma unroll
  for (int k = 0; k < VEC; ++k)
    if (i0 + k >= lo && i0 + k <= hi) b |= 1u << k;
  return b;
}

// R rows per wave, a compile-time constant so that the row march unrolls and
// the register windows slide by renaming instead of copies.
template <typename S, typename W, typename C, int VEC, bool SR, int R>
__global__ void __launch_bounds__(512)
sweep_pair(const PairArgs<S, W, C> A, const int n_strips, const int n_chunks) {
  const SweepArgs<S, W, C> &a = A.s0;
  const Plate p = a.p;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int task = (int)xcd_contiguous_block() * (int)(blockDim.x >> 6) + wave;
  if (task >= n_strips * n_chunks) return;
  const int strip = task % n_strips;
  const int jb = (task / n_strips) * R;
  const int je = min(jb + R, p.ny);  // rows jb .. je - 1 are finished here
  constexpr int OW = kOwnLanes * VEC;
  const int i0 = strip * OW - VEC + lane * VEC;  // first site of this lane (may be < 0)
  const bool inplate = i0 >= 0 && i0 < p.nx;
  const bool own = lane >= 1 && lane <= kOwnLanes && inplate;
  const bool loadable = i0 >= 0 && i0 < (int)p.pitch;
  const uint32_t il = loadable ? (uint32_t)i0 : 0u;
  const uint32_t pitch = p.pitch;
  const Level<C> L0 = level_of(A.s0), L1 = level_of(A.s1);

  // severed vertical links of the crack row for step n, and for step n + 1
  // those plus the ones step n's crack step severs (prescribed growth)
  uint32_t cut0 = 0u, cut1 = 0u;
  if (A.crack) {
    if (loadable && i0 < p.nx)
      cut0 = (a.mV[(size_t)p.j0 * p.mw + (il >> 5)] >> (il & 31)) & ((1u << VEC) - 1u);
    cut1 = cut0;
    if (A.grow) {
#pragma clang fp contract(off)
      const DevCrack c = *A.st;
      if (!(c.flags & core::kFlagWall)) {
        double a_new = c.tip + (A.v_rel * A.cs) * A.dt;
        if (a_new >= A.a_hi) a_new = A.a_hi;
        cut1 |= range_bits<VEC>(i0, (int)floor(c.tip) + 1, min((int)floor(a_new), p.nx - 1));
      }
      if (A.both && !(c.flagsL & core::kFlagWall)) {
        double a_new = c.tipL - (A.v_rel * A.cs) * A.dt;
        if (a_new <= A.a_lo) a_new = A.a_lo;
        cut1 |= range_bits<VEC>(i0, max((int)ceil(a_new), 0), (int)ceil(c.tipL) - 1);
      }
    }
  }
  const int jc = A.crack ? p.j0 : -2;  // crack row (its up-links) and jc + 1 (its down-links)
  // the wave's columns i0 of lanes 0 .. 63 include site 0 or site nx - 1
  const bool edge_strip = strip == 0 || (strip + 1) * OW + VEC > p.nx - 1;

  // register window: state rows r-2, r-1, r (w) and r-1, r (g); step-n rows
  // r-3, r-2, r-1 (w) and r-2, r-1 (g)
  C w_m2[VEC], w_m1[VEC], w_0[VEC], g_m1[VEC], g_0[VEC];
  C v_m3[VEC], v_m2[VEC], h_m2[VEC];
  core::zero_row(w_m2);
  core::zero_row(w_m1);
  core::zero_row(g_m1);
  core::zero_row(v_m3);
  core::zero_row(v_m2);
  core::zero_row(h_m2);
#pragma unroll
  for (int rr = 0; rr < R + 4; ++rr) {
    const int r = jb - 2 + rr;
    if (r > je + 1) break;
    // load state row r
    if (r >= 0 && r < p.ny && loadable) {
      const uint32_t o = (uint32_t)r * pitch + il;
      core::load_row<W, C, VEC>(a.win, o, w_0);
      core::load_row<S, C, VEC>(a.fin, o, g_0);
    } else {
      core::zero_row(w_0);
      core::zero_row(g_0);
    }
    // step n for row r - 1
    const int q = r - 1;
    C v_new[VEC], h_new[VEC];
    if (q >= 0 && q < p.ny && q >= jb - 1) {
      const bool er = q == 0 || q == p.ny - 1 || q == jc || q == jc + 1;
      step_row<S, W, C, VEC>(a, L0, q, i0, w_m2, w_m1, w_0, g_m1, q == jc ? cut0 : 0u,
                             q == jc + 1 ? cut0 : 0u, er, edge_strip, h_new, v_new);
      if (own && (q == jc || q == jc + 1) && q >= jb && q < je)
        core::store_row<W, C, VEC>(A.wmid, (uint32_t)(q - jc) * pitch + il, v_new);
    } else {
      core::zero_row(v_new);
      core::zero_row(h_new);
    }
    // step n + 1 for row r - 2, stored
    const int t = r - 2;
    if (t >= jb && t < je) {
      C g2[VEC], w2[VEC];
      const bool er = t == 0 || t == p.ny - 1 || t == jc || t == jc + 1;
      step_row<S, W, C, VEC>(A.s1, L1, t, i0, v_m3, v_m2, v_new, h_m2, t == jc ? cut1 : 0u,
                             t == jc + 1 ? cut1 : 0u, er, edge_strip, g2, w2);
      if (i0 + VEC - 1 > p.nx - 1) {
#pragma unroll
        for (int k = 0; k < VEC; ++k)
          if (i0 + k > p.nx - 1) g2[k] = w2[k] = C(0);  // padding stays zero
      }
      if (own) {
        const uint32_t o = (uint32_t)t * pitch + il;
        core::store_pops<S, C, VEC, SR, true>(a.fout, p.plane, o, g2, g2, g2, g2, g2,
                                              (uint32_t)t * p.nx + (uint32_t)i0, A.s1.rkey);
        core::store_row<W, C, VEC>(a.wout, o, w2);
      }
    }
    // slide the windows
    copy_row(w_m2, w_m1);
    copy_row(w_m1, w_0);
    copy_row(g_m1, g_0);
    copy_row(v_m3, v_m2);
    copy_row(v_m2, v_new);
    copy_row(h_m2, h_new);
  }
}

template <typename S, typename W, typename C, int VEC, bool SR, int R>
hipError_t pair_t(const PairArgs<S, W, C> &A, int waves, hipStream_t st) {
  const Plate &p = A.s0.p;
  const int n_strips = (p.nx + kOwnLanes * VEC - 1) / (kOwnLanes * VEC);
  const int n_chunks = (p.ny + R - 1) / R;
  const long tasks = (long)n_strips * n_chunks;
  const unsigned blocks = (unsigned)((tasks + waves - 1) / waves);
  hipLaunchKernelGGL((sweep_pair<S, W, C, VEC, SR, R>), dim3(blocks), dim3(64 * waves), 0, st, A,
                     n_strips, n_chunks);
  return hipGetLastError();
}

template <typename S, typename W, typename C, int VEC, bool SR>
hipError_t pair_rows(const PairArgs<S, W, C> &A, int rows, int waves, hipStream_t st) {
  switch (rows) {
    case 4: return pair_t<S, W, C, VEC, SR, 4>(A, waves, st);
    case 8: return pair_t<S, W, C, VEC, SR, 8>(A, waves, st);
    case 16: return pair_t<S, W, C, VEC, SR, 16>(A, waves, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename S, typename W, typename C, int VEC>
hipError_t pair_r(const void *args, int rows, int waves, hipStream_t st) {
  const auto &A = *static_cast<const PairArgs<S, W, C> *>(args);
  if constexpr (sizeof(S) == 2) {
    if (A.s0.sr) return pair_rows<S, W, C, VEC, true>(A, rows, waves, st);
  }
  return pair_rows<S, W, C, VEC, false>(A, rows, waves, st);
}

}  // namespace

hipError_t launch_sweep_pair(Store s, const void *args, int rows, int waves, hipStream_t st) {
  if ((rows != 4 && rows != 8 && rows != 16) || (waves != 1 && waves != 2 && waves != 4 && waves != 8))
    return hipErrorInvalidValue;
  switch (s) {
    case Store::F64S: return pair_r<double, double, double, 2>(args, rows, waves, st);
    case Store::F32S: return pair_r<float, float, float, 4>(args, rows, waves, st);
    case Store::F16S: return pair_r<_Float16, float, float, 4>(args, rows, waves, st);
    case Store::BF16S: return pair_r<__bf16, float, float, 4>(args, rows, waves, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lbmk
