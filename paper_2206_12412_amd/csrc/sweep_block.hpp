// T time steps in one sweep (time blocking, T = 2 .. 8) for the
// equilibrium layout: each wave loads the rest population and w of its rows
// once, computes step n for them and their neighbours in registers, then step
// n + 1 from those, and so on, and stores once, so a step moves 1 / T of the
// bytes of the one-step sweep.  The per-site arithmetic is that of the
// one-step sweep (site_update, sweep_core.hpp) with the same arguments, so
// FP32 and FP64 results are bit for bit those of T one-step sweeps; 16-bit
// storages round only after the last step (the intermediate levels stay in
// FP32), which is more accurate than rounding every step.
//
// Scope: walls (no periodic wrap), no crack or a crack along +x on its row
// with prescribed or no growth.  The links step n + k sees severed are those
// of step n plus the ones the crack steps of n .. n + k - 1 will sever; with
// a prescribed speed they follow from the tips alone, computed here with the
// crack step's own FP64 expressions.  The T crack steps run afterwards, in
// order (K of step n + k < n + T - 1 from the w of the crack rows after that
// step, which this kernel also writes out).
//
// Geometry: a wave owns the columns of a strip of (64 - 2H) * VEC sites and
// loads H extra lanes of VEC sites on either side, H = ceil(T / VEC) (the
// values there go wrong by one site per step from the outer end, so T steps
// leave the owned columns exact); it marches rows jb - T .. jb + R + T - 1 to
// finish rows jb .. jb + R - 1 (R = 4, 8 or 16).  Level k of the march holds
// the rows after step n + k - 1; level k computes row r - k when state row r
// arrives.  x-neighbours move between lanes with DPP; the plate edges and the
// severed links are handled per site as in the one-step sweep.
//
// Two launches: the fast chunks (rows away from the plate's top and bottom
// and the crack rows) of the strips without a plate edge, with only the
// interior arithmetic compiled in; and, on a side stream beside it, the slow
// chunk rows of every strip with the general march and the other chunks of
// the strips with a plate edge, whose march adds the left and right edge
// treatment to the fast one.
#pragma once

#include "crack_core.hpp"
#include "sweep_core.hpp"

namespace lbmk {
namespace blk {

using core::lane_next;
using core::lane_prev;

// Workgroups go to the 8 XCDs round robin (workgroup b to XCD b mod 8), each
// XCD with its own L2.  Renumbering so that XCD x takes a contiguous range of
// the task order puts vertically adjacent row chunks, which read each other's
// halo rows, on the same XCD shortly after one another, so those re-reads
// hit its L2 instead of HBM.
__device__ __forceinline__ unsigned xcd_contiguous_block() {
  const unsigned nb = gridDim.x, b = blockIdx.x;
  const unsigned x = b % 8u, s = b / 8u;
  const unsigned q = nb / 8u, r = nb % 8u;
  return x * q + min(x, r) + s;
}

// The finished rows are stored through buffer resources: a lane that owns no
// columns (a halo lane) passes an offset beyond the resource's size, and the
// hardware drops such a store, so the row march has no branch around its
// stores and the compiler can schedule the loads of later rows across them.
constexpr uint32_t kDropOffset = 0xffffff80u;  // >= the size of any plane (< 4 GiB, 128-byte rows)
constexpr int kNonTemporal = 2;                // cache policy bit "nt"

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, 0x00020000);
}

template <typename T, int VEC>
__device__ __forceinline__ void buffer_store_row(__amdgpu_buffer_rsrc_t rs, uint32_t byte_off,
                                                 const core::Pack<T, VEC> &pk) {
  if constexpr (sizeof(pk) == 16) {
    core::u32x4 v;
    __builtin_memcpy(&v, &pk, 16);
    __builtin_amdgcn_raw_buffer_store_b128(v, rs, (int)byte_off, 0, kNonTemporal);
  } else if constexpr (sizeof(pk) == 8) {
    core::u32x2 v;
    __builtin_memcpy(&v, &pk, 8);
    __builtin_amdgcn_raw_buffer_store_b64(v, rs, (int)byte_off, 0, kNonTemporal);
  } else {
    static_assert(sizeof(pk) == 4, "rows are stored in 4-, 8- or 16-byte pieces");
    uint32_t v;
    __builtin_memcpy(&v, &pk, 4);
    __builtin_amdgcn_raw_buffer_store_b32(v, rs, (int)byte_off, 0, kNonTemporal);
  }
}

// One row of VEC values in the storage type (one 8- or 16-byte load).
template <typename T, int VEC>
__device__ __forceinline__ void load_raw(const T *__restrict__ base, uint32_t off, T (&out)[VEC]) {
  const core::Pack<T, VEC> pk = *reinterpret_cast<const core::Pack<T, VEC> *>(core::at(base, off));
#pragma unroll
  for (int k = 0; k < VEC; ++k) out[k] = pk.v[k];
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
__device__ __forceinline__ void step_row(const SweepArgs<S, W, C> &a, const StepLevel<C> &L, int j,
                                         int i0, const C (&wm)[VEC], const C (&wc)[VEC],
                                         const C (&wp)[VEC], const C (&g)[VEC], uint32_t cut_up,
                                         uint32_t cut_dn, bool edge_row, bool edge_strip,
                                         C (&g_out)[VEC], C (&w_out)[VEC]) {
  const Plate p = a.p;
  const int last = p.nx - 1;
  const C wL = lane_prev(wc[VEC - 1]);
  const C wR = lane_next(wc[0]);
  if (!edge_row) {
    // every vertical link intact and no traction: the interior arithmetic,
    // with the neighbour beyond a left or right plate edge replaced (the
    // site itself for bounce-back, 2 w* - w for a Dirichlet edge)
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
      C wl = (k == 0) ? wL : wc[k - 1];
      C wr = (k == VEC - 1) ? wR : wc[k + 1];
      if (edge_strip) {
        if (i0 + k == 0) wl = (a.dmask & core::kEdgeLeft) ? C(2) * L.wD_left - wc[k] : wc[k];
        if (i0 + k == last) wr = (a.dmask & core::kEdgeRight) ? C(2) * L.wD_right - wc[k] : wc[k];
      }
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

// The row march of one wave: state rows jb - T .. jb + R + T - 1 loaded,
// level k (step n + k - 1) computed for rows jb - (T - k) .. jb + R - 1 +
// (T - k), level T stored for rows jb .. jb + R - 1.  FAST (wave-uniform):
// every row the wave loads lies in the plate, none of the rows it steps is an
// edge or crack row, and its columns hold no plate edge, so every lane loads,
// no row needs a range check and every site takes the interior arithmetic.
// XEDGE: the rows as for FAST, but the columns may hold a plate edge (lanes
// outside the plate, the left and right edge treatment).
template <typename S, typename W, typename C, int VEC, bool SR, int R, int T, bool FAST,
          bool XEDGE = false>
__device__ __forceinline__ void march(const BlockArgs<S, W, C> &A, const int strip, const int jb,
                                      const int lane, const bool edge_strip) {
  static_assert(!(FAST && XEDGE), "FAST columns hold no plate edge");
  constexpr bool ROWS = FAST || XEDGE;  // the rows of a fast chunk
  constexpr int H = (T + VEC - 1) / VEC;  // halo lanes on either side
  constexpr int OW = (64 - 2 * H) * VEC;  // owned columns of a strip
  constexpr int NR = R + 2 * T;           // state rows loaded
  constexpr int D = NR < 6 ? NR : 6;      // rows loaded ahead of their first use
  const SweepArgs<S, W, C> &a = A.s0;
  const Plate p = a.p;
  const int je = ROWS ? jb + R : min(jb + R, p.ny);  // rows jb .. je - 1 are finished here
  const int i0 = strip * OW - H * VEC + lane * VEC;  // first site of this lane (may be < 0)
  const bool inplate = FAST || ((uint32_t)i0 < (uint32_t)p.nx);
  // (one unsigned compare and a bitwise and: no branch)
  const bool own = ((uint32_t)(lane - H) < (uint32_t)(64 - 2 * H)) & inplate;
  const bool loadable = FAST || (i0 >= 0 && i0 < (int)p.pitch);
  const uint32_t il = loadable ? (uint32_t)i0 : 0u;
  const uint32_t pitch = p.pitch;
  const uint32_t rows_elems = pitch * (uint32_t)p.ny;
  const __amdgpu_buffer_rsrc_t rf = plane_rsrc(a.fout, rows_elems * (uint32_t)sizeof(S));
  const __amdgpu_buffer_rsrc_t rw = plane_rsrc(a.wout, rows_elems * (uint32_t)sizeof(W));

  // severed vertical links of the crack row at step n + k: those of step n
  // plus the ones the crack steps of n .. n + k - 1 sever (the tip advance,
  // wall clamp and cut columns of the crack step, at the prescribed speed or,
  // under the K criterion, at each tip's last speed: a prediction the crack
  // steps check)
  uint32_t cut[T];
#pragma unroll
  for (int k = 0; k < T; ++k) cut[k] = 0u;
  if (!ROWS && A.crack) {
    if (loadable && i0 < p.nx)
      cut[0] = (a.mV[(size_t)p.j0 * p.mw + (il >> 5)] >> (il & 31)) & ((1u << VEC) - 1u);
#pragma unroll
    for (int k = 1; k < T; ++k) cut[k] = cut[0];
    if (A.grow) {
#pragma clang fp contract(off)
      const DevCrack c = *A.st;
      const double da = ((A.sif ? c.v : A.v_rel) * A.cs) * A.dt;
      const double daL = ((A.sif ? c.vL : A.v_rel) * A.cs) * A.dt;
      double tip = c.tip, tipL = c.tipL;
      bool wall = (c.flags & core::kFlagWall) != 0, wallL = (c.flagsL & core::kFlagWall) != 0;
#pragma unroll
      for (int k = 1; k < T; ++k) {
        uint32_t add = 0u;
        if (!wall) {
          double a_new = tip + da;
          if (a_new >= A.a_hi) {
            a_new = A.a_hi;
            wall = true;
          }
          add |= range_bits<VEC>(i0, (int)floor(tip) + 1, min((int)floor(a_new), p.nx - 1));
          tip = a_new;
        }
        if (A.both && !wallL) {
          double a_new = tipL - daL;
          if (a_new <= A.a_lo) {
            a_new = A.a_lo;
            wallL = true;
          }
          add |= range_bits<VEC>(i0, max((int)ceil(a_new), 0), (int)ceil(tipL) - 1);
          tipL = a_new;
        }
#pragma unroll
        for (int m = k; m < T; ++m) cut[m] |= add;
      }
    }
  }
  const int jc = A.crack ? p.j0 : -2;  // crack row (its up-links) and jc + 1 (its down-links)

  // state rows in the storage types, D of them in flight ahead of their use:
  // on this hardware a wait for a load also waits for every store issued
  // before it, so each load is issued D rows before the stores it must not
  // wait for.  In a march of more than 28 fast-chunk rows, row rr goes to slot
  // rr % 8 (an array of NR rows was kept in scratch memory for NR = 44 and
  // more); elsewhere each row has its own (with slots the boundary launch
  // took 45 % longer).
  constexpr int RING = (ROWS && NR > 28) ? 8 : NR;
  static_assert(D < RING || RING == NR, "a slot is reused only after its row was taken");
  W wl_[RING][VEC];
  S gl_[RING][VEC];
  auto load = [&](int rr) {
    const int r = jb - T + rr;
    // (XEDGE: the lanes outside the row load its first columns instead; no
    // site of the plate reads them, the edge treatment replaces its
    // neighbours beyond an edge)
    if (ROWS || (r >= 0 && r < p.ny && r <= je + T - 1 && loadable)) {
      const uint32_t o = (uint32_t)r * pitch + il;
      load_raw<W, VEC>(a.win, o, wl_[rr % RING]);
      load_raw<S, VEC>(a.fin, o, gl_[rr % RING]);
    } else {
#pragma unroll
      for (int k = 0; k < VEC; ++k) {
        wl_[rr % RING][k] = W(0);
        gl_[rr % RING][k] = S(0);
      }
    }
  };
#pragma unroll
  for (int rr = 0; rr < D; ++rr) load(rr);

  // level k >= 1 windows: w of its three newest rows (0 = newest), g of its
  // two newest
  C wv[T][3][VEC], gv[T][2][VEC];
#pragma unroll
  for (int k = 0; k < T; ++k) {
    core::zero_row(wv[k][0]);
    core::zero_row(wv[k][1]);
    core::zero_row(wv[k][2]);
    core::zero_row(gv[k][0]);
    core::zero_row(gv[k][1]);
  }
#pragma unroll
  for (int rr = 0; rr < NR; ++rr) {
    const int r = jb - T + rr;
    if (!ROWS && r > je + T - 1) break;
    if (rr + D < NR) load(rr + D);
    // level 0: the state rows r - 2, r - 1, r
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
      wv[0][2][k] = wv[0][1][k];
      wv[0][1][k] = wv[0][0][k];
      wv[0][0][k] = core::to_c(wl_[rr % RING][k]);
      gv[0][1][k] = gv[0][0][k];
      gv[0][0][k] = core::to_c(gl_[rr % RING][k]);
      // 16-bit rows of sweeps of seven and eight steps: the rest population
      // is converted to FP32 where its row arrives, not folded into the
      // mixed-precision FMAs that use it (FP16 T = 8 holds 179 VGPRs instead
      // of 202; 467 against 496 us per sweep, BF16 T = 7 382 against 428;
      // at T = 6 it gains nothing)
      if constexpr (sizeof(S) == 2 && T >= 7) asm volatile("" : "+v"(gv[0][0][k]));
    }
#pragma unroll
    for (int lv = 1; lv <= T; ++lv) {
      const int q = r - lv;  // the row level lv computes now
      const bool valid = rr >= 2 * lv && (ROWS || (q >= 0 && q < p.ny));
      const bool er = !ROWS && (q == 0 || q == p.ny - 1 || q == jc || q == jc + 1);
      const uint32_t cu = (!ROWS && q == jc) ? cut[lv - 1] : 0u;
      const uint32_t cd = (!ROWS && q == jc + 1) ? cut[lv - 1] : 0u;
      C g2[VEC], w2[VEC];
      if (valid) {
        step_row<S, W, C, VEC>(a, A.lv[lv - 1], q, i0, wv[lv - 1][2], wv[lv - 1][1], wv[lv - 1][0],
                               gv[lv - 1][1], cu, cd, er, !FAST && edge_strip, g2, w2);
      } else {
        core::zero_row(g2);
        core::zero_row(w2);
      }
      if (lv < T) {
        // w of the crack rows after step n + lv - 1, for its crack step
        if (!ROWS && valid && own && (q == jc || q == jc + 1) && q >= jb && q < je)
          core::store_row<W, C, VEC>(A.wmid, (uint32_t)(2 * (lv - 1) + q - jc) * pitch + il, w2);
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
          wv[lv][2][k] = wv[lv][1][k];
          wv[lv][1][k] = wv[lv][0][k];
          wv[lv][0][k] = w2[k];
          gv[lv][1][k] = gv[lv][0][k];
          gv[lv][0][k] = g2[k];
        }
      } else if (rr >= 2 * T && (ROWS || q < je)) {
        // the last level: rows jb .. je - 1, stored
        if (!FAST && i0 + VEC - 1 > p.nx - 1) {
#pragma unroll
          for (int k = 0; k < VEC; ++k)
            if (i0 + k > p.nx - 1) g2[k] = w2[k] = C(0);  // padding stays zero
        }
        const uint32_t o = (uint32_t)q * pitch + il;
        core::Pack<S, VEC> pg;
        if constexpr (SR) {
          uint32_t rd[VEC];
          core::sr_draws0<VEC>(core::sr_pair(q, i0, p.nx), A.rkey_last, rd);
          pg = core::pack_row_sr<S, C, VEC>(g2, rd);
        } else {
          pg = core::pack_row<S, C, VEC>(g2);
        }
        buffer_store_row<S, VEC>(rf, own ? o * (uint32_t)sizeof(S) : kDropOffset, pg);
        buffer_store_row<W, VEC>(rw, own ? o * (uint32_t)sizeof(W) : kDropOffset,
                                 core::pack_row<W, C, VEC>(w2));
      }
    }
  }
}

// Whether a strip's columns include site 0 or site nx - 1, and whether a
// chunk (rows jb .. jb + R - 1) of a strip without such a column takes the
// fast path: every row it loads lies in the plate and none of the rows it
// steps is an edge or crack row.
template <int VEC, int T>
__host__ __device__ inline bool edge_strip_of(int strip, int nx) {
  constexpr int H = (T + VEC - 1) / VEC;
  constexpr int OW = (64 - 2 * H) * VEC;
  return strip == 0 || (strip + 1) * OW + H * VEC - 1 >= nx - 1;
}
template <int R, int T>
__host__ __device__ inline bool fast_rows(int jb, int ny, int jc) {
  return jb >= T && jb + R + T - 1 <= ny - 1 && (jc + 1 < jb - (T - 1) || jc > jb + R + T - 2);
}

// The chunk rows that strips without a plate edge cannot take on the fast
// path (the first and last chunk rows, those around the crack rows), for the
// boundary launch.
constexpr int kMaxSlowChunks = 24;
struct SlowChunks {
  int n;
  int c[kMaxSlowChunks];
};

// The fast launch: strips s_lo .. s_hi - 1 (no plate edge) times every chunk
// row (the slow chunk rows return at once: a few per strip).  Only the fast
// march is compiled in, so the kernel is sized for the registers of that
// path alone (in one kernel with the boundary path every wave was sized for
// the larger of the two).  R rows per wave, a compile-time constant so that
// the row march unrolls and the register windows slide by renaming instead
// of copies.  The waves of a workgroup take neighbouring strips of one chunk
// row.  (Tried: the waves of a workgroup on consecutive chunks of one strip,
// the odd ones marching upwards so that both waves at a chunk boundary read
// the rows around it at the same time: 7 % slower.)
template <typename S, typename W, typename C, int VEC, bool SR, int R, int T>
__global__ void __launch_bounds__(512)
sweep_block(const BlockArgs<S, W, C> A, const int s_lo, const int s_hi, const int n_chunks) {
  if (A.gate && *A.gate == 0) return;  // a sweep queued after a wrong prediction
  const Plate p = A.s0.p;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int task = (int)xcd_contiguous_block() * (int)(blockDim.x >> 6) + wave;
  const int n_int = s_hi - s_lo;
  if (task >= n_int * n_chunks) return;
  const int strip = s_lo + task % n_int;
  const int jb = (task / n_int) * R;
  if (!fast_rows<R, T>(jb, p.ny, A.crack ? p.j0 : -2)) return;
  march<S, W, C, VEC, SR, R, T, true>(A, strip, jb, lane, false);
}

// The runs of consecutive fast chunk rows (at most kMaxRuns: the crack rows
// split the plate in two), cut into groups of G chunks (a run's last chunk
// when its length is odd in G goes to the boundary launch); group g of run k
// (g0[k] <= g < g0[k + 1]) starts at chunk c0[k] + (g - g0[k]) G.
constexpr int kMaxRuns = 4;
struct FastRuns {
  int n, G, n_groups;
  int c0[kMaxRuns], g0[kMaxRuns];
};

// The fast launch with waves of G = RF / R chunks: strips s_lo .. s_hi - 1
// times the groups of fast chunk rows, each wave marching its RF rows in one
// pass (the rows around them are loaded and stepped once per RF rows instead
// of once per R: per 16 rows march loads 16 + 2T rows and steps
// sum_k (16 + 2 (T - k)), i.e. at T = 6 it loads 1.75 and steps 1.31 times
// the rows it finishes, at RF = 32 1.38 and 1.16).  The march stays
// unrolled: RF = 64 overflows the instruction cache (three times slower), and
// as a loop over row blocks the rows loaded ahead for the next pass needed
// register copies at the back edge, or waits for every load and store in
// flight at each row.
template <typename S, typename W, typename C, int VEC, bool SR, int R, int RF, int T>
__global__ void __launch_bounds__(512)
sweep_block_tall(const BlockArgs<S, W, C> A, const int s_lo, const int s_hi, const FastRuns fr) {
  if (A.gate && *A.gate == 0) return;  // a sweep queued after a wrong prediction
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int task = (int)xcd_contiguous_block() * (int)(blockDim.x >> 6) + wave;
  const int n_int = s_hi - s_lo;
  if (task >= n_int * fr.n_groups) return;
  const int strip = s_lo + task % n_int;
  const int g = task / n_int;
  int k = 0;
  while (k + 1 < fr.n && g >= fr.g0[k + 1]) ++k;
  const int c = fr.c0[k] + (g - fr.g0[k]) * (RF / R);
  march<S, W, C, VEC, SR, RF, T, true>(A, strip, c * R, lane, false);
}

// The boundary launch: first the slow chunk rows (the first and last ones,
// those around the crack rows, and the fast ones a run of the fast launch
// leaves over) of every strip, with the general march; then the other chunk
// rows of the strips with a plate edge (strips below s_lo and from s_hi on),
// whose rows are those of a fast chunk, so their march needs the left and
// right edge treatment and range checks on its columns only.  (Taken by the
// general march, these chunks held most of this launch's time: it keeps
// about 180 registers and spills.  As a launch of their own after this one,
// on the same side stream, they cost a launch gap on small plates.)
template <typename S, typename W, typename C, int VEC, bool SR, int R, int T>
__global__ void __launch_bounds__(256)
sweep_block_edges(const BlockArgs<S, W, C> A, const int n_strips, const int s_lo, const int s_hi,
                  const int n_chunks, const SlowChunks sc) {
  if (A.gate && *A.gate == 0) return;
  const Plate p = A.s0.p;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int task = (int)(blockIdx.x * (blockDim.x >> 6)) + wave;
  const int n_slow = n_strips * sc.n;
  if (task < n_slow) {
    const int strip = task % n_strips;
    const int chunk = sc.c[task / n_strips];
    march<S, W, C, VEC, SR, R, T, false>(A, strip, chunk * R, lane,
                                         edge_strip_of<VEC, T>(strip, p.nx));
    return;
  }
  const int t = task - n_slow;
  const int n_edge = n_strips - (s_hi - s_lo);
  if (t >= n_edge * n_chunks) return;
  const int e = t % n_edge;
  const int strip = e < s_lo ? e : s_hi + (e - s_lo);
  const int chunk = t / n_edge;
  if (!fast_rows<R, T>(chunk * R, p.ny, A.crack ? p.j0 : -2)) return;
  for (int k = 0; k < sc.n; ++k)
    if (sc.c[k] == chunk) return;  // a slow chunk row, taken above
  march<S, W, C, VEC, SR, R, T, false, true>(A, strip, chunk * R, lane, true);
}

// RF: rows per wave of the fast launch, R (sweep_block) or a multiple of R
// (sweep_block_tall); the boundary launch takes chunks of R rows.
template <typename S, typename W, typename C, int VEC, bool SR, int R, int RF, int T>
hipError_t block_t(const BlockArgs<S, W, C> &A, int waves, hipStream_t st, const SideStream &ss) {
  constexpr int H = (T + VEC - 1) / VEC;
  constexpr int OW = (64 - 2 * H) * VEC;
  constexpr int G = RF / R;
  static_assert(RF % R == 0, "a fast wave takes whole chunks");
  const Plate &p = A.s0.p;
  const int n_strips = (p.nx + OW - 1) / OW;
  const int n_chunks = (p.ny + R - 1) / R;
  // the strips without a plate edge, s_lo .. s_hi - 1 (the edge strips are
  // strip 0 and a suffix)
  const int s_lo = std::min(1, n_strips);
  int s_hi = n_strips;
  while (s_hi > s_lo && edge_strip_of<VEC, T>(s_hi - 1, p.nx)) --s_hi;
  // their slow chunk rows: the first and last ones and those around the
  // crack rows (every chunk row outside these ranges is fast)
  SlowChunks sc{};
  const int jc = A.crack ? p.j0 : -2;
  bool ok = true;
  auto add = [&](int c, bool fast_too) {
    if (c < 0 || c >= n_chunks || (!fast_too && fast_rows<R, T>(c * R, p.ny, jc))) return;
    for (int k = 0; k < sc.n; ++k)
      if (sc.c[k] == c) return;
    if (sc.n == kMaxSlowChunks) {
      ok = false;
      return;
    }
    sc.c[sc.n++] = c;
  };
  for (int c = 0; c <= T / R + 1; ++c) {
    add(c, false);
    add(n_chunks - 1 - c, false);
  }
  if (A.crack)
    for (int c = (jc - R - T) / R - 1; c <= (jc + T) / R + 1; ++c) add(c, false);
  // the runs of fast chunk rows, in groups of G (the last chunks of a run
  // that do not fill a group go to the boundary launch)
  FastRuns fr{};
  fr.G = G;
  if constexpr (G > 1) {
    for (int c = 0; c < n_chunks && ok;) {
      if (!fast_rows<R, T>(c * R, p.ny, jc)) {
        ++c;
        continue;
      }
      int e = c;
      while (e < n_chunks && fast_rows<R, T>(e * R, p.ny, jc)) ++e;
      const int groups = (e - c) / G;
      if (groups > 0) {
        if (fr.n == kMaxRuns) {
          ok = false;
          break;
        }
        fr.c0[fr.n] = c;
        fr.g0[fr.n] = fr.n_groups;
        fr.n_groups += groups;
        fr.n++;
      }
      for (int k = c + groups * G; k < e; ++k) add(k, true);
      c = e;
    }
  }
  if (!ok) return hipErrorInvalidValue;
  // the boundary launch goes first, on the side stream, so that its few
  // long waves run beside the fast launch instead of after it
  // (always there when a side stream exists: the crack steps of the previous
  // sweep may still run on it, and only the boundary launch reads what they
  // write)
  const long etasks = (long)n_strips * sc.n + (long)(n_strips - (s_hi - s_lo)) * n_chunks;
  const bool fork = ss.side != nullptr && etasks > 0;
  hipStream_t est = fork ? ss.side : st;
  if (fork) {
    hipError_t e = hipEventRecord(ss.fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(ss.side, ss.fork, 0);
    if (e != hipSuccess) return e;
  }
  if (etasks > 0) {
    const unsigned blocks = (unsigned)((etasks + 3) / 4);
    hipLaunchKernelGGL((sweep_block_edges<S, W, C, VEC, SR, R, T>), dim3(blocks), dim3(256), 0, est,
                       A, n_strips, s_lo, s_hi, n_chunks, sc);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  // dynamic LDS only to cap the resident waves (s0.lds_bytes, 0 = no cap)
  if constexpr (G > 1) {
    if (s_hi > s_lo && fr.n_groups > 0) {
      const long tasks = (long)(s_hi - s_lo) * fr.n_groups;
      const unsigned blocks = (unsigned)((tasks + waves - 1) / waves);
      hipLaunchKernelGGL((sweep_block_tall<S, W, C, VEC, SR, R, RF, T>), dim3(blocks),
                         dim3(64 * waves), (unsigned)A.s0.lds_bytes, st, A, s_lo, s_hi, fr);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  } else {
    if (s_hi > s_lo) {
      const long tasks = (long)(s_hi - s_lo) * n_chunks;
      const unsigned blocks = (unsigned)((tasks + waves - 1) / waves);
      hipLaunchKernelGGL((sweep_block<S, W, C, VEC, SR, R, T>), dim3(blocks), dim3(64 * waves),
                         (unsigned)A.s0.lds_bytes, st, A, s_lo, s_hi, n_chunks);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  if (fork) {
    hipError_t e = hipEventRecord(ss.join, ss.side);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, ss.join, 0);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// rows 4, 8 or 16 (T >= 6: 16 or more; shorter chunks would recompute their
// halo levels more often than they advance their own rows), or 32 for the
// fast launch (chunks of 16 rows, two per wave; the boundary launch keeps 16)
template <typename S, typename W, typename C, int VEC, bool SR, int T>
hipError_t block_rows(const BlockArgs<S, W, C> &A, int rows, int waves, hipStream_t st,
                      const SideStream &ss) {
  switch (rows) {
    case 4:
      if constexpr (T <= 5) return block_t<S, W, C, VEC, SR, 4, 4, T>(A, waves, st, ss);
      return hipErrorInvalidValue;
    case 8:
      if constexpr (T <= 5) return block_t<S, W, C, VEC, SR, 8, 8, T>(A, waves, st, ss);
      return hipErrorInvalidValue;
    case 16: return block_t<S, W, C, VEC, SR, 16, 16, T>(A, waves, st, ss);
    case 24:
      if constexpr (T >= 6) return block_t<S, W, C, VEC, SR, 8, 24, T>(A, waves, st, ss);
      return hipErrorInvalidValue;
    case 32: return block_t<S, W, C, VEC, SR, 16, 32, T>(A, waves, st, ss);
    default: return hipErrorInvalidValue;
  }
}

// T = TLO .. THI only (a translation unit may hold some of the step counts,
// built with other compiler limits)
template <typename S, typename W, typename C, int VEC, bool SR, int TLO, int THI>
hipError_t block_steps(const BlockArgs<S, W, C> &A, int rows, int waves, hipStream_t st,
                       const SideStream &ss) {
  const int T = A.steps;
  if (T < TLO || T > THI) return hipErrorInvalidValue;
  switch (T) {
    case 2: if constexpr (TLO <= 2 && 2 <= THI) return block_rows<S, W, C, VEC, SR, 2>(A, rows, waves, st, ss); break;
    case 3: if constexpr (TLO <= 3 && 3 <= THI) return block_rows<S, W, C, VEC, SR, 3>(A, rows, waves, st, ss); break;
    case 4: if constexpr (TLO <= 4 && 4 <= THI) return block_rows<S, W, C, VEC, SR, 4>(A, rows, waves, st, ss); break;
    case 5: if constexpr (TLO <= 5 && 5 <= THI) return block_rows<S, W, C, VEC, SR, 5>(A, rows, waves, st, ss); break;
    case 6: if constexpr (TLO <= 6 && 6 <= THI) return block_rows<S, W, C, VEC, SR, 6>(A, rows, waves, st, ss); break;
    case 7: if constexpr (TLO <= 7 && 7 <= THI) return block_rows<S, W, C, VEC, SR, 7>(A, rows, waves, st, ss); break;
    case 8: if constexpr (TLO <= 8 && 8 <= THI) return block_rows<S, W, C, VEC, SR, 8>(A, rows, waves, st, ss); break;
    default: break;
  }
  return hipErrorInvalidValue;
}

template <typename S, typename W, typename C, int VEC, int TLO = 2, int THI = kMaxTimeBlock>
hipError_t block_r(const void *args, int rows, int waves, hipStream_t st, const SideStream &ss) {
  const auto &A = *static_cast<const BlockArgs<S, W, C> *>(args);
  if constexpr (sizeof(S) == 2) {
    if (A.s0.sr) return block_steps<S, W, C, VEC, true, TLO, THI>(A, rows, waves, st, ss);
  }
  return block_steps<S, W, C, VEC, false, TLO, THI>(A, rows, waves, st, ss);
}

}  // namespace blk
}  // namespace lbmk
