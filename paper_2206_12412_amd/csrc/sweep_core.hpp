// Device building blocks of the fused collide-stream sweep (gfx950), shared
// by the single-plate kernels (sweep.hip) and the batched kernels (batch.hip).
//
// One step updates every site (paper Sec. 3): pull-stream with bounce-back on
// severed or outside links (eq. LBE, streaming part; Sec. 4.1 "no information
// is exchanged" along a severed link), wdot = sum of the populations
// (eq. distrib-macro), w += dt wdot (eq. integration), BGK collision towards
// f_eq(w, wdot) (eq. LBE, f-eq).
//
// Layout: populations structure-of-arrays, plane a at fin + a * plane, rows of
// `pitch` elements (multiple of 64, 256-byte aligned); w in its own plane;
// populations and w are double-buffered (source -> destination).  In-plane
// byte offsets are 32-bit (a plane spans < 4 GiB) and every plane base is
// wave-uniform, so loads and stores can use the scalar-base addressing mode.
//
// Work split: a wave owns a strip of 64 * VEC consecutive sites of a row; lane
// l holds sites i0 .. i0 + VEC - 1, i0 = strip * 64 * VEC + l * VEC, so every
// plane row is read and written with one 16-byte (8-byte for 16-bit storage)
// access per lane.  x-neighbours across lanes come from DPP wave shifts
// (v_mov_b32_dpp wave_shr / wave_shl); the strip-edge elements come from one
// per-row halo load whose lanes 0..2 carry them (read back with readlane).
//
// Interior rows (every vertical link intact) and boundary rows (plate edges,
// crack rows) are separate work items with separate code, so the interior
// code carries no bounce-back logic and few registers.
//
// EQ (equilibrium layout, shifted storage only): at omega = dt / tau = 1 (the
// paper's tau = dt, the only stable choice) the collision returns every
// population to its equilibrium, so the shifted moving populations g^1..g^4 =
// f^k - Ak w_emit of every reachable state are exactly zero and each pulled
// population is rebuilt from the w of its emitting site.  The sweep then reads
// and writes plane 0 and w only (the moving planes keep their zeros); the
// arithmetic is the same with the g^k terms dropped.
#pragma once

#include <algorithm>

#include "lbm_internal.hpp"

namespace lbmk {
namespace core {

template <typename S, int N>
struct alignas(N * sizeof(S)) Pack {
  S v[N];
};

__device__ __forceinline__ float to_c(float x) { return x; }
__device__ __forceinline__ double to_c(double x) { return x; }
__device__ __forceinline__ float to_c(_Float16 x) { return static_cast<float>(x); }
__device__ __forceinline__ float to_c(__bf16 x) { return static_cast<float>(x); }

template <typename S> __device__ __forceinline__ S from_c(float x);
template <> __device__ __forceinline__ float from_c<float>(float x) { return x; }
template <> __device__ __forceinline__ _Float16 from_c<_Float16>(float x) { return static_cast<_Float16>(x); }
template <> __device__ __forceinline__ __bf16 from_c<__bf16>(float x) { return static_cast<__bf16>(x); }
template <typename S> __device__ __forceinline__ S from_c(double x);
template <> __device__ __forceinline__ double from_c<double>(double x) { return x; }

// Lane l receives the value of lane l-1 (lane 0 receives 0).
__device__ __forceinline__ float lane_prev(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x138, 0xf, 0xf, false));
}
// Lane l receives the value of lane l+1 (lane 63 receives 0).
__device__ __forceinline__ float lane_next(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ double lane_prev(double x) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  lo = __builtin_amdgcn_update_dpp(0, lo, 0x138, 0xf, 0xf, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, 0x138, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_next(double x) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  lo = __builtin_amdgcn_update_dpp(0, lo, 0x130, 0xf, 0xf, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, 0x130, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
// Value of lane k, broadcast (k is a compile-time constant here).
__device__ __forceinline__ float lane_value(float x, int k) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), k));
}
__device__ __forceinline__ double lane_value(double x, int k) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), k);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), k);
  return __hiloint2double(hi, lo);
}

// base + off with the byte offset formed in 32 bits (a plane spans < 4 GiB), so
// that a uniform base and a 32-bit per-lane offset address the access
template <typename S>
__device__ __forceinline__ const S *at(const S *base, uint32_t off) {
  return reinterpret_cast<const S *>(reinterpret_cast<const char *>(base) + off * (uint32_t)sizeof(S));
}
template <typename S>
__device__ __forceinline__ S *at(S *base, uint32_t off) {
  return reinterpret_cast<S *>(reinterpret_cast<char *>(base) + off * (uint32_t)sizeof(S));
}

template <typename S, typename C, int VEC>
__device__ __forceinline__ void load_row(const S *__restrict__ base, uint32_t off, C (&out)[VEC]) {
  const Pack<S, VEC> pk = *reinterpret_cast<const Pack<S, VEC> *>(at(base, off));
#pragma unroll
  for (int k = 0; k < VEC; ++k) out[k] = to_c(pk.v[k]);
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Rows are written once per step and read back only in the next step, after
// the whole plate has streamed through the caches: store them non-temporally.
template <typename S, typename C, int VEC>
__device__ __forceinline__ void store_row(S *__restrict__ base, uint32_t off, const C (&in)[VEC]) {
  Pack<S, VEC> pk;
#pragma unroll
  for (int k = 0; k < VEC; ++k) pk.v[k] = from_c<S>(in[k]);
  S *ptr = at(base, off);
  if constexpr (sizeof(pk) % 16 == 0) {
#pragma unroll
    for (int c = 0; c < (int)(sizeof(pk) / 16); ++c) {
      u32x4 v;
      __builtin_memcpy(&v, reinterpret_cast<const char *>(&pk) + 16 * c, 16);
      __builtin_nontemporal_store(v, reinterpret_cast<u32x4 *>(ptr) + c);
    }
  } else {
    static_assert(sizeof(pk) == 8, "rows are stored in 8- or 16-byte pieces");
    u32x2 v;
    __builtin_memcpy(&v, &pk, 8);
    __builtin_nontemporal_store(v, reinterpret_cast<u32x2 *>(ptr));
  }
}

// Stochastic rounding to 16 bits with random bits r (FP16 uses the low 13,
// BF16 all 16): adding them to the FP32 bit pattern, at the width of the
// mantissa field the conversion drops, and truncating rounds the magnitude up
// with probability (dropped part) / (16-bit ulp), which makes the rounding
// unbiased at FP32 resolution.  Below the smallest FP16 normal (abs(x) <
// 2^-14, fixed ulp 2^-24) x is first moved by c = +-2^-14 into the binade
// [2^-14, 2^-13), where the FP32 bit 13 is worth 2^-24 as well, and moved back
// after the truncation (exact).
template <typename S> __device__ __forceinline__ S round_sr(float x, uint32_t r);
template <> __device__ __forceinline__ _Float16 round_sr<_Float16>(float x, uint32_t r) {
  const float c = (__builtin_fabsf(x) < 0x1p-14f) ? __builtin_copysignf(0x1p-14f, x) : 0.0f;
  const uint32_t b = (__float_as_uint(x + c) + (r & 0x1fffu)) & 0xffffe000u;
  return static_cast<_Float16>(__uint_as_float(b) - c);  // exact
}
template <> __device__ __forceinline__ __bf16 round_sr<__bf16>(float x, uint32_t r) {
  const uint32_t b = (__float_as_uint(x) + (r & 0xffffu)) & 0xffff0000u;
  return static_cast<__bf16>(__uint_as_float(b));  // exact
}

template <typename S, typename C, int VEC>
__device__ __forceinline__ Pack<S, VEC> pack_row(const C (&in)[VEC]) {
  Pack<S, VEC> pk;
#pragma unroll
  for (int k = 0; k < VEC; ++k) pk.v[k] = from_c<S>(in[k]);
  return pk;
}
template <typename S, typename C, int VEC>
__device__ __forceinline__ Pack<S, VEC> pack_row_sr(const C (&in)[VEC], const uint32_t (&r)[VEC]) {
  Pack<S, VEC> pk;
#pragma unroll
  for (int k = 0; k < VEC; ++k) pk.v[k] = round_sr<S>(in[k], r[k]);
  return pk;
}

template <typename S, typename C, int VEC>
__device__ __forceinline__ void store_row_sr(S *__restrict__ base, uint32_t off, const C (&in)[VEC],
                                             const uint32_t (&r)[VEC]) {
  const Pack<S, VEC> pk = pack_row_sr<S, C, VEC>(in, r);
  static_assert(sizeof(pk) == 8, "16-bit rows are stored in 8-byte pieces");
  u32x2 v;
  __builtin_memcpy(&v, &pk, 8);
  __builtin_nontemporal_store(v, reinterpret_cast<u32x2 *>(at(base, off)));
}

// The rounding draws.  One 32-bit hash serves two horizontally adjacent sites
// (i even and i + 1 of one row) of one plane: the even site takes bits 0..15,
// the odd site bits 16..31.  The pairs of a plate are numbered row by row,
// pair = j * ceil(nx / 2) + i / 2; plane 0's hash of a pair is
// mix32(pair ^ rkey), plane a's is mix32(plane a - 1's ^ kPlaneSalt).
constexpr uint32_t kPlaneSalt = 0x68e31da4u;
__host__ __device__ inline uint32_t sr_pair(uint32_t j, uint32_t i, uint32_t nx) {
  return j * ((nx + 1u) >> 1) + (i >> 1);
}
__device__ __forceinline__ uint32_t sr_half(uint32_t h, uint32_t odd) {
  return odd ? (h >> 16) : (h & 0xffffu);
}
// plane 0's draws of the VEC sites of a lane (pair0: the pair of its first site)
template <int VEC>
__device__ __forceinline__ void sr_draws0(uint32_t pair0, uint32_t rkey, uint32_t (&r)[VEC]) {
  static_assert(VEC % 2 == 0, "rounding draws come in pairs of sites");
#pragma unroll
  for (int k = 0; k < VEC / 2; ++k) {
    const uint32_t h = mix32((pair0 + k) ^ rkey);
    r[2 * k] = sr_half(h, 0u);
    r[2 * k + 1] = sr_half(h, 1u);
  }
}

// The five population rows of a lane's sites (pair0 = the rounding pair of
// the lane's first site, whose column is even); in the equilibrium layout
// plane 0 only, with the same rounding draws as plane 0 of the five-plane
// store.
template <typename S, typename C, int VEC, bool SR, bool EQ = false>
__device__ __forceinline__ void store_pops(S *__restrict__ fout, size_t P, uint32_t o,
                                           const C (&o0)[VEC], const C (&o1)[VEC],
                                           const C (&o2)[VEC], const C (&o3)[VEC],
                                           const C (&o4)[VEC], uint32_t pair0, uint32_t rkey) {
  if constexpr (SR) {
    static_assert(VEC % 2 == 0, "rounding draws come in pairs of sites");
    uint32_t h[VEC / 2], r[VEC];
#pragma unroll
    for (int k = 0; k < VEC / 2; ++k) h[k] = mix32((pair0 + k) ^ rkey);
#pragma unroll
    for (int a = 0; a < (EQ ? 1 : 5); ++a) {
      if (a > 0) {
#pragma unroll
        for (int k = 0; k < VEC / 2; ++k) h[k] = mix32(h[k] ^ kPlaneSalt);
      }
#pragma unroll
      for (int k = 0; k < VEC; ++k) r[k] = sr_half(h[k >> 1], k & 1);
      const C(&oa)[VEC] = a == 0 ? o0 : a == 1 ? o1 : a == 2 ? o2 : a == 3 ? o3 : o4;
      store_row_sr<S, C, VEC>(fout + a * P, o, oa, r);
    }
  } else if constexpr (EQ) {
    store_row<S, C, VEC>(fout, o, o0);
  } else {
    store_row<S, C, VEC>(fout, o, o0);
    store_row<S, C, VEC>(fout + P, o, o1);
    store_row<S, C, VEC>(fout + 2 * P, o, o2);
    store_row<S, C, VEC>(fout + 3 * P, o, o3);
    store_row<S, C, VEC>(fout + 4 * P, o, o4);
  }
}

template <typename C, int VEC>
__device__ __forceinline__ void zero_row(C (&out)[VEC]) {
#pragma unroll
  for (int k = 0; k < VEC; ++k) out[k] = C(0);
}

__device__ __forceinline__ bool in_range(int j, int lo, int hi) { return j >= lo && j <= hi; }

constexpr int kEdgeBottom = 1, kEdgeTop = 2, kEdgeLeft = 4, kEdgeRight = 8;

// 2 f_eq^k(w*, 0) = (2 Ak) w*, the constant of the anti-bounce-back of a
// Dirichlet edge (stored populations f; shifted storage carries it in w_src)
template <typename A, typename C>
__device__ __forceinline__ C dirichlet_term(const A &a, C wstar) {
#pragma clang fp contract(off)
  return (C(2) * a.Ak) * wstar;
}

// One site: wdot, Euler update and collision from the pulled populations.
// gl, gr, gd, gu are the values pulled along +x, -x, +y, -y (already bounced
// where the link is severed); for shifted storage wl .. wup are the w of the
// emitting sites (w0 where bounced); bd / bu say that the +y / -y pull bounced
// and then carries the traction term td / tu.
//
// SHIFT = false: the stored values are the post-collision populations f
// themselves (FP64 and plain FP32), evaluated in the paper's order of
// operations without contraction.  SHIFT = true: the stored values are
// g = f - E(w_emit), E the static equilibrium (E^0 = -A0 w, E^k = Ak w) of
// the emitting site; wdot and the collision are the same arithmetic regrouped
// in these variables so that no large term cancels in FP32 (A0 = 4 Ak).
//
// The five-point difference is written with the forward differences of the
// row and of the column, (wr - w0) - (w0 - wl) and (wup - w0) - (w0 - wdn):
// a site's (w0 - wl) is bit for bit its left neighbour's (wr - w0), and its
// (w0 - wdn) the lower neighbour's (wup - w0), so a sweep computes one new
// difference per direction and site.  A traction term is added only where a
// link bounced (it is zero elsewhere).
template <typename C>
__device__ __forceinline__ C lap5(C w0, C wl, C wr, C wdn, C wup) {
  return ((wr - w0) - (w0 - wl)) + ((wup - w0) - (w0 - wdn));
}

template <typename C, bool SHIFT, bool EQ = false, typename A>
__device__ __forceinline__ void site_update(const A &a, C f0, C gl, C gr, C gd, C gu, C w0, C wl,
                                            C wr, C wdn, C wup, bool bd, bool bu, C td, C tu,
                                            C &o0, C &o1, C &o2, C &o3, C &o4, C &wo) {
  static_assert(SHIFT || !EQ, "the equilibrium layout is a shifted layout");
  if constexpr (EQ) {
    // g^1..g^4 = 0: the five-plane expression below without them; at
    // omega = 1 the relaxed shifted rest population is wdot itself
#pragma clang fp contract(fast)
    C wd = f0 + a.Ak * lap5(w0, wl, wr, wdn, wup);
    if (bd || bu) wd = wd + (td + tu);
    o0 = wd;
    o1 = o2 = o3 = o4 = C(0);
    wo = w0 + a.dt * wd;
  } else if constexpr (SHIFT) {
#pragma clang fp contract(fast)
    C wd = f0 + ((gl + gr) + (gd + gu)) + a.Ak * lap5(w0, wl, wr, wdn, wup);
    if (bd || bu) wd = wd + (td + tu);
    const C wn = w0 + a.dt * wd;
    const C om1 = C(1) - a.omega;
    o0 = om1 * (f0 + a.A0 * (wn - w0)) + a.omega * wd;
    o1 = om1 * (gl + a.Ak * (wl - wn));
    o2 = om1 * (gd + a.Ak * (wdn - wn) + td);
    o3 = om1 * (gr + a.Ak * (wr - wn));
    o4 = om1 * (gu + a.Ak * (wup - wn) + tu);
    wo = wn;
  } else {
#pragma clang fp contract(off)
    const C fi2 = bd ? gd + td : gd;
    const C fi4 = bu ? gu + tu : gu;
    const C wd = f0 + gl + fi2 + gr + fi4;
    const C wn = w0 + a.dt * wd;
    const C e0 = wd - a.A0 * wn;
    const C ek = a.Ak * wn;
    o0 = f0 - a.omega * (f0 - e0);
    o1 = gl - a.omega * (gl - ek);
    o2 = fi2 - a.omega * (fi2 - ek);
    o3 = gr - a.omega * (gr - ek);
    o4 = fi4 - a.omega * (fi4 - ek);
    wo = wn;
  }
}

// ------------------------------------------------------------- task maps --
// (the task maps, InteriorMap and BoundaryMap, are in lbm_internal.hpp: the
// host builds them for the batched descriptors too)

// ----------------------------------------------------------------- interior --
// Rows jb .. jlast of one strip, all of them interior rows (every vertical
// link intact); the left and right plate edges (or the periodic wrap) and the
// ragged end of the last strip are per-lane fix-ups.
template <typename S, typename W, typename C, int VEC, bool SHIFT, bool SR = false, bool EQ = false>
__device__ __forceinline__ void interior_rows(const S *__restrict__ fin, S *__restrict__ fout,
                                              const W *__restrict__ win, W *__restrict__ wout,
                                              const SweepArgs<S, W, C> &a, const int strip,
                                              const int jb, const int jlast) {
  const Plate p = a.p;
  const int lane = threadIdx.x & 63;
  constexpr int SW = 64 * VEC;
  const int last = p.nx - 1;
  const int is = strip * SW;
  const int i0 = is + lane * VEC;
  const bool act = i0 < p.nx;
  const uint32_t il = act ? i0 : is;  // inactive lanes read their strip's first vector
  const bool left_edge = strip == 0;          // holds site 0
  const bool right_edge = is + SW > last;     // holds site nx-1 (and maybe padding)
  const uint32_t pitch = p.pitch;
  const size_t P = p.plane;
  const S *__restrict__ F0 = fin;
  const S *__restrict__ F1 = fin + P;
  const S *__restrict__ F2 = fin + 2 * P;
  const S *__restrict__ F3 = fin + 3 * P;
  const S *__restrict__ F4 = fin + 4 * P;
  // halo: lane 0 the site left of the strip (plane 1; the periodic wrap for
  // the first strip), lane 1 the site right of it (plane 3), lane 2 site 0
  // (plane 3: the periodic neighbour of the last site)
  const S *__restrict__ Fh = (lane == 0) ? F1 : F3;
  const uint32_t hx = (lane == 0) ? (is > 0 ? is - 1 : (p.periodic ? last : 0))
                                  : (lane == 1 && is + SW <= last ? is + SW : 0);

  C wm[VEC], wc[VEC];
  if (SHIFT) {
    load_row<W, C, VEC>(win, (uint32_t)jb * pitch + il, wc);
    load_row<W, C, VEC>(win, (uint32_t)(jb - 1) * pitch + il, wm);
  }
  for (int j = jb; j <= jlast; ++j) {
    const uint32_t o = (uint32_t)j * pitch + il;
    C f0[VEC], f1[VEC], f3[VEC], f2d[VEC], f4u[VEC], wp[VEC], wself[VEC];
    load_row<S, C, VEC>(F0, o, f0);
    if constexpr (EQ) {  // the moving planes hold zeros: not read
      zero_row(f1);
      zero_row(f3);
      zero_row(f2d);
      zero_row(f4u);
    } else {
      load_row<S, C, VEC>(F1, o, f1);
      load_row<S, C, VEC>(F3, o, f3);
      load_row<S, C, VEC>(F2, o - pitch, f2d);
      load_row<S, C, VEC>(F4, o + pitch, f4u);
    }
    if (SHIFT) load_row<W, C, VEC>(win, o + pitch, wp);
    else load_row<W, C, VEC>(win, o, wself);
    const uint32_t ho = (uint32_t)j * pitch + hx;
    C hs = C(0);
    if constexpr (!EQ) hs = to_c(*at(Fh, ho));
    C hw = C(0);
    if (SHIFT) hw = to_c(*at(win, ho));

    // pulled x-neighbours of every site: gl[k] along +x, gr[k] along -x
    C gl[VEC], gr[VEC], wl[VEC], wr[VEC];
    {
      if constexpr (EQ) {
        zero_row(gl);
        zero_row(gr);
      } else {
        const C f1L = lane_prev(f1[VEC - 1]);
        const C f3R = lane_next(f3[0]);
        const C s_left = lane_value(hs, 0), s_right = lane_value(hs, 1);
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
          gl[k] = (k == 0) ? ((lane == 0) ? s_left : f1L) : f1[k - 1];
          gr[k] = (k == VEC - 1) ? ((lane == 63) ? s_right : f3R) : f3[k + 1];
        }
      }
      if (SHIFT) {
        const C wL = lane_prev(wc[VEC - 1]);
        const C wR = lane_next(wc[0]);
        const C w_left = lane_value(hw, 0), w_right = lane_value(hw, 1);
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
          wl[k] = (k == 0) ? ((lane == 0) ? w_left : wL) : wc[k - 1];
          wr[k] = (k == VEC - 1) ? ((lane == 63) ? w_right : wR) : wc[k + 1];
        }
      }
      // the left edge bounces site 0 (or wraps to nx-1, which the halo holds);
      // a Dirichlet edge anti-bounces: f_in = -f^opp + 2 Ak w*, i.e. the
      // ghost site carries 2 w* - w (shifted storage: g = -g^opp, w_src = 2 w* - w)
      if (left_edge && !p.periodic && lane == 0) {
        const C w0 = SHIFT ? wc[0] : wself[0];
        if (a.dmask & kEdgeLeft) {
          gl[0] = SHIFT ? -f3[0] : -f3[0] + dirichlet_term(a, a.wD_left);
          if (SHIFT) wl[0] = C(2) * a.wD_left - w0;
        } else {
          gl[0] = f3[0];
          if (SHIFT) wl[0] = w0;
        }
      }
      // the right edge bounces site nx-1 or wraps to site 0
      if (right_edge) {
        const C s_wrap = EQ ? C(0) : lane_value(hs, 2);
        const C w_wrap = SHIFT ? lane_value(hw, 2) : C(0);
        const bool dr = !p.periodic && (a.dmask & kEdgeRight);
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
          if (i0 + k == last) {
            const C w0 = SHIFT ? wc[k] : wself[k];
            if (dr) {
              gr[k] = SHIFT ? -f1[k] : -f1[k] + dirichlet_term(a, a.wD_right);
              if (SHIFT) wr[k] = C(2) * a.wD_right - w0;
            } else {
              gr[k] = p.periodic ? s_wrap : f1[k];
              if (SHIFT) wr[k] = p.periodic ? w_wrap : w0;
            }
          }
        }
      }
    }

    C o0[VEC], o1[VEC], o2[VEC], o3[VEC], o4[VEC], wo[VEC];
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
      const C w0 = SHIFT ? wc[k] : wself[k];
      const C wdn = SHIFT ? wm[k] : w0;
      const C wup = SHIFT ? wp[k] : w0;
      site_update<C, SHIFT, EQ>(a, f0[k], gl[k], gr[k], f2d[k], f4u[k], w0, SHIFT ? wl[k] : w0,
                            SHIFT ? wr[k] : w0, wdn, wup, false, false, C(0), C(0), o0[k], o1[k],
                            o2[k], o3[k], o4[k], wo[k]);
    }
    if (right_edge) {
#pragma unroll
      for (int k = 0; k < VEC; ++k)
        if (i0 + k > last) o0[k] = o1[k] = o2[k] = o3[k] = o4[k] = wo[k] = C(0);
    }
    if (act) {
      store_pops<S, C, VEC, SR, EQ>(fout, P, o, o0, o1, o2, o3, o4, sr_pair(j, i0, p.nx), a.rkey);
      store_row<W, C, VEC>(wout, o, wo);
    }
    if (SHIFT) {
#pragma unroll
      for (int k = 0; k < VEC; ++k) {
        wm[k] = wc[k];
        wc[k] = wp[k];
      }
    }
  }
}

// ----------------------------------------------------------------- boundary --
// Row j of one strip with the full boundary treatment: bounce-back at the
// plate edges and on severed links (read from the cut bitmask in the rows the
// mask-row range names), traction terms, periodic wrap-around.
// The vertical links of one lattice row (links (i, row)-(i, row + 1)) that a
// crack step running beside the sweep in the same launch severs: columns
// lo_r..hi_r and lo_l..hi_l (lo > hi: none).  row < 0: no such crack step.
struct CutForecast {
  int row = -1;
  int lo_r = 1, hi_r = 0, lo_l = 1, hi_l = 0;

  // bit k: the link of column i + k in link row r is among them
  template <int VEC>
  __device__ __forceinline__ uint32_t bits(int r, uint32_t i) const {
    if (r != row) return 0u;
    uint32_t b = 0u;
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
      const int c = (int)i + k;
      if ((c >= lo_r && c <= hi_r) || (c >= lo_l && c <= hi_l)) b |= 1u << k;
    }
    return b;
  }
};

template <typename S, typename W, typename C, int VEC, bool SHIFT, bool SR = false, bool EQ = false>
__device__ __forceinline__ void boundary_row(const S *__restrict__ fin, S *__restrict__ fout,
                                             const W *__restrict__ win, W *__restrict__ wout,
                                             const uint32_t *__restrict__ mV,
                                             const uint32_t *__restrict__ mH,
                                             const MaskRows *__restrict__ mrows,
                                             const SweepArgs<S, W, C> &a, const int strip,
                                             const int j, const CutForecast &cf = CutForecast{}) {
  const Plate p = a.p;
  const int lane = threadIdx.x & 63;
  constexpr int SW = 64 * VEC;
  const int is = strip * SW;
  const int i0 = is + lane * VEC;
  const bool act = i0 < p.nx;
  const uint32_t il = act ? i0 : is;  // inactive lanes read their strip's first vector
  const int last = p.nx - 1;
  const uint32_t pitch = p.pitch;
  const size_t P = p.plane;
  MaskRows mr = *mrows;
  if (cf.row >= 0) {  // the forecast row counts as a row with severed links
    if (mr.vlo > mr.vhi) {
      mr.vlo = mr.vhi = cf.row;
    } else {
      mr.vlo = min(mr.vlo, cf.row);
      mr.vhi = max(mr.vhi, cf.row);
    }
  }
  const int jm = j > 0 ? j - 1 : (p.periodic ? p.ny - 1 : -1);
  const int jp = j < p.ny - 1 ? j + 1 : (p.periodic ? 0 : -1);
  const uint32_t o = (uint32_t)j * pitch + il;
  const uint32_t rj = (uint32_t)j * pitch;

  C f0[VEC], f1[VEC], f3[VEC], f2d[VEC], f4u[VEC], f2own[VEC], f4own[VEC];
  C wc[VEC], wm[VEC], wp[VEC];
  // (equilibrium layout: the moving planes hold zeros and are not read)
  load_row<S, C, VEC>(fin, o, f0);
  if (!EQ) load_row<S, C, VEC>(fin + P, o, f1);
  else zero_row(f1);
  if (!EQ) load_row<S, C, VEC>(fin + 3 * P, o, f3);
  else zero_row(f3);
  load_row<W, C, VEC>(win, o, wc);
  if (jm >= 0) {
    if (!EQ) load_row<S, C, VEC>(fin + 2 * P, (uint32_t)jm * pitch + il, f2d);
    else zero_row(f2d);
    if (SHIFT) load_row<W, C, VEC>(win, (uint32_t)jm * pitch + il, wm);
    else zero_row(wm);
  } else {
    zero_row(f2d);
    zero_row(wm);
  }
  if (jp >= 0) {
    if (!EQ) load_row<S, C, VEC>(fin + 4 * P, (uint32_t)jp * pitch + il, f4u);
    else zero_row(f4u);
    if (SHIFT) load_row<W, C, VEC>(win, (uint32_t)jp * pitch + il, wp);
    else zero_row(wp);
  } else {
    zero_row(f4u);
    zero_row(wp);
  }
  // own-row f^2 / f^4 for the bounced vertical pulls
  const bool up_mask = in_range(j, mr.vlo, mr.vhi);
  const bool dn_mask = jm >= 0 && in_range(jm, mr.vlo, mr.vhi);
  if (!EQ && (jp < 0 || up_mask)) load_row<S, C, VEC>(fin + 2 * P, o, f2own);
  else zero_row(f2own);
  if (!EQ && (jm < 0 || dn_mask)) load_row<S, C, VEC>(fin + 4 * P, o, f4own);
  else zero_row(f4own);
  // halo: lane 0 left of the strip (or the periodic wrap), lane 1 right of
  // the strip, lane 2 site 0 (the periodic neighbour of the last site)
  const int hl = is > 0 ? is - 1 : (p.periodic ? last : 0);
  const int hr = is + SW <= last ? is + SW : 0;
  const uint32_t hx = (lane == 0) ? hl : (lane == 1 ? hr : 0);
  const S *__restrict__ Fh = (lane == 0) ? fin + P : fin + 3 * P;
  const C hs = EQ ? C(0) : to_c(*at(Fh, rj + hx));
  const C hw = to_c(*at(win, rj + hx));
  // severed-link bits of the lane's sites (bit k = site i0 + k)
  const uint32_t lanebits = (1u << VEC) - 1u;
  uint32_t bup = 0u, bdn = 0u, bri = 0u, ble = 0u;
  if (up_mask) bup = ((mV[(size_t)j * p.mw + (il >> 5)] >> (il & 31)) | cf.bits<VEC>(j, il)) & lanebits;
  if (dn_mask) bdn = ((mV[(size_t)jm * p.mw + (il >> 5)] >> (il & 31)) | cf.bits<VEC>(jm, il)) & lanebits;
  if (in_range(j, mr.hlo, mr.hhi)) {
    const uint32_t *h = mH + (size_t)j * p.mw;
    bri = (h[il >> 5] >> (il & 31)) & lanebits;
    const int ilm = il > 0 ? (int)il - 1 : (p.periodic ? last : -1);
    const uint32_t l0 = ilm >= 0 ? (h[ilm >> 5] >> (ilm & 31)) & 1u : 0u;
    ble = ((bri << 1) | l0) & lanebits;
  }

  const C s_left = lane_value(hs, 0), s_right = lane_value(hs, 1), s_wrap = lane_value(hs, 2);
  const C w_left = lane_value(hw, 0), w_right = lane_value(hw, 1), w_wrap = lane_value(hw, 2);
  C f1L = EQ ? C(0) : lane_prev(f1[VEC - 1]);
  C f3R = EQ ? C(0) : lane_next(f3[0]);
  C wL = lane_prev(wc[VEC - 1]);
  C wR = lane_next(wc[0]);
  if (lane == 0) {
    f1L = s_left;
    wL = w_left;
  }
  if (lane == 63) {
    f3R = s_right;
    wR = w_right;
  }

  C o0[VEC], o1[VEC], o2[VEC], o3[VEC], o4[VEC], wo[VEC];
#pragma unroll
  for (int k = 0; k < VEC; ++k) {
    const int i = i0 + k;
    const C w0 = wc[k];
    // pull along +x (f^1 from i-1)
    const bool dl = i == 0 && !p.periodic && (a.dmask & kEdgeLeft);
    const bool bl = (i == 0 && !p.periodic) || ((ble >> k) & 1u);
    C gl = bl ? f3[k] : ((k == 0) ? f1L : f1[k - 1]);
    C wl = (!SHIFT || bl) ? w0 : ((k == 0) ? wL : wc[k - 1]);
    if (dl) {  // Dirichlet edge: anti-bounce-back (ghost 2 w* - w)
      gl = SHIFT ? -f3[k] : -f3[k] + dirichlet_term(a, a.wD_left);
      wl = SHIFT ? C(2) * a.wD_left - w0 : w0;
    }
    // pull along -x (f^3 from i+1)
    const bool dr = i == last && !p.periodic && (a.dmask & kEdgeRight);
    const bool br = (i == last && !p.periodic) || ((bri >> k) & 1u);
    const bool wrap = (i == last) && !br;
    C gr = br ? f1[k] : (wrap ? s_wrap : ((k == VEC - 1) ? f3R : f3[k + 1]));
    C wr = (!SHIFT || br) ? w0 : (wrap ? w_wrap : ((k == VEC - 1) ? wR : wc[k + 1]));
    if (dr) {
      gr = SHIFT ? -f1[k] : -f1[k] + dirichlet_term(a, a.wD_right);
      wr = SHIFT ? C(2) * a.wD_right - w0 : w0;
    }
    // pull along +y (f^2 from j-1); a Dirichlet bottom edge: f_in^2 =
    // -f^4 + 2 Ak w* (the constant rides in td for stored f, in wdn for g)
    const bool db = jm < 0 && (a.dmask & kEdgeBottom);
    const bool bd = (jm < 0) || ((bdn >> k) & 1u);
    const C td = db ? (SHIFT ? C(0) : dirichlet_term(a, a.wD_bot))
                    : ((jm < 0) ? a.t_bot : (bd ? a.t_up : C(0)));
    const C gd = db ? -f4own[k] : (bd ? f4own[k] : f2d[k]);
    const C wdn = db ? (SHIFT ? C(2) * a.wD_bot - w0 : w0) : ((!SHIFT || bd) ? w0 : wm[k]);
    // pull along -y (f^4 from j+1); a Dirichlet top edge likewise
    const bool dt_ = jp < 0 && (a.dmask & kEdgeTop);
    const bool bu = (jp < 0) || ((bup >> k) & 1u);
    const C tu = dt_ ? (SHIFT ? C(0) : dirichlet_term(a, a.wD_top))
                     : ((jp < 0) ? a.t_top : (bu ? a.t_lo : C(0)));
    const C gu = dt_ ? -f2own[k] : (bu ? f2own[k] : f4u[k]);
    const C wup = dt_ ? (SHIFT ? C(2) * a.wD_top - w0 : w0) : ((!SHIFT || bu) ? w0 : wp[k]);
    site_update<C, SHIFT, EQ>(a, f0[k], gl, gr, gd, gu, w0, wl, wr, wdn, wup, bd, bu, td, tu, o0[k],
                          o1[k], o2[k], o3[k], o4[k], wo[k]);
    if (i > last) {  // padding past the row end stays zero
      o0[k] = o1[k] = o2[k] = o3[k] = o4[k] = wo[k] = C(0);
    }
  }
  if (act) {
    store_pops<S, C, VEC, SR, EQ>(fout, P, o, o0, o1, o2, o3, o4, sr_pair(j, i0, p.nx), a.rkey);
    store_row<W, C, VEC>(wout, o, wo);
  }
}

}  // namespace core
}  // namespace lbmk
