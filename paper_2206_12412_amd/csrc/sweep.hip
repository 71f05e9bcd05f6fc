// Fused collide-stream sweep of the D2Q5 wave-equation LBM for gfx950.
//
// One launch performs one time step for every site (paper Sec. 3):
//   pull-stream with bounce-back on severed or outside links (eq. LBE,
//   streaming part; Sec. 4.1 "no information is exchanged" along a severed
//   link), wdot = sum of the populations (eq. distrib-macro), w += dt wdot
//   (eq. integration), BGK collision towards f_eq(w, wdot) (eq. LBE, f-eq).
//
// Layout: populations structure-of-arrays, plane a at fin + a * plane, rows
// of `pitch` elements (multiple of 64, 256-byte aligned); w in its own plane;
// populations and w are double-buffered (source -> destination).
// Work split: a wave owns a strip of 64 * VEC consecutive sites of a row and
// marches `rows` rows upwards; lane l holds sites i0 .. i0 + VEC - 1 with
// i0 = strip * 64 * VEC + l * VEC, so every plane row is read and written
// with one 16-byte access per lane (8-byte for 16-bit storage, whose FP32 w
// rows are 16 bytes per lane).  x-neighbours across lanes come from DPP
// wave shifts (v_mov_b32_dpp wave_shr / wave_shl); the two strip-edge
// elements and the wrap-around element of periodic rows come from a single
// per-row halo load whose lanes 0..2 carry them (read back with readlane).
// Rows j-1 and j+1 of w stay in registers while marching.
// Links are tested against the plate edges by index and against the per-link
// cut bitmask (bit i of word i/32 of row j: V = link (i,j)-(i,j+1),
// H = link (i,j)-(i+1,j)) only in the rows the mask-row range names, so the
// sweep away from the crack never reads the mask.
#include "lbm_internal.hpp"

namespace lbmk {
namespace {

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

template <typename S, typename C, int VEC>
__device__ __forceinline__ void load_row(const S *__restrict__ ptr, C (&out)[VEC]) {
  const Pack<S, VEC> pk = *reinterpret_cast<const Pack<S, VEC> *>(ptr);
#pragma unroll
  for (int k = 0; k < VEC; ++k) out[k] = to_c(pk.v[k]);
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Rows are written once per step and read back only in the next step, after
// the whole plate has streamed through the caches: store them non-temporally.
template <typename S, typename C, int VEC>
__device__ __forceinline__ void store_row(S *__restrict__ ptr, const C (&in)[VEC]) {
  Pack<S, VEC> pk;
#pragma unroll
  for (int k = 0; k < VEC; ++k) pk.v[k] = from_c<S>(in[k]);
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

template <typename C, int VEC>
__device__ __forceinline__ void zero_row(C (&out)[VEC]) {
#pragma unroll
  for (int k = 0; k < VEC; ++k) out[k] = C(0);
}

__device__ __forceinline__ bool in_range(int j, int lo, int hi) { return j >= lo && j <= hi; }

// One site: wdot, Euler update and collision from the pulled populations.
// gl, gr, gd, gu are the values pulled along +x, -x, +y, -y (already bounced
// where the link is severed); for shifted storage wl .. wup are the w of the
// emitting sites (w0 where bounced); bd / bu say that the +y / -y pull bounced
// and then carries the traction term td / tu.
template <typename C, bool SHIFT, typename A>
__device__ __forceinline__ void site_update(const A &a, C f0, C gl, C gr, C gd, C gu, C w0, C wl,
                                            C wr, C wdn, C wup, bool bd, bool bu, C td, C tu,
                                            C &o0, C &o1, C &o2, C &o3, C &o4, C &wo) {
#pragma clang fp contract(off)
  if (SHIFT) {
    const C wd = f0 + ((gl + gr) + (gd + gu)) +
                 a.Ak * (((wl - w0) + (wr - w0)) + ((wdn - w0) + (wup - w0))) + (td + tu);
    const C wn = w0 + a.dt * wd;
    const C om1 = C(1) - a.omega;
    o0 = om1 * (f0 + a.A0 * (wn - w0)) + a.omega * wd;
    o1 = om1 * (gl + a.Ak * (wl - wn));
    o2 = om1 * (gd + a.Ak * (wdn - wn) + td);
    o3 = om1 * (gr + a.Ak * (wr - wn));
    o4 = om1 * (gu + a.Ak * (wup - wn) + tu);
    wo = wn;
  } else {
    // the paper's order of operations, as written (no contraction)
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

// ---------------------------------------------------------------------------
// Sweep.  SHIFT = false: the stored values are the post-collision populations
// f^alpha themselves (FP64 and plain FP32), evaluated in the paper's order of
// operations without contraction.  SHIFT = true: the stored values are
// g^alpha = f^alpha - E^alpha(w_emit) with the static equilibrium
// E^0 = -A0 w, E^k = Ak w of the emitting site, whose w (before the step) is
// read from the source w plane; wdot and the collision are evaluated in these
// shifted variables, which is the same arithmetic regrouped so that no large
// term cancels in FP32 (A0 = 4 Ak).
template <typename S, typename W, typename C, int VEC, bool SHIFT>
__global__ void __launch_bounds__(512)
sweep_kernel(const S *__restrict__ fin, S *__restrict__ fout, const W *__restrict__ win,
             W *__restrict__ wout, const uint32_t *__restrict__ mV, const uint32_t *__restrict__ mH,
             const MaskRows *__restrict__ mrows, const SweepArgs<S, W, C> a) {
#pragma clang fp contract(off)
  const Plate p = a.p;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  constexpr int SW = 64 * VEC;
  const int n_strips = (p.nx + SW - 1) / SW;
  const int task = blockIdx.x * a.waves + wave;
  const int strip = task % n_strips;
  const int jb = (task / n_strips) * a.rows;
  if (jb >= p.ny) return;
  const int je = min(jb + a.rows, p.ny);
  const int is = strip * SW;  // first site of the strip
  const int i0 = is + lane * VEC;
  const bool act = i0 < p.nx;
  const int il = act ? i0 : is;  // inactive lanes read their strip's first vector
  const size_t P = p.plane;
  const int last = p.nx - 1;
  const MaskRows mr = *mrows;

  // halo elements of a row: lane 0 the site left of the strip, lane 1 the site
  // right of it, lane 2 site 0 (the periodic neighbour of the last site)
  const int hl = is > 0 ? is - 1 : (p.periodic ? last : 0);
  const int hr = is + SW <= last ? is + SW : 0;
  const size_t hs_off = (lane == 0) ? 1 * P + hl : 3 * P + (lane == 1 ? hr : 0);
  const int hw_off = (lane == 0) ? hl : (lane == 1 ? hr : 0);
  // the strip holds neither plate edge (and every lane is inside the plate)
  const bool interior_strip = is > 0 && is + SW <= last;

  auto jdown = [&](int j) { return j > 0 ? j - 1 : (p.periodic ? p.ny - 1 : -1); };
  auto jup = [&](int j) { return j < p.ny - 1 ? j + 1 : (p.periodic ? 0 : -1); };

  // carried along the march: w of rows j-1 and j (shifted storage), and
  // f^4 / g^4 of row j (loaded as the pull source of row j-1)
  C wm[VEC], wc[VEC], f4own[VEC];
  {
    const int jm = jdown(jb);
    if (SHIFT) {
      load_row<W, C, VEC>(win + (size_t)jb * p.pitch + il, wc);
      if (jm >= 0) load_row<W, C, VEC>(win + (size_t)jm * p.pitch + il, wm);
      else zero_row(wm);
    }
    if (jm < 0 || in_range(jm, mr.vlo, mr.vhi)) load_row<S, C, VEC>(fin + 4 * P + (size_t)jb * p.pitch + il, f4own);
    else zero_row(f4own);
  }

  for (int j = jb; j < je; ++j) {
    const int jm = jdown(j), jp = jup(j);
    const size_t rj = (size_t)j * p.pitch;
    C f0[VEC], f1[VEC], f3[VEC], f2d[VEC], f4u[VEC], f2own[VEC], wp[VEC], wself[VEC];
    load_row<S, C, VEC>(fin + 0 * P + rj + il, f0);
    load_row<S, C, VEC>(fin + 1 * P + rj + il, f1);
    load_row<S, C, VEC>(fin + 3 * P + rj + il, f3);
    if (jm >= 0) load_row<S, C, VEC>(fin + 2 * P + (size_t)jm * p.pitch + il, f2d);
    else zero_row(f2d);
    if (jp >= 0) load_row<S, C, VEC>(fin + 4 * P + (size_t)jp * p.pitch + il, f4u);
    else zero_row(f4u);
    if (SHIFT) {
      if (jp >= 0) load_row<W, C, VEC>(win + (size_t)jp * p.pitch + il, wp);
      else zero_row(wp);
    } else {
      load_row<W, C, VEC>(win + rj + il, wself);
    }
    // f^2 / g^2 of the own row: only where the up link may bounce
    const bool up_mask = in_range(j, mr.vlo, mr.vhi);
    if (jp < 0 || up_mask) load_row<S, C, VEC>(fin + 2 * P + rj + il, f2own);
    else zero_row(f2own);
    const C hs = to_c(fin[rj + hs_off]);
    C hw = C(0);
    if (SHIFT) hw = to_c(win[rj + hw_off]);
    // severed-link bits of the lane's sites (bit k = site i0 + k)
    const uint32_t lanebits = (1u << VEC) - 1u;
    uint32_t bup = 0u, bdn = 0u, bri = 0u, ble = 0u;
    if (up_mask) bup = (mV[(size_t)j * p.mw + (il >> 5)] >> (il & 31)) & lanebits;
    if (jm >= 0 && in_range(jm, mr.vlo, mr.vhi))
      bdn = (mV[(size_t)jm * p.mw + (il >> 5)] >> (il & 31)) & lanebits;
    if (in_range(j, mr.hlo, mr.hhi)) {
      const uint32_t *h = mH + (size_t)j * p.mw;
      bri = (h[il >> 5] >> (il & 31)) & lanebits;
      const int ilm = il > 0 ? il - 1 : (p.periodic ? last : -1);
      const uint32_t l0 = ilm >= 0 ? (h[ilm >> 5] >> (ilm & 31)) & 1u : 0u;
      ble = ((bri << 1) | l0) & lanebits;
    }

    // x-neighbours: the adjacent lane, or the halo for the strip-edge lanes
    const C s_left = lane_value(hs, 0), s_right = lane_value(hs, 1), s_wrap = lane_value(hs, 2);
    C f1L = lane_prev(f1[VEC - 1]);
    C f3R = lane_next(f3[0]);
    if (lane == 0) f1L = s_left;
    if (lane == 63) f3R = s_right;
    C wL = C(0), wR = C(0), w_wrap = C(0);
    if (SHIFT) {
      wL = lane_prev(wc[VEC - 1]);
      wR = lane_next(wc[0]);
      if (lane == 0) wL = lane_value(hw, 0);
      if (lane == 63) wR = lane_value(hw, 1);
      w_wrap = lane_value(hw, 2);
    }

    C o0[VEC], o1[VEC], o2[VEC], o3[VEC], o4[VEC], wo[VEC];
    // interior wave and row (uniform): no plate edge in the strip, no edge row,
    // no severed link possible -> no boundary selects at all
    const bool fast = interior_strip && jm >= 0 && jp >= 0 && !up_mask &&
                      !(in_range(jm, mr.vlo, mr.vhi)) && !(in_range(j, mr.hlo, mr.hhi));
    if (fast) {
#pragma unroll
      for (int k = 0; k < VEC; ++k) {
        const C w0 = SHIFT ? wc[k] : wself[k];
        const C gl = (k == 0) ? f1L : f1[k - 1];
        const C gr = (k == VEC - 1) ? f3R : f3[k + 1];
        C wl = w0, wr = w0, wdn = w0, wup = w0;
        if (SHIFT) {
          wl = (k == 0) ? wL : wc[k - 1];
          wr = (k == VEC - 1) ? wR : wc[k + 1];
          wdn = wm[k];
          wup = wp[k];
        }
        site_update<C, SHIFT>(a, f0[k], gl, gr, f2d[k], f4u[k], w0, wl, wr, wdn, wup, false, false,
                              C(0), C(0), o0[k], o1[k], o2[k], o3[k], o4[k], wo[k]);
      }
    } else {
#pragma unroll
      for (int k = 0; k < VEC; ++k) {
        const int i = i0 + k;
        const C w0 = SHIFT ? wc[k] : wself[k];
        // pull along +x (f^1 from i-1)
        const bool bl = (i == 0 && !p.periodic) || ((ble >> k) & 1u);
        const C gl = bl ? f3[k] : ((k == 0) ? f1L : f1[k - 1]);
        const C wl = (!SHIFT || bl) ? w0 : ((k == 0) ? wL : wc[k - 1]);
        // pull along -x (f^3 from i+1)
        const bool br = (i == last && !p.periodic) || ((bri >> k) & 1u);
        const bool wrap = (i == last) && !br;
        const C gr = br ? f1[k] : (wrap ? s_wrap : ((k == VEC - 1) ? f3R : f3[k + 1]));
        const C wr = (!SHIFT || br) ? w0 : (wrap ? w_wrap : ((k == VEC - 1) ? wR : wc[k + 1]));
        // pull along +y (f^2 from j-1)
        const bool bd = (jm < 0) || ((bdn >> k) & 1u);
        const C td = (jm < 0) ? a.t_bot : (bd ? a.t_up : C(0));
        const C gd = bd ? f4own[k] : f2d[k];
        const C wdn = (!SHIFT || bd) ? w0 : wm[k];
        // pull along -y (f^4 from j+1)
        const bool bu = (jp < 0) || ((bup >> k) & 1u);
        const C tu = (jp < 0) ? a.t_top : (bu ? a.t_lo : C(0));
        const C gu = bu ? f2own[k] : f4u[k];
        const C wup = (!SHIFT || bu) ? w0 : wp[k];
        site_update<C, SHIFT>(a, f0[k], gl, gr, gd, gu, w0, wl, wr, wdn, wup, bd, bu, td, tu, o0[k],
                              o1[k], o2[k], o3[k], o4[k], wo[k]);
        if (i > last) {  // padding past the row end stays zero
          o0[k] = o1[k] = o2[k] = o3[k] = o4[k] = wo[k] = C(0);
        }
      }
    }
    if (act) {
      store_row<S, C, VEC>(fout + 0 * P + rj + i0, o0);
      store_row<S, C, VEC>(fout + 1 * P + rj + i0, o1);
      store_row<S, C, VEC>(fout + 2 * P + rj + i0, o2);
      store_row<S, C, VEC>(fout + 3 * P + rj + i0, o3);
      store_row<S, C, VEC>(fout + 4 * P + rj + i0, o4);
      store_row<W, C, VEC>(wout + rj + i0, wo);
    }
    // march: rows j, j+1 become j-1, j
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
      if (SHIFT) {
        wm[k] = wc[k];
        wc[k] = wp[k];
      }
      f4own[k] = f4u[k];
    }
  }
}

template <typename S, typename W, typename C, int VEC, bool SHIFT>
hipError_t launch_t(const void *args, hipStream_t st) {
  const auto &a = *static_cast<const SweepArgs<S, W, C> *>(args);
  constexpr int SW = 64 * VEC;
  const int n_strips = (a.p.nx + SW - 1) / SW;
  const int n_chunks = (a.p.ny + a.rows - 1) / a.rows;
  const long tasks = (long)n_strips * n_chunks;
  const unsigned blocks = (unsigned)((tasks + a.waves - 1) / a.waves);
  hipLaunchKernelGGL((sweep_kernel<S, W, C, VEC, SHIFT>), dim3(blocks), dim3(64 * a.waves), 0, st,
                     a.fin, a.fout, a.win, a.wout, a.mV, a.mH, a.mrows, a);
  return hipGetLastError();
}

}  // namespace

int sweep_vec(Store s) {
  switch (s) {
    case Store::F64: return 2;
    case Store::F32_PLAIN: return 4;
    case Store::F32S: return 4;
    case Store::F16S: return 4;
    case Store::BF16S: return 4;
  }
  return 0;
}

hipError_t launch_sweep(Store s, const void *args, hipStream_t st) {
  switch (s) {
    case Store::F64: return launch_t<double, double, double, 2, false>(args, st);
    case Store::F32_PLAIN: return launch_t<float, float, float, 4, false>(args, st);
    case Store::F32S: return launch_t<float, float, float, 4, true>(args, st);
    case Store::F16S: return launch_t<_Float16, float, float, 4, true>(args, st);
    case Store::BF16S: return launch_t<__bf16, float, float, 4, true>(args, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace lbmk
