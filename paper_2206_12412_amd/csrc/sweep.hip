// Fused collide-stream sweep of the D2Q5 wave-equation LBM for gfx950.
//
// One launch performs one time step for every site (paper Sec. 3):
//   pull-stream with bounce-back on severed or outside links (eq. LBE,
//   streaming part; Sec. 4.1 "no information is exchanged" along a severed
//   link), wdot = sum of the populations (eq. distrib-macro), w += dt wdot
//   (eq. integration), BGK collision towards f_eq(w, wdot) (eq. LBE, f-eq).
//
// Layout: populations structure-of-arrays, plane a at fin + a * plane, rows
// of `pitch` elements (multiple of 64, 256-byte aligned);  w in its own plane.
// Work split: a wave owns a strip of 64 * VEC consecutive sites of a row and
// marches `rows` rows upwards;  lane l holds sites i0 .. i0 + VEC - 1 with
// i0 = strip * 64 * VEC + l * VEC, so every plane row is read with one
// 16-byte load per lane.  The x-neighbours across lanes come from DPP
// wave-shifts (v_mov_b32_dpp wave_shr / wave_shl), the two strip-edge
// lanes read their halo element from memory.  Rows j-1 and j+1 of w stay in
// registers while marching, so the shifted storage reads every w once.
// Links are tested against the plate edges by index and against the per-link
// cut bitmask (bit i of word i/32 of row j: V = link (i,j)-(i,j+1),
// H = link (i,j)-(i+1,j)); a per-row flag word says whether a row holds any
// severed link, so rows away from the crack never read the mask.
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

template <typename S, typename C, int VEC>
__device__ __forceinline__ void load_row(const S *__restrict__ ptr, C (&out)[VEC]) {
  const Pack<S, VEC> pk = *reinterpret_cast<const Pack<S, VEC> *>(ptr);
#pragma unroll
  for (int k = 0; k < VEC; ++k) out[k] = to_c(pk.v[k]);
}

template <typename S, typename C, int VEC>
__device__ __forceinline__ void store_row(S *__restrict__ ptr, const C (&in)[VEC]) {
  Pack<S, VEC> pk;
#pragma unroll
  for (int k = 0; k < VEC; ++k) pk.v[k] = from_c<S>(in[k]);
  *reinterpret_cast<Pack<S, VEC> *>(ptr) = pk;
}

// Severed-link bits of the VEC sites of a lane in row j.
struct LinkBits {
  uint32_t up, dn, right, left;  // bit k = link of site i0 + k is severed
};

__device__ __forceinline__ uint32_t mask_bit(const uint32_t *row, int i) {
  return (row[i >> 5] >> (i & 31)) & 1u;
}

template <int VEC>
__device__ __forceinline__ LinkBits link_bits(const uint32_t *__restrict__ mV,
                                              const uint32_t *__restrict__ mH,
                                              const uint32_t *__restrict__ rowflags, const Plate &p,
                                              int j, int jm, int il) {
  LinkBits b{0u, 0u, 0u, 0u};
  const uint32_t fj = rowflags[j];
  const uint32_t fm = (jm >= 0) ? rowflags[jm] : 0u;
  const uint32_t lanebits = (VEC == 32) ? 0xffffffffu : ((1u << VEC) - 1u);
  if (fj & 2u) b.up = (mV[(size_t)j * p.mw + (il >> 5)] >> (il & 31)) & lanebits;
  if (fm & 2u) b.dn = (mV[(size_t)jm * p.mw + (il >> 5)] >> (il & 31)) & lanebits;
  if (fj & 1u) {
    const uint32_t *h = mH + (size_t)j * p.mw;
    b.right = (h[il >> 5] >> (il & 31)) & lanebits;
    uint32_t l0 = 0u;
    if (il > 0) l0 = mask_bit(h, il - 1);
    else if (p.periodic) l0 = mask_bit(h, p.nx - 1);
    b.left = ((b.right << 1) | l0) & lanebits;
  }
  return b;
}

// ---------------------------------------------------------------------------
// Sweep.  SHIFT = false: the stored values are the post-collision populations
// f^alpha and w is updated in place (FP64 and plain FP32).  SHIFT = true: the
// stored values are g^alpha = f^alpha - E^alpha(w_emit) with the static
// equilibrium E^0 = -A0 w, E^k = Ak w of the emitting site, whose w (before
// the step) is read from the source w plane; the sum wdot and the collision
// are evaluated in these shifted variables, which is the same arithmetic
// regrouped so that no large term cancels in FP32.
template <typename S, typename W, typename C, int VEC, bool SHIFT>
__global__ void __launch_bounds__(512) sweep_kernel(const SweepArgs<S, W, C> a) {
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
  const int i0 = strip * SW + lane * VEC;
  const bool act = i0 < p.nx;
  const int il = act ? i0 : 0;  // load address of the lane (inactive lanes read a valid row start)
  const size_t P = p.plane;
  const int last = p.nx - 1;

  const S *__restrict__ fin = a.fin;
  S *__restrict__ fout = a.fout;
  const W *__restrict__ win = a.win;
  W *__restrict__ wout = a.wout;

  auto row_of = [&](int j) -> size_t { return (size_t)j * p.pitch; };
  auto jdown = [&](int j) { return j > 0 ? j - 1 : (p.periodic ? p.ny - 1 : -1); };
  auto jup = [&](int j) { return j < p.ny - 1 ? j + 1 : (p.periodic ? 0 : -1); };

  // Registers carried along the march: w of rows j-1, j (shifted storage
  // only) and f^4 / g^4 of row j (loaded as the pull source of row j-1).
  C wm[VEC], wc[VEC], f4own[VEC];
  {
    const int j = jb, jm = jdown(j);
    if (SHIFT) {
      load_row<W, C, VEC>(win + row_of(j) + il, wc);
      if (jm >= 0) load_row<W, C, VEC>(win + row_of(jm) + il, wm);
      else
#pragma unroll
        for (int k = 0; k < VEC; ++k) wm[k] = 0;
    }
    const bool need4 = (jm < 0) || (a.rowflags[jm] & 2u);
    if (need4) load_row<S, C, VEC>(fin + 4 * P + row_of(j) + il, f4own);
    else
#pragma unroll
      for (int k = 0; k < VEC; ++k) f4own[k] = 0;
  }

  for (int j = jb; j < je; ++j) {
    const int jm = jdown(j), jp = jup(j);
    const size_t rj = row_of(j);
    C f0[VEC], f1[VEC], f3[VEC], f2d[VEC], f4u[VEC], wp[VEC], wself[VEC];
    load_row<S, C, VEC>(fin + 0 * P + rj + il, f0);
    load_row<S, C, VEC>(fin + 1 * P + rj + il, f1);
    load_row<S, C, VEC>(fin + 3 * P + rj + il, f3);
    if (jm >= 0) load_row<S, C, VEC>(fin + 2 * P + row_of(jm) + il, f2d);
    if (jp >= 0) load_row<S, C, VEC>(fin + 4 * P + row_of(jp) + il, f4u);
    if (SHIFT) {
      if (jp >= 0) load_row<W, C, VEC>(win + row_of(jp) + il, wp);
    } else {
      load_row<W, C, VEC>(win + rj + il, wself);
    }
    const LinkBits lb = link_bits<VEC>(a.mV, a.mH, a.rowflags, p, j, jm, il);
    // f^2 / g^2 of the own row is needed only where the up link bounces.
    C f2own[VEC];
    if (jp < 0 || (a.rowflags[j] & 2u)) load_row<S, C, VEC>(fin + 2 * P + rj + il, f2own);

    // x-neighbours: from the adjacent lane, strip-edge lanes from memory.
    C f1L = lane_prev(f1[VEC - 1]);
    C f3R = lane_next(f3[0]);
    C wL = 0, wR = 0;
    if (SHIFT) {
      wL = lane_prev(wc[VEC - 1]);
      wR = lane_next(wc[0]);
    }
    if (lane == 0 && act) {
      const int il1 = i0 > 0 ? i0 - 1 : (p.periodic ? last : -1);
      if (il1 >= 0) {
        f1L = to_c(fin[1 * P + rj + il1]);
        if (SHIFT) wL = to_c(win[rj + il1]);
      }
    }
    if (lane == 63 && i0 + VEC <= last) {
      f3R = to_c(fin[3 * P + rj + i0 + VEC]);
      if (SHIFT) wR = to_c(win[rj + i0 + VEC]);
    }

    C o0[VEC], o1[VEC], o2[VEC], o3[VEC], o4[VEC], wo[VEC];
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
      const int i = i0 + k;
      const C w0 = SHIFT ? wc[k] : wself[k];
      // pull along +x (f^1 from i-1)
      C gl, wl = w0;
      if ((i == 0 && !p.periodic) || ((lb.left >> k) & 1u)) {
        gl = f3[k];
      } else {
        gl = (k == 0) ? f1L : f1[k - 1];
        if (SHIFT) wl = (k == 0) ? wL : wc[k - 1];
      }
      // pull along -x (f^3 from i+1)
      C gr, wr = w0;
      if ((i == last && !p.periodic) || ((lb.right >> k) & 1u)) {
        gr = f1[k];
      } else if (i == last) {
        gr = to_c(fin[3 * P + rj + 0]);
        if (SHIFT) wr = to_c(win[rj + 0]);
      } else {
        gr = (k == VEC - 1) ? f3R : f3[k + 1];
        if (SHIFT) wr = (k == VEC - 1) ? wR : wc[k + 1];
      }
      // pull along +y (f^2 from j-1)
      C gd, wdn = w0, td = 0;
      bool bd = false;
      if (jm < 0) { gd = f4own[k]; td = a.t_bot; bd = true; }
      else if ((lb.dn >> k) & 1u) { gd = f4own[k]; td = a.t_up; bd = true; }
      else { gd = f2d[k]; if (SHIFT) wdn = wm[k]; }
      // pull along -y (f^4 from j+1)
      C gu, wup = w0, tu = 0;
      bool bu = false;
      if (jp < 0) { gu = f2own[k]; tu = a.t_top; bu = true; }
      else if ((lb.up >> k) & 1u) { gu = f2own[k]; tu = a.t_lo; bu = true; }
      else { gu = f4u[k]; if (SHIFT) wup = wp[k]; }

      if (SHIFT) {
        const C wd = f0[k] + ((gl + gr) + (gd + gu)) +
                     a.Ak * (((wl - w0) + (wr - w0)) + ((wdn - w0) + (wup - w0))) + (td + tu);
        const C wn = w0 + a.dt * wd;
        const C om1 = C(1) - a.omega;
        o0[k] = om1 * (f0[k] + a.A0 * (wn - w0)) + a.omega * wd;
        o1[k] = om1 * (gl + a.Ak * (wl - wn));
        o2[k] = om1 * (gd + a.Ak * (wdn - wn) + td);
        o3[k] = om1 * (gr + a.Ak * (wr - wn));
        o4[k] = om1 * (gu + a.Ak * (wup - wn) + tu);
        wo[k] = wn;
      } else {
        // the paper's order of operations, as written (no contraction)
        const C fi0 = f0[k], fi1 = gl, fi3 = gr;
        const C fi2 = bd ? gd + td : gd;
        const C fi4 = bu ? gu + tu : gu;
        const C wd = fi0 + fi1 + fi2 + fi3 + fi4;
        const C wn = w0 + a.dt * wd;
        const C e0 = wd - a.A0 * wn;
        const C ek = a.Ak * wn;
        o0[k] = fi0 - a.omega * (fi0 - e0);
        o1[k] = fi1 - a.omega * (fi1 - ek);
        o2[k] = fi2 - a.omega * (fi2 - ek);
        o3[k] = fi3 - a.omega * (fi3 - ek);
        o4[k] = fi4 - a.omega * (fi4 - ek);
        wo[k] = wn;
      }
      if (i > last) {  // padding past the row end stays zero
        o0[k] = o1[k] = o2[k] = o3[k] = o4[k] = wo[k] = 0;
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
  hipLaunchKernelGGL((sweep_kernel<S, W, C, VEC, SHIFT>), dim3(blocks), dim3(64 * a.waves), 0, st, a);
  return hipGetLastError();
}

}  // namespace

int sweep_vec(Store s) {
  switch (s) {
    case Store::F64: return 2;
    case Store::F32_PLAIN: return 4;
    case Store::F32S: return 4;
    case Store::F16S: return 8;
    case Store::BF16S: return 8;
  }
  return 0;
}

hipError_t launch_sweep(Store s, const void *args, hipStream_t st) {
  switch (s) {
    case Store::F64: return launch_t<double, double, double, 2, false>(args, st);
    case Store::F32_PLAIN: return launch_t<float, float, float, 4, false>(args, st);
    case Store::F32S: return launch_t<float, float, float, 4, true>(args, st);
    case Store::F16S: return launch_t<_Float16, float, float, 8, true>(args, st);
    case Store::BF16S: return launch_t<__bf16, float, float, 8, true>(args, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace lbmk
