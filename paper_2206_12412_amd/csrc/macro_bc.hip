// The macroscopic boundary scheme of Sec. 3.1, applied after a step's sweep
// and before its crack step.
//
// A boundary point is a site with a severed link or a link leaving the
// plate.  Its displacement is not taken from the lattice Boltzmann update but
// from a quadratic polynomial along the inward normal of each missing link,
// fixed by the boundary condition on the wall or crack face (half a spacing
// beyond the point, s = 0) and by this step's w at the next two lattice
// points inward (s = 3/2 and 5/2); the point sits at s = 1/2.  With several
// missing links (a corner) the point takes the mean of their polynomials.
// Written out (Lagrange basis on the nodes 0, 3/2, 5/2, evaluated at 1/2):
//   prescribed w*:     w_B = 8/15 w* + 2/3 w_I - 1/5 w_II,
//   traction t*:       p = a + q s + c s^2 with the slope q = -t*/mu along
//                      the inward normal gives w_B = 3/2 w_I - 1/2 w_II - 1/2 q.
// Where w_I or w_II belongs to a boundary point itself (next to a corner, a
// lateral edge beside the crack faces), its polynomial value is used: the
// system S w_B = R is solved by substitution, which ends after two levels
// for a rectangular plate with a crack along +x at least three rows from
// either edge (the host checks that geometry).  A dependency deeper than
// that raises the error flag instead.
//
// With w_B known, eq. (f-macro-bc) fills the missing populations so that
// they sum to wdot_B = (w_B(t + dt) - w_B(t)) / dt, and at omega = 1 the
// collision sets every population of the point to f_eq(w_B, wdot_B): the
// rest population wdot_B - A0 w_B and the moving ones Ak w_B, i.e. in the
// shifted storages (g = f - E(w_B)) wdot_B and zeros.  So the kernel writes
// w_B and plane 0 (and, for the unshifted storages, the four moving planes);
// the moving planes of the shifted storages already hold the zeros the sweep
// wrote at omega = 1.
#include "lbm_internal.hpp"
#include "sweep_core.hpp"

namespace lbmk {
namespace {

template <typename W>
struct MacroView {
  const MacroArgs &a;
  const W *__restrict__ w;  // w after the sweep (interior values are final)

  __device__ bool cut_v(int i, int j) const {  // vertical link (i, j)-(i, j + 1) severed
    return a.has_crack && j == a.p.j0 && ((a.mV[(size_t)j * a.p.mw + (i >> 5)] >> (i & 31)) & 1u);
  }
  // missing links of site (i, j) as outward directions (dx, dy)
  __device__ int missing(int i, int j, int (&dx)[4], int (&dy)[4]) const {
    int m = 0;
    if (i == 0) { dx[m] = -1; dy[m++] = 0; }
    if (i == a.p.nx - 1) { dx[m] = 1; dy[m++] = 0; }
    if (j == 0 || (j == a.p.j0 + 1 && cut_v(i, a.p.j0))) { dx[m] = 0; dy[m++] = -1; }
    if (j == a.p.ny - 1 || (j == a.p.j0 && cut_v(i, a.p.j0))) { dx[m] = 0; dy[m++] = 1; }
    return m;
  }
};

// The estimate of one missing link (outward (dx, dy)) of boundary point
// (i, j) from the values v1, v2 of its two interior points.
template <typename C>
__device__ __forceinline__ C link_estimate(const MacroArgs &a, int i, int j, int dx, int dy, C v1,
                                           C v2) {
  const bool wall = (i + dx < 0) || (i + dx >= a.p.nx) || (j + dy < 0) || (j + dy >= a.p.ny);
  if (wall) {
    const int edge = dy < 0 ? 1 : dy > 0 ? 2 : dx < 0 ? 4 : 8;  // LBM_EDGE_* bit
    if (a.dmask & edge) {
      const double g = edge == 1 ? a.wD[0] : edge == 2 ? a.wD[1] : edge == 4 ? a.wD[2] : a.wD[3];
      return C(8.0 / 15.0) * (C)g + C(2.0 / 3.0) * v1 + C(-0.2) * v2;
    }
  }
  // traction t* = mu dw/dn on the outward normal: top +tau, bottom -tau,
  // lateral edges free; the face below the crack (outward +y) -tau*, the
  // face above (outward -y) +tau*
  double t = 0.0;
  if (wall) t = dy > 0 ? a.t_top : dy < 0 ? a.t_bot : 0.0;
  else t = dy > 0 ? -a.t_face : a.t_face;
  const C q = (C)(-t / a.mu);
  return C(-0.5) * q + C(1.5) * v1 + C(-0.5) * v2;
}

template <typename C, typename W, int D>
__device__ C point_value(const MacroView<W> &v, int i, int j, int *err);

// w of site (i, j) after the step: the sweep's value at an interior site, the
// polynomial value (D more levels allowed) at a boundary point
template <typename C, typename W, int D>
__device__ __forceinline__ C site_value(const MacroView<W> &v, int i, int j, int *err) {
  int dx[4], dy[4];
  if (v.missing(i, j, dx, dy) == 0) return (C)v.w[(size_t)j * v.a.p.pitch + i];
  if constexpr (D > 0) {
    return point_value<C, W, D - 1>(v, i, j, err);
  } else {
    *err = 1;  // deeper than the geometry the host admits
    return (C)v.w[(size_t)j * v.a.p.pitch + i];
  }
}

template <typename C, typename W, int D>
__device__ C point_value(const MacroView<W> &v, int i, int j, int *err) {
  int dx[4], dy[4];
  const int m = v.missing(i, j, dx, dy);
  C sum = C(0);
  for (int k = 0; k < m; ++k) {
    const C v1 = site_value<C, W, D>(v, i - dx[k], j - dy[k], err);
    const C v2 = site_value<C, W, D>(v, i - 2 * dx[k], j - 2 * dy[k], err);
    sum += link_estimate<C>(v.a, i, j, dx[k], dy[k], v1, v2);
  }
  return m == 1 ? sum : sum / (C)m;
}

// Candidate sites: rows 0 and ny - 1, columns 0 and nx - 1 of the other rows,
// and the inner columns of the two crack rows.
__device__ __forceinline__ bool candidate(const MacroArgs &a, int64_t t, int *i, int *j) {
  const int nx = a.p.nx, ny = a.p.ny;
  if (t < 2 * (int64_t)nx) {
    *i = (int)(t % nx);
    *j = t < nx ? 0 : ny - 1;
    return true;
  }
  t -= 2 * (int64_t)nx;
  if (t < 2 * (int64_t)(ny - 2)) {
    *j = 1 + (int)(t % (ny - 2));
    *i = t < ny - 2 ? 0 : nx - 1;
    return true;
  }
  t -= 2 * (int64_t)(ny - 2);
  if (a.has_crack && t < 2 * (int64_t)(nx - 2)) {
    *i = 1 + (int)(t % (nx - 2));
    *j = t < nx - 2 ? a.p.j0 : a.p.j0 + 1;
    return true;
  }
  return false;
}

template <typename S, typename W, typename C, bool SHIFT, bool SR, bool EQ>
__global__ void __launch_bounds__(256) macro_bc_kernel(MacroArgs a) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int i, j;
  if (!candidate(a, t, &i, &j)) return;
  const MacroView<W> v{a, static_cast<const W *>(a.wout)};
  int dx[4], dy[4];
  if (v.missing(i, j, dx, dy) == 0) return;
  int err = 0;
  const C wb = point_value<C, W, 2>(v, i, j, &err);
  if (err) a.err[0] = 1;
  const size_t x = (size_t)j * a.p.pitch + i;
  const C wold = (C) static_cast<const W *>(a.win)[x];
  const C wd = (wb - wold) / (C)a.dt;
  static_cast<W *>(a.wout)[x] = (W)wb;
  S *f = static_cast<S *>(a.fout);
  C f0;
  if constexpr (SHIFT) {
    f0 = wd;
  } else {
    f0 = wd - (C)a.A0 * wb;
  }
  if constexpr (SR) {
    const uint32_t h = mix32(core::sr_pair((uint32_t)j, (uint32_t)i, (uint32_t)a.p.nx) ^ a.rkey);
    f[x] = core::round_sr<S>((float)f0, core::sr_half(h, (uint32_t)i & 1u));
  } else {
    f[x] = core::from_c<S>(f0);
  }
  if constexpr (!SHIFT && !EQ) {
    const C ek = (C)a.Ak * wb;
    for (int k = 1; k < 5; ++k) f[x + (size_t)k * a.p.plane] = core::from_c<S>(ek);
  }
}

template <typename S, typename W, typename C, bool SHIFT, bool SR, bool EQ>
hipError_t launch_t(const MacroArgs &a, hipStream_t st) {
  const int64_t n = 2 * (int64_t)a.p.nx + 2 * (int64_t)(a.p.ny - 2) + (a.has_crack ? 2 * (int64_t)(a.p.nx - 2) : 0);
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((macro_bc_kernel<S, W, C, SHIFT, SR, EQ>), dim3((unsigned)((n + 255) / 256)),
                     dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename S, typename W, typename C, bool SHIFT>
hipError_t launch_r(int sr, bool eq, const MacroArgs &a, hipStream_t st) {
  if constexpr (sizeof(S) == 2) {
    if (sr) return eq ? launch_t<S, W, C, SHIFT, true, true>(a, st) : launch_t<S, W, C, SHIFT, true, false>(a, st);
  }
  return eq ? launch_t<S, W, C, SHIFT, false, true>(a, st) : launch_t<S, W, C, SHIFT, false, false>(a, st);
}

}  // namespace

hipError_t launch_macro_bc(Store s, int sr, bool eq, const MacroArgs &a, hipStream_t st) {
  switch (s) {
    case Store::F64: return launch_r<double, double, double, false>(0, false, a, st);
    case Store::F64S: return launch_r<double, double, double, true>(0, eq, a, st);
    case Store::F32_PLAIN: return launch_r<float, float, float, false>(0, false, a, st);
    case Store::F32S: return launch_r<float, float, float, true>(0, eq, a, st);
    case Store::F16S: return launch_r<_Float16, float, float, true>(sr, eq, a, st);
    case Store::BF16S: return launch_r<__bf16, float, float, true>(sr, eq, a, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace lbmk
