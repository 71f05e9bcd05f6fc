// Discrete adjoint of the collide-stream step (the transpose of the affine
// map of one time step, Sec. 3 eq. LBE with eq. f-eq, eq. distrib-macro and
// eq. integration, and the bounce-back of Sec. 4.1), one fused sweep per step.
//
// Forward step n, per site x:  f_in^a(x) = f^a(x - c^a) over an intact link,
// else f^abar(x) + coef t*;  wdot = sum_a f_in^a;  w' = w + dt wdot;
// f'^a = (1 - omega) f_in^a + omega f_eq^a(w', wdot) with f_eq^0 = wdot - A0 w',
// f_eq^k = Ak w'.
//
// The adjoint state stored between sweeps is (mu, W): mu^a(x) the adjoint of
// f_in^a(x) of a step and W(x) the adjoint of w(x) through that step.  Sweep
// m reads mu_m, W_m (+ the loss gradient at the sensors, added beforehand)
// and writes mu_{m-1}, W_{m-1}:
//   streaming transposed: the adjoint of the post-collision f^b(y) is
//     mu^b(y + c^b) if the link (y, y + c^b) is intact, else mu^bbar(y)
//     (the population a site bounces back is its own);
//   then the transposed local map with l = that adjoint and b = W:
//     G = b + omega (-A0 l^0 + Ak (l^1 + l^2 + l^3 + l^4))   (adjoint of w)
//     D = omega l^0 + dt G                                    (adjoint of wdot)
//     mu^a = (1 - omega) l^a + D.
// The traction links make dL/dtau_m = coef (sum over the top row of mu^4
// - sum over the bottom row of mu^2).  The last sweep (m = 0) applies the
// transpose of the initial equilibrium f^0 = wdot_0 - A0 w_0, f^k = Ak w_0,
// which is the same map with omega = 1 and dt = 0: it leaves dL/dwdot_0 in
// plane 0 and dL/dw_0 in W.
//
// Interior rows (all vertical links intact) run the strip code of the
// forward sweep with the neighbour directions reversed (DPP lane shifts for
// x, rows j +- 1 for y); the edge and crack rows run one thread per site, in
// the same launch.  The loss gradient of the state a sweep produces is added
// to W by the thread that writes it (the sensors are indexed by row).
// FP64 is evaluated without contraction in the order written above.
//
// At omega = 1 every mu^a a sweep writes equals D, so the five planes hold
// the same values.  The equilibrium-layout sweep (EQ) keeps plane 0 only and
// reads it for every direction: the same numbers from a fifth of the
// population traffic.
#include "sweep_core.hpp"

namespace lbmk {
namespace {

using core::lane_next;
using core::lane_prev;
using core::lane_value;
using core::load_row;
using core::store_row;

// The transposed local map.  FP64 follows the order written above, without
// contraction.  FP32 uses A0 = 4 Ak (the D2Q5 equilibrium) to write
// -A0 l^0 + Ak sum_k l^k as Ak sum_k (l^k - l^0): the adjoint of a smooth
// field then enters as small differences instead of a cancelling sum of large
// terms (the same regrouping as the shifted FP32 forward sweep).
__device__ __forceinline__ void adj_local_t(const AdjArgs<double> &a, double l0, double l1,
                                            double l2, double l3, double l4, double b, double &G,
                                            double &D) {
#pragma clang fp contract(off)
  G = b + a.omega * (-a.A0 * l0 + a.Ak * (l1 + l2 + l3 + l4));
  D = a.omega * l0 + a.dt * G;
}
__device__ __forceinline__ void adj_local_t(const AdjArgs<float> &a, float l0, float l1, float l2,
                                            float l3, float l4, float b, float &G, float &D) {
#pragma clang fp contract(fast)
  G = b + a.omega * (a.Ak * (((l1 - l0) + (l2 - l0)) + ((l3 - l0) + (l4 - l0))));
  D = a.omega * l0 + a.dt * G;
}

template <typename C>
__device__ __forceinline__ void adj_local(const AdjArgs<C> &a, C l0, C l1, C l2, C l3, C l4, C b,
                                          C &o0, C &o1, C &o2, C &o3, C &o4, C &wo) {
#pragma clang fp contract(off)
  C G, D;
  adj_local_t(a, l0, l1, l2, l3, l4, b, G, D);
  const C om1 = C(1) - a.omega;
  o0 = om1 * l0 + D;
  o1 = om1 * l1 + D;
  o2 = om1 * l2 + D;
  o3 = om1 * l3 + D;
  o4 = om1 * l4 + D;
  wo = G;
}

template <typename C, int VEC, bool EQ>
__device__ __forceinline__ void adj_interior_row(const AdjArgs<C> &a, int strip, int j) {
  const Plate p = a.p;
  const int lane = threadIdx.x & 63;
  constexpr int SW = 64 * VEC;
  const int last = p.nx - 1;
  const int is = strip * SW;
  const int i0 = is + lane * VEC;
  const bool act = i0 < p.nx;
  const uint32_t il = act ? i0 : is;
  const uint32_t pitch = p.pitch;
  const size_t P = p.plane;
  const size_t Q = EQ ? 0 : P;  // plane stride of the reads (EQ: every direction from plane 0)
  const C *__restrict__ M0 = a.min;
  const C *__restrict__ M1 = a.min + Q;
  const C *__restrict__ M2 = a.min + 2 * Q;
  const C *__restrict__ M3 = a.min + 3 * Q;
  const C *__restrict__ M4 = a.min + 4 * Q;
  const uint32_t o = (uint32_t)j * pitch + il;

  C m0[VEC], m1[VEC], m3[VEC], m2u[VEC], m4d[VEC], b[VEC];
  load_row<C, C, VEC>(M0, o, m0);
  if constexpr (EQ) {
#pragma unroll
    for (int k = 0; k < VEC; ++k) m1[k] = m3[k] = m0[k];
  } else {
    load_row<C, C, VEC>(M1, o, m1);
    load_row<C, C, VEC>(M3, o, m3);
  }
  load_row<C, C, VEC>(M2, o + pitch, m2u);  // mu^2 of the site above
  load_row<C, C, VEC>(M4, o - pitch, m4d);  // mu^4 of the site below
  load_row<C, C, VEC>(a.win, o, b);
  // halo: lane 0 mu^3 left of the strip (the periodic wrap for the first
  // strip), lane 1 mu^1 right of the strip, lane 2 mu^1 of site 0 (the
  // periodic neighbour of the last site)
  const C *__restrict__ Mh = (lane == 0) ? M3 : M1;
  const uint32_t hx = (lane == 0) ? (is > 0 ? is - 1 : (p.periodic ? last : 0))
                                  : (lane == 1 && is + SW <= last ? is + SW : 0);
  const C hs = *core::at(Mh, (uint32_t)j * pitch + hx);
  const C s_left = lane_value(hs, 0), s_right = lane_value(hs, 1), s_wrap = lane_value(hs, 2);
  const C m1R = lane_next(m1[0]);
  const C m3L = lane_prev(m3[VEC - 1]);

  C o0[VEC], o1[VEC], o2[VEC], o3[VEC], o4[VEC], wo[VEC];
#pragma unroll
  for (int k = 0; k < VEC; ++k) {
    const int i = i0 + k;
    // adjoint of f^1(i): mu^1 of the right neighbour (the +x link)
    C l1 = (k == VEC - 1) ? ((lane == 63) ? s_right : m1R) : m1[k + 1];
    // adjoint of f^3(i): mu^3 of the left neighbour (the -x link)
    C l3 = (k == 0) ? ((lane == 0) ? s_left : m3L) : m3[k - 1];
    // outside links: bounce-back returns the opposite direction's adjoint,
    // a Dirichlet edge (anti-bounce-back) with the opposite sign
    if (i == last) l1 = p.periodic ? s_wrap : ((a.dmask & core::kEdgeRight) ? -m3[k] : m3[k]);
    if (i == 0 && !p.periodic) l3 = (a.dmask & core::kEdgeLeft) ? -m1[k] : m1[k];
    adj_local<C>(a, m0[k], l1, m2u[k], l3, m4d[k], b[k], o0[k], o1[k], o2[k], o3[k], o4[k], wo[k]);
    if (i > last) o0[k] = o1[k] = o2[k] = o3[k] = o4[k] = wo[k] = C(0);
  }
  if (a.g) {  // the loss gradient at this row's sensors (a wave-uniform loop)
    const int e0 = a.srow[j], e1 = a.srow[j + 1];
    for (int e = e0; e < e1; ++e) {
      const int ci = a.srt[2 * e];
      const double gv = a.g[a.srt[2 * e + 1]];
#pragma unroll
      for (int k = 0; k < VEC; ++k)
        if (ci == i0 + k) wo[k] = (C)((double)wo[k] + gv);
    }
  }
  if (act) {
    store_row<C, C, VEC>(a.mout, o, o0);
    if constexpr (!EQ) {
      store_row<C, C, VEC>(a.mout + P, o, o1);
      store_row<C, C, VEC>(a.mout + 2 * P, o, o2);
      store_row<C, C, VEC>(a.mout + 3 * P, o, o3);
      store_row<C, C, VEC>(a.mout + 4 * P, o, o4);
    }
    store_row<C, C, VEC>(a.wout, o, wo);
  }
}

__device__ __forceinline__ double block_sum(double x, double *lds) {
  for (int s = 32; s >= 1; s >>= 1) x += __shfl_xor(x, s, 64);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) lds[wave] = x;
  __syncthreads();
  return ((lds[0] + lds[1]) + lds[2]) + lds[3];
}

// Edge and crack row j, one thread per site i (part = block of the row).
template <typename C, bool EQ>
__device__ __forceinline__ void adj_boundary_site(const AdjArgs<C> &a, int r, int j, int part,
                                                  double *red) {
  const Plate p = a.p;
  const int i = part * 256 + threadIdx.x;
  const int last = p.nx - 1;
  const size_t P = EQ ? 0 : p.plane;  // plane stride of the reads (EQ: plane 0 only)
  double dtau = 0.0;
  if (i < p.nx) {
    const size_t pitch = p.pitch;
    const size_t x = (size_t)j * pitch + i;
    const int jm = j > 0 ? j - 1 : (p.periodic ? p.ny - 1 : -1);
    const int jp = j < p.ny - 1 ? j + 1 : (p.periodic ? 0 : -1);
    // the crack-row link (i, j0)-(i, j0 + 1) is severed for step m's
    // streaming if it was cut before step m
    const bool cut = a.has_crack && a.cutstep[i] < a.m;
    const bool cut_up = cut && j == p.j0;
    const bool cut_dn = cut && j == p.j0 + 1;
    const C *M = a.min;
    const C l0 = M[x];
    // outside links of a Dirichlet edge: anti-bounce-back, sign -1
    const C sr = (a.dmask & core::kEdgeRight) ? C(-1) : C(1);
    const C sl = (a.dmask & core::kEdgeLeft) ? C(-1) : C(1);
    const C st = (jp < 0 && (a.dmask & core::kEdgeTop)) ? C(-1) : C(1);
    const C sb = (jm < 0 && (a.dmask & core::kEdgeBottom)) ? C(-1) : C(1);
    const C l1 = i < last ? M[P + x + 1] : (p.periodic ? M[P + (size_t)j * pitch] : sr * M[3 * P + x]);
    const C l3 = i > 0 ? M[3 * P + x - 1] : (p.periodic ? M[3 * P + (size_t)j * pitch + last] : sl * M[P + x]);
    const C l2 = (jp >= 0 && !cut_up) ? M[2 * P + (size_t)jp * pitch + i] : st * M[4 * P + x];
    const C l4 = (jm >= 0 && !cut_dn) ? M[4 * P + (size_t)jm * pitch + i] : sb * M[2 * P + x];
    C o0, o1, o2, o3, o4, wo;
    adj_local<C>(a, l0, l1, l2, l3, l4, a.win[x], o0, o1, o2, o3, o4, wo);
    if (a.g) {
      for (int e = a.srow[j]; e < a.srow[j + 1]; ++e)
        if (a.srt[2 * e] == i) wo = (C)((double)wo + a.g[a.srt[2 * e + 1]]);
    }
    a.mout[x] = o0;
    if constexpr (!EQ) {
      a.mout[P + x] = o1;
      a.mout[2 * P + x] = o2;
      a.mout[3 * P + x] = o3;
      a.mout[4 * P + x] = o4;
    }
    a.wout[x] = wo;
    if (a.traction) {  // traction-loaded edges only (not the Dirichlet ones)
      if (j == p.ny - 1 && !(a.dmask & core::kEdgeTop)) dtau += a.coef * (double)M[4 * P + x];
      if (j == 0 && !(a.dmask & core::kEdgeBottom)) dtau -= a.coef * (double)M[2 * P + x];
    }
  }
  const double s = block_sum(dtau, red);
  if (threadIdx.x == 0) a.dtau_part[r * a.n_parts + part] = s;
}

// One adjoint sweep: the first nb * n_parts workgroups take the boundary rows
// (one thread per site), the rest the interior strips (4 waves each).
template <typename C, int VEC, bool EQ>
__global__ void __launch_bounds__(256) adj_step(const AdjArgs<C> a, const core::InteriorMap m,
                                                const core::BoundaryMap bm, long n_tasks) {
  __shared__ double red[4];
  const unsigned nbb = (unsigned)(bm.nb * a.n_parts);
  if (blockIdx.x < nbb) {
    const int r = blockIdx.x / a.n_parts;
    adj_boundary_site<C, EQ>(a, r, core::boundary_row_of(bm, r), blockIdx.x % a.n_parts, red);
    return;
  }
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const long task = (long)(blockIdx.x - nbb) * 4 + wave;
  if (task >= n_tasks) return;
  const int strip = (int)(task % m.n_strips);
  const int chunk = (int)(task / m.n_strips);
  const int j = chunk < m.nc1 ? m.lo1 + chunk : m.lo2 + (chunk - m.nc1);
  adj_interior_row<C, VEC, EQ>(a, strip, j);
}

template <typename C>
__global__ void adj_inject(C *w, Plate p, const int32_t *sens, int n, const double *g) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= n) return;
  const size_t x = (size_t)sens[2 * s + 1] * p.pitch + sens[2 * s];
  w[x] = (C)((double)w[x] + g[s]);
}

template <typename C>
__global__ void adj_export(const C *plane, Plate p, double *out) {
  const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (size_t)p.nx * p.ny) return;
  const size_t j = t / p.nx, i = t % p.nx;
  out[t] = (double)plane[j * p.pitch + i];
}

template <typename C, int VEC, bool EQ>
hipError_t sweep_t(const AdjArgs<C> &a, hipStream_t st) {
  const core::InteriorMap m = core::interior_map(a.p.nx, a.p.ny, VEC, 1, a.skip_lo, a.skip_hi);
  const core::BoundaryMap bm = core::boundary_map(a.p.nx, a.p.ny, VEC, a.skip_lo, a.skip_hi);
  const long tasks = core::interior_task_count(m);
  const unsigned blocks = (unsigned)(bm.nb * a.n_parts + (tasks + 3) / 4);
  hipLaunchKernelGGL((adj_step<C, VEC, EQ>), dim3(blocks), dim3(256), 0, st, a, m, bm, tasks);
  return hipGetLastError();
}

}  // namespace

int adjoint_parts(int nx) { return (nx + 255) / 256; }

hipError_t launch_adjoint_sweep(bool fp64, bool eq, const void *args, hipStream_t st) {
  if (fp64) {
    const auto &a = *static_cast<const AdjArgs<double> *>(args);
    return eq ? sweep_t<double, 2, true>(a, st) : sweep_t<double, 2, false>(a, st);
  }
  const auto &a = *static_cast<const AdjArgs<float> *>(args);
  return eq ? sweep_t<float, 4, true>(a, st) : sweep_t<float, 4, false>(a, st);
}

hipError_t launch_adjoint_inject(bool fp64, void *w, const Plate &p, const int32_t *sens, int n,
                                 const double *g, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (fp64)
    hipLaunchKernelGGL(adj_inject<double>, dim3(blocks), dim3(256), 0, st, static_cast<double *>(w), p,
                       sens, n, g);
  else
    hipLaunchKernelGGL(adj_inject<float>, dim3(blocks), dim3(256), 0, st, static_cast<float *>(w), p,
                       sens, n, g);
  return hipGetLastError();
}

hipError_t launch_adjoint_export(bool fp64, const void *plane, const Plate &p, double *out,
                                 hipStream_t st) {
  const size_t n = (size_t)p.nx * p.ny;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (fp64)
    hipLaunchKernelGGL(adj_export<double>, dim3(blocks), dim3(256), 0, st,
                       static_cast<const double *>(plane), p, out);
  else
    hipLaunchKernelGGL(adj_export<float>, dim3(blocks), dim3(256), 0, st,
                       static_cast<const float *>(plane), p, out);
  return hipGetLastError();
}

}  // namespace lbmk
