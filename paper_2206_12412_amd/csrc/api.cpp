// Host side of the C-ABI declared in include/lbm.h: validation, device
// layout, launch order and queries.  All arithmetic of a time step runs in
// the kernels of sweep.hip and crack.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "crack_geom.hpp"
#include "lbm.h"
#include "lbm_internal.hpp"

using lbmk::Store;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(LBM_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));              \
  } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Layout {
  size_t elem = 0, welem = 0;
  int pitch = 0, mw = 0;
  size_t plane = 0;             // elements between planes
  size_t off_f[2] = {0, 0};
  size_t off_w[2] = {0, 0};
  size_t off_mV = 0, off_mH = 0, off_rf = 0, off_crack = 0, off_crack2 = 0, off_fargs = 0;
  size_t off_trK = 0, off_trA = 0, off_trV = 0, off_trF = 0;
  size_t off_trKL = 0, off_trAL = 0, off_trVL = 0, off_trFL = 0;
  size_t off_evS = 0, off_evC = 0, off_evJ = 0, off_evO = 0, off_stage = 0;
  size_t off_sens = 0, off_trS = 0, off_wmid = 0, off_spec = 0, off_merr = 0;
  int64_t event_cap = 0;
  int stage_rows = 0;
  size_t total = 0;
};

// storage and layout -> storage scheme (FP64 in the equilibrium layout is
// kept in the shifted form)
bool store_of(int32_t s, int32_t layout, Store *out) {
  switch (s) {
    case LBM_F64: *out = layout == LBM_LAYOUT_EQ ? Store::F64S : Store::F64; return true;
    case LBM_F32: *out = Store::F32S; return true;
    case LBM_F16S: *out = Store::F16S; return true;
    case LBM_BF16S: *out = Store::BF16S; return true;
    case LBM_F32_PLAIN: *out = Store::F32_PLAIN; return true;
    default: return false;
  }
}

bool is_fp64(Store s) { return s == Store::F64 || s == Store::F64S; }

size_t elem_size(Store s) {
  switch (s) {
    case Store::F64: case Store::F64S: return 8;
    case Store::F32_PLAIN: case Store::F32S: return 4;
    case Store::F16S: case Store::BF16S: return 2;
  }
  return 0;
}

Layout make_layout(const lbm_config &c, Store s) {
  Layout L;
  L.elem = elem_size(s);
  L.welem = is_fp64(s) ? 8 : 4;
  L.pitch = (int)align_up((size_t)c.nx, 64);
  L.mw = (int)align_up(((size_t)c.nx + 31) / 32, 2);
  // planes 256-byte aligned with a 1 KiB skew between consecutive planes
  const size_t plane_bytes = align_up((size_t)L.pitch * c.ny * L.elem, 256) + 1024;
  L.plane = plane_bytes / L.elem;
  size_t o = 0;
  for (int b = 0; b < 2; ++b) {
    L.off_f[b] = o;
    o += 5 * plane_bytes;
  }
  const size_t wbytes = align_up((size_t)L.pitch * c.ny * L.welem, 256) + 1024;
  for (int b = 0; b < 2; ++b) {
    L.off_w[b] = o;
    o += wbytes;
  }
  const size_t mbytes = align_up((size_t)c.ny * L.mw * 4, 256);
  L.off_mV = o; o += mbytes;
  L.off_mH = o; o += mbytes;
  L.off_rf = o; o += 256;
  L.off_crack = o; o += 256;
  L.off_crack2 = o; o += 256;  // second slot: a crack step folded into the next sweep
  const size_t tc = c.trace_cap > 0 ? (size_t)c.trace_cap : 1;
  L.off_trK = o; o += align_up(tc * 8, 256);
  L.off_trA = o; o += align_up(tc * 8, 256);
  L.off_trV = o; o += align_up(tc * 8, 256);
  L.off_trF = o; o += align_up(tc * 4, 256);
  const size_t tl = c.both_tips ? tc : 1;  // left-tip traces (two tips)
  L.off_trKL = o; o += align_up(tl * 8, 256);
  L.off_trAL = o; o += align_up(tl * 8, 256);
  L.off_trVL = o; o += align_up(tl * 8, 256);
  L.off_trFL = o; o += align_up(tl * 4, 256);
  // a straight crack severs at most one link per lattice line it crosses
  L.event_cap = 2 * ((int64_t)c.nx + c.ny) + 16;
  L.off_evS = o; o += align_up((size_t)L.event_cap * 8, 256);
  L.off_evC = o; o += align_up((size_t)L.event_cap * 4, 256);
  L.off_evJ = o; o += align_up((size_t)L.event_cap * 4, 256);
  L.off_evO = o; o += align_up((size_t)L.event_cap * 4, 256);
  // T-step sweep: the crack rows after steps n .. n + T - 2
  L.off_wmid = o; o += align_up((size_t)2 * (lbmk::kMaxTimeBlock - 1) * L.pitch * L.welem, 256);
  // speculative T-step sweep (K criterion): the crack state and crack-row mask of step n
  // (and the gate of the speculative sweeps in flight)
  L.off_spec = o; o += align_up(sizeof(lbmk::SpecSlot), 256) + align_up((size_t)L.mw * 4, 256) + 256;
  L.off_sens = o; o += align_up((size_t)std::max(c.n_sensors, 1) * 8, 256);
  L.off_trS = o; o += align_up(tc * (size_t)std::max(c.n_sensors, 1) * 8, 256);
  L.stage_rows = (int)std::max<int64_t>(1, std::min<int64_t>(c.ny, (1 << 20) / std::max(1, c.nx)));
  L.off_stage = o;
  o += align_up((size_t)5 * L.stage_rows * c.nx * 8, 256);
  L.off_merr = o;  // error flag of the macroscopic boundary scheme
  o += 256;
  // the arguments of a crack step folded into the next sweep, per (current
  // buffer, state slot): device addresses of this handle, so after the part
  // a checkpoint holds (off_mV .. off_stage)
  L.off_fargs = o;
  o += 4 * align_up(sizeof(lbmk::CrackArgs), 256);
  L.total = o;
  return L;
}

// The crack line of a configuration: start point, unit growth direction
// (exact along the axes) and the line coordinates where the line leaves the
// plate (the walls the tips stop at).
void crack_line(const lbm_config &c, lbmk::geom::Line *L, double *a_lo, double *a_hi) {
  const int j0 = c.crack_row >= 0 ? c.crack_row : c.ny / 2 - 1;
  L->x0 = c.crack_x0;
  L->yc = j0 + 0.5;
  L->aligned = (c.crack_dy == 0.0 && c.crack_dx >= 0.0);
  if (L->aligned) {
    L->ux = 1.0;
    L->uy = 0.0;
    *a_lo = -0.5;
    *a_hi = c.nx - 0.5;
    return;
  }
  const double n = std::sqrt(c.crack_dx * c.crack_dx + c.crack_dy * c.crack_dy);
  L->ux = c.crack_dx / n;
  L->uy = c.crack_dy / n;
  if (c.crack_dx == 0.0) {
    L->ux = 0.0;
    L->uy = c.crack_dy > 0 ? 1.0 : -1.0;
  }
  if (c.crack_dy == 0.0) {
    L->uy = 0.0;
    L->ux = c.crack_dx > 0 ? 1.0 : -1.0;
  }
  *a_hi = L->x0 + lbmk::geom::wall_distance(c.nx, c.ny, L->x0, L->yc, L->ux, L->uy);
  *a_lo = L->x0 - lbmk::geom::wall_distance(c.nx, c.ny, L->x0, L->yc, -L->ux, -L->uy);
}

int validate(const lbm_config *c, Store *s) {
  if (!c) return fail(LBM_EINVAL, "null config");
  if (c->layout != LBM_LAYOUT_FULL && c->layout != LBM_LAYOUT_EQ)
    return fail(LBM_EINVAL, "unknown layout %d", c->layout);
  if (!store_of(c->storage, c->layout, s)) return fail(LBM_EINVAL, "unknown storage %d", c->storage);
  if (c->layout == LBM_LAYOUT_EQ && *s == Store::F32_PLAIN)
    return fail(LBM_EINVAL, "the equilibrium layout needs a shifted storage (not F32_PLAIN)");
  if (c->nx < 1 || c->ny < 1 || c->nx > (1 << 24) || c->ny > (1 << 24))
    return fail(LBM_EINVAL, "plate size %d x %d out of range", c->nx, c->ny);
  // in-plane byte offsets are 32-bit: one plane (populations or w) < 4 GiB
  {
    const size_t e = (c->storage == LBM_F64) ? 8 : 4;
    if (align_up((size_t)c->nx, 64) * (size_t)c->ny * e >= (size_t(1) << 32))
      return fail(LBM_EINVAL, "plate of %d x %d sites: one plane would exceed 4 GiB", c->nx, c->ny);
  }
  if (c->bc_mode != LBM_BC_WALLS && c->bc_mode != LBM_BC_PERIODIC)
    return fail(LBM_EINVAL, "unknown bc_mode %d", c->bc_mode);
  if (!(c->mu > 0) || !(c->rho > 0) || !std::isfinite(c->mu) || !std::isfinite(c->rho))
    return fail(LBM_EINVAL, "mu and rho must be positive");
  if (!(c->kappa > 0) || !std::isfinite(c->kappa)) return fail(LBM_EINVAL, "kappa must be positive");
  if (c->omega != 1.0)
    return fail(LBM_EUNSTABLE, "omega = %g: with w integrated into f_eq the scheme is stable only at tau = dt", c->omega);
  if (c->kappa * c->kappa <= 2.0)
    return fail(LBM_EUNSTABLE, "kappa = %g: the scheme needs kappa > sqrt(2)", c->kappa);
  if (c->crack_row < -1) return fail(LBM_EINVAL, "crack_row must be -1 (mid-line) or a row");
  if (c->has_crack) {
    if (c->crack_row < 0 && (c->ny < 2 || c->ny % 2))
      return fail(LBM_EINVAL, "a crack on the mid-line needs an even ny >= 2");
    if (c->crack_row > c->ny - 2) return fail(LBM_EINVAL, "crack_row must be in 0..ny-2");
    if (!std::isfinite(c->crack_dx) || !std::isfinite(c->crack_dy))
      return fail(LBM_EINVAL, "bad crack direction");
    const bool aligned = c->crack_dy == 0.0 && c->crack_dx >= 0.0;
    if (!(c->crack_x0 >= -0.5) || !(c->crack_x0 <= c->nx - 0.5) || !(c->crack_tip >= c->crack_x0) ||
        (aligned && !(c->crack_tip <= c->nx - 0.5)))
      return fail(LBM_ECRACK, "crack [%g, %g] not inside [-0.5, %g]", c->crack_x0, c->crack_tip, c->nx - 0.5);
    if (!aligned) {
      lbmk::geom::Line L;
      double a_lo, a_hi;
      crack_line(*c, &L, &a_lo, &a_hi);
      if (!(c->crack_tip <= a_hi))
        return fail(LBM_ECRACK, "crack tip %g beyond the plate (line coordinate <= %g)", c->crack_tip, a_hi);
      if (c->k_band != 1) return fail(LBM_EINVAL, "a crack along another direction than +x needs k_band = 1");
      if (c->bc_mode == LBM_BC_PERIODIC) return fail(LBM_EINVAL, "a crack along another direction needs walls");
    }
    if (!(c->r0 > 0)) return fail(LBM_EINVAL, "r0 must be positive");
    if (c->k_band < 1 || c->k_band > 64) return fail(LBM_EINVAL, "k_band must be in 1..64");
  }
  if (c->growth != LBM_GROW_NONE && c->growth != LBM_GROW_PRESCRIBED && c->growth != LBM_GROW_SIF)
    return fail(LBM_EINVAL, "unknown growth %d", c->growth);
  if (c->growth != LBM_GROW_NONE && (!c->has_crack || c->bc_mode == LBM_BC_PERIODIC))
    return fail(LBM_EINVAL, "growth needs a crack and walls");
  if (c->growth == LBM_GROW_PRESCRIBED && !(c->v_rel >= 0 && c->v_rel < 1))
    return fail(LBM_EINVAL, "prescribed speed must be in [0, 1)");
  if (c->growth == LBM_GROW_SIF && !(c->K_C > 0 && c->v_max >= 0 && c->v_max < 1))
    return fail(LBM_EINVAL, "K criterion needs K_C > 0 and v_max in [0, 1)");
  if (c->n_hist < 0 || (c->n_hist > 0 && !c->tau_hist)) return fail(LBM_EINVAL, "bad traction history");
  if (c->trace_cap < 0) return fail(LBM_EINVAL, "negative trace_cap");
  if (c->both_tips && !c->has_crack) return fail(LBM_EINVAL, "both_tips needs a crack");
  if (c->dirichlet < 0 || c->dirichlet > 15) return fail(LBM_EINVAL, "dirichlet holds edge bits 1..8");
  if (c->dirichlet && c->bc_mode == LBM_BC_PERIODIC)
    return fail(LBM_EINVAL, "a periodic lattice has no edges");
  if (c->dirichlet && (c->n_wD < 1 || !c->wD_hist))
    return fail(LBM_EINVAL, "Dirichlet edges need a wall-displacement history");
  if (c->n_sensors < 0 || c->n_sensors > (1 << 20) || (c->n_sensors > 0 && !c->sensors))
    return fail(LBM_EINVAL, "bad sensor list");
  if (c->n_sensors > 0) {
    std::vector<int64_t> ids;
    ids.reserve(c->n_sensors);
    for (int k = 0; k < c->n_sensors; ++k) {
      const int i = c->sensors[2 * k], j = c->sensors[2 * k + 1];
      if (i < 0 || i >= c->nx || j < 0 || j >= c->ny)
        return fail(LBM_EINVAL, "sensor %d at (%d, %d) is outside the plate", k, i, j);
      ids.push_back((int64_t)j * c->nx + i);
    }
    std::sort(ids.begin(), ids.end());
    if (std::adjacent_find(ids.begin(), ids.end()) != ids.end())
      return fail(LBM_EINVAL, "sensor sites must be distinct");
  }
  if (c->bc_scheme != LBM_BC_LINK && c->bc_scheme != LBM_BC_MACRO)
    return fail(LBM_EINVAL, "unknown bc_scheme %d", c->bc_scheme);
  if (c->bc_scheme == LBM_BC_MACRO) {
    if (c->bc_mode == LBM_BC_PERIODIC) return fail(LBM_EINVAL, "the macroscopic scheme needs walls");
    if (c->nx < 3 || c->ny < 3) return fail(LBM_EINVAL, "the macroscopic scheme needs nx, ny >= 3");
    if (c->has_crack) {
      if (!(c->crack_dy == 0.0 && c->crack_dx >= 0.0))
        return fail(LBM_EINVAL, "the macroscopic scheme takes cracks along +x only");
      // three rows on either side of the crack line: every boundary point's
      // two interior points then resolve within two levels
      const int j0 = c->crack_row >= 0 ? c->crack_row : c->ny / 2 - 1;
      if (j0 < 3 || j0 + 4 > c->ny - 1)
        return fail(LBM_EINVAL, "the macroscopic scheme needs three rows on either side of the crack line");
    }
  }
  if (c->rounding != LBM_ROUND_NEAREST && c->rounding != LBM_ROUND_STOCHASTIC)
    return fail(LBM_EINVAL, "unknown rounding %d", c->rounding);
  if (c->rounding == LBM_ROUND_STOCHASTIC && c->storage != LBM_F16S && c->storage != LBM_BF16S)
    return fail(LBM_EINVAL, "stochastic rounding applies to the 16-bit storages only");
  return LBM_OK;
}

}  // namespace

// K-criterion T-step sweeps in flight at once (see spec_pipeline)
constexpr int kSpecDepth = 4;

struct lbm_handle {
  lbm_config cfg{};
  Store store = Store::F64;
  Layout L;
  lbmk::Plate plate{};
  hipStream_t stream = nullptr;
  std::vector<double> tau;
  double cs = 0, c = 0, dt = 0, lambda = 0, A0 = 0, Ak = 0, coef = 0;
  char *base = nullptr;
  int cur = 0;        // buffer (populations and w) holding the current state
  int64_t step = 0;
  int rows = 1, waves = 4, occ = 0;
  int lds_per_cu = 65536;
  bool timing = false;
  int timing_stride = 1;  // record the steps whose index is a multiple of this
  std::vector<hipEvent_t> ev_pool;
  std::vector<hipEvent_t> ev_used;  // per timed step: before, after the sweep, after the crack step
  std::vector<int> ev_steps;        // steps covered by each recorded triple (T: a T-step sweep)
  double t_sweep = 0, t_crack = 0;
  int64_t n_timed = 0;
  lbmk::DevCrack host_crack{};
  lbmk::CrackArgs host_fargs[4]{};  // host side of the fused_args upload
  bool in_batch = false;  // stepped by a batch; lbm_step refuses it
  // equilibrium layout: the sweep touches plane 0 and w only.  The moving
  // planes of both buffers hold zeros in every state reached by a step; until
  // two steps have run since the state was set (init, restore) the five-plane
  // sweep runs, so that initial moving populations (the part of an FP64 w0
  // that FP32 cannot hold) are streamed and both buffers are cleared.
  bool eq = false;
  int full_steps = 0;
  // time blocking: steps per sweep (1, or T = 2..8 with the T-step sweep)
  // and the T-step sweep's rows per wave and waves per workgroup, per T
  int tblock = 1;
  // a call whose step count is not a multiple of T ends with the sweeps of
  // plan_tail (on) or with one shorter sweep (off)
  bool tail_plan = true;
  // speculative T-step sweeps (K criterion) and how many were run again;
  // the length the next one may take (halved by a sweep run again, one more
  // after each sweep that held, at most T)
  int64_t spec_blocks = 0, spec_reruns = 0;
  int spec_cap = lbmk::kMaxTimeBlock;
  // the speculative sweeps' verdicts, written by the crack kernel into pinned
  // host memory (allocated with the first such sweep; one per sweep in
  // flight) and their device address
  lbmk::SpecOut *spec_host = nullptr, *spec_dev = nullptr;
  // the gate the T-step launches pass on (null: ungated)
  const int32_t *blk_gate = nullptr;
  // the side stream the T-step sweep's boundary chunks run on beside the
  // rest, with its fork and join events (created with the first T-step
  // sweep, on the device current then; default priority)
  lbmk::SideStream side{nullptr, nullptr, nullptr};
  // a T-step sweep's crack steps under a prescribed speed (or none) run on
  // the side stream right after the sweep's boundary launch (the crack rows
  // and the side buffer of the inner steps are all they read), beside the
  // fast chunks of this sweep and the next, which read neither the crack
  // rows nor the crack state; crack_pending says the side stream holds crack
  // steps the caller's stream has not yet joined
  bool crack_pending = false;
  // one-step sweeps run the crack step of the step before them (fold_crack):
  // crack_deferred says the crack step of step `step - 1` has not run yet; the
  // state before it is in slot cslot (0: off_crack, 1: off_crack2).  Between
  // calls of lbm_step nothing is deferred and the state is in slot 0.
  bool crack_deferred = false;
  int cslot = 0;
  int blk_rows[lbmk::kMaxTimeBlock + 1] = {};
  int blk_waves[lbmk::kMaxTimeBlock + 1] = {};
  int blk_occ[lbmk::kMaxTimeBlock + 1] = {};  // resident waves per SIMD, 0 = no cap
  // crack line, wall limits of the tips and the rows a crack can touch
  lbmk::geom::Line line{1, 0.0, 0.0, 1.0, 0.0};
  double a_lo = -0.5, a_hi = 0.0;
  int skip_lo = 1, skip_hi = 0;
  std::vector<int32_t> sensors;  // host copy of the sensor sites
  std::vector<double> wD;        // host copy of the wall-displacement history [n][4]

  bool macro() const { return cfg.bc_scheme == LBM_BC_MACRO; }
  bool crack_step_needed() const { return cfg.has_crack || cfg.n_sensors > 0; }

  void *fbuf(int b) const { return base + L.off_f[b]; }
  void *wbuf(int b) const { return base + L.off_w[b]; }
  uint32_t *mV() const { return reinterpret_cast<uint32_t *>(base + L.off_mV); }
  uint32_t *mH() const { return reinterpret_cast<uint32_t *>(base + L.off_mH); }
  lbmk::MaskRows *mrows() const { return reinterpret_cast<lbmk::MaskRows *>(base + L.off_rf); }
  lbmk::DevCrack *crack() const { return reinterpret_cast<lbmk::DevCrack *>(base + L.off_crack); }
  // device copy of the arguments of the crack step a one-step sweep runs:
  // w in buffer cur, state in slot cslot, going to the other slot
  const lbmk::CrackArgs *fused_args(int cur_buf, int slot) const {
    return reinterpret_cast<const lbmk::CrackArgs *>(
        base + L.off_fargs + (size_t)(2 * cur_buf + slot) * align_up(sizeof(lbmk::CrackArgs), 256));
  }
  lbmk::DevCrack *crack_slot(int k) const {
    return reinterpret_cast<lbmk::DevCrack *>(base + (k ? L.off_crack2 : L.off_crack));
  }
  // a one-step sweep can run the previous step's crack step itself: a crack
  // along +x or none (sensors only), not under the macroscopic boundary scheme
  // (its kernel runs between the sweep and the crack step)
  bool fold_crack() const {
    return crack_step_needed() && !macro() && (!cfg.has_crack || line.aligned);
  }
  lbmk::SpecSlot *spec_slot() const { return reinterpret_cast<lbmk::SpecSlot *>(base + L.off_spec); }
  uint32_t *spec_mask() const {
    return reinterpret_cast<uint32_t *>(base + L.off_spec + align_up(sizeof(lbmk::SpecSlot), 256));
  }
  int32_t *spec_gate() const {
    return reinterpret_cast<int32_t *>(base + L.off_spec + align_up(sizeof(lbmk::SpecSlot), 256) +
                                       align_up((size_t)L.mw * 4, 256));
  }
  double *stage() const { return reinterpret_cast<double *>(base + L.off_stage); }
  double tau_at(int64_t n) const {
    if (tau.empty()) return 0.0;
    return tau[(size_t)std::min<int64_t>(n, (int64_t)tau.size() - 1)];
  }
};

namespace {

hipEvent_t take_event(lbm_handle *h) {
  if (!h->ev_pool.empty()) {
    hipEvent_t e = h->ev_pool.back();
    h->ev_pool.pop_back();
    return e;
  }
  // timing only (read after a stream synchronisation): no system-scope fence,
  // which would add a cache write-back to every timed interval
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

int harvest_timing(lbm_handle *h) {
  if (h->ev_used.empty()) return LBM_OK;
  HIP_TRY(hipStreamSynchronize(h->stream));
  for (size_t k = 0; k + 2 < h->ev_used.size(); k += 3) {
    float a = 0, c = 0;
    HIP_TRY(hipEventElapsedTime(&a, h->ev_used[k], h->ev_used[k + 1]));
    HIP_TRY(hipEventElapsedTime(&c, h->ev_used[k + 1], h->ev_used[k + 2]));
    h->t_sweep += a;
    h->t_crack += c;
    h->n_timed += h->ev_steps[k / 3];
  }
  for (hipEvent_t e : h->ev_used) h->ev_pool.push_back(e);
  h->ev_used.clear();
  h->ev_steps.clear();
  return LBM_OK;
}

// Sweep arguments of step n (its traction, wall values and rounding key),
// from the current buffers to the other ones.
template <typename S, typename W, typename C>
lbmk::SweepArgs<S, W, C> sweep_args(const lbm_handle *h, int64_t n) {
  lbmk::SweepArgs<S, W, C> a{};
  const int nxt = 1 - h->cur;
  a.fin = static_cast<const S *>(h->fbuf(h->cur));
  a.fout = static_cast<S *>(h->fbuf(nxt));
  a.win = static_cast<const W *>(h->wbuf(h->cur));
  a.wout = static_cast<W *>(h->wbuf(nxt));
  a.mV = h->mV();
  a.mH = h->mH();
  a.mrows = h->mrows();
  a.p = h->plate;
  a.omega = (C)h->cfg.omega;
  a.dt = (C)h->dt;
  a.A0 = (C)h->A0;
  a.Ak = (C)h->Ak;
  const double tau = h->tau_at(n);
  const bool per = h->cfg.bc_mode == LBM_BC_PERIODIC;
  a.t_top = per ? C(0) : (C)(h->coef * tau);
  a.t_bot = per ? C(0) : (C)(h->coef * -tau);
  a.t_up = per ? C(0) : (C)(h->coef * h->cfg.face_traction);
  a.t_lo = per ? C(0) : (C)(h->coef * -h->cfg.face_traction);
  a.rows = h->rows;
  a.waves = h->waves;
  a.lds_bytes = 0;
  if (h->occ > 0) {
    // resident workgroups per CU = occ waves per SIMD x 4 SIMDs / waves per group
    const int groups = std::max(1, (h->occ * 4) / h->waves);
    a.lds_bytes = std::min(65536, (h->lds_per_cu / groups) / 256 * 256);
  }
  // the rows a crack can touch go to the boundary work
  a.skip_lo = h->skip_lo;
  a.skip_hi = h->skip_hi;
  a.sr = h->cfg.rounding == LBM_ROUND_STOCHASTIC;
  a.rkey = lbmk::step_key(h->cfg.seed, n);
  a.dmask = per ? 0 : h->cfg.dirichlet;
  if (a.dmask) {
    const size_t r = 4 * (size_t)std::min<int64_t>(n, h->cfg.n_wD - 1);
    a.wD_bot = (C)h->wD[r];
    a.wD_top = (C)h->wD[r + 1];
    a.wD_left = (C)h->wD[r + 2];
    a.wD_right = (C)h->wD[r + 3];
  } else {
    a.wD_bot = a.wD_top = a.wD_left = a.wD_right = C(0);
  }
  return a;
}

template <typename S, typename W, typename C>
int launch_sweep_typed(lbm_handle *h, const lbmk::CrackArgs *fc) {
  const lbmk::SweepArgs<S, W, C> a = sweep_args<S, W, C>(h, h->step);
  HIP_TRY(lbmk::launch_sweep(h->store, h->eq && h->full_steps == 0, &a, h->stream, fc));
  return LBM_OK;
}

// Steps n .. n + T - 1 in one sweep (time blocking, sweep2.hip).
template <typename S, typename W, typename C>
int launch_block_typed(lbm_handle *h, int T) {
  lbmk::BlockArgs<S, W, C> A{};
  A.s0 = sweep_args<S, W, C>(h, h->step);
  A.s0.lds_bytes = 0;
  if (h->blk_occ[T] > 0) {
    const int groups = std::max(1, (h->blk_occ[T] * 4) / h->blk_waves[T]);
    A.s0.lds_bytes = std::min(65536, (h->lds_per_cu / groups) / 256 * 256);
  }
  for (int k = 0; k < T; ++k) {
    const lbmk::SweepArgs<S, W, C> a = sweep_args<S, W, C>(h, h->step + k);
    A.lv[k] = lbmk::StepLevel<C>{a.t_top, a.t_bot, a.t_up, a.t_lo,
                                 a.wD_bot, a.wD_top, a.wD_left, a.wD_right};
    A.rkey_last = a.rkey;
  }
  A.steps = T;
  A.wmid = reinterpret_cast<W *>(h->base + h->L.off_wmid);
  A.st = h->crack();
  A.crack = h->cfg.has_crack;
  A.both = h->cfg.both_tips;
  A.grow = h->cfg.growth == LBM_GROW_PRESCRIBED || h->cfg.growth == LBM_GROW_SIF;
  A.sif = h->cfg.growth == LBM_GROW_SIF;
  A.v_rel = h->cfg.v_rel;
  A.cs = h->cs;
  A.dt = h->dt;
  A.a_lo = h->a_lo;
  A.a_hi = h->a_hi;
  A.gate = h->blk_gate;
  if (!h->side.side) {
    HIP_TRY(hipStreamCreateWithFlags(&h->side.side, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&h->side.fork, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&h->side.join, hipEventDisableTiming));
  }
  HIP_TRY(lbmk::launch_sweep_block(h->store, &A, h->blk_rows[T], h->blk_waves[T], h->stream,
                                   h->side));
  return LBM_OK;
}

int launch_block_any(lbm_handle *h, int T) {
  switch (h->store) {
    case Store::F64S: return launch_block_typed<double, double, double>(h, T);
    case Store::F32S: return launch_block_typed<float, float, float>(h, T);
    case Store::F16S: return launch_block_typed<_Float16, float, float>(h, T);
    case Store::BF16S: return launch_block_typed<__bf16, float, float>(h, T);
    default: return fail(LBM_EINVAL, "the T-step sweep needs the equilibrium layout");
  }
}

// fc: device copy of the arguments of the previous step's crack step, run
// by this sweep (null: none)
int launch_sweep_any(lbm_handle *h, const lbmk::CrackArgs *fc) {
  switch (h->store) {
    case Store::F64: return launch_sweep_typed<double, double, double>(h, fc);
    case Store::F64S: return launch_sweep_typed<double, double, double>(h, fc);
    case Store::F32_PLAIN: return launch_sweep_typed<float, float, float>(h, fc);
    case Store::F32S: return launch_sweep_typed<float, float, float>(h, fc);
    case Store::F16S: return launch_sweep_typed<_Float16, float, float>(h, fc);
    case Store::BF16S: return launch_sweep_typed<__bf16, float, float>(h, fc);
  }
  return fail(LBM_EINVAL, "bad storage");
}

lbmk::CrackArgs crack_args(const lbm_handle *h) {
  lbmk::CrackArgs a{};
  a.st = h->crack();
  a.w = h->wbuf(1 - h->cur);  // w after the sweep just enqueued
  a.w_is_double = is_fp64(h->store);
  a.mV = h->mV();
  a.mH = h->mH();
  a.mrows = h->mrows();
  a.trK = reinterpret_cast<double *>(h->base + h->L.off_trK);
  a.trA = reinterpret_cast<double *>(h->base + h->L.off_trA);
  a.trV = reinterpret_cast<double *>(h->base + h->L.off_trV);
  a.trF = reinterpret_cast<int32_t *>(h->base + h->L.off_trF);
  a.trKL = reinterpret_cast<double *>(h->base + h->L.off_trKL);
  a.trAL = reinterpret_cast<double *>(h->base + h->L.off_trAL);
  a.trVL = reinterpret_cast<double *>(h->base + h->L.off_trVL);
  a.trFL = reinterpret_cast<int32_t *>(h->base + h->L.off_trFL);
  a.evStep = reinterpret_cast<int64_t *>(h->base + h->L.off_evS);
  a.evCol = reinterpret_cast<int32_t *>(h->base + h->L.off_evC);
  a.evRow = reinterpret_cast<int32_t *>(h->base + h->L.off_evJ);
  a.evOri = reinterpret_cast<int32_t *>(h->base + h->L.off_evO);
  a.sens = reinterpret_cast<const int32_t *>(h->base + h->L.off_sens);
  a.trS = reinterpret_cast<double *>(h->base + h->L.off_trS);
  a.n_sens = h->cfg.n_sensors;
  a.p = h->plate;
  a.c.crack = h->cfg.has_crack;
  a.c.both = h->cfg.both_tips;
  a.c.growth = h->cfg.growth;
  a.c.band = h->cfg.k_band;
  a.c.v_rel = h->cfg.v_rel;
  a.c.K_C = h->cfg.K_C;
  a.c.r0 = h->cfg.r0;
  a.c.v_max = h->cfg.v_max;
  a.c.cs = h->cs;
  a.c.dt = h->dt;
  a.c.mu = h->cfg.mu;
  a.c.x0 = h->cfg.crack_x0;
  a.c.aligned = h->line.aligned;
  a.c.yc = h->line.yc;
  a.c.ux = h->line.ux;
  a.c.uy = h->line.uy;
  a.c.a_lo = h->a_lo;
  a.c.a_hi = h->a_hi;
  a.c.trace_cap = h->cfg.trace_cap;
  a.c.event_cap = h->L.event_cap;
  return a;
}

int launch_crack_step(lbm_handle *h) {
  const lbmk::CrackArgs a = crack_args(h);
  HIP_TRY(lbmk::launch_crack(a, h->stream));
  return LBM_OK;
}

// The arguments of the crack step of step h->step - 1, deferred by the last
// one-step sweep: the current w is the w after that step, the state before
// it is in slot cslot.
lbmk::CrackArgs deferred_crack_args(const lbm_handle *h) {
  lbmk::CrackArgs a = crack_args(h);
  a.w = h->wbuf(h->cur);
  a.st = h->crack_slot(h->cslot);
  return a;
}

// The deferred crack step (if any) on its own, its state going to slot 0.
int flush_deferred_crack(lbm_handle *h) {
  if (!h->crack_deferred) return LBM_OK;
  lbmk::CrackArgs a = deferred_crack_args(h);
  a.st_out = h->cslot ? h->crack_slot(0) : nullptr;
  HIP_TRY(lbmk::launch_crack(a, h->stream));
  h->crack_deferred = false;
  h->cslot = 0;
  return LBM_OK;
}

// The pinned verdict buffers of the speculative sweeps (one per sweep in
// flight), made with the first such sweep.
int ensure_spec_out(lbm_handle *h) {
  if (h->spec_dev) return LBM_OK;  // both pointers or neither
  lbmk::SpecOut *hp = nullptr;
  void *dp = nullptr;
  HIP_TRY(hipHostMalloc((void **)&hp, kSpecDepth * sizeof(lbmk::SpecOut),
                        hipHostMallocMapped | hipHostMallocCoherent));
  if (hipHostGetDevicePointer(&dp, hp, 0) != hipSuccess || !dp) {
    (void)hipHostFree(hp);
    return fail(LBM_EHIP, "no device address for the pinned verdict buffer");
  }
  h->spec_host = hp;
  h->spec_dev = static_cast<lbmk::SpecOut *>(dp);
  return LBM_OK;
}

// The crack steps of a T-step sweep of ns steps just enqueued: steps
// n .. n + ns - 2 from the crack rows after each (the side buffer), the last
// from the new state.
lbmk::CrackSeq crack_seq_args(const lbm_handle *h, int ns) {
  lbmk::CrackSeq q{};
  q.a = crack_args(h);
  q.n = ns;
  for (int m = 0; m < ns; ++m) {
    const bool mid = m + 1 < ns;
    q.w[m] = mid ? (const void *)(h->base + h->L.off_wmid + (size_t)2 * m * h->L.pitch * h->L.welem)
                 : q.a.w;
    q.w_row0[m] = mid ? h->plate.j0 : 0;
  }
  return q;
}

// K-criterion T-step sweeps with up to kSpecDepth of them in flight.  A
// speculative sweep is right or is run again with the steps its crack
// sequence found right (see lbm_step); instead of waiting for each verdict
// before queueing the next sweep, the host queues the next sweeps on the
// assumption that the pending ones hold, each gated on a device word: a
// crack sequence that finds a prediction wrong puts the start state back and
// closes the gate, so that everything queued after it returns at once and
// leaves buffers, mask and crack state as they were.  The host reads the
// verdicts in order (an event after each crack sequence); at a wrong one it
// rewinds to that sweep's start, opens the gate and queues the steps found
// right.  The kernels, their arguments and their order on the stream are
// those of one sweep at a time, so the results are the same bits.  The host
// polls the pinned verdicts (an event per verdict put one more marker between
// a crack sequence and the next sweep).  Returns in *done the steps advanced
// (every sweep resolved).
int spec_pipeline(lbm_handle *h, int64_t max_steps, int64_t *done) {
  *done = 0;
  int rc = ensure_spec_out(h);
  if (rc != LBM_OK) return rc;
  int32_t *gate = h->spec_gate();
  HIP_TRY(lbmk::launch_set_flag(gate, 1, h->stream));
  struct Pending {
    int64_t step0;
    int cur0, ns, slot;
  };
  Pending q[kSpecDepth];
  int qh = 0, qn = 0, next_slot = 0;
  int64_t queued = 0;  // steps queued (resolved or not)
  int force = 0;       // the next sweep's length after a wrong one (0: planned)
  h->blk_gate = gate;
  for (;;) {
    while (qn < kSpecDepth && (force > 0 || max_steps - queued >= 2)) {
      int ns = force > 0 ? force
                         : (int)std::min<int64_t>(std::min(h->tblock, std::max(2, h->spec_cap)),
                                                  max_steps - queued);
      force = 0;
      if (ns == 1) {
        // one step found right: the one-step sweep and its crack step
        rc = launch_sweep_any(h, nullptr);
        if (rc == LBM_OK) rc = launch_crack_step(h);
        if (rc != LBM_OK) break;
        h->cur = 1 - h->cur;
        h->step += 1;
        queued += 1;
        *done += 1;
        continue;
      }
      const int slot = next_slot;
      next_slot = (next_slot + 1) % kSpecDepth;
      *(volatile int32_t *)&h->spec_host[slot].valid = -1;
      rc = launch_block_any(h, ns);
      if (rc != LBM_OK) break;
      lbmk::CrackSeq cs = crack_seq_args(h, ns);
      cs.spec_out = h->spec_dev + slot;
      cs.spec = h->spec_slot();
      cs.spec_mask = h->spec_mask();
      cs.gate = gate;
      if (lbmk::launch_crack_seq(cs, h->stream) != hipSuccess) {
        rc = fail(LBM_EHIP, "queueing a speculative sweep failed");
        break;
      }
      q[(qh + qn) % kSpecDepth] = Pending{h->step, h->cur, ns, slot};
      qn++;
      h->cur = 1 - h->cur;
      h->step += ns;
      queued += ns;
    }
    if (rc != LBM_OK || qn == 0) break;
    const Pending f = q[qh];
    // the oldest verdict: its crack sequence runs (every one before it held),
    // and writes it into pinned memory; the host polls for it (a stream that
    // is idle with no verdict would be a fault, not a wait)
    int32_t valid = -1;
    for (int64_t it = 0;; ++it) {
      valid = *(volatile int32_t *)&h->spec_host[f.slot].valid;
      if (valid != -1) break;
      if ((it & 1023) == 1023) {
        const hipError_t e = hipStreamQuery(h->stream);
        if (e == hipSuccess) {
          valid = *(volatile int32_t *)&h->spec_host[f.slot].valid;
          if (valid == -1) rc = fail(LBM_EHIP, "a speculative sweep left no verdict");
          break;
        }
        if (e != hipErrorNotReady) {
          rc = fail(LBM_EHIP, "waiting for a speculative sweep failed: %s", hipGetErrorString(e));
          break;
        }
      }
    }
    if (rc != LBM_OK) break;
    if (valid < 1 || valid > f.ns) {
      rc = fail(LBM_EHIP, "bad speculation count %d", valid);
      break;
    }
    h->spec_blocks++;
    qh = (qh + 1) % kSpecDepth;
    qn--;
    if (valid == f.ns) {
      h->spec_cap = std::min(h->tblock, h->spec_cap + 1);
      *done += f.ns;
      continue;
    }
    // wrong from crack step `valid` on: the sweeps queued after it did nothing
    h->spec_reruns++;
    h->spec_cap = std::max(2, f.ns / 2);
    h->cur = f.cur0;
    h->step = f.step0;
    queued = *done;
    qn = 0;
    qh = 0;
    if (lbmk::launch_set_flag(gate, 1, h->stream) != hipSuccess) {
      rc = fail(LBM_EHIP, "reopening the gate failed");
      break;
    }
    force = valid;
  }
  h->blk_gate = nullptr;
  return rc;
}

// The macroscopic boundary scheme of step n = h->step on the buffers the
// sweep just wrote (Sec. 3.1).
int launch_macro(lbm_handle *h) {
  lbmk::MacroArgs m{};
  const int nxt = 1 - h->cur;
  m.fout = h->fbuf(nxt);
  m.win = h->wbuf(h->cur);
  m.wout = h->wbuf(nxt);
  m.mV = h->mV();
  m.p = h->plate;
  m.has_crack = h->cfg.has_crack;
  m.dmask = h->cfg.dirichlet;
  if (h->cfg.dirichlet) {
    const size_t r = 4 * (size_t)std::min<int64_t>(h->step, h->cfg.n_wD - 1);
    for (int k = 0; k < 4; ++k) m.wD[k] = h->wD[r + k];
  }
  const double tau = h->tau_at(h->step);
  m.t_top = tau;
  m.t_bot = -tau;
  m.t_face = h->cfg.face_traction;
  m.mu = h->cfg.mu;
  m.dt = h->dt;
  m.A0 = h->A0;
  m.Ak = h->Ak;
  m.rkey = lbmk::step_key(h->cfg.seed, h->step);
  m.err = reinterpret_cast<int *>(h->base + h->L.off_merr);
  HIP_TRY(lbmk::launch_macro_bc(h->store, h->cfg.rounding == LBM_ROUND_STOCHASTIC,
                                h->eq && h->full_steps == 0, m, h->stream));
  return LBM_OK;
}

// Reports (and clears) the macroscopic scheme's error flag; synchronises.
int check_macro(lbm_handle *h) {
  if (!h->macro()) return LBM_OK;
  int err = 0;
  HIP_TRY(hipMemcpyAsync(&err, h->base + h->L.off_merr, sizeof err, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (err) return fail(LBM_EHIP, "a boundary point of the macroscopic scheme depends deeper than two levels");
  return LBM_OK;
}

// Times each launch shape of a fixed grid over trial_steps whole steps and
// keeps the fastest.  set(rows, waves, occ) applies a shape, run(n) enqueues n
// steps on the stream.
template <typename Set, typename Run>
int tune_shapes(hipStream_t st, int32_t trial_steps, Set set, Run run, int32_t *rows_out,
                int32_t *waves_out, int32_t *occ_out, double *ms_out) {
  if (trial_steps < 1 || trial_steps > 1000) return fail(LBM_EINVAL, "trial_steps must be in 1..1000");
  static const int kRows[] = {1, 2, 4, 8};
  static const int kWaves[] = {1, 2, 4, 8};
  static const int kOcc[] = {0, 2, 3, 4, 5, 6};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return fail(LBM_EHIP, "event creation failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(LBM_EHIP, "event creation failed");
  }
  int rc = LBM_OK;
  float best = -1.0f;
  int br = 1, bw = 4, bo = 0;
  for (int r : kRows) {
    for (int w : kWaves) {
      for (int o : kOcc) {
        rc = set(r, w, o);
        if (rc == LBM_OK) rc = run(1);
        if (rc == LBM_OK && hipEventRecord(e0, st) != hipSuccess) rc = fail(LBM_EHIP, "event record failed");
        if (rc == LBM_OK) rc = run(trial_steps);
        if (rc == LBM_OK && hipEventRecord(e1, st) != hipSuccess) rc = fail(LBM_EHIP, "event record failed");
        float t = 0.0f;
        if (rc == LBM_OK && (hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&t, e0, e1) != hipSuccess))
          rc = fail(LBM_EHIP, "event timing failed");
        if (rc != LBM_OK) break;
        if (best < 0.0f || t < best) {
          best = t;
          br = r;
          bw = w;
          bo = o;
        }
      }
      if (rc != LBM_OK) break;
    }
    if (rc != LBM_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != LBM_OK) return rc;
  rc = set(br, bw, bo);
  if (rc != LBM_OK) return rc;
  if (rows_out) *rows_out = br;
  if (waves_out) *waves_out = bw;
  if (occ_out) *occ_out = bo;
  if (ms_out) *ms_out = (double)best / trial_steps;
  return LBM_OK;
}

// Time of one sweep of T = 1 .. 8 steps with the default shapes, in
// microseconds, measured on a 16384 x 8192 plate in the equilibrium layout
// with a crack growing at a prescribed speed (per-sweep HIP events over
// twenty sweeps in one call, best of three).  The sweep of six or eight
// steps costs little more than a short one: it moves the same bytes.  Only
// the ratios matter to the tail plan.
const double kSweepUs[4][lbmk::kMaxTimeBlock] = {
    {269.3, 317.4, 322.0, 342.6, 337.3, 347.9, 374.8, 408.4},   // FP16
    {270.0, 315.1, 325.1, 347.3, 338.6, 348.6, 364.8, 392.9},   // BF16
    {354.9, 389.6, 407.1, 417.3, 408.7, 421.3, 427.3, 446.8},   // FP32
    {686.0, 854.3, 844.3, 846.7, 882.9, 898.1, 862.6, 852.0}};  // FP64

int cost_row(Store s) {
  switch (s) {
    case Store::F16S: return 0;
    case Store::BF16S: return 1;
    case Store::F32S:
    case Store::F32_PLAIN: return 2;
    default: return 3;
  }
}

constexpr int kMaxTail = 32;  // 3 sweeps of at most 8 steps and a rest of at most 7

// The sweeps that end a call of n steps at T steps per sweep: the call runs
// (n - their sum) / T sweeps of T steps, then these.  A call whose step count
// is a multiple of T ends with none.  Otherwise the rest n mod T and the last
// j = 0 .. 3 sweeps of T steps before it are split anew into sweeps of 1 .. 8
// steps, taking the split of least predicted time over every j (ties: the
// smaller j); the sweeps come longest first.  Returns their number.
int plan_tail(int row, int T, int64_t n, int32_t *tail) {
  if (T < 2 || n <= 0 || n % T == 0) return 0;
  const double *c = kSweepUs[row];
  const int64_t q = n / T;
  const int r = (int)(n % T);
  const int jmax = (int)std::min<int64_t>(q, 3);
  const int mmax = jmax * T + r;
  // best[m]: least time of m steps in sweeps of 1 .. 8 steps; first[m]: one
  // sweep of that split (the longest where several splits tie)
  double best[kMaxTail] = {0.0};
  int first[kMaxTail] = {0};
  for (int m = 1; m <= mmax; ++m) {
    best[m] = 1e300;
    for (int t = std::min(m, lbmk::kMaxTimeBlock); t >= 1; --t) {
      const double v = c[t - 1] + best[m - t];
      if (v < best[m]) {
        best[m] = v;
        first[m] = t;
      }
    }
  }
  int jbest = 0;
  double vbest = 1e300;
  for (int j = 0; j <= jmax; ++j) {
    const double v = (double)(jmax - j) * c[T - 1] + best[j * T + r];
    if (v < vbest) {
      vbest = v;
      jbest = j;
    }
  }
  int k = 0;
  for (int m = jbest * T + r; m > 0; m -= first[m]) tail[k++] = first[m];
  std::sort(tail, tail + k, [](int32_t a, int32_t b) { return a > b; });
  return k;
}

}  // namespace

extern "C" {

const char *lbm_last_error(void) { return g_err.c_str(); }

size_t lbm_state_bytes(const lbm_config *cfg) {
  Store s;
  if (validate(cfg, &s) != LBM_OK) return 0;
  return make_layout(*cfg, s).total;
}

int lbm_init(const lbm_config *cfg, lbm_handle **out) {
  if (!out) return fail(LBM_EINVAL, "null output handle");
  *out = nullptr;
  Store s;
  int rc = validate(cfg, &s);
  if (rc != LBM_OK) return rc;
  Layout L = make_layout(*cfg, s);
  if (!cfg->dev_buf) return fail(LBM_EINVAL, "null dev_buf");
  if (reinterpret_cast<uintptr_t>(cfg->dev_buf) % 256)
    return fail(LBM_EINVAL, "dev_buf must be 256-byte aligned");
  if (cfg->dev_bytes < L.total)
    return fail(LBM_ENOMEM, "dev_bytes %zu < required %zu", cfg->dev_bytes, L.total);

  lbm_handle *h = new lbm_handle();
  h->cfg = *cfg;
  h->store = s;
  h->L = L;
  h->eq = cfg->layout == LBM_LAYOUT_EQ;
  // shifted FP64 holds w0 exactly: its initial moving populations are zero
  h->full_steps = (h->eq && s != Store::F64S) ? 2 : 0;
  h->stream = static_cast<hipStream_t>(cfg->stream);
  if (cfg->n_hist > 0) h->tau.assign(cfg->tau_hist, cfg->tau_hist + cfg->n_hist);
  h->cfg.tau_hist = nullptr;
  h->cfg.w0 = nullptr;
  h->cfg.wdot0 = nullptr;
  if (cfg->n_sensors > 0) h->sensors.assign(cfg->sensors, cfg->sensors + 2 * (size_t)cfg->n_sensors);
  h->cfg.sensors = nullptr;
  if (cfg->dirichlet) h->wD.assign(cfg->wD_hist, cfg->wD_hist + 4 * (size_t)cfg->n_wD);
  h->cfg.wD_hist = nullptr;
  h->base = static_cast<char *>(cfg->dev_buf);
  // lattice constants (Sec. 3): c = kappa c_s, dt = dh / c with dh = 1,
  // lambda = c_s^2 / (dt (1/omega - 1/2)), f_eq^0 = wdot - A0 w, f_eq^k = Ak w,
  // traction coefficient dt / (rho dh)
  h->cs = std::sqrt(cfg->mu / cfg->rho);
  h->c = cfg->kappa * h->cs;
  h->dt = 1.0 / h->c;
  h->lambda = h->cs * h->cs / (h->dt * (1.0 / cfg->omega - 0.5));
  h->A0 = 2.0 * h->lambda / (h->c * h->c);
  h->Ak = h->lambda / (2.0 * h->c * h->c);
  h->coef = h->dt / (cfg->rho * 1.0);
  lbmk::Plate &p = h->plate;
  p.nx = cfg->nx;
  p.ny = cfg->ny;
  p.pitch = L.pitch;
  p.mw = L.mw;
  p.j0 = cfg->crack_row >= 0 ? cfg->crack_row : cfg->ny / 2 - 1;
  p.periodic = cfg->bc_mode == LBM_BC_PERIODIC;
  p.plane = L.plane;
  // default launch shape, the fastest of the autotuner's grid on MI355X for a
  // 16384 x 8192 plate (much larger than the caches).  Five planes: one row
  // per wave, and a cap on the resident waves per SIMD -- 1-wave workgroups
  // with at most 2 resident waves per SIMD for 8- and 4-byte storage, 4-wave
  // workgroups with at most 4 for 16-bit storage.  Equilibrium layout (fewer
  // loads per row, so more rows and waves in flight pay): FP64 4 rows per
  // wave, 1-wave groups, at most 2 per SIMD; FP32 1 row, 8-wave groups, no
  // cap (with the crack step run by the sweep; 4-wave groups are 1 % faster
  // without it); 16-bit 2 rows, 8-wave groups, no cap.  lbm_autotune searches
  // the same grid for other plates.
  {
    const bool half = (s == Store::F16S || s == Store::BF16S);
    if (!h->eq) {
      h->rows = 1;
      h->waves = half ? 4 : 1;
      h->occ = half ? 4 : 2;
    } else if (is_fp64(s)) {
      h->rows = 4;
      h->waves = 1;
      h->occ = 2;
    } else {
      h->rows = half ? 2 : 1;
      h->waves = 8;
      h->occ = 0;
    }
    // T-step sweep (lbm_set_time_block): rows per wave, waves per group and
    // the cap on resident waves per SIMD of the fast launch (0 = none) for
    // T = 2 .. 8, the fastest measured on a 16384 x 8192 plate
    static_assert(lbmk::kMaxTimeBlock == 8, "one shape per T = 2 .. 8");
    static const int kShape[3][7][3] = {
        {{4, 4, 3}, {8, 4, 2}, {8, 4, 0}, {16, 2, 3}, {16, 4, 0}, {24, 4, 3}, {24, 4, 3}},   // 16-bit
        {{4, 4, 3}, {4, 4, 2}, {8, 4, 3}, {16, 4, 3}, {32, 4, 3}, {32, 4, 3}, {24, 4, 3}},   // FP32
        {{8, 2, 0}, {8, 2, 2}, {8, 4, 2}, {16, 4, 3}, {16, 4, 3}, {16, 4, 3}, {32, 4, 3}}};  // FP64
    const int kind = half ? 0 : (is_fp64(s) ? 2 : 1);
    for (int T = 2; T <= lbmk::kMaxTimeBlock; ++T) {
      h->blk_rows[T] = kShape[kind][T - 2][0];
      h->blk_waves[T] = kShape[kind][T - 2][1];
      h->blk_occ[T] = kShape[kind][T - 2][2];
    }
    // FP16 at T = 6: two chunks per fast wave, 58.1 against 59.4 us per step
    // (BF16, with more code per row, and 16-bit T = 7 / 8 are slower that
    // way); rows 32 in the table: FP32 T = 6 70.5 against 71.3 us, T = 7
    // 61.9 against 66.1, FP64 T = 8 106.6 against 110.4 (FP32 T = 8 is
    // slower: 86.1 against 59.3)
    if (s == Store::F16S) h->blk_rows[6] = 32;
    // rows 24 in the table (three 8-row chunks per fast wave): FP16 T = 7
    // 53.5 against 56.1 us per step with 16 rows, T = 8 51.0 against 54.3,
    // BF16 T = 7 51.9 against 54.5, T = 8 49.0 against 55.9, FP32 T = 8 56.2
    // against 58.8; not for FP32 T = 7 (62.8 against 62.1 with 32 rows) or
    // FP64 T = 8 (107.5 against 106.4)
  }

  {
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) ==
            hipSuccess && lds > 0)
      h->lds_per_cu = lds;
  }

  auto bail = [&](int code) {
    delete h;
    return code;
  };
  hipStream_t st = h->stream;
  if (lbmk::launch_zero(h->base, L.total, st) != hipSuccess)
    return bail(fail(LBM_EHIP, "zero fill failed: %s", hipGetErrorString(hipGetLastError())));
  // initial fields, staged through device memory in row chunks
  double *stage = h->stage();
  const size_t rowlen = (size_t)cfg->nx;
  for (int r0 = 0; r0 < cfg->ny; r0 += L.stage_rows) {
    const int nr = std::min(L.stage_rows, cfg->ny - r0);
    double *dw = nullptr, *dwd = nullptr;
    if (cfg->w0) {
      dw = stage;
      if (hipMemcpyAsync(dw, cfg->w0 + (size_t)r0 * rowlen, nr * rowlen * 8, hipMemcpyHostToDevice, st) != hipSuccess)
        return bail(fail(LBM_EHIP, "upload of w0 failed"));
    }
    if (cfg->wdot0) {
      dwd = stage + (size_t)L.stage_rows * rowlen;
      if (hipMemcpyAsync(dwd, cfg->wdot0 + (size_t)r0 * rowlen, nr * rowlen * 8, hipMemcpyHostToDevice, st) != hipSuccess)
        return bail(fail(LBM_EHIP, "upload of wdot0 failed"));
    }
    if (lbmk::launch_init_rows(s, h->fbuf(0), h->wbuf(0), h->wbuf(1), p, r0, nr, dw, dwd, h->A0, h->Ak, st) != hipSuccess)
      return bail(fail(LBM_EHIP, "init kernel failed"));
    if (hipStreamSynchronize(st) != hipSuccess) return bail(fail(LBM_EHIP, "init sync failed"));
  }
  crack_line(*cfg, &h->line, &h->a_lo, &h->a_hi);
  int64_t n_cut0 = 0;
  if (!cfg->has_crack) {
    h->skip_lo = 1;
    h->skip_hi = 0;
  } else if (h->line.aligned) {
    // links can be severed only on the crack row j0 (vertical links between
    // rows j0 and j0 + 1)
    h->skip_lo = p.j0;
    h->skip_hi = p.j0 + 1;
  } else {
    // every row within reach of the line between the ends the tips can reach
    const double e0 = cfg->both_tips ? h->a_lo : cfg->crack_x0;
    const double e1 = cfg->growth != LBM_GROW_NONE ? h->a_hi : cfg->crack_tip;
    double x, y0, y1;
    lbmk::geom::point_at(h->line, e0, &x, &y0);
    lbmk::geom::point_at(h->line, e1, &x, &y1);
    h->skip_lo = std::max(0, (int)std::ceil(std::fmin(y0, y1)) - 1);
    h->skip_hi = std::min(cfg->ny - 1, (int)std::floor(std::fmax(y0, y1)) + 1);
  }
  if (lbmk::launch_init_mask(h->mV(), h->mH(), h->mrows(), p,
                             cfg->has_crack && h->line.aligned, cfg->crack_x0, cfg->crack_tip,
                             st) != hipSuccess)
    return bail(fail(LBM_EHIP, "mask init failed"));
  if (cfg->has_crack && !h->line.aligned) {
    // the initial crack along another direction: every link the segment
    // x0 .. a0 touches, severed like a grown segment's links (Sec. 4.1), set on the host
    const int rows = p.ny, mw = p.mw;
    std::vector<uint32_t> mv((size_t)rows * mw, 0u), mhv((size_t)rows * mw, 0u);
    lbmk::MaskRows mr{1, 0, 1, 0};
    double xa, ya, xb, yb;
    lbmk::geom::point_at(h->line, cfg->crack_x0, &xa, &ya);
    lbmk::geom::point_at(h->line, cfg->crack_tip, &xb, &yb);
    const int ilo = std::max(0, (int)std::floor(std::fmin(xa, xb)) - 1);
    const int ihi = std::min(p.nx - 1, (int)std::ceil(std::fmax(xa, xb)) + 1);
    const int jlo = std::max(0, (int)std::floor(std::fmin(ya, yb)) - 1);
    const int jhi = std::min(p.ny - 1, (int)std::ceil(std::fmax(ya, yb)) + 1);
    for (int j = jlo; j <= jhi; ++j)
      for (int i = ilo; i <= ihi; ++i) {
        if (j + 1 < p.ny && lbmk::geom::touches_link(h->line, cfg->crack_x0, cfg->crack_tip, i, j, 0, 1)) {
          mv[(size_t)j * mw + (i >> 5)] |= 1u << (i & 31);
          mr.vlo = mr.vlo > mr.vhi ? j : std::min(mr.vlo, j);
          mr.vhi = std::max(mr.vhi, j);
          ++n_cut0;
        }
        if (i + 1 < p.nx && lbmk::geom::touches_link(h->line, cfg->crack_x0, cfg->crack_tip, i, j, 1, 0)) {
          mhv[(size_t)j * mw + (i >> 5)] |= 1u << (i & 31);
          mr.hlo = mr.hlo > mr.hhi ? j : std::min(mr.hlo, j);
          mr.hhi = std::max(mr.hhi, j);
          ++n_cut0;
        }
      }
    const size_t off = (size_t)jlo * mw * 4, len = (size_t)(jhi - jlo + 1) * mw * 4;
    if (hipMemcpyAsync(reinterpret_cast<char *>(h->mV()) + off, mv.data() + (size_t)jlo * mw, len,
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(reinterpret_cast<char *>(h->mH()) + off, mhv.data() + (size_t)jlo * mw, len,
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(h->mrows(), &mr, sizeof mr, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return bail(fail(LBM_EHIP, "upload of the initial crack failed"));
  }
  lbmk::DevCrack &c0 = h->host_crack;
  c0 = lbmk::DevCrack{};
  c0.tip = cfg->has_crack ? cfg->crack_tip : 0.0;
  c0.v = 0.0;
  c0.K = std::nan("");
  c0.r = std::nan("");
  c0.step = 0;
  c0.flags = 0;
  c0.n_events = 0;
  c0.col_K = -1;
  c0.tipL = cfg->has_crack ? cfg->crack_x0 : 0.0;
  c0.vL = 0.0;
  c0.KL = std::nan("");
  c0.rL = std::nan("");
  c0.flagsL = 0;
  c0.col_KL = -1;
  if (cfg->has_crack && h->line.aligned) {
    const int lo = std::max(0, (int)std::ceil(cfg->crack_x0));
    const int hi = std::min(cfg->nx - 1, (int)std::floor(cfg->crack_tip));
    c0.n_cut = hi >= lo ? hi - lo + 1 : 0;
  } else if (cfg->has_crack) {
    c0.n_cut = (int32_t)n_cut0;
  }
  if (hipMemcpyAsync(h->crack(), &c0, sizeof c0, hipMemcpyHostToDevice, st) != hipSuccess)
    return bail(fail(LBM_EHIP, "crack state upload failed"));
  if (h->fold_crack()) {
    // the four argument sets of a crack step run by a one-step sweep
    const int cur0 = h->cur, slot0 = h->cslot;
    for (int b = 0; b < 2; ++b)
      for (int k = 0; k < 2; ++k) {
        h->cur = b;
        h->cslot = k;
        lbmk::CrackArgs &a = h->host_fargs[2 * b + k];
        a = deferred_crack_args(h);
        a.st_out = h->crack_slot(1 - k);
        if (hipMemcpyAsync(const_cast<lbmk::CrackArgs *>(h->fused_args(b, k)), &a, sizeof a,
                           hipMemcpyHostToDevice, st) != hipSuccess)
          return bail(fail(LBM_EHIP, "crack argument upload failed"));
      }
    h->cur = cur0;
    h->cslot = slot0;
  }
  if (!h->sensors.empty() &&
      hipMemcpyAsync(h->base + L.off_sens, h->sensors.data(), h->sensors.size() * 4,
                     hipMemcpyHostToDevice, st) != hipSuccess)
    return bail(fail(LBM_EHIP, "sensor upload failed"));
  if (hipStreamSynchronize(st) != hipSuccess)
    return bail(fail(LBM_EHIP, "init failed: %s", hipGetErrorString(hipGetLastError())));
  *out = h;
  return LBM_OK;
}

int lbm_step(lbm_handle *h, int64_t nsteps) {
  if (!h) return fail(LBM_EINVAL, "null handle");
  if (h->in_batch) return fail(LBM_ESTATE, "this plate is stepped by its batch (lbm_batch_step)");
  if (nsteps < 0) return fail(LBM_EINVAL, "negative step count");
  const bool sif_blocks = h->tblock >= 2 && h->cfg.growth == LBM_GROW_SIF;
  // the sweeps that end this call (planned when the start-up steps are done;
  // the speculative sweeps of the K criterion take lengths of their own)
  int32_t tail[kMaxTail];
  int n_tail = -1, i_tail = 0;
  int64_t tail_steps = 0;
  for (int64_t k = 0; k < nsteps;) {
    // T steps in one sweep when time blocking is on and the moving planes
    // are settled (the five-plane start-up steps run one at a time); fewer
    // at the end of the call
    int ns = h->full_steps == 0 ? (int)std::min<int64_t>(h->tblock, nsteps - k) : 1;
    if (h->full_steps == 0 && h->tblock >= 2 && h->tail_plan && !sif_blocks) {
      if (n_tail < 0) {
        n_tail = plan_tail(cost_row(h->store), h->tblock, nsteps - k, tail);
        for (int m = 0; m < n_tail; ++m) tail_steps += tail[m];
      }
      if (nsteps - k <= tail_steps) {
        if (i_tail >= n_tail) return fail(LBM_EINVAL, "sweep plan out of step");
        ns = tail[i_tail++];
      }
    }
    if (sif_blocks) ns = std::min(ns, std::max(2, h->spec_cap));
    bool timed = false;
    for (int m = 0; m < ns; ++m) timed |= h->timing && (h->step + m) % h->timing_stride == 0;
    // a one-step sweep, a speculative sweep and a timed sweep run their crack
    // steps on the caller's stream: the crack steps still running on the side
    // stream come first (the sweep's crack rows read their mask and state)
    if (h->crack_pending && (ns < 2 || sif_blocks || timed)) {
      HIP_TRY(hipEventRecord(h->side.join, h->side.side));
      HIP_TRY(hipStreamWaitEvent(h->stream, h->side.join, 0));
      h->crack_pending = false;
    }
    // A one-step sweep runs the crack step of the step before it (which then
    // leaves its own to the next sweep, or to the launch at the end); other
    // sweeps find the crack steps done.
    const bool fold = ns < 2 && h->fold_crack();
    if (!fold) {
      const int rc = flush_deferred_crack(h);
      if (rc != LBM_OK) return rc;
    }
    // untimed speculative sweeps: several in flight
    if (sif_blocks && ns >= 2 && !h->timing) {
      int64_t done = 0;
      const int rc = spec_pipeline(h, nsteps - k, &done);
      if (rc != LBM_OK) return rc;
      k += done;
      continue;
    }
    // Under the K criterion the T-step sweep severs links as if each tip kept
    // its last speed; when a crack step before the last leaves a tip in
    // another column, the crack kernel puts back the state of step n and the
    // sweep runs again, from the same source buffers, for the steps that were
    // right (fewer each time, so this ends).
    for (;;) {
      hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
      if (timed) {
        for (auto &e : ev) {
          e = take_event(h);
          if (!e) return fail(LBM_EHIP, "event creation failed");
        }
        HIP_TRY(hipEventRecord(ev[0], h->stream));
      }
      int rc = LBM_OK;
      if (ns >= 2) {
        rc = launch_block_any(h, ns);
      } else if (h->crack_deferred) {
        rc = launch_sweep_any(h, h->fused_args(h->cur, h->cslot));
        if (rc == LBM_OK) {
          h->cslot = 1 - h->cslot;
          h->crack_deferred = false;
        }
      } else {
        rc = launch_sweep_any(h, nullptr);
      }
      if (rc == LBM_OK && h->macro()) rc = launch_macro(h);
      if (rc != LBM_OK) return rc;
      if (timed) HIP_TRY(hipEventRecord(ev[1], h->stream));
      bool spec = false;
      if (h->crack_step_needed()) {
        if (ns >= 2) {
          // steps n .. n + T - 2 from the crack rows after each, then the last
          // from the new state, in one launch
          lbmk::CrackSeq q = crack_seq_args(h, ns);
          spec = h->cfg.growth == LBM_GROW_SIF;
          if (spec) {
            rc = ensure_spec_out(h);
            if (rc != LBM_OK) return rc;
            *(volatile int32_t *)&h->spec_host->valid = -1;
            q.spec_out = h->spec_dev;
            q.spec = h->spec_slot();
            q.spec_mask = h->spec_mask();
          }
          if (!spec && !timed && h->side.side) {
            // on the side stream right after the boundary launch, whose rows
            // are all it reads: beside the rest of this sweep and the next
            HIP_TRY(lbmk::launch_crack_seq(q, h->side.side));
            h->crack_pending = true;
          } else {
            HIP_TRY(lbmk::launch_crack_seq(q, h->stream));
          }
        } else if (fold) {
          h->crack_deferred = true;
        } else {
          rc = launch_crack_step(h);
          if (rc != LBM_OK) return rc;
        }
      }
      if (timed) HIP_TRY(hipEventRecord(ev[2], h->stream));
      int32_t valid = ns;
      if (spec) {
        HIP_TRY(hipStreamSynchronize(h->stream));
        valid = *(volatile int32_t *)&h->spec_host->valid;
        if (valid < 1 || valid > ns) return fail(LBM_EHIP, "bad speculation count %d", valid);
        h->spec_blocks++;
        if (valid < ns) {
          h->spec_reruns++;
          h->spec_cap = std::max(2, ns / 2);
        } else {
          h->spec_cap = std::min(h->tblock, h->spec_cap + 1);
        }
      }
      if (timed) {
        // a sweep that is run again counts its time but not its steps
        for (auto &e : ev) h->ev_used.push_back(e);
        h->ev_steps.push_back(valid == ns ? ns : 0);
        if (h->ev_used.size() >= 3 * 4096) {
          rc = harvest_timing(h);
          if (rc != LBM_OK) return rc;
        }
      }
      if (valid == ns) break;
      ns = valid;
    }
    h->cur = 1 - h->cur;
    h->step += ns;
    k += ns;
    if (h->full_steps > 0) h->full_steps--;
  }
  {
    const int rc = flush_deferred_crack(h);
    if (rc != LBM_OK) return rc;
  }
  if (h->crack_pending) {
    // work the caller enqueues after lbm_step sees every crack step
    HIP_TRY(hipEventRecord(h->side.join, h->side.side));
    HIP_TRY(hipStreamWaitEvent(h->stream, h->side.join, 0));
    h->crack_pending = false;
  }
  return LBM_OK;
}

int lbm_crack_state(lbm_handle *h, lbm_crack_info *out) {
  if (!h || !out) return fail(LBM_EINVAL, "null argument");
  const int rc = check_macro(h);
  if (rc != LBM_OK) return rc;
  lbmk::DevCrack c{};
  HIP_TRY(hipMemcpyAsync(&c, h->crack(), sizeof c, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  out->tip = c.tip;
  out->v = c.v;
  out->K = c.K;
  out->r = c.r;
  out->step = h->cfg.has_crack ? c.step : h->step;
  out->flags = c.flags;
  out->n_events = c.n_events;
  out->col_K = c.col_K;
  out->n_cut = c.n_cut;
  out->tip_left = c.tipL;
  out->v_left = c.vL;
  out->K_left = c.KL;
  out->r_left = c.rL;
  out->flags_left = c.flagsL;
  out->col_K_left = c.col_KL;
  return LBM_OK;
}

static int check_range(lbm_handle *h, int64_t first, int64_t count, bool need_crack = true) {
  if (!h) return fail(LBM_EINVAL, "null handle");
  if (need_crack && !h->cfg.has_crack) return fail(LBM_ESTATE, "no crack: no traces");
  if (first < 0 || count < 0 || first + count > std::min<int64_t>(h->step, h->cfg.trace_cap))
    return fail(LBM_EINVAL, "trace range [%lld, %lld) outside the %lld recorded steps",
                (long long)first, (long long)(first + count),
                (long long)std::min<int64_t>(h->step, h->cfg.trace_cap));
  return LBM_OK;
}

int lbm_sif(lbm_handle *h, double *K_out, int64_t first, int64_t count) {
  int rc = check_range(h, first, count);
  if (rc != LBM_OK) return rc;
  if (count == 0) return LBM_OK;
  if (!K_out) return fail(LBM_EINVAL, "null output");
  HIP_TRY(hipMemcpyAsync(K_out, h->base + h->L.off_trK + first * 8, count * 8, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int lbm_traces(lbm_handle *h, double *tip_out, double *v_out, int32_t *flags_out, int64_t first,
               int64_t count) {
  int rc = check_range(h, first, count);
  if (rc != LBM_OK) return rc;
  if (count == 0) return LBM_OK;
  if (tip_out)
    HIP_TRY(hipMemcpyAsync(tip_out, h->base + h->L.off_trA + first * 8, count * 8, hipMemcpyDeviceToHost, h->stream));
  if (v_out)
    HIP_TRY(hipMemcpyAsync(v_out, h->base + h->L.off_trV + first * 8, count * 8, hipMemcpyDeviceToHost, h->stream));
  if (flags_out)
    HIP_TRY(hipMemcpyAsync(flags_out, h->base + h->L.off_trF + first * 4, count * 4, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int lbm_traces_left(lbm_handle *h, double *K_out, double *tip_out, double *v_out,
                    int32_t *flags_out, int64_t first, int64_t count) {
  int rc = check_range(h, first, count);
  if (rc != LBM_OK) return rc;
  if (!h->cfg.both_tips) return fail(LBM_ESTATE, "the crack has one tip");
  if (count == 0) return LBM_OK;
  const hipStream_t st = h->stream;
  if (K_out) HIP_TRY(hipMemcpyAsync(K_out, h->base + h->L.off_trKL + first * 8, count * 8, hipMemcpyDeviceToHost, st));
  if (tip_out) HIP_TRY(hipMemcpyAsync(tip_out, h->base + h->L.off_trAL + first * 8, count * 8, hipMemcpyDeviceToHost, st));
  if (v_out) HIP_TRY(hipMemcpyAsync(v_out, h->base + h->L.off_trVL + first * 8, count * 8, hipMemcpyDeviceToHost, st));
  if (flags_out) HIP_TRY(hipMemcpyAsync(flags_out, h->base + h->L.off_trFL + first * 4, count * 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return LBM_OK;
}

int lbm_sensor_traces(lbm_handle *h, double *out, int64_t first, int64_t count,
                      int32_t out_on_device) {
  int rc = check_range(h, first, count, false);
  if (rc != LBM_OK) return rc;
  if (h->cfg.n_sensors == 0 || count == 0) return LBM_OK;
  if (!out) return fail(LBM_EINVAL, "null output");
  const size_t row = (size_t)h->cfg.n_sensors * 8;
  HIP_TRY(hipMemcpyAsync(out, h->base + h->L.off_trS + first * row, count * row,
                         out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                         h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int lbm_cut_links(lbm_handle *h, int64_t *steps, int32_t *i_out, int32_t *j_out, int32_t *orient,
                  int64_t cap, int64_t *n) {
  if (!h || !n) return fail(LBM_EINVAL, "null argument");
  lbmk::DevCrack c{};
  HIP_TRY(hipMemcpyAsync(&c, h->crack(), sizeof c, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  const int64_t total = c.n_events;
  const int64_t m = std::min<int64_t>(std::min<int64_t>(total, cap), h->L.event_cap);
  const hipStream_t st = h->stream;
  if (m > 0 && steps) HIP_TRY(hipMemcpyAsync(steps, h->base + h->L.off_evS, m * 8, hipMemcpyDeviceToHost, st));
  if (m > 0 && i_out) HIP_TRY(hipMemcpyAsync(i_out, h->base + h->L.off_evC, m * 4, hipMemcpyDeviceToHost, st));
  if (m > 0 && j_out) HIP_TRY(hipMemcpyAsync(j_out, h->base + h->L.off_evJ, m * 4, hipMemcpyDeviceToHost, st));
  if (m > 0 && orient) HIP_TRY(hipMemcpyAsync(orient, h->base + h->L.off_evO, m * 4, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  *n = total;
  return LBM_OK;
}

int lbm_cut_events(lbm_handle *h, int64_t *steps, int32_t *cols, int64_t cap, int64_t *n) {
  if (!h || !n) return fail(LBM_EINVAL, "null argument");
  lbmk::DevCrack c{};
  HIP_TRY(hipMemcpyAsync(&c, h->crack(), sizeof c, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  const int64_t total = c.n_events;
  const int64_t m = std::min<int64_t>(std::min<int64_t>(total, cap), h->L.event_cap);
  if (m > 0 && steps)
    HIP_TRY(hipMemcpyAsync(steps, h->base + h->L.off_evS, m * 8, hipMemcpyDeviceToHost, h->stream));
  if (m > 0 && cols)
    HIP_TRY(hipMemcpyAsync(cols, h->base + h->L.off_evC, m * 4, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  *n = total;
  return LBM_OK;
}

static int export_rows(lbm_handle *h, double *w_out, double *wd_out, double *f_out) {
  const lbmk::Plate &p = h->plate;
  const int sr = h->L.stage_rows;
  double *stage = h->stage();
  const size_t chunk = (size_t)sr * p.nx;
  const void *f = h->fbuf(h->cur);
  const void *w = h->wbuf(h->cur);
  const size_t n = (size_t)p.nx * p.ny;
  for (int r0 = 0; r0 < p.ny; r0 += sr) {
    const int nr = std::min(sr, p.ny - r0);
    const size_t cnt = (size_t)nr * p.nx;
    double *dw = w_out ? stage : nullptr;
    double *dwd = wd_out ? stage + chunk : nullptr;
    double *df = f_out ? stage : nullptr;  // f export uses the whole stage (5 chunks)
    if (f_out) {
      dw = nullptr;
      dwd = nullptr;
    }
    HIP_TRY(lbmk::launch_export_rows(h->store, f, w, p, r0, nr, h->A0, h->Ak, dw, dwd, df, h->stream));
    if (w_out) HIP_TRY(hipMemcpyAsync(w_out + (size_t)r0 * p.nx, dw, cnt * 8, hipMemcpyDeviceToHost, h->stream));
    if (wd_out) HIP_TRY(hipMemcpyAsync(wd_out + (size_t)r0 * p.nx, dwd, cnt * 8, hipMemcpyDeviceToHost, h->stream));
    if (f_out)
      for (int a = 0; a < 5; ++a)
        HIP_TRY(hipMemcpyAsync(f_out + a * n + (size_t)r0 * p.nx, df + a * cnt, cnt * 8,
                               hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
  }
  return LBM_OK;
}

int lbm_get_fields(lbm_handle *h, double *w_out, double *wdot_out) {
  if (!h) return fail(LBM_EINVAL, "null handle");
  if (!w_out && !wdot_out) return LBM_OK;
  const int rc = check_macro(h);
  if (rc != LBM_OK) return rc;
  return export_rows(h, w_out, wdot_out, nullptr);
}

int lbm_get_populations(lbm_handle *h, double *f_out) {
  if (!h || !f_out) return fail(LBM_EINVAL, "null argument");
  return export_rows(h, nullptr, nullptr, f_out);
}

// Checkpoint layout: a 256-byte header, the five current population planes,
// the current w plane, then the layout region from the cut mask to the sensor
// traces (mask, mask-row range, crack state, traces, events, sensors).
namespace {
struct CkptHeader {
  uint64_t magic;
  int64_t step;
  uint64_t f_bytes, w_bytes, tail_bytes;
  int32_t nx, ny, storage, scheme;  // scheme: the storage scheme (shifted or not)
};
constexpr uint64_t kCkptMagic = 0x4c424d434b505431ull;  // "LBMCKPT1"

void ckpt_sizes(const lbm_handle *h, size_t *f, size_t *w, size_t *tail) {
  *f = h->L.off_f[1] - h->L.off_f[0];
  *w = h->L.off_w[1] - h->L.off_w[0];
  *tail = h->L.off_stage - h->L.off_mV;
}
}  // namespace

size_t lbm_checkpoint_bytes(const lbm_handle *h) {
  if (!h) return 0;
  size_t f, w, tail;
  ckpt_sizes(h, &f, &w, &tail);
  return 256 + f + w + tail;
}

int lbm_checkpoint(lbm_handle *h, void *dst) {
  if (!h || !dst) return fail(LBM_EINVAL, "null argument");
  if (h->in_batch) return fail(LBM_ESTATE, "plates of a batch are not checkpointed one by one");
  size_t f, w, tail;
  ckpt_sizes(h, &f, &w, &tail);
  CkptHeader hd{kCkptMagic, h->step, f, w, tail, h->cfg.nx, h->cfg.ny, h->cfg.storage,
                (int32_t)h->store};
  char *d = static_cast<char *>(dst);
  HIP_TRY(hipMemcpyAsync(d, &hd, sizeof hd, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipMemcpyAsync(d + 256, h->fbuf(h->cur), f, hipMemcpyDeviceToDevice, h->stream));
  HIP_TRY(hipMemcpyAsync(d + 256 + f, h->wbuf(h->cur), w, hipMemcpyDeviceToDevice, h->stream));
  HIP_TRY(hipMemcpyAsync(d + 256 + f + w, h->base + h->L.off_mV, tail, hipMemcpyDeviceToDevice,
                         h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int lbm_restore(lbm_handle *h, const void *src) {
  if (!h || !src) return fail(LBM_EINVAL, "null argument");
  if (h->in_batch) return fail(LBM_ESTATE, "plates of a batch are not restored one by one");
  size_t f, w, tail;
  ckpt_sizes(h, &f, &w, &tail);
  CkptHeader hd{};
  const char *s = static_cast<const char *>(src);
  HIP_TRY(hipMemcpyAsync(&hd, s, sizeof hd, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (hd.magic != kCkptMagic || hd.f_bytes != f || hd.w_bytes != w || hd.tail_bytes != tail ||
      hd.nx != h->cfg.nx || hd.ny != h->cfg.ny || hd.storage != h->cfg.storage ||
      hd.scheme != (int32_t)h->store)
    return fail(LBM_EINVAL, "checkpoint does not belong to a plate of this configuration");
  HIP_TRY(hipMemcpyAsync(h->fbuf(h->cur), s + 256, f, hipMemcpyDeviceToDevice, h->stream));
  HIP_TRY(hipMemcpyAsync(h->wbuf(h->cur), s + 256 + f, w, hipMemcpyDeviceToDevice, h->stream));
  HIP_TRY(hipMemcpyAsync(h->base + h->L.off_mV, s + 256 + f + w, tail, hipMemcpyDeviceToDevice,
                         h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  h->step = hd.step;
  h->full_steps = (h->eq && h->store != Store::F64S) ? 2 : 0;
  return LBM_OK;
}

int lbm_get_mask(lbm_handle *h, uint8_t *cutV, uint8_t *cutH) {
  if (!h) return fail(LBM_EINVAL, "null handle");
  const lbmk::Plate &p = h->plate;
  const size_t n = (size_t)p.nx * p.ny;
  // bytes staged through the FP64 stage area in row chunks
  const size_t cap = (size_t)h->L.stage_rows * p.nx * 8 * 5;
  const int rows = (int)std::max<size_t>(1, std::min<size_t>(p.ny, cap / (2 * (size_t)p.nx)));
  uint8_t *sv = reinterpret_cast<uint8_t *>(h->stage());
  for (int r0 = 0; r0 < p.ny; r0 += rows) {
    const int nr = std::min(rows, p.ny - r0);
    lbmk::Plate q = p;
    q.ny = nr;
    const size_t cnt = (size_t)nr * p.nx;
    HIP_TRY(lbmk::launch_export_mask(h->mV() + (size_t)r0 * p.mw, h->mH() + (size_t)r0 * p.mw, q,
                                     cutV ? sv : nullptr, cutH ? sv + cnt : nullptr, h->stream));
    if (cutV) HIP_TRY(hipMemcpyAsync(cutV + (size_t)r0 * p.nx, sv, cnt, hipMemcpyDeviceToHost, h->stream));
    if (cutH) HIP_TRY(hipMemcpyAsync(cutH + (size_t)r0 * p.nx, sv + cnt, cnt, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
  }
  (void)n;
  return LBM_OK;
}

int lbm_timing(lbm_handle *h, int32_t enable, double *sweep_ms, double *crack_ms, int64_t *n_timed) {
  if (!h) return fail(LBM_EINVAL, "null handle");
  int rc = harvest_timing(h);
  if (rc != LBM_OK) return rc;
  if (sweep_ms) *sweep_ms = h->t_sweep;
  if (crack_ms) *crack_ms = h->t_crack;
  if (n_timed) *n_timed = h->n_timed;
  if (enable < 0) return fail(LBM_EINVAL, "negative timing stride");
  if (enable && !h->timing) {
    h->t_sweep = h->t_crack = 0;
    h->n_timed = 0;
  }
  h->timing = enable != 0;
  if (enable) h->timing_stride = enable;
  return LBM_OK;
}

int lbm_get_launch(lbm_handle *h, int32_t *vec, int32_t *rows, int32_t *waves, int32_t *occupancy) {
  if (!h) return fail(LBM_EINVAL, "null handle");
  if (vec) *vec = lbmk::sweep_vec(h->store);
  if (rows) *rows = h->rows;
  if (waves) *waves = h->waves;
  if (occupancy) *occupancy = h->occ;
  return LBM_OK;
}

int lbm_set_launch(lbm_handle *h, int32_t rows, int32_t waves, int32_t occupancy) {
  if (!h) return fail(LBM_EINVAL, "null handle");
  if (rows < 1 || rows > 4096) return fail(LBM_EINVAL, "rows must be in 1..4096");
  if (waves != 1 && waves != 2 && waves != 4 && waves != 8) return fail(LBM_EINVAL, "waves must be 1, 2, 4 or 8");
  if (occupancy < 0 || occupancy > 8) return fail(LBM_EINVAL, "occupancy must be in 0..8");
  h->rows = rows;
  h->waves = waves;
  h->occ = occupancy;
  return LBM_OK;
}

int lbm_set_time_block(lbm_handle *h, int32_t steps, int32_t rows, int32_t waves) {
  if (!h) return fail(LBM_EINVAL, "null handle");
  if (steps < 1 || steps > lbmk::kMaxTimeBlock)
    return fail(LBM_EINVAL, "steps per sweep must be 1 to 8");
  if (rows != 0 && rows != 4 && rows != 8 && rows != 16 && rows != 24 && rows != 32)
    return fail(LBM_EINVAL, "rows must be 4, 8, 16, 24 (T >= 6) or 32 (0 = keep)");
  if (waves != 0 && waves != 1 && waves != 2 && waves != 4 && waves != 8)
    return fail(LBM_EINVAL, "waves must be 0 (keep), 1, 2, 4 or 8");
  if (rows == 24 && steps < 6) return fail(LBM_EINVAL, "24 rows per wave: sweeps of six or more steps");
  if (steps >= 6 && rows != 0 && rows < 16)
    return fail(LBM_EINVAL, "sweeps of six or more steps take 16 or more rows per wave");
  if (steps == 1 && (rows != 0 || waves != 0))
    return fail(LBM_EINVAL, "rows and waves shape the T-step sweep (steps 2..8)");
  if (steps >= 2) {
    if (!h->eq || h->store == Store::F32_PLAIN || h->store == Store::F64)
      return fail(LBM_EINVAL, "the T-step sweep needs the equilibrium layout");
    if (h->cfg.bc_mode == LBM_BC_PERIODIC) return fail(LBM_EINVAL, "the T-step sweep needs walls");
    if (h->cfg.has_crack && !h->line.aligned)
      return fail(LBM_EINVAL, "the T-step sweep takes a crack along +x only");
    if (h->cfg.n_sensors > 0) return fail(LBM_EINVAL, "the T-step sweep records no sensors");
    if (h->macro()) return fail(LBM_EINVAL, "the macroscopic boundary scheme runs one step per sweep");
  }
  HIP_TRY(hipStreamSynchronize(h->stream));
  h->tblock = steps;
  h->spec_cap = steps;
  if (rows > 0) h->blk_rows[steps] = rows;
  if (waves > 0) h->blk_waves[steps] = waves;
  return LBM_OK;
}

int lbm_set_tail_plan(lbm_handle *h, int32_t on) {
  if (!h) return fail(LBM_EINVAL, "null handle");
  if (on != 0 && on != 1) return fail(LBM_EINVAL, "on must be 0 or 1");
  h->tail_plan = on != 0;
  return LBM_OK;
}

int lbm_plan_tail(int32_t storage, int32_t steps_per_sweep, int64_t nsteps, int32_t *tail,
                  int32_t *n_tail) {
  if (storage < LBM_F64 || storage > LBM_F32_PLAIN) return fail(LBM_EINVAL, "unknown storage %d", storage);
  if (steps_per_sweep < 1 || steps_per_sweep > lbmk::kMaxTimeBlock)
    return fail(LBM_EINVAL, "steps per sweep must be 1 to 8");
  if (nsteps < 0) return fail(LBM_EINVAL, "negative step count");
  if (!tail || !n_tail) return fail(LBM_EINVAL, "null output");
  const Store s = storage == LBM_F16S ? Store::F16S : storage == LBM_BF16S ? Store::BF16S
                  : storage == LBM_F64 ? Store::F64S : Store::F32S;
  *n_tail = plan_tail(cost_row(s), steps_per_sweep, nsteps, tail);
  return LBM_OK;
}

int lbm_sweep_cost(int32_t storage, int32_t steps, double *us) {
  if (storage < LBM_F64 || storage > LBM_F32_PLAIN) return fail(LBM_EINVAL, "unknown storage %d", storage);
  if (steps < 1 || steps > lbmk::kMaxTimeBlock) return fail(LBM_EINVAL, "steps must be 1 to 8");
  if (!us) return fail(LBM_EINVAL, "null output");
  const Store s = storage == LBM_F16S ? Store::F16S : storage == LBM_BF16S ? Store::BF16S
                  : storage == LBM_F64 ? Store::F64S : Store::F32S;
  *us = kSweepUs[cost_row(s)][steps - 1];
  return LBM_OK;
}

int lbm_time_block_stats(lbm_handle *h, int64_t *sweeps, int64_t *reruns) {
  if (!h) return fail(LBM_EINVAL, "null handle");
  if (sweeps) *sweeps = h->spec_blocks;
  if (reruns) *reruns = h->spec_reruns;
  return LBM_OK;
}

int lbm_round16(const float *x, void *out, int64_t n, int32_t storage, int32_t rounding,
                int32_t plane, uint32_t seed, int64_t step, void *stream) {
  if (n < 0 || (n > 0 && (!x || !out))) return fail(LBM_EINVAL, "bad arrays");
  if (n > (int64_t)UINT32_MAX) return fail(LBM_EINVAL, "site indices are 32-bit");
  if (storage != LBM_F16S && storage != LBM_BF16S) return fail(LBM_EINVAL, "16-bit storages only");
  if (rounding != LBM_ROUND_NEAREST && rounding != LBM_ROUND_STOCHASTIC)
    return fail(LBM_EINVAL, "unknown rounding %d", rounding);
  if (plane < 0 || plane > 4) return fail(LBM_EINVAL, "plane must be in 0..4");
  const Store s = storage == LBM_F16S ? Store::F16S : Store::BF16S;
  HIP_TRY(lbmk::launch_round16(s, rounding == LBM_ROUND_STOCHASTIC, x, out, n, plane,
                               lbmk::step_key(seed, step), static_cast<hipStream_t>(stream)));
  return LBM_OK;
}

int lbm_autotune(lbm_handle *h, int32_t trial_steps, int32_t *rows, int32_t *waves,
                 int32_t *occupancy, double *ms_per_step) {
  if (!h) return fail(LBM_EINVAL, "null handle");
  if (h->in_batch) return fail(LBM_ESTATE, "plate belongs to a batch: tune the batch");
  const bool was_timing = h->timing;
  h->timing = false;
  const int rc = tune_shapes(
      h->stream, trial_steps, [h](int r, int w, int o) { return lbm_set_launch(h, r, w, o); },
      [h](int64_t n) { return lbm_step(h, n); }, rows, waves, occupancy, ms_per_step);
  h->timing = was_timing;
  return rc;
}

int lbm_autotune_time_block(lbm_handle *h, int32_t steps, int32_t trial_sweeps, int32_t *rows,
                            int32_t *waves, double *ms_per_step) {
  if (!h) return fail(LBM_EINVAL, "null handle");
  if (h->in_batch) return fail(LBM_ESTATE, "plates of a batch step one time step per sweep");
  if (steps < 2 || steps > lbmk::kMaxTimeBlock) return fail(LBM_EINVAL, "steps must be 2 to 8");
  if (trial_sweeps < 1 || trial_sweeps > 1000)
    return fail(LBM_EINVAL, "trial_sweeps must be in 1..1000");
  static const int kRows[] = {4, 8, 16, 24, 32};
  static const int kWaves[] = {1, 2, 4, 8};
  int rc = lbm_set_time_block(h, steps, 0, 0);  // refuses plates the T-step sweep cannot take
  if (rc != LBM_OK) return rc;
  const bool was_timing = h->timing;
  h->timing = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    h->timing = was_timing;
    return fail(LBM_EHIP, "event creation failed");
  }
  float best = -1.0f;
  int br = h->blk_rows[steps], bw = h->blk_waves[steps];
  for (int r : kRows) {
    if ((steps >= 6 && r < 16) || (steps < 6 && r == 24)) continue;
    for (int w : kWaves) {
      rc = lbm_set_time_block(h, steps, r, w);
      if (rc == LBM_OK) rc = lbm_step(h, steps);
      if (rc == LBM_OK && hipEventRecord(e0, h->stream) != hipSuccess)
        rc = fail(LBM_EHIP, "event record failed");
      if (rc == LBM_OK) rc = lbm_step(h, (int64_t)trial_sweeps * steps);
      if (rc == LBM_OK && hipEventRecord(e1, h->stream) != hipSuccess)
        rc = fail(LBM_EHIP, "event record failed");
      float t = 0.0f;
      if (rc == LBM_OK && (hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&t, e0, e1) != hipSuccess))
        rc = fail(LBM_EHIP, "event timing failed");
      if (rc != LBM_OK) break;
      if (best < 0.0f || t < best) {
        best = t;
        br = r;
        bw = w;
      }
    }
    if (rc != LBM_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->timing = was_timing;
  if (rc != LBM_OK) return rc;
  rc = lbm_set_time_block(h, steps, br, bw);
  if (rc != LBM_OK) return rc;
  if (rows) *rows = br;
  if (waves) *waves = bw;
  if (ms_per_step) *ms_per_step = (double)best / ((double)trial_sweeps * steps);
  return LBM_OK;
}

double lbm_bytes_per_site(const lbm_handle *h) {
  if (!h) return 0.0;
  const double e = (double)elem_size(h->store), we = is_fp64(h->store) ? 8.0 : 4.0;
  return 2.0 * ((h->eq ? 1.0 : 5.0) * e + we) / h->tblock;
}

void lbm_free(lbm_handle *h) {
  if (!h) return;
  if (!h->ev_used.empty() || h->side.side) (void)hipStreamSynchronize(h->stream);
  for (hipEvent_t e : h->ev_used) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  if (h->side.side) {
    (void)hipStreamSynchronize(h->side.side);
    (void)hipEventDestroy(h->side.fork);
    (void)hipEventDestroy(h->side.join);
    (void)hipStreamDestroy(h->side.side);
  }
  if (h->spec_host) (void)hipHostFree(h->spec_host);
  delete h;
}

}  // extern "C"

// ------------------------------------------------------------------ batches --

struct lbm_batch {
  std::vector<lbm_handle *> plates;
  Store store = Store::F32S;
  hipStream_t stream = nullptr;
  char *base = nullptr;
  size_t off_desc = 0, off_tau = 0, off_sync = 0, total = 0;
  std::vector<size_t> off_plate;
  std::vector<size_t> off_tau_plate;
  std::vector<lbmk::BatchPlate> desc;
  int64_t n_int = 0, n_bnd = 0;
  int rows = 1, waves = 4, occ = 0, lds_per_cu = 65536;
  int cur = 0;
  int64_t step = 0;
  bool timing = false;
  std::vector<hipEvent_t> ev_pool, ev_used;
  double t_ms = 0;
  int64_t n_timed = 0;
  int persistent_blocks = 0;
  int sr = 0;  // stochastic rounding (same for every plate)
  bool eq = false;     // equilibrium layout (same for every plate)
  int full_steps = 0;  // five-plane steps still to run (see lbm_handle)
  int device = 0;      // the GPU the batch's memory is on (current at lbm_batch_init)
  // fold: every plate that has a crack step has its crack along +x, so the
  // sweep of step n + 1 runs the crack steps of step n (as a single plate's
  // one-step sweeps do); crack_deferred and cslot as in lbm_handle.  Between
  // calls nothing is deferred and every state is in slot 0.
  bool fold = false;
  bool crack_deferred = false;
  int cslot = 0;
};

namespace {

struct BatchLayout {
  std::vector<size_t> off_plate, off_tau_plate;
  size_t off_desc = 0, off_tau = 0, off_sync = 0, total = 0;
};

// offset of a plate's wall-displacement history inside its history block
size_t wd_offset(const lbm_config &c) {
  return align_up(sizeof(double) * (size_t)std::max<int64_t>(c.n_hist, 1), 256);
}

int batch_layout(const lbm_config *cfgs, int32_t n, BatchLayout *B, Store *store) {
  if (!cfgs || n < 1 || n > 65536) return fail(LBM_EINVAL, "a batch needs 1..65536 plates");
  size_t o = 0;
  for (int k = 0; k < n; ++k) {
    Store s;
    int rc = validate(&cfgs[k], &s);
    if (rc != LBM_OK) return fail(rc, "plate %d: %s", k, g_err.c_str());
    if (cfgs[k].bc_scheme != LBM_BC_LINK)
      return fail(LBM_EINVAL, "plate %d: the batched kernels bounce back per link (bc_scheme LINK)", k);
    if (k == 0) *store = s;
    else if (s != *store) return fail(LBM_EINVAL, "plate %d: every plate of a batch needs the same storage", k);
    if (cfgs[k].rounding != cfgs[0].rounding)
      return fail(LBM_EINVAL, "plate %d: every plate of a batch needs the same rounding", k);
    if (cfgs[k].layout != cfgs[0].layout)
      return fail(LBM_EINVAL, "plate %d: every plate of a batch needs the same layout", k);
    B->off_plate.push_back(o);
    o += align_up(make_layout(cfgs[k], s).total, 256);
  }
  B->off_desc = o;
  o += align_up(sizeof(lbmk::BatchPlate) * n, 256);
  B->off_tau = o;
  for (int k = 0; k < n; ++k) {
    B->off_tau_plate.push_back(o);  // traction history, then wall displacements
    o += align_up(sizeof(double) * (size_t)std::max<int64_t>(cfgs[k].n_hist, 1), 256);
    o += align_up(sizeof(double) * 4 * (size_t)std::max<int64_t>(cfgs[k].dirichlet ? cfgs[k].n_wD : 0, 1), 256);
  }
  B->off_sync = o;
  o += align_up(lbmk::persistent_sync_bytes(n), 256);  // the persistent run's synchronisation words
  B->total = o;
  return LBM_OK;
}

int batch_build_desc(lbm_batch *b) {
  const int n = (int)b->plates.size();
  const int vec = lbmk::sweep_vec(b->store);
  b->desc.assign(n, lbmk::BatchPlate{});
  int64_t ti = 0, tb = 0;
  for (int k = 0; k < n; ++k) {
    const lbm_handle *h = b->plates[k];
    lbmk::BatchPlate &d = b->desc[k];
    d.f[0] = h->fbuf(0);
    d.f[1] = h->fbuf(1);
    d.w[0] = h->wbuf(0);
    d.w[1] = h->wbuf(1);
    d.mV = h->mV();
    d.mH = h->mH();
    d.mrows = h->mrows();
    d.p = h->plate;
    d.omega = h->cfg.omega;
    d.dt = h->dt;
    d.A0 = h->A0;
    d.Ak = h->Ak;
    d.coef = h->coef;
    d.face = h->cfg.bc_mode == LBM_BC_PERIODIC ? 0.0 : h->cfg.face_traction;
    d.tau = reinterpret_cast<const double *>(b->base + b->off_tau_plate[k]);
    d.n_hist = (int64_t)h->tau.size();
    d.has_crack = h->cfg.has_crack;
    d.seed = h->cfg.seed;
    d.dmask = h->cfg.bc_mode == LBM_BC_PERIODIC ? 0 : h->cfg.dirichlet;
    d.wD = reinterpret_cast<const double *>(b->base + b->off_tau_plate[k] + wd_offset(h->cfg));
    d.n_wD = (int64_t)h->wD.size() / 4;
    d.skip_lo = h->skip_lo;
    d.skip_hi = h->skip_hi;
    // the same task maps as the single-plate kernels
    d.im = lbmk::core::interior_map(h->plate.nx, h->plate.ny, vec, b->rows, d.skip_lo, d.skip_hi);
    d.bm = lbmk::core::boundary_map(h->plate.nx, h->plate.ny, vec, d.skip_lo, d.skip_hi);
    d.itask0 = ti;
    d.btask0 = tb;
    ti += lbmk::core::interior_task_count(d.im);
    tb += lbmk::core::boundary_task_count(d.bm);
    d.crack = crack_args(h);
    d.st2 = h->crack_slot(1);
    for (int c = 0; c < 2; ++c)
      for (int k2 = 0; k2 < 2; ++k2) d.fargs[2 * c + k2] = h->fused_args(c, k2);
  }
  bool any = false, all = true;
  for (const lbm_handle *h : b->plates) {
    any |= h->crack_step_needed();
    all &= !h->crack_step_needed() || h->fold_crack();
  }
  b->fold = any && all;
  b->n_int = ti;
  b->n_bnd = tb;
  HIP_TRY(hipMemcpyAsync(b->base + b->off_desc, b->desc.data(), sizeof(lbmk::BatchPlate) * n,
                         hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  return LBM_OK;
}

void batch_sync_handles(lbm_batch *b) {
  for (lbm_handle *h : b->plates) {
    h->cur = b->cur;
    h->step = b->step;
  }
}

int batch_lds(const lbm_batch *b) {
  if (b->occ <= 0) return 0;
  const int groups = std::max(1, (b->occ * 4) / b->waves);
  return std::min(65536, (b->lds_per_cu / groups) / 256 * 256);
}

}  // namespace

extern "C" {

size_t lbm_batch_state_bytes(const lbm_config *cfgs, int32_t n) {
  BatchLayout B;
  Store s;
  if (batch_layout(cfgs, n, &B, &s) != LBM_OK) return 0;
  return B.total;
}

int lbm_batch_init(const lbm_config *cfgs, int32_t n, void *dev_buf, size_t dev_bytes, void *stream,
                   lbm_batch **out) {
  if (!out) return fail(LBM_EINVAL, "null output batch");
  *out = nullptr;
  BatchLayout B;
  Store s;
  int rc = batch_layout(cfgs, n, &B, &s);
  if (rc != LBM_OK) return rc;
  if (!dev_buf || reinterpret_cast<uintptr_t>(dev_buf) % 256)
    return fail(LBM_EINVAL, "dev_buf must be a 256-byte aligned device pointer");
  if (dev_bytes < B.total) return fail(LBM_ENOMEM, "dev_bytes %zu < required %zu", dev_bytes, B.total);
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return fail(LBM_EHIP, "no current device");
  {  // the fixed scratch of lbm_batch_run_persistent_static: its address on this device
    void *sp = nullptr;
    size_t sbytes = 0;
    const hipError_t e = lbmk::static_scratch(&sp, &sbytes);
    if (e != hipSuccess) return fail(LBM_EHIP, "static scratch lookup failed: %s", hipGetErrorString(e));
  }
  lbm_batch *b = new lbm_batch();
  b->device = device;
  b->store = s;
  b->sr = cfgs[0].rounding == LBM_ROUND_STOCHASTIC;
  b->eq = cfgs[0].layout == LBM_LAYOUT_EQ;
  b->full_steps = (b->eq && s != Store::F64S) ? 2 : 0;
  b->stream = static_cast<hipStream_t>(stream);
  b->base = static_cast<char *>(dev_buf);
  b->off_plate = B.off_plate;
  b->off_tau_plate = B.off_tau_plate;
  b->off_desc = B.off_desc;
  b->off_tau = B.off_tau;
  b->off_sync = B.off_sync;
  b->total = B.total;
  auto bail = [&](int code) {
    for (lbm_handle *h : b->plates) lbm_free(h);
    delete b;
    return code;
  };
  for (int k = 0; k < n; ++k) {
    lbm_config c = cfgs[k];
    c.dev_buf = b->base + B.off_plate[k];
    c.dev_bytes = (k + 1 < n ? B.off_plate[k + 1] : B.off_desc) - B.off_plate[k];
    c.stream = stream;
    lbm_handle *h = nullptr;
    rc = lbm_init(&c, &h);
    if (rc != LBM_OK) return bail(fail(rc, "plate %d: %s", k, g_err.c_str()));
    h->in_batch = true;
    b->plates.push_back(h);
    if (!h->tau.empty() &&
        hipMemcpy(b->base + B.off_tau_plate[k], h->tau.data(), sizeof(double) * h->tau.size(),
                  hipMemcpyHostToDevice) != hipSuccess)
      return bail(fail(LBM_EHIP, "upload of the traction history failed"));
    if (!h->wD.empty() &&
        hipMemcpy(b->base + B.off_tau_plate[k] + wd_offset(cfgs[k]), h->wD.data(),
                  sizeof(double) * h->wD.size(), hipMemcpyHostToDevice) != hipSuccess)
      return bail(fail(LBM_EHIP, "upload of the wall displacements failed"));
  }
  // launch shape: that of a plate of the batch's storage and layout
  b->rows = b->plates[0]->rows;
  b->waves = b->plates[0]->waves;
  b->occ = b->plates[0]->occ;
  b->lds_per_cu = b->plates[0]->lds_per_cu;
  rc = batch_build_desc(b);
  if (rc != LBM_OK) return bail(rc);
  *out = b;
  return LBM_OK;
}

int lbm_batch_step(lbm_batch *b, int64_t nsteps) {
  if (!b) return fail(LBM_EINVAL, "null batch");
  if (nsteps < 0) return fail(LBM_EINVAL, "negative step count");
  const auto *d = reinterpret_cast<const lbmk::BatchPlate *>(b->base + b->off_desc);
  const int n = (int)b->plates.size();
  const int lds = batch_lds(b);
  for (int64_t k = 0; k < nsteps; ++k) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (b->timing) {
      if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(LBM_EHIP, "event creation failed");
      HIP_TRY(hipEventRecord(e0, b->stream));
    }
    // with fold: this sweep runs the crack steps of the step before it (if
    // deferred) and leaves its own to the next sweep or to the launch after
    // the call's last step
    const int slot = b->fold && b->crack_deferred ? b->cslot : -1;
    HIP_TRY(lbmk::launch_batch_sweep(b->store, b->sr, b->eq && b->full_steps == 0, d, n, b->n_int,
                                     b->n_bnd, b->cur, b->step, b->waves, lds, slot, b->stream));
    if (slot >= 0) b->cslot = 1 - b->cslot;
    b->cur = 1 - b->cur;
    b->step++;
    if (b->full_steps > 0) b->full_steps--;
    if (b->fold) b->crack_deferred = true;
    if (!b->fold || k + 1 == nsteps) {
      HIP_TRY(lbmk::launch_batch_crack(d, n, b->cur, b->cslot, b->stream));
      b->crack_deferred = false;
      b->cslot = 0;
    }
    if (b->timing) {
      HIP_TRY(hipEventRecord(e1, b->stream));
      b->ev_used.push_back(e0);
      b->ev_used.push_back(e1);
    }
  }
  batch_sync_handles(b);
  return LBM_OK;
}

int lbm_batch_run_persistent(lbm_batch *b, int64_t nsteps) {
  if (!b) return fail(LBM_EINVAL, "null batch");
  if (nsteps < 0) return fail(LBM_EINVAL, "negative step count");
  if (nsteps == 0) return LBM_OK;
  if (b->full_steps > 0) {  // the five-plane steps of a fresh state run one launch each
    const int64_t k = std::min<int64_t>(nsteps, b->full_steps);
    const int rc = lbm_batch_step(b, k);
    if (rc != LBM_OK || k == nsteps) return rc;
    nsteps -= k;
  }
  const auto *d = reinterpret_cast<const lbmk::BatchPlate *>(b->base + b->off_desc);
  unsigned *sync = reinterpret_cast<unsigned *>(b->base + b->off_sync);
  HIP_TRY(lbmk::launch_zero(sync, lbmk::persistent_sync_bytes((int)b->plates.size()), b->stream));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (b->timing) {
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
      return fail(LBM_EHIP, "event creation failed");
    HIP_TRY(hipEventRecord(e0, b->stream));
  }
  int blocks = 0;
  hipError_t e = lbmk::launch_batch_persistent(b->store, b->sr, b->eq, d, (int)b->plates.size(), b->n_int, b->n_bnd,
                                               b->cur, b->step, nsteps, sync, &blocks, b->stream);
  if (e != hipSuccess) return fail(LBM_EHIP, "persistent launch failed: %s", hipGetErrorString(e));
  b->persistent_blocks = blocks;
  if (b->timing) {
    HIP_TRY(hipEventRecord(e1, b->stream));
    b->ev_used.push_back(e0);
    b->ev_used.push_back(e1);
  }
  unsigned flag = 0;
  HIP_TRY(hipMemcpyAsync(&flag, sync + 64, sizeof flag, hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  b->cur = (int)((b->cur + nsteps) & 1);
  b->step += nsteps;
  batch_sync_handles(b);
  if (flag) return fail(LBM_EHIP, "grid barrier timed out: the persistent run is invalid");
  return LBM_OK;
}

int lbm_batch_run_persistent_static(lbm_batch *b, int64_t nsteps) {
  if (!b) return fail(LBM_EINVAL, "null batch");
  if (nsteps < 0) return fail(LBM_EINVAL, "negative step count");
  if (nsteps == 0) return LBM_OK;
  const int n = (int)b->plates.size();
  const size_t need = lbmk::persistent_sync_bytes(n);
  int prev = -1;
  HIP_TRY(hipGetDevice(&prev));
  if (prev != b->device) HIP_TRY(hipSetDevice(b->device));
  struct Restore {  // the caller's current device, whatever the return path
    int dev, was;
    ~Restore() {
      if (dev != was) (void)hipSetDevice(was);
    }
  } restore{b->device, prev};
  void *sp = nullptr;
  size_t cap = 0;
  const hipError_t le = lbmk::static_scratch(&sp, &cap);
  if (le != hipSuccess) return fail(LBM_EHIP, "static scratch lookup failed: %s", hipGetErrorString(le));
  if (need > cap)
    return fail(LBM_EINVAL, "a batch of %d plates needs %zu bytes of static scratch; it holds %zu", n,
                need, cap);
  // no events here (they would be created): timing stays off for this call
  const bool timing = b->timing;
  b->timing = false;
  int rc = LBM_OK;
  if (b->full_steps > 0) {  // the five-plane steps of a fresh state run one launch each
    const int64_t k = std::min<int64_t>(nsteps, b->full_steps);
    rc = lbm_batch_step(b, k);
    nsteps -= k;
  }
  b->timing = timing;
  if (rc != LBM_OK || nsteps == 0) return rc;
  const auto *d = reinterpret_cast<const lbmk::BatchPlate *>(b->base + b->off_desc);
  unsigned *sync = static_cast<unsigned *>(sp);
  // the array keeps the last call's contents: the words that must start at
  // zero are cleared by a fill kernel (no memset node, so a captured graph
  // replays it correctly)
  HIP_TRY(lbmk::launch_zero(sync, need, b->stream));
  int blocks = 0;
  const hipError_t e = lbmk::launch_batch_persistent(b->store, b->sr, b->eq, d, n, b->n_int, b->n_bnd,
                                                     b->cur, b->step, nsteps, sync, &blocks, b->stream);
  if (e != hipSuccess) return fail(LBM_EHIP, "persistent launch failed: %s", hipGetErrorString(e));
  b->persistent_blocks = blocks;
  unsigned flag = 0;
  HIP_TRY(hipMemcpyAsync(&flag, sync + 64, sizeof flag, hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  b->cur = (int)((b->cur + nsteps) & 1);
  b->step += nsteps;
  batch_sync_handles(b);
  if (flag) return fail(LBM_EHIP, "grid barrier timed out: the persistent run is invalid");
  return LBM_OK;
}

lbm_handle *lbm_batch_plate(lbm_batch *b, int32_t k) {
  if (!b || k < 0 || k >= (int32_t)b->plates.size()) {
    fail(LBM_EINVAL, "no plate %d in this batch", k);
    return nullptr;
  }
  return b->plates[k];
}

int lbm_batch_set_launch(lbm_batch *b, int32_t rows, int32_t waves, int32_t occupancy) {
  if (!b) return fail(LBM_EINVAL, "null batch");
  if (rows < 1 || rows > 4096) return fail(LBM_EINVAL, "rows must be in 1..4096");
  if (waves != 1 && waves != 2 && waves != 4 && waves != 8) return fail(LBM_EINVAL, "waves must be 1, 2, 4 or 8");
  if (occupancy < 0 || occupancy > 8) return fail(LBM_EINVAL, "occupancy must be in 0..8");
  HIP_TRY(hipStreamSynchronize(b->stream));
  b->rows = rows;
  b->waves = waves;
  b->occ = occupancy;
  return batch_build_desc(b);
}

int lbm_batch_get_launch(lbm_batch *b, int32_t *rows, int32_t *waves, int32_t *occupancy,
                         int32_t *persistent_blocks) {
  if (!b) return fail(LBM_EINVAL, "null batch");
  if (rows) *rows = b->rows;
  if (waves) *waves = b->waves;
  if (occupancy) *occupancy = b->occ;
  if (persistent_blocks) *persistent_blocks = b->persistent_blocks;
  return LBM_OK;
}

int lbm_batch_autotune(lbm_batch *b, int32_t trial_steps, int32_t *rows, int32_t *waves,
                       int32_t *occupancy, double *ms_per_step) {
  if (!b) return fail(LBM_EINVAL, "null batch");
  const bool was_timing = b->timing;
  b->timing = false;
  const int rc = tune_shapes(
      b->stream, trial_steps, [b](int r, int w, int o) { return lbm_batch_set_launch(b, r, w, o); },
      [b](int64_t n) { return lbm_batch_step(b, n); }, rows, waves, occupancy, ms_per_step);
  b->timing = was_timing;
  return rc;
}

int lbm_batch_timing(lbm_batch *b, int32_t enable, double *ms, int64_t *n_timed) {
  if (!b) return fail(LBM_EINVAL, "null batch");
  if (!b->ev_used.empty()) {
    HIP_TRY(hipStreamSynchronize(b->stream));
    for (size_t k = 0; k + 1 < b->ev_used.size(); k += 2) {
      float t = 0;
      HIP_TRY(hipEventElapsedTime(&t, b->ev_used[k], b->ev_used[k + 1]));
      b->t_ms += t;
      b->n_timed += 1;
    }
    for (hipEvent_t e : b->ev_used) (void)hipEventDestroy(e);
    b->ev_used.clear();
  }
  if (ms) *ms = b->t_ms;
  if (n_timed) *n_timed = b->n_timed;
  if (enable && !b->timing) {
    b->t_ms = 0;
    b->n_timed = 0;
  }
  b->timing = enable != 0;
  return LBM_OK;
}

int64_t lbm_batch_sites(const lbm_batch *b) {
  if (!b) return 0;
  int64_t s = 0;
  for (const lbm_handle *h : b->plates) s += (int64_t)h->plate.nx * h->plate.ny;
  return s;
}

void lbm_batch_free(lbm_batch *b) {
  if (!b) return;
  if (!b->ev_used.empty()) (void)hipStreamSynchronize(b->stream);
  for (hipEvent_t e : b->ev_used) (void)hipEventDestroy(e);
  for (lbm_handle *h : b->plates) lbm_free(h);
  delete b;
}

}  // extern "C"

// ------------------------------------------------------------------ adjoint --

struct lbm_adjoint {
  lbm_handle *h = nullptr;
  bool fp64 = false;
  lbmk::Plate p{};       // the plate with pitch / plane in adjoint elements
  char *base = nullptr;
  size_t off_m[2] = {0, 0}, off_w[2] = {0, 0}, off_cut = 0, off_part = 0, off_srow = 0,
         off_srt = 0, total = 0;
  int n_parts = 0;
  int64_t cap = 0;       // sweeps the partial-sum table holds (trace_cap + 1)
  const double *g = nullptr;  // loss gradient of the current run
  double ms = 0;
  int64_t sweeps = 0;
};

namespace {

struct AdjLayout {
  size_t esize = 0, plane = 0, off_m[2] = {0, 0}, off_w[2] = {0, 0}, off_cut = 0, off_part = 0,
         off_srow = 0, off_srt = 0, total = 0;
  int n_parts = 0;
  int64_t cap = 0;
};

AdjLayout adjoint_layout(const lbm_handle *h) {
  AdjLayout A;
  A.esize = is_fp64(h->store) ? 8 : 4;
  const size_t pb = align_up((size_t)h->L.pitch * h->cfg.ny * A.esize, 256) + 1024;
  A.plane = pb / A.esize;
  size_t o = 0;
  for (int b = 0; b < 2; ++b) {
    A.off_m[b] = o;
    o += 5 * pb;
  }
  for (int b = 0; b < 2; ++b) {
    A.off_w[b] = o;
    o += pb;
  }
  A.off_cut = o;
  o += align_up((size_t)h->cfg.nx * 4, 256);
  A.n_parts = lbmk::adjoint_parts(h->cfg.nx);
  A.cap = std::max<int64_t>(h->cfg.trace_cap, 0) + 1;
  A.off_part = o;
  o += align_up((size_t)A.cap * 4 * A.n_parts * 8, 256);
  A.off_srow = o;  // sensors by row: first entry of each row, ny + 1 values
  o += align_up(((size_t)h->cfg.ny + 1) * 4, 256);
  A.off_srt = o;   // (column, sensor index) sorted by row
  o += align_up((size_t)std::max(h->cfg.n_sensors, 1) * 8, 256);
  A.total = o;
  return A;
}

template <typename C>
int adjoint_sweep(lbm_adjoint *a, int cur, int64_t m) {
  const lbm_handle *h = a->h;
  lbmk::AdjArgs<C> g{};
  g.min = reinterpret_cast<const C *>(a->base + a->off_m[cur]);
  g.mout = reinterpret_cast<C *>(a->base + a->off_m[1 - cur]);
  g.win = reinterpret_cast<const C *>(a->base + a->off_w[cur]);
  g.wout = reinterpret_cast<C *>(a->base + a->off_w[1 - cur]);
  g.p = a->p;
  const bool init = m == 0;  // transpose of the initial equilibrium
  g.omega = init ? C(1) : (C)h->cfg.omega;
  g.dt = init ? C(0) : (C)h->dt;
  g.A0 = (C)h->A0;
  g.Ak = (C)h->Ak;
  g.m = m;
  g.cutstep = reinterpret_cast<const int32_t *>(a->base + a->off_cut);
  g.has_crack = h->cfg.has_crack;
  g.traction = h->cfg.bc_mode != LBM_BC_PERIODIC;
  g.dmask = h->cfg.bc_mode == LBM_BC_PERIODIC ? 0 : h->cfg.dirichlet;
  g.coef = h->coef;
  g.dtau_part = reinterpret_cast<double *>(a->base + a->off_part) + (size_t)m * 4 * a->n_parts;
  g.n_parts = a->n_parts;
  if (h->cfg.has_crack) {
    g.skip_lo = h->plate.j0;
    g.skip_hi = h->plate.j0 + 1;
  } else {
    g.skip_lo = 1;
    g.skip_hi = 0;
  }
  // the sweep writes the adjoint of w after step m - 1; the loss gradient of
  // that trace row (step m - 2 of the trace) joins it there (m - 1 >= 1)
  const int ns = h->cfg.n_sensors;
  g.g = (ns > 0 && m >= 2) ? a->g + (size_t)(m - 2) * ns : nullptr;
  g.srow = reinterpret_cast<const int32_t *>(a->base + a->off_srow);
  g.srt = reinterpret_cast<const int32_t *>(a->base + a->off_srt);
  HIP_TRY(lbmk::launch_adjoint_sweep(a->fp64, h->eq, &g, h->stream));
  return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_adjoint_bytes(const lbm_handle *h) {
  if (!h) return 0;
  return adjoint_layout(h).total;
}

int lbm_adjoint_init(lbm_handle *h, void *dev_buf, size_t dev_bytes, lbm_adjoint **out) {
  if (!h || !out) return fail(LBM_EINVAL, "null argument");
  *out = nullptr;
  const AdjLayout A = adjoint_layout(h);
  if (!dev_buf || reinterpret_cast<uintptr_t>(dev_buf) % 256)
    return fail(LBM_EINVAL, "dev_buf must be a 256-byte aligned device pointer");
  if (dev_bytes < A.total) return fail(LBM_ENOMEM, "dev_bytes %zu < required %zu", dev_bytes, A.total);
  if (h->macro())
    return fail(LBM_EINVAL, "the adjoint transposes the per-link boundary scheme only (bc_scheme LINK)");
  if (h->cfg.has_crack && !h->line.aligned)
    return fail(LBM_EINVAL, "the adjoint takes cracks along +x only (the cut steps are kept per column)");
  lbm_adjoint *a = new lbm_adjoint();
  a->h = h;
  a->fp64 = is_fp64(h->store);
  a->p = h->plate;
  a->p.plane = A.plane;
  a->base = static_cast<char *>(dev_buf);
  for (int b = 0; b < 2; ++b) {
    a->off_m[b] = A.off_m[b];
    a->off_w[b] = A.off_w[b];
  }
  a->off_cut = A.off_cut;
  a->off_part = A.off_part;
  a->off_srow = A.off_srow;
  a->off_srt = A.off_srt;
  a->total = A.total;
  a->n_parts = A.n_parts;
  a->cap = A.cap;
  *out = a;
  return LBM_OK;
}

int lbm_adjoint_run(lbm_adjoint *a, const double *g, double *dL_dtau, double *dL_dwdot0,
                    double *dL_dw0) {
  if (!a) return fail(LBM_EINVAL, "null adjoint");
  lbm_handle *h = a->h;
  const int64_t T = h->step;
  if (T < 1) return fail(LBM_ESTATE, "the handle has taken no step");
  if (T > h->cfg.trace_cap || T + 1 > a->cap)
    return fail(LBM_ESTATE, "%lld steps taken, but the traces hold %lld", (long long)T,
                (long long)h->cfg.trace_cap);
  const int ns = h->cfg.n_sensors;
  if (ns > 0 && !g) return fail(LBM_EINVAL, "null loss gradient");
  hipStream_t st = h->stream;
  // the step at which each crack-row link was severed (-1: initially)
  std::vector<int32_t> cut(h->cfg.nx, INT32_MAX);
  if (h->cfg.has_crack) {
    const int lo = std::max(0, (int)std::ceil(h->cfg.crack_x0));
    const int hi = std::min(h->cfg.nx - 1, (int)std::floor(h->cfg.crack_tip));
    for (int i = lo; i <= hi; ++i) cut[i] = -1;
    lbmk::DevCrack c{};
    HIP_TRY(hipMemcpyAsync(&c, h->crack(), sizeof c, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const int64_t ne = std::min<int64_t>(c.n_events, h->L.event_cap);
    if (ne > 0) {
      std::vector<int64_t> es(ne);
      std::vector<int32_t> ec(ne);
      HIP_TRY(hipMemcpyAsync(es.data(), h->base + h->L.off_evS, ne * 8, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipMemcpyAsync(ec.data(), h->base + h->L.off_evC, ne * 4, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      for (int64_t k = 0; k < ne; ++k)
        if (ec[k] >= 0 && ec[k] < h->cfg.nx) cut[ec[k]] = (int32_t)es[k];
    }
  }
  // lambda_T = (0, dL/dw_T): a zero state (and zero partial sums), then the
  // last trace row's gradient
  HIP_TRY(lbmk::launch_zero(a->base, a->total, st));
  HIP_TRY(hipMemcpyAsync(a->base + a->off_cut, cut.data(), cut.size() * 4, hipMemcpyHostToDevice, st));
  // sensors indexed by row for the in-sweep injection of the loss gradient
  std::vector<int32_t> srow(h->cfg.ny + 1, 0), srt(2 * (size_t)std::max(ns, 1), 0);
  {
    std::vector<int32_t> order(ns);
    for (int k = 0; k < ns; ++k) order[k] = k;
    std::sort(order.begin(), order.end(), [&](int x, int y) {
      const int jx = h->sensors[2 * x + 1], jy = h->sensors[2 * y + 1];
      return jx != jy ? jx < jy : h->sensors[2 * x] < h->sensors[2 * y];
    });
    for (int e = 0; e < ns; ++e) {
      srt[2 * e] = h->sensors[2 * order[e]];
      srt[2 * e + 1] = order[e];
      srow[h->sensors[2 * order[e] + 1] + 1] += 1;
    }
    for (int j = 0; j < h->cfg.ny; ++j) srow[j + 1] += srow[j];
  }
  HIP_TRY(hipMemcpyAsync(a->base + a->off_srow, srow.data(), srow.size() * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(a->base + a->off_srt, srt.data(), srt.size() * 4, hipMemcpyHostToDevice, st));
  a->g = g;
  const int32_t *sens = reinterpret_cast<const int32_t *>(h->base + h->L.off_sens);
  if (ns > 0)
    HIP_TRY(lbmk::launch_adjoint_inject(a->fp64, a->base + a->off_w[0], a->p, sens, ns,
                                        g + (size_t)(T - 1) * ns, st));
  struct Events {  // destroyed on every return path
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Events() {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  } ev;
  HIP_TRY(hipEventCreate(&ev.e0));
  HIP_TRY(hipEventCreate(&ev.e1));
  hipEvent_t e0 = ev.e0, e1 = ev.e1;
  HIP_TRY(hipEventRecord(e0, st));
  int cur = 0;
  for (int64_t m = T; m >= 0; --m) {
    const int rc = a->fp64 ? adjoint_sweep<double>(a, cur, m) : adjoint_sweep<float>(a, cur, m);
    if (rc != LBM_OK) return rc;
    cur = 1 - cur;
  }
  HIP_TRY(hipEventRecord(e1, st));
  if (dL_dwdot0) HIP_TRY(lbmk::launch_adjoint_export(a->fp64, a->base + a->off_m[cur], a->p, dL_dwdot0, st));
  if (dL_dw0) HIP_TRY(lbmk::launch_adjoint_export(a->fp64, a->base + a->off_w[cur], a->p, dL_dw0, st));
  std::vector<double> parts;
  if (dL_dtau) {
    parts.resize((size_t)T * 4 * a->n_parts);
    HIP_TRY(hipMemcpyAsync(parts.data(), a->base + a->off_part, parts.size() * 8, hipMemcpyDeviceToHost, st));
  }
  HIP_TRY(hipStreamSynchronize(st));
  float ms = 0;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  a->ms = ms;
  a->sweeps = T + 1;
  if (dL_dtau) {
    // rows the boundary kernel did not use hold zeros
    for (int64_t n = 0; n < T; ++n) {
      double s = 0.0;
      for (int r = 0; r < 4; ++r)
        for (int b = 0; b < a->n_parts; ++b) s += parts[((size_t)n * 4 + r) * a->n_parts + b];
      dL_dtau[n] = s;
    }
  }
  return LBM_OK;
}

int lbm_adjoint_timing(lbm_adjoint *a, double *ms, int64_t *sweeps) {
  if (!a) return fail(LBM_EINVAL, "null adjoint");
  if (ms) *ms = a->ms;
  if (sweeps) *sweeps = a->sweeps;
  return LBM_OK;
}

void lbm_adjoint_free(lbm_adjoint *a) { delete a; }

}  // extern "C"
