// Internal declarations of liblbmcrack: device-side layout, kernel argument
// blocks and the launch functions of the HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace lbmk {

// Crack state kept on the device and updated by the one-wavefront crack
// kernel after each sweep (Alg. 1, CrackGrowth).
struct DevCrack {
  double tip;        // a_n
  double v;          // speed of the last step / c_s
  double K;          // K_III of the last step
  double r;          // distance used for K
  int64_t step;      // steps completed
  int32_t flags;     // LBM_FLAG_* of the last step (WALL is sticky)
  int32_t n_events;  // cut events recorded
  int32_t col_K;     // column of the last K (-1: undefined)
  int32_t n_cut;     // severed links on the crack row
  // the left end: a second tip growing in -x when both tips grow
  double tipL, vL, KL, rL;
  int32_t flagsL, col_KL;
};

// Static description of one plate's lattice as the kernels see it.
struct Plate {
  int nx, ny;        // sites
  int pitch;         // elements per row (multiple of 64)
  int mw;            // mask words per row (multiple of 2)
  int j0;            // crack row (the crack line is y = j0 + 1/2)
  int periodic;      // both axes wrap
  size_t plane;      // elements between population planes
};

namespace core {

// Interior work of a plate: the strips of 64 * VEC sites times the chunks of
// `rows` consecutive interior rows, which are 1 .. skip_lo-1 and
// skip_hi+1 .. ny-2 (the rows skip_lo .. skip_hi and the two edge rows belong
// to the boundary work).  Task t -> strip t % n_strips, chunk t / n_strips.
struct InteriorMap {
  int n_strips, rows, lo1, hi1, lo2, hi2, nc1, nc2;
};

__host__ __device__ inline InteriorMap interior_map(int nx, int ny, int vec, int rows, int skip_lo,
                                                    int skip_hi) {
  InteriorMap m;
  m.n_strips = (nx + 64 * vec - 1) / (64 * vec);
  m.rows = rows;
  const bool has_skip = skip_lo <= skip_hi;
  m.lo1 = 1;
  m.hi1 = has_skip ? skip_lo - 1 : ny - 2;
  m.lo2 = has_skip ? skip_hi + 1 : ny;
  m.hi2 = ny - 2;
  m.nc1 = m.hi1 >= m.lo1 ? (m.hi1 - m.lo1 + rows) / rows : 0;
  m.nc2 = m.hi2 >= m.lo2 ? (m.hi2 - m.lo2 + rows) / rows : 0;
  return m;
}

__host__ __device__ inline long interior_task_count(const InteriorMap &m) {
  return (long)m.n_strips * (m.nc1 + m.nc2);
}

// Boundary work of a plate: every strip of each boundary row, the rows being
// row 0, the skipped rows lo .. hi (the rows a crack can ever touch) and row
// ny - 1, each once, in that order.  Task t -> row row_of(t / n_strips).
struct BoundaryMap {
  int n_strips, nb;
  int c0;      // 1 if row 0 comes first (it is not inside lo .. hi)
  int lo, hi;  // skipped rows (lo > hi: none)
  int top;     // row ny - 1 (listed last when it is not row 0 or inside lo .. hi)
};

__host__ __device__ inline BoundaryMap boundary_map(int nx, int ny, int vec, int skip_lo,
                                                    int skip_hi) {
  BoundaryMap m;
  m.n_strips = (nx + 64 * vec - 1) / (64 * vec);
  m.lo = skip_lo < 0 ? 0 : skip_lo;
  m.hi = skip_hi > ny - 1 ? ny - 1 : skip_hi;
  const bool has = m.lo <= m.hi;
  if (!has) {
    m.lo = 1;
    m.hi = 0;
  }
  m.c0 = (!has || m.lo > 0) ? 1 : 0;
  const bool top = ny - 1 > 0 && (!has || m.hi < ny - 1);
  m.top = ny - 1;
  m.nb = m.c0 + (has ? m.hi - m.lo + 1 : 0) + (top ? 1 : 0);
  return m;
}

__host__ __device__ inline int boundary_row_of(const BoundaryMap &m, int r) {
  if (r < m.c0) return 0;
  r -= m.c0;
  const int mid = m.hi >= m.lo ? m.hi - m.lo + 1 : 0;
  return r < mid ? m.lo + r : m.top;
}

__host__ __device__ inline long boundary_task_count(const BoundaryMap &m) {
  return (long)m.n_strips * m.nb;
}

}  // namespace core

// Parameters of the crack step.
struct CrackParams {
  int crack;         // the plate has a crack (else only the sensors are recorded)
  int both;          // the left end grows as well (two tips)
  int growth;        // LBM_GROW_*
  int band;          // columns in the K fit
  double v_rel, K_C, r0, v_max;
  double cs, dt, mu;
  double x0;         // left end of the crack line
  int aligned;       // the crack grows along +x on its row
  double yc;         // y of the start point (x0, yc)
  double ux, uy;     // unit growth direction of the right tip
  double a_lo, a_hi; // line coordinates where the line leaves the plate
  int64_t trace_cap;
  int64_t event_cap;
};

// Rows of the cut bitmask that may hold a severed link: vertical links in
// rows vlo..vhi, horizontal links in rows hlo..hhi (lo > hi: none).  Kept on
// the device next to the mask and widened by the crack kernel; the sweep
// reads it once per wave, so rows away from the crack never touch the mask.
struct MaskRows {
  int32_t vlo, vhi, hlo, hhi;
};

// Per-launch arguments of the sweep.  S is the storage type of the
// populations, W the storage type of w, C the compute type.  The source and
// destination buffers are distinct (populations and w are double-buffered).
template <typename S, typename W, typename C>
struct SweepArgs {
  const S *fin;      // plane 0 of the source populations
  S *fout;           // plane 0 of the destination populations
  const W *win;      // w before the step
  W *wout;           // w after the step
  const uint32_t *mV, *mH;
  const MaskRows *mrows;
  Plate p;
  C omega, dt, A0, Ak;
  C t_top, t_bot;    // coef * traction on top / bottom edge links
  C t_up, t_lo;      // coef * traction on the crack face above / below
  int rows;          // rows marched by one wave of the interior kernel
  int waves;         // waves per workgroup of the interior kernel
  int lds_bytes;     // LDS reserved per interior workgroup (caps resident waves; 0 = none)
  // rows the interior kernel leaves to the boundary kernel besides the two
  // edge rows: the rows next to severable links (crack rows), lo > hi = none
  int skip_lo, skip_hi;
  int sr;            // 16-bit storage: stochastic rounding of the stores
  uint32_t rkey;     // per-step key of the rounding bits (step_key)
  int dmask;         // edges with a prescribed w (LBM_EDGE_* bits)
  C wD_bot, wD_top, wD_left, wD_right;  // their wall values this step
};

// Per-step values of one time level of the T-step sweep.
template <typename C>
struct StepLevel {
  C t_top, t_bot, t_up, t_lo;
  C wD_bot, wD_top, wD_left, wD_right;
};

constexpr int kMaxTimeBlock = 8;

// Arguments of the T-step sweep (sweep2.hip): the per-step values of the T
// steps (their traction and wall values differ), the rounding key of the last
// (the only stores), and the crack state the later steps' cut links follow
// from.
template <typename S, typename W, typename C>
struct BlockArgs {
  SweepArgs<S, W, C> s0;              // step n: buffers, shape, constants
  StepLevel<C> lv[kMaxTimeBlock];     // steps n .. n + T - 1
  int steps;                          // T = 2 .. 8
  uint32_t rkey_last;                 // rounding key of step n + T - 1
  W *wmid;                            // w after steps n .. n + T - 2 on rows j0, j0 + 1 ([T - 1][2][pitch])
  const DevCrack *st;                 // crack state before step n's crack step
  int crack, both, grow;              // crack present, two tips, growing tips
  int sif;                            // K criterion: each tip keeps its last speed (predicted)
  double v_rel, cs, dt, a_lo, a_hi;
  // K criterion, several sweeps in flight: the sweep runs only while *gate is
  // nonzero (a crack sequence that found a prediction wrong closes it, and the
  // sweeps queued after it return at once); null = always
  const int32_t *gate;
};

// Counter-based randomness of the stochastic rounding: the integer hash
// "lowbias32" (C. Wellons' hash-prospector, 2018), and the key of one step.
__host__ __device__ inline uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}
__host__ __device__ inline uint32_t step_key(uint32_t seed, int64_t step) {
  return mix32(mix32(seed ^ 0x9e3779b9u) ^ (uint32_t)step ^ mix32((uint32_t)(step >> 32)));
}

struct CrackArgs {
  DevCrack *st;      // the crack state before the step
  DevCrack *st_out;  // where the state after it goes (null: st)
  const void *w;     // w after the sweep (double or float, see w_is_double)
  int w_is_double;
  int w_row0;        // row of the plate that w's first row holds (0: the whole plane)
  uint32_t *mV, *mH;  // cut bits of the vertical / horizontal links
  MaskRows *mrows;
  double *trK, *trA, *trV;
  int32_t *trF;
  double *trKL, *trAL, *trVL;  // left-tip traces (two tips)
  int32_t *trFL;
  int64_t *evStep;
  int32_t *evCol;    // site (i, j) of the link and its orientation
  int32_t *evRow;    // (0: vertical (i,j)-(i,j+1), 1: horizontal (i,j)-(i+1,j))
  int32_t *evOri;
  const int32_t *sens;  // sensor sites [n_sens][2] = (i, j)
  double *trS;          // sensor traces [trace_cap][n_sens]
  int n_sens;
  Plate p;
  CrackParams c;
};

// One plate of a batch as the batched kernels see it (device memory).  The
// per-step values (buffer parity, step index) come with each launch.
struct BatchPlate {
  const void *f[2];     // population buffers (plane 0), indexed by parity
  const void *w[2];     // w buffers, indexed by parity
  const uint32_t *mV, *mH;
  MaskRows *mrows;
  Plate p;
  double omega, dt, A0, Ak, coef;
  double face;          // crack-face traction (0 in periodic mode)
  const double *tau;    // device copy of the traction history
  int64_t n_hist;
  int has_crack, skip_lo, skip_hi;
  uint32_t seed;        // stochastic rounding seed (the batch decides whether it is used)
  int dmask;            // Dirichlet edges
  const double *wD;     // device copy of the wall-displacement history [n_wD][4]
  int64_t n_wD;
  // task maps (the single-plate maps of this plate)
  core::InteriorMap im;
  core::BoundaryMap bm;
  int64_t itask0, btask0;  // first interior / boundary task of this plate in the batch
  CrackArgs crack;      // w is set per step from the parity
  DevCrack *st2;        // the second crack-state slot (crack.st is the first)
  // device arguments of a crack step folded into a sweep, [2 * cur + slot]:
  // w in buffer cur, state in slot `slot`, going to the other slot
  const CrackArgs *fargs[4];
};

// Per-sweep arguments of the adjoint (adjoint.hip).  C is the adjoint's
// arithmetic and storage type (double for FP64 plates, float otherwise).
// Sweep m applies the transpose of step m's streaming to the adjoint of the
// post-streaming populations of step m (min, 5 planes) and then the
// transposed collision / Euler / moment map of step m - 1 (m = 0: of the
// initial equilibrium, omega = 1, dt = 0).
template <typename C>
struct AdjArgs {
  const C *min;          // plane 0 of the source adjoint populations
  C *mout;               // plane 0 of the destination
  const C *win;          // adjoint of w (source)
  C *wout;               // destination
  Plate p;               // pitch / plane in elements of C
  C omega, dt, A0, Ak;
  int64_t m;             // sweep index
  const int32_t *cutstep;  // per column: step of the cut of the crack-row link (-1 initial)
  int has_crack;
  int traction;          // the edges carry tau (walls): derivative wanted
  int dmask;             // Dirichlet edges: their anti-bounce-back has sign -1
  double coef;           // traction coefficient dt / (rho dh)
  double *dtau_part;     // partial sums of dL/dtau_m: [4 rows][n_parts]
  int n_parts;           // blocks per boundary row
  int skip_lo, skip_hi;  // crack rows, handled by the boundary kernel
  // loss gradient added to the written W at the sensors (g == nullptr: none);
  // the sensors of row j are srt[srow[j] .. srow[j + 1]), entries (i, index)
  const double *g;
  const int32_t *srow;
  const int32_t *srt;
};

// ---- launchers (adjoint.hip) ----
// one adjoint sweep (boundary rows and interior strips in one launch)
// eq: the adjoint populations kept in plane 0 only (they are all equal at
// omega = 1)
hipError_t launch_adjoint_sweep(bool fp64, bool eq, const void *args, hipStream_t st);
// w[sensor s] += g[s] (the loss gradient of the last step, before the first sweep)
hipError_t launch_adjoint_inject(bool fp64, void *w, const Plate &p, const int32_t *sens, int n,
                                 const double *g, hipStream_t st);
// dense FP64 [ny][nx] copy of one adjoint plane
hipError_t launch_adjoint_export(bool fp64, const void *plane, const Plate &p, double *out,
                                 hipStream_t st);
// blocks per boundary row of the adjoint boundary kernel
int adjoint_parts(int nx);

// ---- launchers (sweep.hip) ----
// F64S: FP64 in the shifted form (the equilibrium layout of FP64)
enum class Store { F64, F64S, F32_PLAIN, F32S, F16S, BF16S };

int sweep_vec(Store s);  // sites per lane
// one sweep step (interior strips and boundary rows in one launch); eq: the
// equilibrium layout (plane 0 and w only; shifted storages)
// fused: null, or the DEVICE address of the arguments of a crack step that
// this sweep runs besides (single plate, one-step sweeps, a crack along +x or
// none): one more wave of the boundary part executes it, and the crack-row
// waves forecast the links it severs from the same state and field, so that
// the sweep's bounce-back already sees them.  Its w is the sweep's source w
// (w after the step the crack step belongs to), st the state before it and
// st_out a second slot for the state after it (the forecast reads st while
// the crack wave runs).
hipError_t launch_sweep(Store s, bool eq, const void *args, hipStream_t st,
                        const CrackArgs *fused = nullptr);
// T = 2 .. 8 steps in one sweep (equilibrium layout, walls, a crack along
// +x with prescribed or no growth); args is a BlockArgs of the storage's types.
// The chunks of the strips without a plate edge run on st; the others (edge
// strips, the first and last chunk rows, the crack rows) on the side stream
// side, forked from st by the event fork and joined back into st by join
// (side == nullptr: both on st, one after the other).
struct SideStream {
  hipStream_t side;
  hipEvent_t fork, join;
};
hipError_t launch_sweep_block(Store s, const void *args, int rows, int waves, hipStream_t st,
                              const SideStream &ss);
// the 16-bit store conversion of the sweep applied to x[0..n) (F16S / BF16S)
hipError_t launch_round16(Store s, int sr, const float *x, void *out, int64_t n, int plane,
                          uint32_t rkey, hipStream_t st);

// ---- launchers (crack.hip) ----
// Speculative T-step sweep under the K criterion: the sweep severs the links
// of steps n + 1 .. n + T - 1 as if each tip kept the speed of its last step,
// which holds while every crack step of n .. n + T - 2 leaves its tip in the
// column that prediction gives.  The crack steps stop at the first one that
// does not, put back the crack state, mask-row range and crack-row mask of
// step n, and report how many steps were right (the sweep is then run again
// with that many).
struct SpecSlot {
  DevCrack st;
  MaskRows mr;
};
// What the host reads after the launch (pinned host memory, written by the
// kernel so that no copy has to be queued).
struct SpecOut {
  int32_t valid;   // steps found right (n when every prediction held)
};
hipError_t launch_crack(const CrackArgs &a, hipStream_t st);
// the crack steps of the n <= kMaxTimeBlock time steps of one T-step sweep,
// in order, in one launch
struct CrackSeq {
  CrackArgs a;                       // w and w_row0 replaced per step
  const void *w[kMaxTimeBlock];
  int32_t w_row0[kMaxTimeBlock];
  int n;
  SpecSlot *spec;                    // non-null: the sweep assumed no cuts (K criterion)
  uint32_t *spec_mask;               // mw words: the crack row's mask at the start
  SpecOut *spec_out;                 // device address of the host's SpecOut
  // with several sweeps in flight (see BlockArgs::gate): the sequence runs only
  // while *gate is nonzero, and closes it when it puts the start state back
  int32_t *gate;
};
hipError_t launch_crack_seq(const CrackSeq &s, hipStream_t st);
// *p = v by a kernel (capturable, unlike a memset node)
hipError_t launch_set_flag(int32_t *p, int32_t v, hipStream_t st);
hipError_t launch_init_mask(uint32_t *mV, uint32_t *mH, MaskRows *mrows, const Plate &p,
                            int has_crack, double x0, double a0, hipStream_t st);

// ---- launchers (batch.hip) ----
// The sweep of one step of every plate (boundary and interior tasks).  cur =
// parity of the source buffers, step = step index.  fused_slot >= 0 folds in
// the crack step of the step before (every plate's crack along +x, or none):
// one wave per plate runs it on the source w from its state in that slot
// (0: crack.st, 1: st2) into the other slot, and the crack-row tasks forecast
// the links it severs.  fused_slot < 0: the sweep alone.
hipError_t launch_batch_sweep(Store s, int sr, bool eq, const BatchPlate *d, int n_plates,
                              int64_t n_int_tasks, int64_t n_bnd_tasks, int cur, int64_t step,
                              int waves, int lds_bytes, int fused_slot, hipStream_t st);
// The crack step of every plate, one wave each, on w buffer wbuf, from the
// state in slot `slot` into slot 0.
hipError_t launch_batch_crack(const BatchPlate *d, int n_plates, int wbuf, int slot, hipStream_t st);
// nsteps steps in one cooperative launch with grid barriers; sync is a
// zeroed 512-byte device scratch (barrier counter, generation and time-out
// flag at words 0, 32 and 64).  Returns hipErrorCooperativeLaunchTooLarge if
// the grid cannot be co-resident.
hipError_t launch_batch_persistent(Store s, int sr, bool eq, const BatchPlate *d, int n_plates, int64_t n_int_tasks,
                                   int64_t n_bnd_tasks, int cur, int64_t step, int64_t nsteps,
                                   unsigned *sync, int *blocks_used, hipStream_t st);

// Bytes of synchronisation words the persistent launch needs for n_plates.
size_t persistent_sync_bytes(int n_plates);
// The device address of this library's fixed scratch array on the current
// device (looked up once per device with hipGetSymbolAddress) and its size;
// the no-allocation persistent run keeps its synchronisation words there.
hipError_t static_scratch(void **ptr, size_t *bytes);

// ---- launchers (macro_bc.hip) ----
// The macroscopic boundary scheme of Sec. 3.1 after a one-step sweep: w and
// the rest population (all five populations for the unshifted storages) of
// every boundary point from the boundary conditions (see macro_bc.hip).
struct MacroArgs {
  void *fout;           // plane 0 of the destination populations
  const void *win;      // w before the step
  void *wout;           // w after the step: the sweep's values, boundary points replaced
  const uint32_t *mV;   // cut bits of the vertical links
  Plate p;
  int has_crack;        // the crack row j0 may hold severed links
  int dmask;            // edges with a prescribed w (LBM_EDGE_* bits)
  double wD[4];         // their wall values this step (bottom, top, left, right)
  double t_top, t_bot;  // traction t* of the top / bottom edge this step
  double t_face;        // traction t* of the crack face above the crack (-t_face below)
  double mu, dt, A0, Ak;
  uint32_t rkey;        // rounding key of the step (stochastic rounding of plane 0)
  int *err;             // set to 1 if a boundary point depends deeper than two levels
};
hipError_t launch_macro_bc(Store s, int sr, bool eq, const MacroArgs &a, hipStream_t st);

// ---- launchers (io.hip) ----
// Initial populations and w of rows [row0, row0 + nrows) from FP64 staging
// (w0, wd0 may be null = 0).
hipError_t launch_init_rows(Store s, void *f, void *w, void *w2, const Plate &p, int row0,
                            int nrows, const double *w0, const double *wd0, double A0, double Ak,
                            hipStream_t st);
// FP64 export of rows [row0, row0 + nrows): w, wdot, or the five populations.
hipError_t launch_export_rows(Store s, const void *f, const void *w, const Plate &p, int row0,
                              int nrows, double A0, double Ak, double *w_out, double *wd_out,
                              double *f_out, hipStream_t st);
hipError_t launch_export_mask(const uint32_t *mV, const uint32_t *mH, const Plate &p,
                              uint8_t *v_out, uint8_t *h_out, hipStream_t st);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t st);

}  // namespace lbmk
