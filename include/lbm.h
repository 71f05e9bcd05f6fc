/*
 * lbm.h -- C-ABI of liblbmcrack: an MI355X (gfx950) lattice Boltzmann solver
 * for antiplane shear with a dynamically growing mode III crack, after
 * H. Mueller, A. Touil, A. Schlueter, R. Mueller, "Dynamic Propagation of
 * Mode III Cracks in a Lattice Boltzmann Method for Solids", arXiv:2206.12412.
 *
 * The method (paper Sec. 3 and Sec. 4):
 *   - D2Q5 lattice, populations f^alpha, alpha = 0 rest, 1 +x, 2 +y, 3 -x, 4 -y
 *     (Sec. 3, lattice velocities);
 *   - BGK lattice Boltzmann equation (Sec. 3, eq. LBE) with
 *     wdot = sum_alpha f^alpha (eq. distrib-macro), the Euler update
 *     w <- w + dt wdot (eq. integration) and the wave-equation equilibrium
 *     f_eq^0 = wdot - 2 lambda w / c^2, f_eq^k = lambda w / (2 c^2) (eq. f-eq,
 *     with the zeroth moment of f_eq equal to wdot), lambda = c_s^2 / (dt (tau/dt - 1/2)),
 *     c_s = sqrt(mu / rho), c = kappa c_s, dt = dh / c, dh = 1;
 *   - a straight crack (by default along the mid-line y = ny/2 - 1/2; any
 *     row, a second tip and any prescribed direction are configuration) whose
 *     severed links exchange nothing (Sec. 4.1): the population is bounced
 *     back (traction-free face), as at the plate edges;  a traction t* on a
 *     link adds (dt / (rho dh)) t* to the bounced population;  the top edge
 *     carries sigma_yz = +tau_n, the bottom edge -tau_n, the lateral edges are
 *     free, unless an edge holds a prescribed w (Sec. 5.1, 5.2);
 *   - the crack step appended after the time integration (Alg. 1): K_III from
 *     the crack opening at the column i_K = floor(a - r_min), r = a - i_K
 *     (eq. sif, eq. r(v)); growth at a prescribed speed or while K > K_C
 *     with v = v_max tanh(sqrt((K/K_C)^4 - 1)) (eq. sifCriterion, eq. v-tanh);
 *     tip a <- a + (v c_s) dt in FP64; every link the new crack segment
 *     touches is severed (CheckLinks / ProcessPoints; along +x the vertical
 *     links of the crack row with a_prev < i <= a).
 *
 * Conventions: sites (i, j), i = 0..nx-1 along x, j = 0..ny-1 along y; all
 * host arrays are FP64 row-major [ny][nx] (populations [5][ny][nx]); lengths
 * are in lattice spacings, times in steps unless stated.
 *
 * Memory and streams: the caller owns the device memory (one block of
 * lbm_state_bytes() bytes, 256-byte aligned) and the HIP stream; the library
 * keeps borrowed pointers and never allocates or frees device memory.  The
 * T-step sweep (lbm_set_time_block) runs its boundary chunks on a side stream
 * that the handle creates with its first such sweep (default priority), forked
 * from and joined back into the caller's stream, so that work enqueued on the
 * caller's stream after lbm_step still follows all of it; under the K
 * criterion it also allocates a small pinned host buffer (hipHostMalloc) that
 * the crack kernel writes each speculative sweep's verdict to, freed by
 * lbm_free.  Host arrays passed
 * to lbm_init are copied.  All calls on one handle must come
 * from one host thread at a time.
 *
 * Errors: every int-returning call returns 0 (LBM_OK) or a negative
 * lbm_status; lbm_last_error() gives a message for the calling thread.
 * lbm_step only enqueues work; a failure of enqueued work surfaces at the next
 * call that synchronises (lbm_crack_state, lbm_sif, lbm_traces, lbm_get_*).
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum lbm_status {
  LBM_OK = 0,
  LBM_EINVAL = -1,    /* invalid argument or configuration                  */
  LBM_ENOMEM = -2,    /* dev_bytes smaller than lbm_state_bytes()           */
  LBM_EHIP = -3,      /* a HIP runtime call failed                          */
  LBM_EUNSTABLE = -4, /* omega != 1 or kappa <= sqrt(2): the scheme diverges */
  LBM_ECRACK = -5,    /* crack outside the plate                            */
  LBM_ESTATE = -6     /* handle in a state that does not allow the call     */
};

/* Storage of the populations.  LBM_F64 and LBM_F32_PLAIN store the
 * post-collision f^alpha themselves; LBM_F32, LBM_F16S and LBM_BF16S store
 * g^alpha = f^alpha - E^alpha(w), E the static equilibrium f_eq(w, 0) of the
 * emitting site, with w kept in FP32 and all arithmetic in FP32. */
enum lbm_storage { LBM_F64 = 0, LBM_F32 = 1, LBM_F16S = 2, LBM_BF16S = 3, LBM_F32_PLAIN = 4 };
enum lbm_growth { LBM_GROW_NONE = 0, LBM_GROW_PRESCRIBED = 1, LBM_GROW_SIF = 2 };
enum lbm_bc { LBM_BC_WALLS = 0, LBM_BC_PERIODIC = 1 /* both axes wrap; no edge loads */ };
enum lbm_flags { LBM_FLAG_GREW = 1, LBM_FLAG_WALL = 2, LBM_FLAG_K_UNDEF = 4 };
/* Rounding of the FP32 results to the 16-bit storages (LBM_F16S, LBM_BF16S).
 * NEAREST: round to nearest even.  STOCHASTIC: round up or down to a
 * neighbouring 16-bit value with probability proportional to the distance
 * (random bits added below the kept mantissa: 13 for FP16, 16 for BF16,
 * exactly the bits the conversion drops, so the rounding is unbiased at FP32
 * resolution, FP16 subnormals included; one counter-based hash per pair of
 * horizontally adjacent sites, keyed by the pair's plate-local index, the
 * step and cfg->seed), so that rounding errors do not accumulate coherently
 * over steps.  Results stay deterministic: they depend on (site, step, seed),
 * not on the launch. */
enum lbm_rounding { LBM_ROUND_NEAREST = 0, LBM_ROUND_STOCHASTIC = 1 };
/* Plate edges.  An edge is traction-loaded by default (top +tau_n, bottom
 * -tau_n, lateral edges free); an edge whose bit is set in cfg->dirichlet
 * holds a prescribed displacement w* at the wall (the link midpoint) by
 * anti-bounce-back, f_in^alpha = -f^opp + 2 f_eq^alpha(w*, 0) (the ghost site
 * then carries 2 w* - w), as the lower and upper edges of Sec. 5.2. */
enum lbm_edge { LBM_EDGE_BOTTOM = 1, LBM_EDGE_TOP = 2, LBM_EDGE_LEFT = 4, LBM_EDGE_RIGHT = 8 };
/* Layout of the state in device memory.  FULL: the five populations and w
 * (Sec. 3, eq. LBE), each read and written once per step.  EQ: at omega = 1
 * (tau = dt, Sec. 3) the collision sets every population to its equilibrium,
 * so each moving population that streams is f_eq^k(w) = Ak w of its emitting
 * site: the sweep reads and writes only the rest population (shifted: wdot)
 * and w, and rebuilds the moving ones from the w of the neighbours.  Needs a
 * shifted storage (LBM_F32, LBM_F16S, LBM_BF16S; LBM_F64 is then kept in the
 * shifted form too).  Results equal those of FULL in the same storage (the
 * moving shifted populations are exactly zero), except that FP64 in EQ is
 * the shifted FP64 arithmetic (within rounding of FULL's FP64).  The moving
 * planes stay allocated and zero, so the population and checkpoint views are
 * the same for both layouts. */
enum lbm_layout { LBM_LAYOUT_FULL = 0, LBM_LAYOUT_EQ = 1 };
/* Treatment of boundary points (sites with a severed link or a link leaving
 * the plate).  LINK: per link, bounce-back at the link midpoint (with the
 * traction term) or, at a prescribed-w edge, anti-bounce-back.  MACRO: the
 * macroscopic scheme of Sec. 3.1: w at a boundary point from a quadratic
 * polynomial along the inward normal of each missing link, through the
 * boundary condition on the wall or crack face half a spacing beyond the
 * point (w* or the traction slope -t* / mu) and this step's w at the next two
 * lattice points inward (the mean over several missing links); the missing
 * populations then follow from eq. (f-macro-bc), so that they sum to
 * (w_B(t + dt) - w_B(t)) / dt.  MACRO needs walls, no crack or a crack
 * along +x with at least three rows on either side of the crack line, and
 * one step per sweep; no batches, no adjoint. */
enum lbm_bc_scheme { LBM_BC_LINK = 0, LBM_BC_MACRO = 1 };

typedef struct lbm_config {
  int32_t nx, ny;          /* sites; ny even and >= 2 when there is a crack      */
  int32_t storage;         /* enum lbm_storage                                   */
  int32_t bc_mode;         /* enum lbm_bc                                        */
  double kappa;            /* c / c_s (> sqrt(2)); Sec. 3                        */
  double omega;            /* dt / tau; the paper's tau = dt gives 1 (required)  */
  double mu, rho;          /* shear modulus, density (> 0)                       */
  int32_t has_crack;       /* 0: no crack (no crack step, no traces)             */
  double crack_x0;         /* left end of the crack line; -0.5 = left edge       */
  double crack_tip;        /* initial tip a_0, crack_x0 <= a_0 <= nx - 1/2       */
  int32_t growth;          /* enum lbm_growth                                    */
  double v_rel;            /* prescribed speed a_dot / c_s in [0, 1)             */
  double K_C;              /* critical K_III of the criterion (> 0 for SIF)      */
  double r0;               /* r_min at v = 0 (eq. r(v)), > 0                     */
  double v_max;            /* maximum speed of the tanh law, in [0, 1)           */
  int32_t k_band;          /* columns in the K fit, 1..64 (1 = eq. sif)          */
  double face_traction;    /* tau* on the crack faces (suddenly loaded faces)    */
  const double *tau_hist;  /* host, n_hist values: step n uses                   */
  int64_t n_hist;          /* tau_hist[min(n, n_hist - 1)]; 0 = unloaded          */
  const double *w0;        /* host [ny][nx] initial displacement, NULL = 0       */
  const double *wdot0;     /* host [ny][nx] initial velocity, NULL = 0           */
  int64_t trace_cap;       /* per-step K / tip / speed traces kept on device     */
  int32_t rounding;        /* enum lbm_rounding; 16-bit storages only            */
  uint32_t seed;           /* seed of the stochastic rounding                    */
  int32_t n_sensors;       /* sensor sites: w there is recorded after each step  */
  const int32_t *sensors;  /* host [n_sensors][2] = (i, j), distinct; copied     */
  int32_t crack_row;       /* j0 of the crack line y = j0 + 1/2 (0..ny-2); -1 =  */
                           /* the mid-line ny/2 - 1 (then ny must be even)       */
  int32_t both_tips;       /* 1: the left end crack_x0 is a tip too and grows in */
                           /* -x by the same rule (Sec. 5.2: two tips)           */
  int32_t dirichlet;       /* enum lbm_edge bits: edges holding a prescribed w   */
  const double *wD_hist;   /* host [n_wD][4]: w* of (bottom, top, left, right);  */
  int64_t n_wD;            /* step n uses row min(n, n_wD - 1); copied           */
  int32_t layout;          /* enum lbm_layout                                    */
  double crack_dx, crack_dy; /* growth direction of the (right) tip, Alg. 1's   */
                           /* input d: (0, 0) or (1, 0) = +x along crack_row;     */
                           /* otherwise the crack is the straight segment through */
                           /* S = (crack_x0, crack_row + 1/2) along d, the tips   */
                           /* given by line coordinates a (the point              */
                           /* S + (a - crack_x0) d/|d|), every vertical or        */
                           /* horizontal link it touches severed; k_band = 1,     */
                           /* walls only, no adjoint                             */
  int32_t bc_scheme;       /* enum lbm_bc_scheme                                 */
  void *dev_buf;           /* device memory, >= lbm_state_bytes(cfg), 256-aligned */
  size_t dev_bytes;
  void *stream;            /* hipStream_t; NULL = the null stream                */
} lbm_config;

typedef struct lbm_crack_info {
  double tip;      /* current tip a_n                                       */
  double v;        /* speed of the last step (relative to c_s)              */
  double K;        /* K_III of the last step (NaN if undefined)             */
  double r;        /* distance used for that K                              */
  int64_t step;    /* steps completed                                       */
  int32_t flags;   /* enum lbm_flags of the last step                       */
  int32_t n_events;/* cut events recorded so far                            */
  int32_t col_K;   /* column used for that K (-1 if undefined)              */
  int32_t n_cut;   /* severed links on the crack row                        */
  /* the left end (a tip when cfg->both_tips; otherwise crack_x0, at rest) */
  double tip_left, v_left, K_left, r_left;
  int32_t flags_left, col_K_left;
} lbm_crack_info;

typedef struct lbm_handle lbm_handle;

/* Bytes of device memory lbm_init needs for cfg (0 if cfg is invalid). */
size_t lbm_state_bytes(const lbm_config *cfg);

/* Validate cfg, lay the state out in cfg->dev_buf and enqueue its
 * initialisation on cfg->stream: f = f_eq(w0, wdot0), w = w0, the links
 * severed by the initial crack segment (Sec. 4.1 severs them the same way as
 * those a growing tip crosses).
 * Returns LBM_EINVAL / LBM_EUNSTABLE / LBM_ECRACK / LBM_ENOMEM without
 * touching the GPU when cfg is unusable. */
int lbm_init(const lbm_config *cfg, lbm_handle **out);

/* Enqueue nsteps time steps (fused collide-stream sweep, then the crack step
 * of Alg. 1) on the handle's stream.  Asynchronous. */
int lbm_step(lbm_handle *h, int64_t nsteps);

/* Crack state after the last step (synchronises the stream). */
int lbm_crack_state(lbm_handle *h, lbm_crack_info *out);

/* K_III trace (eq. sif) of steps [first, first + count) into host K_out;
 * entries past the steps taken or past trace_cap are LBM_EINVAL. */
int lbm_sif(lbm_handle *h, double *K_out, int64_t first, int64_t count);

/* Tip position after each step, speed and flags, same indexing as lbm_sif;
 * any output pointer may be NULL. */
int lbm_traces(lbm_handle *h, double *tip_out, double *v_out, int32_t *flags_out,
               int64_t first, int64_t count);

/* K, position, speed and flags of the left tip (cfg->both_tips), same
 * indexing; any output pointer may be NULL. */
int lbm_traces_left(lbm_handle *h, double *K_out, double *tip_out, double *v_out,
                    int32_t *flags_out, int64_t first, int64_t count);

/* Sensor traces: w at the sensor sites after each step, rows [first,
 * first + count) of the [trace_cap][n_sensors] FP64 table (row n = after step
 * n).  out is a host pointer, or a device pointer if out_on_device != 0. */
int lbm_sensor_traces(lbm_handle *h, double *out, int64_t first, int64_t count,
                      int32_t out_on_device);

/* Cut events: (step, column) of every link severed by growth, in order;
 * writes min(cap, total) entries and the total into *n. */
int lbm_cut_events(lbm_handle *h, int64_t *steps, int32_t *cols, int64_t cap, int64_t *n);

/* Cut events with the severed link itself (Alg. 1, ProcessPoints): step,
 * site (i, j) and orientation (0: vertical link (i,j)-(i,j+1), 1: horizontal
 * link (i,j)-(i+1,j)); a crack along +x severs vertical links of its row only.
 * Any output pointer may be NULL; writes min(cap, total) entries and the total
 * into *n. */
int lbm_cut_links(lbm_handle *h, int64_t *steps, int32_t *i, int32_t *j, int32_t *orient,
                  int64_t cap, int64_t *n);

/* Host FP64 snapshot of w and wdot = sum_alpha f^alpha (either may be NULL). */
int lbm_get_fields(lbm_handle *h, double *w_out, double *wdot_out);

/* Host FP64 snapshot of the post-collision populations f^alpha, [5][ny][nx]
 * (shifted storage is converted back: f = g + E(w)). */
int lbm_get_populations(lbm_handle *h, double *f_out);

/* Severed links as bytes: cutV[j][i] is the link (i,j)-(i,j+1), cutH[j][i]
 * the link (i,j)-(i+1,j) (the wrap-around link (nx-1,j)-(0,j) in periodic
 * mode), either may be NULL. */
int lbm_get_mask(lbm_handle *h, uint8_t *cutV, uint8_t *cutH);

/* Checkpoint and restart.  lbm_checkpoint copies the state after the steps
 * taken so far (current populations and w, cut mask, crack state, traces, cut
 * events, sensor traces, step count) into dst, a device buffer of
 * lbm_checkpoint_bytes(h) bytes (256-byte aligned; the caller owns it);
 * lbm_restore makes a handle continue from such a checkpoint: the handle must
 * have been initialised from the same configuration (checked through the
 * recorded sizes), and its next steps then reproduce bit for bit the steps
 * that followed the checkpoint.  Both are enqueued on h's stream and
 * synchronise it. */
size_t lbm_checkpoint_bytes(const lbm_handle *h);
int lbm_checkpoint(lbm_handle *h, void *dst);
int lbm_restore(lbm_handle *h, const void *src);

/* Kernel timing with HIP events on the handle's stream.  A step launches the
 * sweep kernel (interior strips and boundary rows in one launch) and the
 * crack kernel; a one-step sweep of a plate whose crack runs along +x (or
 * that has none) runs the crack step of the step before it instead, so its
 * time counts as sweep time and the crack time of such steps is about zero
 * (the crack launch that ends each lbm_step call is not timed).
 * enable = n > 0 starts recording (and clears the sums) on
 * every step whose index is a multiple of n (n > 1 samples the steps, so that
 * the events cost less); 0 stops.  Returns the summed durations (ms) of the
 * two kernels over the timed steps and their number (synchronises the
 * stream).  With time blocking a sweep and its crack steps are timed
 * together when one of its steps is sampled; a speculative sweep that is run
 * again (K criterion) adds its time but not its steps.  Any output pointer
 * may be NULL. */
int lbm_timing(lbm_handle *h, int32_t enable, double *sweep_ms, double *crack_ms, int64_t *n_timed);

/* Launch shape of the sweep: sites per lane along x (vec, fixed by the
 * storage), rows marched per wave (rows), waves per workgroup (waves) and the
 * cap on resident waves per SIMD (occupancy; 0 = no cap), which the library
 * enforces by reserving LDS per workgroup.  lbm_set_launch accepts rows in
 * 1..4096, waves in {1, 2, 4, 8} and occupancy in 0..8.  Results do not
 * depend on the launch shape. */
int lbm_get_launch(lbm_handle *h, int32_t *vec, int32_t *rows, int32_t *waves,
                   int32_t *occupancy);
int lbm_set_launch(lbm_handle *h, int32_t rows, int32_t waves, int32_t occupancy);

/* Time blocking: with steps = T (2 to 8), lbm_step advances T time steps
 * per sweep (each wave computes step n for its rows and their neighbours in
 * registers, then step n + 1 from those, and so on, then stores), so a step
 * moves 1 / T of the bytes of the one-step sweep; the crack steps of all T
 * time steps still run, in order (K of step n + k from the crack rows after
 * step n + k; Alg. 1 takes one crack step per time step).  FP32 and FP64
 * results are bit for bit those of steps = 1; 16-bit storages round only at
 * the end of each sweep.  Needs the equilibrium layout, walls, no sensors,
 * and no crack or a crack along +x.  Prescribed growth: the sweep derives
 * the links severed at steps n + 1 .. n + T - 1 from the prescribed advance.
 * K criterion (eq. sifCriterion): the sweep severs links as if each tip kept
 * the speed of its last step; when the crack step of some step n + m before
 * the last leaves a tip in another column than that prediction, the state of
 * step n is put back and the sweep runs again for m + 1 steps (lbm_step
 * queues up to four such sweeps ahead of the verdicts it has read, gated on a
 * device word that a wrong one closes, and rewinds at a wrong one; while
 * per-kernel timing is on it waits for each verdict instead; after a sweep
 * that was run again the next may take half as many steps, growing back by
 * one per sweep that held).
 * rows / waves: rows finished per wave (4, 8 or 16; or 32: chunks of 16
 * rows, two per wave of the launch away from the plate edges and crack rows,
 * which loads and steps the rows around them once per wave instead of once
 * per chunk; or, for T >= 6, 24: chunks of 8 rows, three per such wave) and
 * waves per workgroup (1, 2, 4 or 8)
 * of the T-step sweep for this T (0 = keep; T >= 6: 16 rows or more; the
 * defaults, and
 * a cap on the resident waves per SIMD, are the fastest measured on a
 * 16384 x 8192 plate).  A call whose step count is
 * not a multiple of T ends with the sweeps lbm_plan_tail gives (or, with
 * lbm_set_tail_plan(h, 0), with one shorter sweep; a sweep of one step is
 * the one-step sweep); under the K criterion the speculative sweeps choose
 * their own lengths.  steps = 1 restores the one-step sweep. */
int lbm_set_time_block(lbm_handle *h, int32_t steps, int32_t rows, int32_t waves);

/* The end of a call whose step count is not a multiple of T.  A sweep moves
 * the same bytes whatever its step count, so on a large plate a sweep of two
 * steps costs nearly as much as one of six: a call of 20 steps at T = 6 runs
 * faster as 7 + 7 + 6 than as 6 + 6 + 6 + 2.  With on = 1 (the default)
 * lbm_step re-splits the rest and up to three T-step sweeps before it into
 * the sweeps of 1 to 8 steps that lbm_plan_tail gives; on = 0 ends the call
 * with one shorter sweep.  FP32 and FP64 results are the same bit for bit
 * either way; the 16-bit storages round once per sweep, so their results
 * follow the split (as for calls of other lengths).  EINVAL for on other
 * than 0 or 1. */
int lbm_set_tail_plan(lbm_handle *h, int32_t on);

/* Host only (no device work).  The sweeps, longest first, that end a call of
 * nsteps steps at steps_per_sweep = T on a plate of this storage (an enum
 * lbm_storage; the T-step sweep runs FP64 plates in the shifted storage)
 * while the tail plan is on: the call runs (nsteps - sum of tail) / T sweeps
 * of T steps, then tail[0 .. *n_tail - 1] (each 1 to 8 steps; at most 32
 * entries: the caller's array holds 32).  A step count that is a multiple of
 * T, and T = 1, give no tail.  Otherwise the rest nsteps mod T and the last
 * j = 0 .. 3 sweeps of T steps before it are split into the sweeps of least
 * total time by lbm_sweep_cost, over every j (ties: the smaller j).  EINVAL
 * for an unknown storage, T outside 1..8, negative nsteps or null outputs. */
int lbm_plan_tail(int32_t storage, int32_t steps_per_sweep, int64_t nsteps, int32_t *tail,
                  int32_t *n_tail);

/* Host only.  The time (us) of one sweep of `steps` (1 to 8) time steps of
 * this storage that lbm_plan_tail works from: per-sweep HIP events with the
 * default shapes on a 16384 x 8192 plate in the equilibrium layout, a crack
 * growing at a prescribed speed.  EINVAL as lbm_plan_tail. */
int lbm_sweep_cost(int32_t storage, int32_t steps, double *us);

/* Times every shape of the T-step sweep for steps = T (rows 4, 8, 16 or 32
 * per wave, 16, 24 or 32 for T >= 6; waves 1, 2, 4 or 8 per workgroup) over
 * trial_sweeps sweeps of h itself (h advances: tune a scratch plate made from
 * the same configuration), then sets the fastest with lbm_set_time_block and
 * returns it with its time per step.  The defaults were measured on a
 * 16384 x 8192 plate; on smaller plates the sweep is bound by the latency of
 * one wave's march rather than by bytes, and another shape can win.  Same
 * refusals as lbm_set_time_block; trial_sweeps in 1..1000. */
int lbm_autotune_time_block(lbm_handle *h, int32_t steps, int32_t trial_sweeps, int32_t *rows,
                            int32_t *waves, double *ms_per_step);

/* Counts since the handle was made: T-step sweeps run under the K criterion
 * (speculative, see lbm_set_time_block) and how many of them were run again
 * with fewer steps because a tip left the predicted column before their last
 * step.  Any
 * output pointer may be NULL. */
int lbm_time_block_stats(lbm_handle *h, int64_t *sweeps, int64_t *reruns);

/* The 16-bit store conversion of the sweep, applied to an array (for
 * inspection and tests of the storage formats): out[i] is the value the sweep
 * of step `step` with seed `seed` stores for a result x[i] at site (i, 0) of
 * population plane `plane` (0..4) of a plate with rows of n sites (the
 * rounding draws depend on the site's row, column and plane, the plate width,
 * the seed and the step).  storage is
 * LBM_F16S or LBM_BF16S, rounding an enum lbm_rounding.  x (FP32) and out
 * (n 16-bit values) are device pointers; enqueued on `stream` (hipStream_t,
 * NULL = the null stream). */
int lbm_round16(const float *x, void *out, int64_t n, int32_t storage, int32_t rounding,
                int32_t plane, uint32_t seed, int64_t step, void *stream);

/* Launch-shape search.  Times every shape of a fixed grid (rows in {1, 2, 4,
 * 8}, waves in {1, 2, 4, 8}, occupancy in {0, 2, 3, 4, 5, 6}) over trial_steps
 * whole steps each (after one untimed step), with HIP events on the handle's
 * stream, and leaves the fastest shape set on h.  The search ADVANCES h by
 * 96 * (trial_steps + 1) steps, so run it on a scratch handle built from the
 * production config and copy the result with lbm_set_launch (results never
 * depend on the launch shape).  trial_steps must be in 1..1000.  Outputs: the
 * chosen shape and its mean step time in ms (any pointer may be NULL).
 * Synchronises the stream. */
int lbm_autotune(lbm_handle *h, int32_t trial_steps, int32_t *rows, int32_t *waves,
                 int32_t *occupancy, double *ms_per_step);

/* Algorithmic bytes moved by one sweep per site (read + write of the stored
 * populations, five or, in the equilibrium layout, one, and of w), for the
 * storage and layout of the handle. */
double lbm_bytes_per_site(const lbm_handle *h);

/* Release the handle (host metadata only; the device block stays the caller's). */
void lbm_free(lbm_handle *h);

/* ---------------------------------------------------------------- batches --
 * Many independent plates (each its own lbm_config: size, load, crack rule)
 * advanced together by batched kernels; every plate of a batch must use the
 * same storage.  Each plate's arithmetic is the single-plate arithmetic, so a
 * plate evolves bit for bit as it does alone.  dev_buf/dev_bytes/stream of
 * the plate configs are ignored: the batch places every plate inside its own
 * device block (lbm_batch_state_bytes bytes, 256-byte aligned, caller-owned)
 * and runs on the given stream. */
typedef struct lbm_batch lbm_batch;

size_t lbm_batch_state_bytes(const lbm_config *cfgs, int32_t n);
int lbm_batch_init(const lbm_config *cfgs, int32_t n, void *dev_buf, size_t dev_bytes, void *stream,
                   lbm_batch **out);

/* nsteps steps; each step is one batched sweep launch (the boundary and
 * interior tasks of every plate) and one batched crack launch (one wavefront
 * per plate).  When every plate's crack runs along +x (or it has none), the
 * crack steps of step n run inside the sweep launch of step n + 1 (one more
 * wavefront per plate; the crack-row tasks take the links it severs) and the
 * call ends with one crack launch; the results are the same bit for bit.
 * Asynchronous. */
int lbm_batch_step(lbm_batch *b, int64_t nsteps);

/* nsteps steps in ONE cooperative (persistent) launch: waves walk the task
 * list of all plates with a grid stride; grid barriers separate the sweep, the
 * crack step and the next sweep.  The barrier waits a bounded time; a time-out
 * ends every wave and returns LBM_EHIP (the state is then invalid).
 * Synchronises the stream. */
int lbm_batch_run_persistent(lbm_batch *b, int64_t nsteps);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): lbm_batch_run_persistent
 * with its synchronisation words (arrival counter, generation, time-out flag)
 * in a fixed 64 KiB device array of the library instead of the batch's
 * device block.  The same kernels, the same results bit for bit.  It calls
 * no allocating routine: no hipMalloc / hipFree, no event or stream creation
 * (per-call timing, lbm_batch_timing, is not recorded for it).  Each GPU the
 * library runs on holds one copy of the array until the process ends; its
 * address is looked up once per device at lbm_batch_init.  Every call on a
 * GPU shares that GPU's copy: its words are cleared by a fill kernel at the
 * start of each call, and calls that overlap on one GPU (from two threads or
 * on two streams) race on it.  Errors: LBM_EINVAL if the batch needs more
 * synchronisation words than the array holds; otherwise as
 * lbm_batch_run_persistent.  Synchronises the stream. */
int lbm_batch_run_persistent_static(lbm_batch *b, int64_t nsteps);

/* Handle of plate k for queries (lbm_crack_state, lbm_sif, lbm_get_fields,
 * ...); owned by the batch (no lbm_free, no lbm_step on it).  NULL if k is out
 * of range. */
lbm_handle *lbm_batch_plate(lbm_batch *b, int32_t k);

/* Launch shape of the batched interior kernel (as lbm_set_launch) and the
 * grid of the last persistent launch (one workgroup per CU: 16 waves in the
 * equilibrium layout, 8 with five planes). */
int lbm_batch_set_launch(lbm_batch *b, int32_t rows, int32_t waves, int32_t occupancy);
int lbm_batch_get_launch(lbm_batch *b, int32_t *rows, int32_t *waves, int32_t *occupancy,
                         int32_t *persistent_blocks);

/* lbm_autotune for a batch (per-step launches): same grid, same contract;
 * the batch advances by 96 * (trial_steps + 1) steps. */
int lbm_batch_autotune(lbm_batch *b, int32_t trial_steps, int32_t *rows, int32_t *waves,
                       int32_t *occupancy, double *ms_per_step);

/* Whole-step timing with HIP events (per-step launches: one interval per
 * step; persistent runs: one interval per run). */
int lbm_batch_timing(lbm_batch *b, int32_t enable, double *ms, int64_t *n_timed);

/* Total sites of all plates. */
int64_t lbm_batch_sites(const lbm_batch *b);

void lbm_batch_free(lbm_batch *b);

/* ------------------------------------------------------------- adjoint --
 * Discrete adjoint of the steps a handle has taken, for a loss L of its
 * sensor traces.  One step maps the state s_n = (f_n, w_n) affinely:
 * s_{n+1} = A_n s_n + b tau_n, where A_n holds the pull streaming with
 * bounce-back on the links severed at step n (Sec. 3 eq. LBE, Sec. 4.1) and
 * the collision / Euler update (eq. f-eq, eq. distrib-macro, eq.
 * integration), and b the traction links of the top (+tau_n) and bottom
 * (-tau_n) edges.  With lambda_T = (0, dL/dw_T) and
 *   lambda_n = A_n^T lambda_{n+1} + (0, dL/dw_n),   dL/dtau_n = b^T lambda_{n+1},
 * the gradient with respect to the initial fields follows from
 * f_0 = f_eq(w_0, wdot_0).  A_n^T is evaluated as one fused sweep per step:
 * the transposed local map, then a pull of the adjoint populations along the
 * reversed lattice directions with the transposed bounce-back (a severed
 * link returns the adjoint to the opposite direction at the same site).
 * The links severed at each step come from the recorded cut events, so the
 * sweep reads no forward state; with the K criterion the cut sequence of the
 * forward run is held fixed (the derivative of the piecewise affine map on
 * the path taken).  The adjoint runs in FP64 for LBM_F64 plates and in FP32
 * otherwise. */
typedef struct lbm_adjoint lbm_adjoint;

/* Device bytes lbm_adjoint_init needs for handle h (0 if h is invalid). */
size_t lbm_adjoint_bytes(const lbm_handle *h);

/* Adjoint workspace for handle h in caller-owned device memory (256-byte
 * aligned), on h's stream.  h must outlive the adjoint object. */
int lbm_adjoint_init(lbm_handle *h, void *dev_buf, size_t dev_bytes, lbm_adjoint **out);

/* Runs the adjoint through every step h has taken (T = steps, 1 <= T <=
 * trace_cap).  g: device FP64 [T][n_sensors], g[n][s] = dL/dw at sensor s
 * after step n (the gradient of L with respect to lbm_sensor_traces).
 * Outputs (any may be NULL): dL_dtau host [T], the derivative with respect to
 * the traction tau_n of step n; dL_dwdot0 and dL_dw0 device FP64 [ny][nx],
 * the derivatives with respect to the initial fields.  Synchronises. */
int lbm_adjoint_run(lbm_adjoint *a, const double *g, double *dL_dtau, double *dL_dwdot0,
                    double *dL_dw0);

/* Adjoint kernel time of the last lbm_adjoint_run (ms, HIP events around the
 * sweeps) and its number of sweeps. */
int lbm_adjoint_timing(lbm_adjoint *a, double *ms, int64_t *sweeps);

void lbm_adjoint_free(lbm_adjoint *a);

/* Message of the last error on the calling thread ("" if none). */
const char *lbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
