/*
 * lbm_oracle.h -- plain FP64 CPU oracle for the D2Q5 lattice Boltzmann method
 * for antiplane shear with a dynamically growing mode III crack
 * (Mueller, Touil, Schlueter, Mueller, arXiv:2206.12412).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this code; only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no source, header, table or constant with
 * the HIP path.
 *
 * Conventions (lattice units, Delta h = 1):
 *   sites (i, j), i = 0..nx-1 along x (fastest in memory), j = 0..ny-1 along y;
 *   arrays are row-major [j][i]; populations are [alpha][j][i];
 *   directions alpha: 0 rest, 1 +x, 2 +y, 3 -x, 4 -y  (Sec. 3, D2Q5 lattice);
 *   walls lie half-way between the outer sites and the (absent) ghost sites;
 *   the crack runs along y_c = j0 + 1/2 (j0 = crack_row, default ny/2 - 1),
 *   from x = crack_x0 to the tip x = a, and grows in +x; with both_tips its
 *   left end is a second tip that grows in -x by the same rule.  With a
 *   growth direction d = (crack_dx, crack_dy) other than +x (Alg. 1 takes the
 *   direction as an input) the crack is the straight segment through
 *   S = (crack_x0, y_c) along d: a tip at line coordinate a sits at
 *   S + (a - crack_x0) d / |d| and advances in a; every link, vertical or
 *   horizontal, that the closed segment touches is severed.
 *   An edge is traction-loaded (default: top +tau, bottom -tau, lateral 0) or,
 *   if its bit is set in `dirichlet`, holds a prescribed displacement w* at
 *   the wall by anti-bounce-back: f_in = -f^opp + 2 f_eq(w*, 0).
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_GROW_NONE = 0, ORC_GROW_PRESCRIBED = 1, ORC_GROW_SIF = 2 };
enum { ORC_FLAG_GREW = 1, ORC_FLAG_WALL = 2, ORC_FLAG_K_UNDEF = 4 };
enum { ORC_EDGE_BOTTOM = 1, ORC_EDGE_TOP = 2, ORC_EDGE_LEFT = 4, ORC_EDGE_RIGHT = 8 };
/* ORC_BC_LINK: a population whose link is severed or leaves the plate is
 * bounced back (anti-bounce-back at a prescribed-w edge), per link.
 * ORC_BC_MACRO: the macroscopic scheme of Sec. 3.1: w at every boundary
 * point from a quadratic polynomial along the boundary normal through the
 * boundary condition and two interior points, assembled into S w_B = R and
 * solved; the missing populations from eq. (f-macro-bc). */
enum { ORC_BC_LINK = 0, ORC_BC_MACRO = 1 };

typedef struct {
  int32_t nx, ny;
  int32_t periodic;        /* 1: both axes wrap around (closed lattice, no walls) */
  double kappa;            /* c / c_s */
  double omega;            /* Delta t / tau */
  double mu, rho;
  int32_t has_crack;
  double crack_x0;         /* left end of the crack line (-0.5 = left wall)      */
  double crack_tip;        /* initial tip position a_0                           */
  int32_t growth;          /* ORC_GROW_*                                         */
  double v_rel;            /* prescribed crack speed / c_s                       */
  double K_C, r0, v_max;   /* K criterion, r_min law and velocity regularisation */
  int32_t k_band;          /* columns used for K (1 = the single pair of eq. sif) */
  double face_traction;    /* traction on the crack faces (suddenly loaded faces) */
  const double *tau_hist;  /* sigma_yz on top/bottom edges, step n uses           */
  int64_t n_hist;          /* tau_hist[min(n, n_hist-1)]; n_hist = 0 -> unloaded  */
  const double *w0;        /* optional initial displacement [ny][nx] (NULL = 0)  */
  const double *wdot0;     /* optional initial velocity [ny][nx] (NULL = 0)      */
  int64_t trace_cap;       /* length of the per-step K / tip / speed traces      */
  int32_t threads;         /* OpenMP threads for the sweep (0 = runtime default) */
  int32_t crack_row;       /* j0 of the crack line y = j0 + 1/2; -1 = ny/2 - 1    */
  int32_t both_tips;       /* 1: the left end crack_x0 grows in -x as well       */
  int32_t dirichlet;       /* ORC_EDGE_* bits of the edges with a prescribed w   */
  const double *wD_hist;   /* [n_wD][4] w* of (bottom, top, left, right); step n  */
  int64_t n_wD;            /* uses row min(n, n_wD - 1)                          */
  double crack_dx, crack_dy; /* growth direction of the right tip; (0, 0) or     */
                             /* (1, 0) = +x along the crack row                  */
  int32_t bc_scheme;       /* ORC_BC_*: how boundary points are treated          */
} orc_config;

typedef struct orc_sim orc_sim;

/* Returns NULL and sets *err (<0) on an invalid configuration. */
orc_sim *orc_create(const orc_config *cfg, int32_t *err);
void orc_free(orc_sim *s);
/* Advance n time steps (LBM step followed by the crack step). */
int32_t orc_step(orc_sim *s, int64_t n);

/* Snapshots, FP64, [ny][nx]; wdot = sum of the post-collision populations. */
void orc_get_fields(const orc_sim *s, double *w, double *wdot);
void orc_get_pops(const orc_sim *s, double *f);            /* [5][ny][nx] */
/* Overwrite the post-collision populations and the displacement. */
void orc_set_state(orc_sim *s, const double *f, const double *w);
/* Link masks: cutV[j][i] is the link (i,j)-(i,j+1), cutH[j][i] is (i,j)-(i+1,j). */
void orc_get_mask(const orc_sim *s, uint8_t *cutV, uint8_t *cutH);
void orc_crack(const orc_sim *s, double *tip, double *v, int64_t *step, int32_t *flags);
int64_t orc_traces(const orc_sim *s, double *K, double *tip, double *v, int32_t *flags,
                   int64_t cap);
/* The same for the left tip (both_tips). */
int64_t orc_traces_left(const orc_sim *s, double *K, double *tip, double *v, int32_t *flags,
                        int64_t cap);
/* Cut events produced by crack growth: step, site (i, j) and orientation
 * (0 = vertical link (i,j)-(i,j+1), 1 = horizontal link (i,j)-(i+1,j)). */
int64_t orc_events(const orc_sim *s, int64_t *step, int32_t *i, int32_t *j, int32_t *orient,
                   int64_t cap);
/* Derived lattice constants: cs, c, dt, lambda, A0 (2 lambda/c^2),
 * Ak (lambda/(2 c^2)), traction coefficient dt/(rho dh). */
void orc_constants(const orc_sim *s, double out[7]);

/* CheckLinks for the crack-line segment between line coordinates a_prev and
 * a_new, run from the boundary points around the crack line at column b_col
 * (a crack along +x) or, for another direction, the four sites of the cell
 * holding the point at a_prev; writes the intersected links (i, j, orient)
 * found by the breadth-first search of Alg. 1 and by an exhaustive scan of every
 * link of the lattice.  Returns the counts through n_bfs / n_all. */
void orc_check_links(const orc_sim *s, double a_prev, double a_new, int32_t b_col,
                     int32_t *bfs_links, int32_t *n_bfs, int32_t *all_links, int32_t *n_all,
                     int32_t cap);

/* K at the current tip from the current displacement, as the crack step
 * computes it, with r_min taken for the crack speed vK (eq. r(v)); the
 * return value is NaN when the evaluation columns leave the crack. */
double orc_eval_K(const orc_sim *s, double vK);

/* eq. (sif): K from the crack opening delta at distance r. */
double orc_sif(double delta, double r, double mu);

/* Discrete adjoint of the affine LBM map (stationary crack, fixed mask;
 * a Dirichlet edge enters with the sign of its anti-bounce-back):
 * given lam_f [5][ny][nx] and lam_w [ny][nx] (adjoint of the state after a step),
 * overwrite them with the adjoint of the state before the step and return the
 * derivative of <lam, state_after> with respect to the step's traction tau. */
double orc_adjoint_step(orc_sim *s, double *lam_f, double *lam_w);

#ifdef __cplusplus
}
#endif
#endif
