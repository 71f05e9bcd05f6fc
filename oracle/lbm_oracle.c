/*
 * lbm_oracle.c -- plain FP64 CPU oracle of the lattice Boltzmann method for
 * antiplane shear with dynamic mode III crack growth (arXiv:2206.12412).
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU
 * baseline of the benchmark; never by the product path.  Slow and literal on
 * purpose: loops over j, i, alpha; no blocking, no fusion beyond the order in
 * which the paper states the steps.
 *
 * One time step (Sec. 3 and Sec. 4.1):
 *   1. streaming of the post-collision populations along the D2Q5 links
 *      (eq. LBE, left-hand side); a population whose link is severed by the
 *      crack or leaves the plate is bounced back (traction-free), plus a
 *      traction term on loaded links;
 *   2. particle velocity wdot = sum_alpha f^alpha          (eq. distrib-macro);
 *   3. Euler update w += dt * wdot                          (eq. integration);
 *   4. BGK collision towards f_eq(w, wdot)                  (eq. LBE, eq. f-eq);
 *   4a. (macroscopic boundary scheme only) w at the boundary points from
 *      the boundary conditions, S w_B = R; missing populations from eq.
 *      (f-macro-bc); collision at those points (Sec. 3.1);
 *   5. crack step appended after the integration (Alg. 1): evaluate the
 *      criterion with K from eq. (sif), advance the tip, find the intersected
 *      links by the breadth-first CheckLinks search, sever them.
 *
 * Readings taken where the paper is silent or garbled (each is listed in the
 * design notes of the repository):
 *   - f_eq^kappa = lambda w / (2 c^2): the printed lambda w / c^2 makes the
 *     zeroth moment of f_eq differ from wdot (eq. f-eq vs eq. distrib-macro);
 *   - lambda = c_s^2 / (dt (1/omega - 1/2)), which is the printed formula for
 *     mu = rho, tau = dt, dh = 1;
 *   - bounce-back at the link midpoint; a traction t* adds
 *     (dt / (rho dh)) t* to the reflected population (momentum balance);
 *   - a vertical link is severed when the closed crack segment touches it;
 *   - K uses the column i_K = floor(a - r_min), r = a - i_K, r_min from
 *     eq. r(v) with the speed of the previous step (mirrored for a left tip:
 *     i_K = ceil(a + r_min), r = i_K - a);
 *   - a Dirichlet edge holds the prescribed w* at the wall (link midpoint) by
 *     anti-bounce-back, f_in^alpha = -f^opp + 2 f_eq^alpha(w*, 0): the ghost
 *     site then carries 2 w* - w (the leapfrog's antisymmetric ghost);
 *   - with two tips, K and the criterion of both are evaluated on the same
 *     field, then both advance, the right tip's cuts recorded first;
 *   - the macroscopic boundary scheme (ORC_BC_MACRO, Sec. 3.1): the two
 *     interior points of a boundary point are the next two lattice points
 *     along the inward normal of its missing link (the boundary half a
 *     spacing beyond the point); a point with several missing links takes
 *     the mean of their polynomials; it applies after the whole sweep, before
 *     the crack step, so K reads the boundary values.
 */
#include "lbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NPOP 5
static const int EX[NPOP] = {0, 1, 0, -1, 0};
static const int EY[NPOP] = {0, 0, 1, 0, -1};
static const int OPP[NPOP] = {0, 3, 4, 1, 2};

typedef struct { int32_t i, j, o; } link_t;  /* o: 0 vertical, 1 horizontal */

/* One crack tip: position, speed of the last step, flags, the boundary points
 * of its previous increment (Alg. 1, B_prev) and its traces.  dir = +1 for
 * the right tip (grows in +x), -1 for the left one. */
typedef struct {
  int dir;
  double a, v;
  int32_t flags;
  int32_t *bprev, nbprev, capbprev;
  double *trK, *trA, *trV;
  int32_t *trF;
} tip_t;

struct orc_sim {
  orc_config cfg;
  double *tau;                       /* private copy of the traction history */
  double *wD;                        /* private copy of the wall displacements */
  double cs, c, dt, lambda, A0, Ak, coef;
  int32_t j0;
  double yc;
  int aligned;                       /* growth along +x on the crack row */
  double ux, uy;                     /* unit growth direction of the right tip */
  double a_lo, a_hi;                 /* line coordinates where the line leaves the plate */
  double *f, *fn, *w;
  uint8_t *cutV, *cutH;
  tip_t tips[2];                     /* [0] right tip, [1] left end / left tip */
  int64_t step;
  /* cut events */
  int64_t *evs;
  int32_t *evi, *evj, *evo;
  int64_t nev, capev;
  /* scratch for the breadth-first search */
  uint8_t *inq, *vis;
  int32_t *queue, *touched;
  /* macroscopic boundary scheme: w before the step, and the weights of the
   * quadratic polynomial for a prescribed w and for a traction */
  double *wold;
  double qw_dir[3], qw_trac[3];
};

static inline size_t IDX(const orc_sim *s, int i, int j) {
  return (size_t)j * (size_t)s->cfg.nx + (size_t)i;
}
static inline double *POP(orc_sim *s, double *base, int a) {
  return base + (size_t)a * (size_t)s->cfg.nx * (size_t)s->cfg.ny;
}

/* ---------------------------------------------------------------- links -- */

/* Link between site (i, j) and its neighbour in direction (dx, dy), |dx|+|dy| = 1.
 * Returns 0 if the neighbour lies outside the plate (walls mode). */
static int link_of(const orc_sim *s, int i, int j, int dx, int dy, link_t *L) {
  const int nx = s->cfg.nx, ny = s->cfg.ny;
  int ni = i + dx, nj = j + dy;
  if (s->cfg.periodic) {
    ni = (ni + nx) % nx;
    nj = (nj + ny) % ny;
  } else if (ni < 0 || ni >= nx || nj < 0 || nj >= ny) {
    return 0;
  }
  if (dy == 0) { /* horizontal link, stored at its left end (i, i+1 mod nx) */
    L->o = 1;
    L->j = j;
    L->i = (dx > 0) ? i : ni;
  } else {       /* vertical link, stored at its lower end */
    L->o = 0;
    L->i = i;
    L->j = (dy > 0) ? j : nj;
  }
  return 1;
}

static int is_cut(const orc_sim *s, const link_t *L) {
  size_t k = (size_t)L->j * (size_t)s->cfg.nx + (size_t)L->i;
  return L->o == 0 ? s->cutV[k] : s->cutH[k];
}

static void set_cut(orc_sim *s, const link_t *L) {
  size_t k = (size_t)L->j * (size_t)s->cfg.nx + (size_t)L->i;
  if (L->o == 0) s->cutV[k] = 1; else s->cutH[k] = 1;
}

/* Segment-segment intersection of closed segments (touching counts). */
static int orient(double px, double py, double qx, double qy, double rx, double ry) {
  double d = (qx - px) * (ry - py) - (qy - py) * (rx - px);
  return (d > 0) - (d < 0);
}
static int on_segment(double px, double py, double qx, double qy, double rx, double ry) {
  /* r collinear with p-q: is it inside the bounding box of p-q? */
  return fmin(px, qx) <= rx && rx <= fmax(px, qx) && fmin(py, qy) <= ry && ry <= fmax(py, qy);
}
static int segments_intersect(double p1x, double p1y, double p2x, double p2y,
                              double q1x, double q1y, double q2x, double q2y) {
  int d1 = orient(q1x, q1y, q2x, q2y, p1x, p1y);
  int d2 = orient(q1x, q1y, q2x, q2y, p2x, p2y);
  int d3 = orient(p1x, p1y, p2x, p2y, q1x, q1y);
  int d4 = orient(p1x, p1y, p2x, p2y, q2x, q2y);
  if (d1 * d2 < 0 && d3 * d4 < 0) return 1;
  if (d1 == 0 && on_segment(q1x, q1y, q2x, q2y, p1x, p1y)) return 1;
  if (d2 == 0 && on_segment(q1x, q1y, q2x, q2y, p2x, p2y)) return 1;
  if (d3 == 0 && on_segment(p1x, p1y, p2x, p2y, q1x, q1y)) return 1;
  if (d4 == 0 && on_segment(p1x, p1y, p2x, p2y, q2x, q2y)) return 1;
  return 0;
}

/* The point of the crack line at line coordinate a: (a, y_c) along +x, else
 * S + (a - x0) u. */
static void crack_point(const orc_sim *s, double a, double *x, double *y) {
  if (s->aligned) {
    *x = a;
    *y = s->yc;
    return;
  }
  const double d = a - s->cfg.crack_x0;
  *x = s->cfg.crack_x0 + d * s->ux;
  *y = s->yc + d * s->uy;
}

/* Does the crack segment between line coordinates a0 and a1 intersect the
 * link from site p to its neighbour n?  Links are the straight lines between
 * lattice points. */
static int seg_hits_link(const orc_sim *s, double a0, double a1, int pi, int pj, int ni, int nj) {
  double x0, y0, x1, y1;
  crack_point(s, a0, &x0, &y0);
  crack_point(s, a1, &x1, &y1);
  return segments_intersect(x0, y0, x1, y1, (double)pi, (double)pj, (double)ni, (double)nj);
}

/* Arc length from (x, y) along (ux, uy) to the plate's wall rectangle
 * [-1/2, nx - 1/2] x [-1/2, ny - 1/2] (the point lies inside it). */
static double exit_length(const orc_sim *s, double x, double y, double ux, double uy) {
  double t = INFINITY;
  if (ux > 0) t = fmin(t, (s->cfg.nx - 0.5 - x) / ux);
  if (ux < 0) t = fmin(t, (-0.5 - x) / ux);
  if (uy > 0) t = fmin(t, (s->cfg.ny - 0.5 - y) / uy);
  if (uy < 0) t = fmin(t, (-0.5 - y) / uy);
  return t;
}

/* ------------------------------------------------------------- creation -- */

/* ------------------------------------------ macroscopic boundary scheme -- */

/* Sec. 3.1: near a boundary point x_B the displacement is approximated by a
 * quadratic polynomial p(s) = c0 + c1 s + c2 s^2 along the inward boundary
 * normal, s the distance from the boundary.  With the lattice-aligned walls
 * and crack of this solver the boundary lies half a spacing beyond x_B
 * (s_B = 1/2), and the two interior points are the next lattice points along
 * the normal, x_I at s = 3/2 and x_II at s = 5/2 (so the bilinear
 * interpolation of the paper returns their lattice values).  The polynomial
 * is fixed by p(0) = w* (prescribed w) or p'(0) = dw/ds (traction) and by
 * p(s_I) = w(x_I), p(s_II) = w(x_II); then w(x_B) = p(s_B) = q[0] b + q[1]
 * w(x_I) + q[2] w(x_II), b the boundary value.  The weights q solve
 * M^T q = (1, s_B, s_B^2), M the 3 x 3 matrix of the three conditions acting
 * on (c0, c1, c2): Gaussian elimination with partial pivoting. */
static void quad_weights(int prescribed_w, double q[3]) {
  const double sB = 0.5, sI = 1.5, sII = 2.5;
  const double M[3][3] = {{prescribed_w ? 1.0 : 0.0, prescribed_w ? 0.0 : 1.0, 0.0},
                          {1.0, sI, sI * sI},
                          {1.0, sII, sII * sII}};
  double A[3][4];
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) A[r][c] = M[c][r]; /* the transpose */
  }
  A[0][3] = 1.0;
  A[1][3] = sB;
  A[2][3] = sB * sB;
  for (int k = 0; k < 3; ++k) {
    int piv = k;
    for (int r = k + 1; r < 3; ++r)
      if (fabs(A[r][k]) > fabs(A[piv][k])) piv = r;
    for (int c = 0; c < 4; ++c) {
      double t = A[k][c]; A[k][c] = A[piv][c]; A[piv][c] = t;
    }
    for (int r = k + 1; r < 3; ++r) {
      const double m = A[r][k] / A[k][k];
      for (int c = k; c < 4; ++c) A[r][c] -= m * A[k][c];
    }
  }
  for (int r = 2; r >= 0; --r) {
    double acc = A[r][3];
    for (int c = r + 1; c < 3; ++c) acc -= A[r][c] * q[c];
    q[r] = acc / A[r][r];
  }
}

orc_sim *orc_create(const orc_config *cfg, int32_t *err) {
  int32_t e = 0;
  if (cfg->nx < 1 || cfg->ny < 1) e = -1;
  else if (!(cfg->kappa > 0) || !(cfg->omega > 0 && cfg->omega < 2)) e = -1;
  else if (!(cfg->mu > 0) || !(cfg->rho > 0)) e = -1;
  /* omega = 1 is the leapfrog scheme: stable only for kappa > sqrt(2). */
  else if (cfg->kappa * cfg->kappa <= 2.0) e = -4;
  else if (cfg->has_crack && cfg->crack_row < 0 && (cfg->ny < 2 || cfg->ny % 2 != 0)) e = -1;
  else if (cfg->has_crack && cfg->crack_row >= 0 && cfg->crack_row > cfg->ny - 2) e = -1;
  else if (cfg->both_tips && !cfg->has_crack) e = -1;
  else if (cfg->dirichlet && (cfg->periodic || cfg->n_wD < 1 || !cfg->wD_hist)) e = -1;
  else if (!(isfinite(cfg->crack_dx) && isfinite(cfg->crack_dy))) e = -1;
  /* the start point inside the plate, the tip on the far side of it (and,
   * along +x, inside the plate; for another direction checked below) */
  else if (cfg->has_crack && !(cfg->crack_x0 >= -0.5 && cfg->crack_x0 <= cfg->nx - 0.5 &&
                               cfg->crack_tip >= cfg->crack_x0 &&
                               (cfg->crack_tip <= cfg->nx - 0.5 ||
                                !(cfg->crack_dy == 0.0 && cfg->crack_dx >= 0.0)))) e = -5;
  else if (cfg->growth != ORC_GROW_NONE && (!cfg->has_crack || cfg->periodic)) e = -1;
  else if (cfg->growth == ORC_GROW_PRESCRIBED && !(cfg->v_rel >= 0 && cfg->v_rel < 1)) e = -1;
  else if (cfg->growth == ORC_GROW_SIF && !(cfg->K_C > 0 && cfg->v_max >= 0 && cfg->v_max < 1))
    e = -1;
  else if (cfg->has_crack && !(cfg->r0 > 0)) e = -1;
  else if (cfg->has_crack && cfg->k_band < 1) e = -1;
  else if (cfg->n_hist < 0 || (cfg->n_hist > 0 && !cfg->tau_hist)) e = -1;
  else if (cfg->bc_scheme != ORC_BC_LINK && cfg->bc_scheme != ORC_BC_MACRO) e = -1;
  /* the macroscopic scheme: walls, a crack along +x, and two interior points
   * along the normal of every boundary point on its own side of the crack */
  else if (cfg->bc_scheme == ORC_BC_MACRO &&
           (cfg->periodic || cfg->nx < 3 || cfg->ny < 3 ||
            (cfg->has_crack && !(cfg->crack_dy == 0.0 && cfg->crack_dx >= 0.0)))) e = -1;
  else if (cfg->bc_scheme == ORC_BC_MACRO && cfg->has_crack) {
    /* three rows on either side of the crack line: the interior points of a
     * crack face are then no edge points (and no edge point reaches back to
     * a face), so S couples no point to itself */
    const int jc = cfg->crack_row >= 0 ? cfg->crack_row : cfg->ny / 2 - 1;
    if (jc < 3 || jc + 4 > cfg->ny - 1) e = -1;
  }
  if (e) {
    if (err) *err = e;
    return NULL;
  }
  orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
  s->cfg = *cfg;
  const size_t n = (size_t)cfg->nx * (size_t)cfg->ny;
  s->tau = NULL;
  if (cfg->n_hist > 0) {
    s->tau = (double *)malloc(sizeof(double) * (size_t)cfg->n_hist);
    memcpy(s->tau, cfg->tau_hist, sizeof(double) * (size_t)cfg->n_hist);
  }
  s->cfg.tau_hist = s->tau;
  s->wD = NULL;
  if (cfg->dirichlet) {
    s->wD = (double *)malloc(sizeof(double) * 4 * (size_t)cfg->n_wD);
    memcpy(s->wD, cfg->wD_hist, sizeof(double) * 4 * (size_t)cfg->n_wD);
  }
  s->cfg.wD_hist = s->wD;
  s->cfg.w0 = NULL;
  s->cfg.wdot0 = NULL;

  /* Lattice constants (Sec. 3): c = kappa c_s, dt = dh / c with dh = 1. */
  s->cs = sqrt(cfg->mu / cfg->rho);
  s->c = cfg->kappa * s->cs;
  s->dt = 1.0 / s->c;
  s->lambda = s->cs * s->cs / (s->dt * (1.0 / cfg->omega - 0.5));
  s->A0 = 2.0 * s->lambda / (s->c * s->c);
  s->Ak = s->lambda / (2.0 * s->c * s->c);
  s->coef = s->dt / (cfg->rho * 1.0);
  s->j0 = cfg->crack_row >= 0 ? cfg->crack_row : cfg->ny / 2 - 1;
  s->yc = s->j0 + 0.5;
  /* growth direction: +x along the crack row unless another one is given */
  s->aligned = (cfg->crack_dy == 0.0 && cfg->crack_dx >= 0.0);
  if (s->aligned) {
    s->ux = 1.0;
    s->uy = 0.0;
    s->a_lo = -0.5;
    s->a_hi = cfg->nx - 0.5;
  } else {
    const double nrm = sqrt(cfg->crack_dx * cfg->crack_dx + cfg->crack_dy * cfg->crack_dy);
    s->ux = cfg->crack_dx / nrm;
    s->uy = cfg->crack_dy / nrm;
    /* exact unit vectors along the axes */
    if (cfg->crack_dx == 0.0) { s->ux = 0.0; s->uy = cfg->crack_dy > 0 ? 1.0 : -1.0; }
    if (cfg->crack_dy == 0.0) { s->uy = 0.0; s->ux = cfg->crack_dx > 0 ? 1.0 : -1.0; }
    s->a_hi = cfg->crack_x0 + exit_length(s, cfg->crack_x0, s->yc, s->ux, s->uy);
    s->a_lo = cfg->crack_x0 - exit_length(s, cfg->crack_x0, s->yc, -s->ux, -s->uy);
    if (cfg->has_crack && (cfg->crack_tip > s->a_hi || cfg->k_band != 1)) {
      free(s->tau);
      free(s->wD);
      free(s);
      if (err) *err = cfg->k_band != 1 ? -1 : -5;
      return NULL;
    }
  }

  s->f = (double *)calloc(NPOP * n, sizeof(double));
  s->fn = (double *)calloc(NPOP * n, sizeof(double));
  s->w = (double *)calloc(n, sizeof(double));
  s->cutV = (uint8_t *)calloc(n, 1);
  s->cutH = (uint8_t *)calloc(n, 1);
  s->inq = (uint8_t *)calloc(n, 1);
  s->vis = (uint8_t *)calloc(n, 1);
  s->queue = (int32_t *)malloc(sizeof(int32_t) * n);
  s->touched = (int32_t *)malloc(sizeof(int32_t) * n);
  if (cfg->bc_scheme == ORC_BC_MACRO) {
    s->wold = (double *)malloc(sizeof(double) * n);
    quad_weights(1, s->qw_dir);
    quad_weights(0, s->qw_trac);
  }

  /* Initial state: at rest or the given fields, populations in equilibrium. */
  for (int j = 0; j < cfg->ny; ++j)
    for (int i = 0; i < cfg->nx; ++i) {
      size_t x = IDX(s, i, j);
      double w = cfg->w0 ? cfg->w0[x] : 0.0;
      double wd = cfg->wdot0 ? cfg->wdot0[x] : 0.0;
      s->w[x] = w;
      POP(s, s->f, 0)[x] = wd - s->A0 * w;
      for (int a = 1; a < NPOP; ++a) POP(s, s->f, a)[x] = s->Ak * w;
    }

  /* Initial crack: every link intersected by the segment x0..a0 is severed. */
  for (int t = 0; t < 2; ++t) {
    tip_t *T = &s->tips[t];
    T->dir = t == 0 ? 1 : -1;
    T->a = t == 0 ? cfg->crack_tip : cfg->crack_x0;
    T->v = 0.0;
    T->flags = 0;
    T->capbprev = 64;
    T->bprev = (int32_t *)malloc(sizeof(int32_t) * 2 * T->capbprev);
    T->nbprev = 0;
    if (cfg->trace_cap > 0) {
      T->trK = (double *)calloc((size_t)cfg->trace_cap, sizeof(double));
      T->trA = (double *)calloc((size_t)cfg->trace_cap, sizeof(double));
      T->trV = (double *)calloc((size_t)cfg->trace_cap, sizeof(double));
      T->trF = (int32_t *)calloc((size_t)cfg->trace_cap, sizeof(int32_t));
    }
  }
  if (cfg->has_crack) {
    for (int j = 0; j < cfg->ny; ++j)
      for (int i = 0; i < cfg->nx; ++i) {
        link_t L;
        if (link_of(s, i, j, 0, 1, &L) && seg_hits_link(s, cfg->crack_x0, cfg->crack_tip, i, j, i, j + 1))
          set_cut(s, &L);
        if (link_of(s, i, j, 1, 0, &L) && seg_hits_link(s, cfg->crack_x0, cfg->crack_tip, i, j, i + 1, j))
          set_cut(s, &L);
      }
    /* B_prev: the pair of sites around the crack line at the tip column
     * (the right tip's floor(a), the left tip's ceil(a)); for another
     * direction the four sites of the lattice cell that holds the tip. */
    for (int t = 0; t < 2; ++t) {
      tip_t *T = &s->tips[t];
      if (s->aligned) {
        int c = t == 0 ? (int)floor(T->a) : (int)ceil(T->a);
        if (c < 0) c = 0;
        if (c > cfg->nx - 1) c = cfg->nx - 1;
        T->bprev[0] = c; T->bprev[1] = s->j0;
        T->bprev[2] = c; T->bprev[3] = s->j0 + 1;
        T->nbprev = 2;
      } else {
        double x, y;
        crack_point(s, T->a, &x, &y);
        const int ci = (int)floor(x), cj = (int)floor(y);
        T->nbprev = 0;
        for (int dj = 0; dj <= 1; ++dj)
          for (int di = 0; di <= 1; ++di) {
            int pi = ci + di, pj = cj + dj;
            if (pi < 0) pi = 0;
            if (pi > cfg->nx - 1) pi = cfg->nx - 1;
            if (pj < 0) pj = 0;
            if (pj > cfg->ny - 1) pj = cfg->ny - 1;
            T->bprev[2 * T->nbprev] = pi;
            T->bprev[2 * T->nbprev + 1] = pj;
            T->nbprev++;
          }
      }
    }
  }

  s->capev = 16;
  s->evs = (int64_t *)malloc(sizeof(int64_t) * s->capev);
  s->evi = (int32_t *)malloc(sizeof(int32_t) * s->capev);
  s->evj = (int32_t *)malloc(sizeof(int32_t) * s->capev);
  s->evo = (int32_t *)malloc(sizeof(int32_t) * s->capev);
  if (err) *err = 0;
  return s;
}

void orc_free(orc_sim *s) {
  if (!s) return;
  free(s->tau); free(s->wD); free(s->f); free(s->fn); free(s->w); free(s->cutV); free(s->cutH);
  free(s->inq); free(s->vis); free(s->queue); free(s->touched);
  for (int t = 0; t < 2; ++t) {
    free(s->tips[t].bprev);
    free(s->tips[t].trK); free(s->tips[t].trA); free(s->tips[t].trV); free(s->tips[t].trF);
  }
  free(s->evs); free(s->evi); free(s->evj); free(s->evo);
  free(s->wold);
  free(s);
}

/* ------------------------------------------------------------ LBM sweep -- */

/* Traction t* on the boundary seen by the population of site (i, j) that is
 * pulled along alpha, when that link is severed or leaves the plate. */
static double traction(const orc_sim *s, int j, int alpha, int outside, double tau) {
  if (s->cfg.periodic) return 0.0;
  if (outside) {
    /* top edge (outward normal +y) carries sigma_yz = tau, bottom edge -tau;
     * the lateral edges are traction-free */
    if (alpha == 4 && j == s->cfg.ny - 1) return tau;
    if (alpha == 2 && j == 0) return -tau;
    return 0.0;
  }
  /* severed link: crack faces, loaded only in the face-traction test mode;
   * the face above the crack has outward normal -y, the one below +y */
  if (alpha == 2) return s->cfg.face_traction;
  if (alpha == 4) return -s->cfg.face_traction;
  return 0.0;
}

static double tau_at(const orc_sim *s, int64_t n) {
  if (s->cfg.n_hist <= 0) return 0.0;
  return s->tau[n < s->cfg.n_hist ? n : s->cfg.n_hist - 1];
}

/* The wall a population pulled along alpha at site (i, j) crosses when its
 * upstream neighbour lies outside the plate (an ORC_EDGE_* bit). */
static int edge_of(const orc_sim *s, int i, int j, int alpha) {
  if (alpha == 1 && i == 0) return ORC_EDGE_LEFT;
  if (alpha == 3 && i == s->cfg.nx - 1) return ORC_EDGE_RIGHT;
  if (alpha == 2 && j == 0) return ORC_EDGE_BOTTOM;
  if (alpha == 4 && j == s->cfg.ny - 1) return ORC_EDGE_TOP;
  return 0;
}

/* Prescribed wall displacement of an edge at step n. */
static double wall_w(const orc_sim *s, int edge, int64_t n) {
  const double *row = s->wD + 4 * (n < s->cfg.n_wD ? n : s->cfg.n_wD - 1);
  switch (edge) {
    case ORC_EDGE_BOTTOM: return row[0];
    case ORC_EDGE_TOP: return row[1];
    case ORC_EDGE_LEFT: return row[2];
    default: return row[3];
  }
}

static int sweep_threads(const orc_sim *s) {
#ifdef _OPENMP
  return s->cfg.threads > 0 ? s->cfg.threads : omp_get_max_threads();
#else
  (void)s;
  return 1;
#endif
}

static void lbm_sweep(orc_sim *s) {
  const int nx = s->cfg.nx, ny = s->cfg.ny;
  const double tau = tau_at(s, s->step);
  const double omega = s->cfg.omega;
#pragma omp parallel for schedule(static) num_threads(sweep_threads(s))
  for (int j = 0; j < ny; ++j) {
    for (int i = 0; i < nx; ++i) {
      const size_t x = IDX(s, i, j);
      double fin[NPOP];
      fin[0] = POP(s, s->f, 0)[x];
      for (int a = 1; a < NPOP; ++a) {
        /* pull from the upstream neighbour y = x - c^alpha */
        link_t L;
        int inside = link_of(s, i, j, -EX[a], -EY[a], &L);
        if (inside && !is_cut(s, &L)) {
          int si = i - EX[a], sj = j - EY[a];
          if (s->cfg.periodic) { si = (si + nx) % nx; sj = (sj + ny) % ny; }
          fin[a] = POP(s, s->f, a)[IDX(s, si, sj)];
        } else if (!inside && (s->cfg.dirichlet & edge_of(s, i, j, a))) {
          /* anti-bounce-back: the wall (link midpoint) holds w*, i.e. the
           * ghost site carries 2 w* - w(x); f_eq^alpha(w*, 0) = Ak w* */
          fin[a] = -POP(s, s->f, OPP[a])[x] + 2.0 * s->Ak * wall_w(s, edge_of(s, i, j, a), s->step);
        } else {
          /* bounce-back: the population that left x towards y returns */
          fin[a] = POP(s, s->f, OPP[a])[x] + s->coef * traction(s, j, a, !inside, tau);
        }
      }
      double wd = fin[0] + fin[1] + fin[2] + fin[3] + fin[4];
      double wn = s->w[x] + s->dt * wd;
      double feq[NPOP];
      feq[0] = wd - s->A0 * wn;
      for (int a = 1; a < NPOP; ++a) feq[a] = s->Ak * wn;
      for (int a = 0; a < NPOP; ++a) POP(s, s->fn, a)[x] = fin[a] - omega * (fin[a] - feq[a]);
      s->w[x] = wn;
    }
  }
  double *t = s->f; s->f = s->fn; s->fn = t;
}

/* Sec. 3.1, after the streaming, moment and integration of every site:
 * boundary points (sites with a severed link or a link leaving the plate)
 * take w from the boundary conditions instead.  For each missing link of
 * x_B, whose outward normal is that link's direction, the polynomial through
 * the boundary condition on it and the interior points x_B - c, x_B - 2c
 * gives one equation; a point with several missing links (a corner) takes
 * the mean of them.  Values at interior points are this step's, and where
 * an interior point is itself a boundary point its w is an unknown: the
 * equations form S w_B = R.  S = I - N, N holding those couplings; the chain
 * of couplings ends at points whose interior points are interior sites, so N
 * is nilpotent and the Jacobi iteration w_B <- R + N w_B reaches the exact
 * solution after at most as many sweeps as the longest chain (it is run
 * until it no longer changes, and fails if it has not stopped after n_B + 2
 * sweeps).  Then the missing populations follow from eq. (f-macro-bc) with
 * wdot_B = (w_B(t + dt) - w_B(t)) / dt, and x_B collides as any site. */
static int macro_boundary(orc_sim *s) {
  const int nx = s->cfg.nx, ny = s->cfg.ny;
  const size_t n = (size_t)nx * ny;
  const double tau = tau_at(s, s->step);
  const double omega = s->cfg.omega;
  int32_t *bidx = (int32_t *)malloc(sizeof(int32_t) * n);
  int32_t nb = 0;
  for (size_t x = 0; x < n; ++x) bidx[x] = -1;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i)
      for (int b = 1; b < NPOP; ++b) {
        link_t L;
        if (!link_of(s, i, j, EX[b], EY[b], &L) || is_cut(s, &L)) {
          bidx[IDX(s, i, j)] = nb++;
          break;
        }
      }
  /* rows of S w_B = R: R[b], and up to 8 couplings (column, weight) */
  double *R = (double *)calloc((size_t)nb + 1, sizeof(double));
  int32_t *ncol = (int32_t *)calloc((size_t)nb + 1, sizeof(int32_t));
  int32_t *col = (int32_t *)malloc(sizeof(int32_t) * 8 * ((size_t)nb + 1));
  double *wt = (double *)malloc(sizeof(double) * 8 * ((size_t)nb + 1));
  size_t *site = (size_t *)malloc(sizeof(size_t) * ((size_t)nb + 1));
  int rc = 0;
  for (int j = 0; j < ny && !rc; ++j)
    for (int i = 0; i < nx && !rc; ++i) {
      const size_t x = IDX(s, i, j);
      const int32_t r = bidx[x];
      if (r < 0) continue;
      site[r] = x;
      int miss[NPOP], m = 0, outside[NPOP];
      for (int b = 1; b < NPOP; ++b) {
        link_t L;
        const int in = link_of(s, i, j, EX[b], EY[b], &L);
        if (!in || is_cut(s, &L)) { outside[m] = !in; miss[m++] = b; }
      }
      for (int k = 0; k < m; ++k) {
        const int b = miss[k];
        /* the interior points, inward along -c_b, on this side of the crack */
        const int i1 = i - EX[b], j1 = j - EY[b], i2 = i - 2 * EX[b], j2 = j - 2 * EY[b];
        link_t L1, L2;
        if (!link_of(s, i, j, -EX[b], -EY[b], &L1) || is_cut(s, &L1) ||
            !link_of(s, i1, j1, -EX[b], -EY[b], &L2) || is_cut(s, &L2)) {
          rc = -7;
          break;
        }
        const double *q;
        double bval;
        /* the population that would have arrived through the missing link
         * is the one pulled along OPP[b]: its edge / traction rules */
        const int edge = outside[k] ? edge_of(s, i, j, OPP[b]) : 0;
        if (edge && (s->cfg.dirichlet & edge)) {
          q = s->qw_dir;
          bval = wall_w(s, edge, s->step);
        } else {
          /* traction t* = mu dw/dn on the outward normal c_b: the slope
           * along the inward normal is -t* / mu */
          q = s->qw_trac;
          bval = -traction(s, j, OPP[b], outside[k], tau) / s->cfg.mu;
        }
        R[r] += q[0] * bval / m;
        const size_t p[2] = {IDX(s, i1, j1), IDX(s, i2, j2)};
        for (int e = 0; e < 2; ++e) {
          const double c = q[1 + e] / m;
          if (bidx[p[e]] >= 0) {
            col[8 * r + ncol[r]] = bidx[p[e]];
            wt[8 * r + ncol[r]] = c;
            ncol[r]++;
          } else {
            R[r] += c * s->w[p[e]];
          }
        }
      }
    }
  double *wb = (double *)malloc(sizeof(double) * ((size_t)nb + 1));
  double *wn = (double *)malloc(sizeof(double) * ((size_t)nb + 1));
  if (!rc) {
    for (int32_t r = 0; r < nb; ++r) wb[r] = R[r];
    int done = 0;
    for (int it = 0; it < nb + 2 && !done; ++it) {
      done = 1;
      for (int32_t r = 0; r < nb; ++r) {
        double acc = R[r];
        for (int k = 0; k < ncol[r]; ++k) acc += wt[8 * r + k] * wb[col[8 * r + k]];
        wn[r] = acc;
        if (acc != wb[r]) done = 0;
      }
      double *t = wb; wb = wn; wn = t;
    }
    if (!done) rc = -7;
  }
  if (!rc) {
    /* eq. (f-macro-bc) and the collision at every boundary point; the
     * source populations of this step are in s->fn (swapped by the sweep) */
    for (int32_t r = 0; r < nb; ++r) {
      const size_t x = site[r];
      const int i = (int)(x % (size_t)nx), j = (int)(x / (size_t)nx);
      const double w_new = wb[r];
      const double wd = (w_new - s->wold[x]) / s->dt;
      double fin[NPOP];
      int known[NPOP];
      double sum_known = POP(s, s->fn, 0)[x];
      int n_miss = 0;
      fin[0] = sum_known;
      known[0] = 1;
      for (int a = 1; a < NPOP; ++a) {
        link_t L;
        const int in = link_of(s, i, j, -EX[a], -EY[a], &L);
        known[a] = in && !is_cut(s, &L);
        if (known[a]) {
          fin[a] = POP(s, s->fn, a)[IDX(s, i - EX[a], j - EY[a])];
          sum_known += fin[a];
        } else {
          n_miss++;
        }
      }
      for (int a = 1; a < NPOP; ++a)
        if (!known[a]) fin[a] = (wd - sum_known) / n_miss;
      double feq[NPOP];
      feq[0] = wd - s->A0 * w_new;
      for (int a = 1; a < NPOP; ++a) feq[a] = s->Ak * w_new;
      for (int a = 0; a < NPOP; ++a) POP(s, s->f, a)[x] = fin[a] - omega * (fin[a] - feq[a]);
      s->w[x] = w_new;
    }
  }
  free(bidx); free(R); free(ncol); free(col); free(wt); free(site); free(wb); free(wn);
  return rc;
}

/* -------------------------------------------------------- crack handling -- */

double orc_sif(double delta, double r, double mu) {
  return delta * (mu / 4.0) * sqrt(2.0 * M_PI / r);
}

/* K at a tip from the displacement jump across the crack faces.  The right
 * tip evaluates at the column i_K = floor(a - r_min) (and i_K - 1, ... for a
 * band), the left tip at the mirrored column ceil(a + r_min) (and + 1, ...);
 * r is the horizontal distance from the tip.  The columns must lie on the
 * crack, i.e. between the two ends. */
/* K at a tip of a crack along another direction than +x.  Along the line,
 * the vertical links cross it at integer x and the horizontal ones at integer
 * y; the pair of sites used is that of the first crossing at or beyond r_min
 * behind the tip (for +x this is the column floor(a - r_min) of the rule
 * above), delta the jump of w between the two sites and r the distance along
 * the line from the tip to the projection of the pair's midpoint (for +x the
 * midpoint lies on the line, at the crossing).  A crossing through a lattice
 * site, off the crack or off the plate leaves K undefined. */
static double evaluate_K_line(const orc_sim *s, const tip_t *T, double vK, int32_t *undef) {
  const double x0 = s->cfg.crack_x0, yc = s->yc, ux = s->ux, uy = s->uy;
  const double rmin = s->cfg.r0 / (1.0 - vK);
  const double st = T->a - x0;                           /* the tip */
  const double so = s->tips[T->dir > 0 ? 1 : 0].a - x0;  /* the crack's other end */
  const double target = T->dir > 0 ? st - rmin : st + rmin;
  *undef = 1;
  /* candidate of each family: the crossing nearest to the target on the
   * side away from the tip */
  int have_v = 0, have_h = 0;
  double sv = 0.0, sh = 0.0, iv = 0.0, jh = 0.0;
  if (ux != 0.0) {
    const double xt = x0 + target * ux;
    iv = ((T->dir > 0) == (ux > 0)) ? floor(xt) : ceil(xt);
    sv = (iv - x0) / ux;
    have_v = 1;
  }
  if (uy != 0.0) {
    const double yt = yc + target * uy;
    jh = ((T->dir > 0) == (uy > 0)) ? floor(yt) : ceil(yt);
    sh = (jh - yc) / uy;
    have_h = 1;
  }
  int vertical;
  if (have_v && have_h) vertical = T->dir > 0 ? (sv >= sh) : (sv <= sh);
  else vertical = have_v;
  const double sc = vertical ? sv : sh;
  if (T->dir > 0 ? sc < so : sc > so) return NAN;  /* off the crack */
  int i0, j0, i1, j1;
  if (vertical) {
    const double y = yc + sc * uy;
    if (y == floor(y)) return NAN;  /* through a lattice site */
    i0 = i1 = (int)iv;
    j0 = (int)floor(y);
    j1 = j0 + 1;
  } else {
    const double x = x0 + sc * ux;
    if (x == floor(x)) return NAN;
    j0 = j1 = (int)jh;
    i0 = (int)floor(x);
    i1 = i0 + 1;
  }
  if (i0 < 0 || i1 > s->cfg.nx - 1 || j0 < 0 || j1 > s->cfg.ny - 1) return NAN;
  *undef = 0;
  const double delta = fabs(s->w[IDX(s, i1, j1)] - s->w[IDX(s, i0, j0)]);
  const double mx = 0.5 * (double)(i0 + i1), my = 0.5 * (double)(j0 + j1);
  const double sm = (mx - x0) * ux + (my - yc) * uy;  /* projection of the midpoint */
  return orc_sif(delta, T->dir > 0 ? st - sm : sm - st, s->cfg.mu);
}

static double evaluate_K(const orc_sim *s, const tip_t *T, double vK, int32_t *undef) {
  if (!s->aligned) return evaluate_K_line(s, T, vK, undef);
  const int nx = s->cfg.nx;
  const double rmin = s->cfg.r0 / (1.0 - vK);
  const int band = s->cfg.k_band;
  const double other = s->tips[T->dir > 0 ? 1 : 0].a;  /* the crack's other end */
  *undef = 1;
  double iKf;
  if (T->dir > 0) {
    iKf = floor(T->a - rmin);
    if (!(iKf - (band - 1) >= 0.0) || !(iKf <= nx - 1) || iKf - (band - 1) < other) return NAN;
  } else {
    iKf = ceil(T->a + rmin);
    if (!(iKf >= 0.0) || !(iKf + (band - 1) <= nx - 1) || iKf + (band - 1) > other) return NAN;
  }
  const int iK = (int)iKf;
  *undef = 0;
  if (band == 1) {
    double delta = fabs(s->w[IDX(s, iK, s->j0 + 1)] - s->w[IDX(s, iK, s->j0)]);
    return orc_sif(delta, T->dir > 0 ? T->a - iK : iK - T->a, s->cfg.mu);
  }
  /* several columns: least-squares fit of delta_i = (4K/mu) sqrt(r_i / 2 pi) */
  double num = 0.0, den = 0.0;
  for (int b = 0; b < band; ++b) {
    int i = iK - T->dir * b;
    double r = T->dir > 0 ? T->a - i : i - T->a;
    double sq = sqrt(r / (2.0 * M_PI));
    double delta = fabs(s->w[IDX(s, i, s->j0 + 1)] - s->w[IDX(s, i, s->j0)]);
    num += delta * sq;
    den += sq * sq;
  }
  return (s->cfg.mu / 4.0) * num / den;
}

/* Alg. 1, CheckLinks: breadth-first search from the neighbours of the
 * previous boundary points; every link of a popped point is tested against
 * the new segment; a hit adds both ends to B and the neighbours of the far
 * end to the queue.  Returns the intersected links (and B through bout). */
static int32_t check_links_bfs(orc_sim *s, double a0, double a1, const int32_t *bprev, int32_t nb,
                               link_t *hits, int32_t caphits, int32_t *bout, int32_t *nbout,
                               int32_t capb) {
  const int nx = s->cfg.nx;
  int32_t head = 0, tail = 0, nt = 0, nh = 0;
  *nbout = 0;
  /* Q <- N(B_prev) */
  for (int p = 0; p < nb; ++p)
    for (int a = 1; a < NPOP; ++a) {
      link_t L;
      int pi = bprev[2 * p], pj = bprev[2 * p + 1];
      if (!link_of(s, pi, pj, EX[a], EY[a], &L)) continue;
      size_t k = IDX(s, pi + EX[a], pj + EY[a]);
      if (!s->inq[k]) { s->inq[k] = 1; s->queue[tail++] = (int32_t)k; s->touched[nt++] = (int32_t)k; }
    }
  while (head < tail) {
    const int32_t k = s->queue[head++]; /* pop p */
    const int pi = k % nx, pj = k / nx;
    s->vis[k] = 1;                     /* mark as visited */
    for (int a = 1; a < NPOP; ++a) {
      link_t L;
      if (!link_of(s, pi, pj, EX[a], EY[a], &L)) continue;
      const int ni = pi + EX[a], nj = pj + EY[a];
      if (!seg_hits_link(s, a0, a1, pi, pj, ni, nj)) continue;
      /* B <- B u {p, n_p} */
      int seen = 0;
      for (int h = 0; h < nh; ++h)
        if (hits[h].i == L.i && hits[h].j == L.j && hits[h].o == L.o) seen = 1;
      if (!seen && nh < caphits) hits[nh++] = L;
      const int ends[2][2] = {{pi, pj}, {ni, nj}};
      for (int e = 0; e < 2; ++e) {
        int dup = 0;
        for (int b = 0; b < *nbout; ++b)
          if (bout[2 * b] == ends[e][0] && bout[2 * b + 1] == ends[e][1]) dup = 1;
        if (!dup && *nbout < capb) {
          bout[2 * *nbout] = ends[e][0];
          bout[2 * *nbout + 1] = ends[e][1];
          ++*nbout;
        }
      }
      /* Q <- Q u N(n_p) \ V */
      for (int b = 1; b < NPOP; ++b) {
        link_t M;
        if (!link_of(s, ni, nj, EX[b], EY[b], &M)) continue;
        size_t q = IDX(s, ni + EX[b], nj + EY[b]);
        if (!s->vis[q] && !s->inq[q]) { s->inq[q] = 1; s->queue[tail++] = (int32_t)q; s->touched[nt++] = (int32_t)q; }
      }
    }
  }
  for (int t = 0; t < nt; ++t) { s->inq[s->touched[t]] = 0; s->vis[s->touched[t]] = 0; }
  return nh;
}

double orc_eval_K(const orc_sim *s, double vK) {
  int32_t undef;
  return evaluate_K(s, &s->tips[0], vK, &undef);
}

static void record_event(orc_sim *s, const link_t *L) {
  if (s->nev == s->capev) {
    s->capev *= 2;
    s->evs = (int64_t *)realloc(s->evs, sizeof(int64_t) * s->capev);
    s->evi = (int32_t *)realloc(s->evi, sizeof(int32_t) * s->capev);
    s->evj = (int32_t *)realloc(s->evj, sizeof(int32_t) * s->capev);
    s->evo = (int32_t *)realloc(s->evo, sizeof(int32_t) * s->capev);
  }
  s->evs[s->nev] = s->step;
  s->evi[s->nev] = L->i;
  s->evj[s->nev] = L->j;
  s->evo[s->nev] = L->o;
  s->nev++;
}

/* EvaluateCriterion for one tip: whether it grows this step and at which
 * speed (relative to c_s). */
static int criterion(const orc_sim *s, const tip_t *T, double K, double *v) {
  const orc_config *cfg = &s->cfg;
  *v = 0.0;
  if (T->flags & ORC_FLAG_WALL) return 0;
  if (cfg->growth == ORC_GROW_PRESCRIBED) {
    *v = cfg->v_rel;
    return 1;
  }
  if (cfg->growth == ORC_GROW_SIF && K > cfg->K_C) {
    /* eq. (v-tanh): crack speed regularised by the overshoot of K */
    double q = K / cfg->K_C;
    double q2 = q * q;
    *v = cfg->v_max * tanh(sqrt(q2 * q2 - 1.0));
    return 1;
  }
  return 0;
}

/* Advance one tip by (v c_s) dt along its direction, find the intersected
 * links with CheckLinks and sever them (ProcessPoints). */
static void advance(orc_sim *s, tip_t *T, double v, int32_t *flags) {
  const double a_prev = T->a;
  double a_new;
  if (T->dir > 0) {
    a_new = a_prev + (v * s->cs) * s->dt;
    if (a_new >= s->a_hi) {
      a_new = s->a_hi;
      *flags |= ORC_FLAG_WALL;
    }
  } else {
    a_new = a_prev - (v * s->cs) * s->dt;
    if (a_new <= s->a_lo) {
      a_new = s->a_lo;
      *flags |= ORC_FLAG_WALL;
    }
  }
  link_t hits[16];
  int32_t bnew[32];
  int32_t nbnew = 0;
  int32_t nh = check_links_bfs(s, a_prev, a_new, T->bprev, T->nbprev, hits, 16, bnew, &nbnew, 16);
  for (int h = 0; h < nh; ++h) {
    if (!is_cut(s, &hits[h])) {
      set_cut(s, &hits[h]);
      record_event(s, &hits[h]);
    }
  }
  if (nbnew > 0) {
    if (nbnew > T->capbprev) {
      T->capbprev = nbnew;
      T->bprev = (int32_t *)realloc(T->bprev, sizeof(int32_t) * 2 * T->capbprev);
    }
    memcpy(T->bprev, bnew, sizeof(int32_t) * 2 * nbnew);
    T->nbprev = nbnew;
  }
  T->a = a_new;
  *flags |= ORC_FLAG_GREW;
}

/* Alg. 1, CrackGrowth, appended after the time integration of the step: K
 * and the criterion at every growing tip on the same field, then the tips
 * advance (the right tip's cuts are recorded first). */
static void crack_step(orc_sim *s) {
  const orc_config *cfg = &s->cfg;
  const int ntips = cfg->both_tips ? 2 : 1;
  double K[2] = {NAN, NAN}, v[2] = {0.0, 0.0};
  int32_t flags[2] = {0, 0};
  int grow[2] = {0, 0};
  for (int t = 0; t < ntips; ++t) {
    tip_t *T = &s->tips[t];
    const double vK = (cfg->growth == ORC_GROW_PRESCRIBED) ? cfg->v_rel : T->v;
    int32_t undef = 0;
    K[t] = evaluate_K(s, T, vK, &undef);
    flags[t] = T->flags & ORC_FLAG_WALL;
    if (undef) flags[t] |= ORC_FLAG_K_UNDEF;
    grow[t] = criterion(s, T, K[t], &v[t]);
  }
  for (int t = 0; t < ntips; ++t) {
    tip_t *T = &s->tips[t];
    if (grow[t]) advance(s, T, v[t], &flags[t]);
    T->v = v[t];
    T->flags = flags[t];
    if (s->step < cfg->trace_cap) {
      T->trK[s->step] = K[t];
      T->trA[s->step] = T->a;
      T->trV[s->step] = v[t];
      T->trF[s->step] = flags[t];
    }
  }
}

int32_t orc_step(orc_sim *s, int64_t n) {
  for (int64_t k = 0; k < n; ++k) {
    const int macro = s->cfg.bc_scheme == ORC_BC_MACRO;
    if (macro) memcpy(s->wold, s->w, sizeof(double) * (size_t)s->cfg.nx * (size_t)s->cfg.ny);
    lbm_sweep(s);
    if (macro) {
      const int rc = macro_boundary(s);
      if (rc) return rc;
    }
    if (s->cfg.has_crack) crack_step(s);
    s->step++;
  }
  return 0;
}

/* --------------------------------------------------------------- adjoint -- */

double orc_adjoint_step(orc_sim *s, double *lam_f, double *lam_w) {
  /* The step is affine in (f, w) and in tau; this applies the transpose of
   * its linear part, site by site, in the order collision -> Euler -> moment
   * -> streaming reversed. */
  const int nx = s->cfg.nx, ny = s->cfg.ny;
  const size_t n = (size_t)nx * ny;
  const double om = s->cfg.omega;
  double *gin = (double *)malloc(sizeof(double) * NPOP * n);
  /* adjoint of collision, Euler update and moment, per site */
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      size_t x = IDX(s, i, j);
      double l[NPOP];
      for (int a = 0; a < NPOP; ++a) l[a] = lam_f[a * n + x];
      double G = lam_w[x] + om * (-s->A0 * l[0] + s->Ak * (l[1] + l[2] + l[3] + l[4]));
      double gwd = om * l[0] + s->dt * G;
      for (int a = 0; a < NPOP; ++a) gin[a * n + x] = (1.0 - om) * l[a] + gwd;
      lam_w[x] = G;
    }
  /* adjoint of streaming with bounce-back */
  double dtau = 0.0;
  for (int a = 0; a < NPOP; ++a)
    for (size_t x = 0; x < n; ++x) lam_f[a * n + x] = 0.0;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      size_t x = IDX(s, i, j);
      lam_f[0 * n + x] += gin[0 * n + x];
      for (int a = 1; a < NPOP; ++a) {
        link_t L;
        int inside = link_of(s, i, j, -EX[a], -EY[a], &L);
        double g = gin[a * n + x];
        if (inside && !is_cut(s, &L)) {
          int si = i - EX[a], sj = j - EY[a];
          if (s->cfg.periodic) { si = (si + nx) % nx; sj = (sj + ny) % ny; }
          lam_f[a * n + IDX(s, si, sj)] += g;
        } else if (!inside && (s->cfg.dirichlet & edge_of(s, i, j, a))) {
          lam_f[OPP[a] * n + x] -= g;  /* anti-bounce-back: f_in = -f^opp + const */
        } else {
          lam_f[OPP[a] * n + x] += g;
          if (!inside && !s->cfg.periodic) {
            if (a == 4 && j == ny - 1) dtau += s->coef * g;
            if (a == 2 && j == 0) dtau -= s->coef * g;
          }
        }
      }
    }
  free(gin);
  return dtau;
}

/* ------------------------------------------------------------- queries -- */

void orc_get_fields(const orc_sim *s, double *w, double *wdot) {
  const size_t n = (size_t)s->cfg.nx * s->cfg.ny;
  for (size_t x = 0; x < n; ++x) {
    if (w) w[x] = s->w[x];
    if (wdot) {
      double acc = 0.0;
      for (int a = 0; a < NPOP; ++a) acc += s->f[a * n + x];
      wdot[x] = acc;
    }
  }
}

void orc_get_pops(const orc_sim *s, double *f) {
  memcpy(f, s->f, sizeof(double) * NPOP * (size_t)s->cfg.nx * s->cfg.ny);
}

void orc_set_state(orc_sim *s, const double *f, const double *w) {
  const size_t n = (size_t)s->cfg.nx * s->cfg.ny;
  if (f) memcpy(s->f, f, sizeof(double) * NPOP * n);
  if (w) memcpy(s->w, w, sizeof(double) * n);
}

void orc_get_mask(const orc_sim *s, uint8_t *cutV, uint8_t *cutH) {
  const size_t n = (size_t)s->cfg.nx * s->cfg.ny;
  if (cutV) memcpy(cutV, s->cutV, n);
  if (cutH) memcpy(cutH, s->cutH, n);
}

void orc_crack(const orc_sim *s, double *tip, double *v, int64_t *step, int32_t *flags) {
  if (tip) *tip = s->tips[0].a;
  if (v) *v = s->tips[0].v;
  if (step) *step = s->step;
  if (flags) *flags = s->tips[0].flags;
}

static int64_t tip_traces(const orc_sim *s, const tip_t *T, double *K, double *tip, double *v,
                          int32_t *flags, int64_t cap) {
  int64_t n = s->step < s->cfg.trace_cap ? s->step : s->cfg.trace_cap;
  if (n > cap) n = cap;
  for (int64_t k = 0; k < n; ++k) {
    if (K) K[k] = T->trK[k];
    if (tip) tip[k] = T->trA[k];
    if (v) v[k] = T->trV[k];
    if (flags) flags[k] = T->trF[k];
  }
  return n;
}

int64_t orc_traces(const orc_sim *s, double *K, double *tip, double *v, int32_t *flags,
                   int64_t cap) {
  return tip_traces(s, &s->tips[0], K, tip, v, flags, cap);
}

int64_t orc_traces_left(const orc_sim *s, double *K, double *tip, double *v, int32_t *flags,
                        int64_t cap) {
  return tip_traces(s, &s->tips[1], K, tip, v, flags, cap);
}

int64_t orc_events(const orc_sim *s, int64_t *step, int32_t *i, int32_t *j, int32_t *orient,
                   int64_t cap) {
  int64_t n = s->nev < cap ? s->nev : cap;
  for (int64_t k = 0; k < n; ++k) {
    if (step) step[k] = s->evs[k];
    if (i) i[k] = s->evi[k];
    if (j) j[k] = s->evj[k];
    if (orient) orient[k] = s->evo[k];
  }
  return s->nev;
}

void orc_constants(const orc_sim *s, double out[7]) {
  out[0] = s->cs; out[1] = s->c; out[2] = s->dt; out[3] = s->lambda;
  out[4] = s->A0; out[5] = s->Ak; out[6] = s->coef;
}

void orc_check_links(const orc_sim *s_in, double a_prev, double a_new, int32_t b_col,
                     int32_t *bfs_links, int32_t *n_bfs, int32_t *all_links, int32_t *n_all,
                     int32_t cap) {
  orc_sim *s = (orc_sim *)s_in;
  link_t hits[64];
  int32_t bp[8] = {b_col, s->j0, b_col, s->j0 + 1};
  int32_t nbp = 2;
  if (!s->aligned) {  /* the cell holding the point at a_prev */
    double x, y;
    crack_point(s, a_prev, &x, &y);
    nbp = 0;
    for (int dj = 0; dj <= 1; ++dj)
      for (int di = 0; di <= 1; ++di) {
        int pi = (int)floor(x) + di, pj = (int)floor(y) + dj;
        pi = pi < 0 ? 0 : (pi > s->cfg.nx - 1 ? s->cfg.nx - 1 : pi);
        pj = pj < 0 ? 0 : (pj > s->cfg.ny - 1 ? s->cfg.ny - 1 : pj);
        bp[2 * nbp] = pi;
        bp[2 * nbp + 1] = pj;
        ++nbp;
      }
  }
  int32_t bout[128], nbout = 0;
  int32_t nh = check_links_bfs(s, a_prev, a_new, bp, nbp, hits, 64, bout, &nbout, 64);
  *n_bfs = 0;
  for (int h = 0; h < nh && h < cap; ++h) {
    bfs_links[3 * h] = hits[h].i; bfs_links[3 * h + 1] = hits[h].j; bfs_links[3 * h + 2] = hits[h].o;
    ++*n_bfs;
  }
  *n_all = 0;
  for (int j = 0; j < s->cfg.ny; ++j)
    for (int i = 0; i < s->cfg.nx; ++i) {
      link_t L;
      if (link_of(s, i, j, 0, 1, &L) && seg_hits_link(s, a_prev, a_new, i, j, i, j + 1) && *n_all < cap) {
        all_links[3 * *n_all] = L.i; all_links[3 * *n_all + 1] = L.j; all_links[3 * *n_all + 2] = 0;
        ++*n_all;
      }
      if (link_of(s, i, j, 1, 0, &L) && seg_hits_link(s, a_prev, a_new, i, j, i + 1, j) && *n_all < cap) {
        all_links[3 * *n_all] = L.i; all_links[3 * *n_all + 1] = L.j; all_links[3 * *n_all + 2] = 1;
        ++*n_all;
      }
    }
}
