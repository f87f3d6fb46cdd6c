/* FP64 CPU oracle of the exhaustive RKN seed scan -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * call this file. It shares no code with the GPU library.
 *
 * Built with -O2 -ffp-contract=off so that every operation rounds as written.
 * Each function cites the passage of the paper (sections and Eq. 1) it follows;
 * where the paper is silent the reading taken is stated beside the code.
 *
 * Parity status of each part:
 *   field, seed state, RKN step, trace ...... pinned (closed-form helix, order 4,
 *                                              |T| and Busch invariants)
 *   segment/wire distance, DOCA ............. pinned (skew-line and axial-wire closed
 *                                              forms, dense sampling)
 *   score, argmin ........................... pinned (truth seed, symmetries, brute
 *                                              force through an independent path)
 *   band pruning ............................ pinned (bit-identical to brute force)
 *   Hough accumulator and peaks ............. pinned (independent brute force,
 *                                              hits on a known circle)
 *   candidate -> window (constants) ......... parity unpinned as to quality: its
 *                                              constants are free readings
 *   coarse-to-fine rescan loop .............. pinned (one round = the k lowest of an
 *                                              independent window scan; truth on the
 *                                              grid found and kept; rounds compose)
 */
#include "rkn_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Field (section 2.2 sends "the magnetic field" to the device: a uniform value or
 * an (r, z) map). Reading: bilinear in (r, z), clamped to the edge outside the
 * grid; B_phi = 0; B_x = B_r x / r, B_y = B_r y / r, zero on the axis.          */
void orc_field_eval(const orc_field *f, const double x[3], double B[3]) {
  if (f->kind == 0) {
    B[0] = 0.0; B[1] = 0.0; B[2] = f->bz;
    return;
  }
  double r = sqrt(x[0] * x[0] + x[1] * x[1]);
  double dr = (f->r1 - f->r0) / (double)(f->nr - 1);
  double dz = (f->z1 - f->z0) / (double)(f->nz - 1);
  double u = (r - f->r0) / dr;
  double v = (x[2] - f->z0) / dz;
  int i = (int)floor(u), j = (int)floor(v);
  if (i < 0) i = 0;
  if (i > f->nr - 2) i = f->nr - 2;
  if (j < 0) j = 0;
  if (j > f->nz - 2) j = f->nz - 2;
  double a = u - i, b = v - j;
  if (a < 0.0) a = 0.0;
  if (a > 1.0) a = 1.0;
  if (b < 0.0) b = 0.0;
  if (b > 1.0) b = 1.0;
  int n00 = j * f->nr + i, n01 = j * f->nr + i + 1;
  int n10 = (j + 1) * f->nr + i, n11 = (j + 1) * f->nr + i + 1;
  double br = (1.0 - b) * ((1.0 - a) * (double)f->br[n00] + a * (double)f->br[n01]) +
              b * ((1.0 - a) * (double)f->br[n10] + a * (double)f->br[n11]);
  double bz = (1.0 - b) * ((1.0 - a) * (double)f->bzg[n00] + a * (double)f->bzg[n01]) +
              b * ((1.0 - a) * (double)f->bzg[n10] + a * (double)f->bzg[n11]);
  if (r < 1e-9) {
    B[0] = 0.0; B[1] = 0.0;
  } else {
    B[0] = br * x[0] / r;
    B[1] = br * x[1] / r;
  }
  B[2] = bz;
}

/* ------------------------------------------------------------------------- */
/* Section 2.1: the seed holds (R0, theta0, z0) in cylindrical and (px0, py0, pz0)
 * in Cartesian coordinates with R0 fixed, so five parameters are scanned.
 * State: position, unit direction T = p/|p|, Lambda = kappa q / |p|.          */
int orc_seed_state(const orc_params *p, const double seed[5], double x[3], double T[3], double *Lam) {
  double pm = sqrt(seed[2] * seed[2] + seed[3] * seed[3] + seed[4] * seed[4]);
  if (!(pm >= 1e-3)) return 0;
  x[0] = p->R0 * cos(seed[0]);
  x[1] = p->R0 * sin(seed[0]);
  x[2] = seed[1];
  T[0] = seed[2] / pm;
  T[1] = seed[3] / pm;
  T[2] = seed[4] / pm;
  *Lam = ORC_KAPPA * p->charge / pm;
  return 1;
}

/* x'' = Lam T x B(x): the Lorentz force on a unit-speed parametrisation. */
static void accel(const orc_field *f, double Lam, const double x[3], const double T[3], double k[3]) {
  double B[3];
  orc_field_eval(f, x, B);
  k[0] = Lam * (T[1] * B[2] - T[2] * B[1]);
  k[1] = Lam * (T[2] * B[0] - T[0] * B[2]);
  k[2] = Lam * (T[0] * B[1] - T[1] * B[0]);
}

/* Section 2.2: RKN track propagation. Classical fourth-order Runge-Kutta-Nystrom
 * formula for y'' = f(y, y') (Abramowitz & Stegun 25.5.20), fixed step h, three
 * field evaluations (start, middle, end). No renormalisation of T.            */
void orc_rkn_step(const orc_field *f, double Lam, double h, double x[3], double T[3]) {
  double k1[3], k2[3], k3[3], k4[3], xm[3], xe[3], Tt[3];
  int c;
  accel(f, Lam, x, T, k1);
  for (c = 0; c < 3; ++c) xm[c] = x[c] + 0.5 * h * T[c] + 0.125 * h * h * k1[c];
  for (c = 0; c < 3; ++c) Tt[c] = T[c] + 0.5 * h * k1[c];
  accel(f, Lam, xm, Tt, k2);
  for (c = 0; c < 3; ++c) Tt[c] = T[c] + 0.5 * h * k2[c];
  accel(f, Lam, xm, Tt, k3);
  for (c = 0; c < 3; ++c) xe[c] = x[c] + h * T[c] + 0.5 * h * h * k3[c];
  for (c = 0; c < 3; ++c) Tt[c] = T[c] + h * k3[c];
  accel(f, Lam, xe, Tt, k4);
  for (c = 0; c < 3; ++c) {
    x[c] = x[c] + h * T[c] + (h * h / 6.0) * (k1[c] + k2[c] + k3[c]);
    T[c] = T[c] + (h / 6.0) * (k1[c] + 2.0 * k2[c] + 2.0 * k3[c] + k4[c]);
  }
}

/* Section 2.3 and section 4.2 (the propagation runs to the end of the turn
 * partition). Reading: with turn_stop set, the partition ends with the first step
 * whose end point lies inside the seed cylinder r < R0 (the track has left the
 * chamber inwards); that step's chord is the last one. */
static int turn_ended(const orc_params *p, const double x[3]) {
  return p->turn_stop && x[0] * x[0] + x[1] * x[1] < p->R0 * p->R0;
}

int orc_trace(const orc_field *f, const orc_params *p, int64_t n_seeds, const double *seeds5,
              int32_t n_sel, const int32_t *step_idx, double *states) {
  int64_t s;
  for (s = 0; s < n_seeds; ++s) {
    double x[3], T[3], Lam;
    double *out = states + s * (int64_t)n_sel * 6;
    int32_t k, n = 0, ended = 0;
    if (!orc_seed_state(p, seeds5 + 5 * s, x, T, &Lam)) {
      for (k = 0; k < 6 * n_sel; ++k) out[k] = NAN;
      continue;
    }
    for (k = 0; k < n_sel; ++k) {
      while (n < step_idx[k] && !ended) {
        orc_rkn_step(f, Lam, p->step_mm, x, T);
        ++n;
        ended = turn_ended(p, x);
      }
      out[6 * k + 0] = x[0]; out[6 * k + 1] = x[1]; out[6 * k + 2] = x[2];
      out[6 * k + 3] = T[0]; out[6 * k + 4] = T[1]; out[6 * k + 5] = T[2];
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Section 2.2: distance of closest approach between the extrapolated track and a
 * wire. Reading: the track between steps is its chord [p0, p1]; the wire is the
 * finite segment m + t u, |t| <= L. The squared distance F(s, t) = |r + s d - t u|^2
 * (r = p0 - m, d = p1 - p0) is a convex quadratic on [0,1] x [-L, L], so its
 * minimum is the interior stationary point when that lies inside, otherwise the
 * smallest of the four edge minima (each a clamped 1-D convex quadratic).      */
static double f_at(const double r[3], const double d[3], const double u[3], double s, double t) {
  double v0 = r[0] + s * d[0] - t * u[0];
  double v1 = r[1] + s * d[1] - t * u[1];
  double v2 = r[2] + s * d[2] - t * u[2];
  return v0 * v0 + v1 * v1 + v2 * v2;
}
static double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

static double seg_wire_best(const double p0[3], const double p1[3], const double m[3], const double u[3],
                            double L, double *s_best, double *t_best);

double orc_seg_wire_dist2(const double p0[3], const double p1[3], const double m[3],
                          const double u[3], double L) {
  double sb, tb;
  return seg_wire_best(p0, p1, m, u, L, &sb, &tb);
}

/* Same minimum, also returning the minimising parameters (s on the chord, t on the
 * wire). Candidates are tried in a fixed order; the first smallest one wins.     */
static double seg_wire_best(const double p0[3], const double p1[3], const double m[3], const double u[3],
                            double L, double *s_best, double *t_best) {
  double r[3] = {p0[0] - m[0], p0[1] - m[1], p0[2] - m[2]};
  double d[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
  double a = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  double b = d[0] * u[0] + d[1] * u[1] + d[2] * u[2];
  double c = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  double e = d[0] * r[0] + d[1] * r[1] + d[2] * r[2];
  double g = u[0] * r[0] + u[1] * r[1] + u[2] * r[2];
  double best = INFINITY, v, s, t;
  double det = a * c - b * b;
#define ORC_TAKE(S, T)              \
  do {                              \
    v = f_at(r, d, u, (S), (T));    \
    if (v < best) {                 \
      best = v;                     \
      *s_best = (S);                \
      *t_best = (T);                \
    }                               \
  } while (0)
  *s_best = 0.0;
  *t_best = 0.0;
  if (det > 1e-14 * a * c) {          /* non-parallel: interior stationary point */
    s = (b * g - c * e) / det;
    t = (a * g - b * e) / det;
    if (s >= 0.0 && s <= 1.0 && t >= -L && t <= L) ORC_TAKE(s, t);
  }
  /* edges s = 0 and s = 1: minimise over t */
  t = clampd(g / c, -L, L);
  ORC_TAKE(0.0, t);
  t = clampd((g + b) / c, -L, L);
  ORC_TAKE(1.0, t);
  /* edges t = -L and t = +L: minimise over s */
  if (a > 0.0) {
    s = clampd(-(e + L * b) / a, 0.0, 1.0);
    ORC_TAKE(s, -L);
    s = clampd(-(e - L * b) / a, 0.0, 1.0);
    ORC_TAKE(s, L);
  }
#undef ORC_TAKE
  return best;
}

static void wire_of(const orc_geometry *g, int32_t w, double m[3], double u[3], double *L) {
  m[0] = g->mx[w]; m[1] = g->my[w]; m[2] = g->mz[w];
  u[0] = g->ux[w]; u[1] = g->uy[w]; u[2] = g->uz[w];
  *L = g->half_len[w];
}

int orc_doca2(const orc_geometry *g, const orc_field *f, const orc_params *p, const double seed[5],
              int32_t n_hits, const int32_t *wire_id, double *d2) {
  double x[3], T[3], Lam, xo[3];
  int32_t i, n;
  for (i = 0; i < n_hits; ++i) d2[i] = INFINITY;
  if (!orc_seed_state(p, seed, x, T, &Lam)) return 0;
  for (n = 0; n < p->n_steps; ++n) {
    xo[0] = x[0]; xo[1] = x[1]; xo[2] = x[2];
    orc_rkn_step(f, Lam, p->step_mm, x, T);
    for (i = 0; i < n_hits; ++i) {
      double m[3], u[3], L, v;
      wire_of(g, wire_id[i], m, u, &L);
      v = orc_seg_wire_dist2(xo, x, m, u, L);
      if (v < d2[i]) d2[i] = v;
    }
    if (turn_ended(p, x)) break;
  }
  return 1;
}

/* Radial extent of a chord: the largest radius is at an endpoint, the smallest
 * is the clamped foot of the perpendicular from the z axis in the xy plane.   */
static void chord_radial_range(const double p0[3], const double p1[3], double *rmin, double *rmax) {
  double dx = p1[0] - p0[0], dy = p1[1] - p0[1];
  double r0 = sqrt(p0[0] * p0[0] + p0[1] * p0[1]);
  double r1 = sqrt(p1[0] * p1[0] + p1[1] * p1[1]);
  double dd = dx * dx + dy * dy, s = 0.0, qx, qy;
  if (dd > 0.0) s = clampd(-(p0[0] * dx + p0[1] * dy) / dd, 0.0, 1.0);
  qx = p0[0] + s * dx;
  qy = p0[1] + s * dy;
  *rmax = r0 > r1 ? r0 : r1;
  *rmin = sqrt(qx * qx + qy * qy);
}

/* Eq. (1): E = sum over fired wires of min(d_L^2, d_R^2, lambda). Reading: with
 * D the DCA of the track to the wire and d the measured drift distance, the left
 * and right candidates give d_L,R = D -+ d, so min(d_L^2, d_R^2) = (D - d)^2.
 * Hits with (D - d)^2 < lambda are classified to the track (section 2.2).
 *
 * Band pruning (mode 1) is exact: a pair (chord, hit) can lower the hit's term
 * below lambda only if the chord passes within d + sqrt(lambda) of the wire, which
 * needs the chord's radial range to meet the layer's radial extent widened by
 * that distance; a 1 mm margin keeps the rounding of borderline terms identical. */
double orc_score(const orc_geometry *g, const orc_field *f, const orc_params *p, const double seed[5],
                 int32_t n_hits, const int32_t *wire_id, const float *drift, int32_t mode,
                 int32_t *n_in, int64_t *pairs) {
  double x[3], T[3], Lam, xo[3], E = 0.0;
  double *d2 = (double *)malloc(sizeof(double) * (n_hits > 0 ? n_hits : 1));
  double sl = sqrt(p->lambda_mm2);
  int64_t np = 0;
  int32_t i, n, cnt = 0;
  for (i = 0; i < n_hits; ++i) d2[i] = INFINITY;
  if (!orc_seed_state(p, seed, x, T, &Lam)) {
    free(d2);
    if (n_in) *n_in = 0;
    if (pairs) *pairs = 0;
    return INFINITY;
  }
  for (n = 0; n < p->n_steps; ++n) {
    double rmin = 0.0, rmax = 0.0;
    xo[0] = x[0]; xo[1] = x[1]; xo[2] = x[2];
    orc_rkn_step(f, Lam, p->step_mm, x, T);
    if (mode == 1) chord_radial_range(xo, x, &rmin, &rmax);
    for (i = 0; i < n_hits; ++i) {
      double m[3], u[3], L, v;
      int32_t w = wire_id[i];
      if (mode == 1) {
        int32_t l = g->layer_of[w];
        double dc = (double)drift[i] + sl + 1.0;
        if (rmax < g->layer_rmin[l] - dc || rmin > g->layer_rmax[l] + dc) continue;
      }
      wire_of(g, w, m, u, &L);
      v = orc_seg_wire_dist2(xo, x, m, u, L);
      ++np;
      if (v < d2[i]) d2[i] = v;
    }
    if (turn_ended(p, x)) break;
  }
  for (i = 0; i < n_hits; ++i) {
    double r = sqrt(d2[i]) - (double)drift[i];
    double t = r * r;
    if (t < p->lambda_mm2) {
      E += t;
      ++cnt;
    } else {
      E += p->lambda_mm2;
    }
  }
  free(d2);
  if (n_in) *n_in = cnt;
  if (pairs) *pairs = np;
  return E;
}

/* Seed grids: per dimension an inclusive linspace c - w + 2 w k / (n - 1)
 * (n = 1 gives c); flat index with theta slowest and pz fastest.             */
void orc_window_seed(const orc_window *w, int64_t flat, double seed[5]) {
  int64_t k[5];
  int d;
  for (d = 4; d >= 0; --d) {
    k[d] = flat % w->count[d];
    flat /= w->count[d];
  }
  for (d = 0; d < 5; ++d) {
    if (w->count[d] <= 1)
      seed[d] = w->center[d];
    else
      seed[d] = w->center[d] - w->half_width[d] +
                2.0 * w->half_width[d] * (double)k[d] / (double)(w->count[d] - 1);
  }
}

static int64_t window_size(const orc_window *w) {
  return (int64_t)w->count[0] * w->count[1] * w->count[2] * w->count[3] * w->count[4];
}

/* Section 2.2: the candidate seeds with the lowest E are kept. Reading: exact ties
 * go to the lowest global seed index.                                          */
int orc_scan_windows(const orc_geometry *g, const orc_field *f, const orc_params *p,
                     int32_t n_events, const int32_t *ev_off, const int32_t *wire_id, const float *drift,
                     int32_t n_windows, const orc_window *w, int32_t mode,
                     double *score, int32_t *n_in, int64_t *best_index, double *best_score,
                     int64_t *pairs_total) {
  int64_t *base = (int64_t *)malloc(sizeof(int64_t) * (n_windows + 1));
  int64_t total, s, ptot = 0;
  int32_t e, k;
  base[0] = 0;
  for (k = 0; k < n_windows; ++k) base[k + 1] = base[k] + window_size(&w[k]);
  total = base[n_windows];
  for (e = 0; e < n_events; ++e) {
    best_index[e] = -1;
    best_score[e] = INFINITY;
  }
#pragma omp parallel for schedule(static) reduction(+ : ptot)
  for (s = 0; s < total; ++s) {
    int32_t kw = 0, ev, ni = 0;
    int64_t np = 0;
    double seed[5], E;
    while (base[kw + 1] <= s) ++kw;
    ev = w[kw].event;
    orc_window_seed(&w[kw], s - base[kw], seed);
    E = orc_score(g, f, p, seed, ev_off[ev + 1] - ev_off[ev], wire_id + ev_off[ev], drift + ev_off[ev],
                  mode, &ni, &np);
    score[s] = E;
    if (n_in) n_in[s] = ni;
    ptot += np;
  }
  for (s = 0; s < total; ++s) {
    int32_t kw = 0, ev;
    while (base[kw + 1] <= s) ++kw;
    ev = w[kw].event;
    if (best_index[ev] < 0 || score[s] < best_score[ev]) {
      best_score[ev] = score[s];
      best_index[ev] = s;
    }
  }
  if (pairs_total) *pairs_total = ptot;
  free(base);
  return 0;
}

int orc_scan_seeds(const orc_geometry *g, const orc_field *f, const orc_params *p,
                   int32_t n_events, const int32_t *ev_off, const int32_t *wire_id, const float *drift,
                   int64_t n_seeds, const int32_t *seed_event, const double *theta, const double *z,
                   const double *px, const double *py, const double *pz, int32_t mode,
                   double *score, int32_t *n_in, int64_t *best_index, double *best_score,
                   int64_t *pairs_total) {
  int64_t s, ptot = 0;
  int32_t e;
  for (e = 0; e < n_events; ++e) {
    best_index[e] = -1;
    best_score[e] = INFINITY;
  }
#pragma omp parallel for schedule(static) reduction(+ : ptot)
  for (s = 0; s < n_seeds; ++s) {
    int32_t ev = seed_event[s], ni = 0;
    int64_t np = 0;
    double seed[5] = {theta[s], z[s], px[s], py[s], pz[s]};
    score[s] = orc_score(g, f, p, seed, ev_off[ev + 1] - ev_off[ev], wire_id + ev_off[ev],
                         drift + ev_off[ev], mode, &ni, &np);
    if (n_in) n_in[s] = ni;
    ptot += np;
  }
  if (pairs_total) *pairs_total = ptot;
  for (s = 0; s < n_seeds; ++s) {
    int32_t ev = seed_event[s];
    if (best_index[ev] < 0 || score[s] < best_score[ev]) {
      best_score[ev] = score[s];
      best_index[ev] = s;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Section 2.1: the transverse seed ranges come from a circle Hough transform of
 * the hits. Readings: each hit votes with its wire's waist (x, y) quantised to
 * 2^-8 mm (round half to even); the accumulator spans circle centres on an
 * n_xy x n_xy grid and radii in n_r bins; a hit votes in every centre cell at the
 * radius bin that contains its distance to the cell centre. All operands are
 * multiples of 2^-8 mm, so the squared distance is an exact integer in units of
 * 2^-16 mm^2 and the vote is exact.                                            */
static int hough_geometry_ok(const orc_hough_params *hp) {
  double wxy = 2.0 * hp->xy_half / hp->n_xy, wr = (hp->r_max - hp->r_min) / hp->n_r;
  double a = hp->xy_half * 256.0, b = wxy * 256.0, c = hp->r_min * 256.0, d = wr * 256.0;
  return hp->n_xy > 0 && hp->n_r > 0 && a == floor(a) && b == floor(b) && c == floor(c) &&
         d == floor(d) && hp->r_min >= 0.0 && hp->r_max > hp->r_min;
}

int orc_hough_accumulate(const orc_geometry *g, const orc_hough_params *hp, int32_t n_hits,
                         const int32_t *wire_id, uint32_t *acc) {
  int64_t nbins = (int64_t)hp->n_xy * hp->n_xy * hp->n_r;
  int64_t wxy_q = (int64_t)llround(2.0 * hp->xy_half / hp->n_xy * 256.0);
  int64_t half_q = (int64_t)llround(hp->xy_half * 256.0);
  int64_t rmin_q = (int64_t)llround(hp->r_min * 256.0);
  int64_t wr_q = (int64_t)llround((hp->r_max - hp->r_min) / hp->n_r * 256.0);
  int64_t *edge = (int64_t *)malloc(sizeof(int64_t) * (hp->n_r + 1));
  int32_t i, a, b, k;
  if (!hough_geometry_ok(hp)) {
    free(edge);
    return -1;
  }
  memset(acc, 0, sizeof(uint32_t) * nbins);
  for (k = 0; k <= hp->n_r; ++k) {
    int64_t rk = rmin_q + wr_q * k;
    edge[k] = rk * rk;
  }
  for (i = 0; i < n_hits; ++i) {
    int64_t X = (int64_t)nearbyint(g->mx[wire_id[i]] * 256.0);
    int64_t Y = (int64_t)nearbyint(g->my[wire_id[i]] * 256.0);
    for (a = 0; a < hp->n_xy; ++a) {
      /* centre of cell a, times 256: -xy_half + wxy (a + 1/2) */
      int64_t XC2 = -2 * half_q + wxy_q * (2 * a + 1);   /* twice the centre, exact */
      int64_t DX = 2 * X - XC2;                          /* twice the offset        */
      for (b = 0; b < hp->n_xy; ++b) {
        int64_t YC2 = -2 * half_q + wxy_q * (2 * b + 1);
        int64_t DY = 2 * Y - YC2;
        int64_t rho2x4 = DX * DX + DY * DY;              /* 4 * rho^2               */
        int32_t lo = 0, hi = hp->n_r;                    /* find edge[k] <= rho^2 < edge[k+1] */
        if (rho2x4 < 4 * edge[0] || rho2x4 >= 4 * edge[hp->n_r]) continue;
        while (hi - lo > 1) {
          int32_t mid = (lo + hi) / 2;
          if (4 * edge[mid] <= rho2x4)
            lo = mid;
          else
            hi = mid;
        }
        acc[((int64_t)a * hp->n_xy + b) * hp->n_r + lo] += 1u;
      }
    }
  }
  free(edge);
  return 0;
}

/* Readings (the paper gives none): threshold max(min_votes, ceil(max/2)); a bin is
 * a peak if it is at least every one of its 26 neighbours and strictly above the
 * neighbours with a smaller flat index (plateaus keep their first bin); peaks are
 * ordered by count (descending) then flat index (ascending).                   */
static int is_peak(const orc_hough_params *hp, const uint32_t *acc, int a, int b, int k) {
  int64_t me = ((int64_t)a * hp->n_xy + b) * hp->n_r + k;
  uint32_t c = acc[me];
  int da, db, dk;
  for (da = -1; da <= 1; ++da)
    for (db = -1; db <= 1; ++db)
      for (dk = -1; dk <= 1; ++dk) {
        int aa = a + da, bb = b + db, kk = k + dk;
        int64_t nb;
        if (!da && !db && !dk) continue;
        if (aa < 0 || bb < 0 || kk < 0 || aa >= hp->n_xy || bb >= hp->n_xy || kk >= hp->n_r) continue;
        nb = ((int64_t)aa * hp->n_xy + bb) * hp->n_r + kk;
        if (acc[nb] > c) return 0;
        if (acc[nb] == c && nb < me) return 0;
      }
  return 1;
}

typedef struct { uint32_t count; int64_t flat; } orc_peak;

static int peak_order(const void *pa, const void *pb) {
  const orc_peak *a = (const orc_peak *)pa, *b = (const orc_peak *)pb;
  if (a->count != b->count) return a->count > b->count ? -1 : 1;
  return a->flat < b->flat ? -1 : (a->flat > b->flat ? 1 : 0);
}

int orc_hough_peaks(const orc_hough_params *hp, const uint32_t *acc, int32_t max_out,
                    int64_t *peak_flat, uint32_t *peak_count) {
  int64_t nbins = (int64_t)hp->n_xy * hp->n_xy * hp->n_r, v, n = 0, cap = 64;
  orc_peak *list = (orc_peak *)malloc(sizeof(orc_peak) * cap);
  uint32_t mx = 0, thr;
  int32_t j, nout;
  for (v = 0; v < nbins; ++v)
    if (acc[v] > mx) mx = acc[v];
  thr = (mx + 1u) / 2u;                               /* ceil(max / 2) */
  if (thr < (uint32_t)hp->min_votes) thr = (uint32_t)hp->min_votes;
  if (thr < 1u) thr = 1u;
  for (v = 0; v < nbins; ++v) {
    int a, b, k;
    if (acc[v] < thr) continue;
    a = (int)(v / ((int64_t)hp->n_xy * hp->n_r));
    b = (int)((v / hp->n_r) % hp->n_xy);
    k = (int)(v % hp->n_r);
    if (!is_peak(hp, acc, a, b, k)) continue;
    if (n == cap) {
      cap *= 2;
      list = (orc_peak *)realloc(list, sizeof(orc_peak) * cap);
    }
    list[n].count = acc[v];
    list[n].flat = v;
    ++n;
  }
  qsort(list, (size_t)n, sizeof(orc_peak), peak_order);
  nout = n < max_out ? (int32_t)n : max_out;
  for (j = 0; j < nout; ++j) {
    peak_flat[j] = list[j].flat;
    peak_count[j] = list[j].count;
  }
  free(list);
  return nout;
}

/* Section 2.1 (Fig. 4): transverse seeds extracted from the found circle. The
 * circle (centre c, radius R) gives pT = kappa b_ref R; the seed point is the
 * circle's crossing of r = R0 where the particle moves outward (for q < 0 it
 * turns counter-clockwise seen from +z, velocity z^ x (P - c) / R). The window
 * width grows with the peak's half-maximum extent (readings, see the params). */
static int half_max_extent(const orc_hough_params *hp, const uint32_t *acc, int a, int b, int k,
                           int axis) {
  uint32_t c = acc[((int64_t)a * hp->n_xy + b) * hp->n_r + k];
  int n = 1, dir, lim = axis == 2 ? hp->n_r : hp->n_xy;
  for (dir = -1; dir <= 1; dir += 2) {
    int step;
    for (step = 1;; ++step) {
      int aa = a, bb = b, kk = k, pos;
      if (axis == 0) aa += dir * step;
      if (axis == 1) bb += dir * step;
      if (axis == 2) kk += dir * step;
      pos = axis == 0 ? aa : (axis == 1 ? bb : kk);
      if (pos < 0 || pos >= lim) break;
      if (2u * acc[((int64_t)aa * hp->n_xy + bb) * hp->n_r + kk] < c) break;
      ++n;
    }
  }
  return n;
}

int orc_hough_window(const orc_hough_params *hp, const uint32_t *acc, int64_t peak_flat,
                     orc_window *w) {
  int a = (int)(peak_flat / ((int64_t)hp->n_xy * hp->n_r));
  int b = (int)((peak_flat / hp->n_r) % hp->n_xy);
  int k = (int)(peak_flat % hp->n_r);
  double wxy = 2.0 * hp->xy_half / hp->n_xy, wr = (hp->r_max - hp->r_min) / hp->n_r;
  double xc = -hp->xy_half + wxy * (a + 0.5), yc = -hp->xy_half + wxy * (b + 0.5);
  double R = hp->r_min + wr * (k + 0.5);
  double d = sqrt(xc * xc + yc * yc), R0 = hp->R0;
  double pt = ORC_KAPPA * hp->b_ref * R;
  double al, h, cx, cy, P[2][2], best_dot = 0.0;
  int j, pick = -1, s, e1, e2, e3, d_;
  int64_t prod;
  if (!(d > 0.0) || d > R + R0 || d < fabs(R - R0)) return 0;
  al = (R0 * R0 - R * R + d * d) / (2.0 * d);
  h = R0 * R0 - al * al;
  h = h > 0.0 ? sqrt(h) : 0.0;
  cx = xc / d;
  cy = yc / d;
  P[0][0] = al * cx - h * cy; P[0][1] = al * cy + h * cx;
  P[1][0] = al * cx + h * cy; P[1][1] = al * cy - h * cx;
  for (j = 0; j < 2; ++j) {
    double vx = -(P[j][1] - yc) / R, vy = (P[j][0] - xc) / R;   /* z^ x (P - c) / R */
    double dot;
    if (hp->charge > 0.0) { vx = -vx; vy = -vy; }
    dot = vx * P[j][0] + vy * P[j][1];
    if (dot > best_dot) {
      best_dot = dot;
      pick = j;
      w->center[2] = pt * vx;
      w->center[3] = pt * vy;
    }
  }
  if (pick < 0) return 0;
  w->center[0] = atan2(P[pick][1], P[pick][0]);
  w->center[1] = hp->center_z;
  w->center[4] = hp->center_pz;
  e1 = half_max_extent(hp, acc, a, b, k, 0);
  e2 = half_max_extent(hp, acc, a, b, k, 1);
  e3 = half_max_extent(hp, acc, a, b, k, 2);
  s = e1 > e2 ? e1 : e2;
  if (e3 > s) s = e3;
  for (d_ = 0; d_ < 5; ++d_) {
    int n = hp->count[d_] + hp->grow[d_] * (s - 1);
    if (n > hp->count_max) n = hp->count_max;
    if (n < 1) n = 1;
    w->count[d_] = n;
  }
  for (;;) {
    int big = 0;
    prod = (int64_t)w->count[0] * w->count[1] * w->count[2] * w->count[3] * w->count[4];
    if (prod <= hp->max_seeds_window) break;
    for (d_ = 1; d_ < 5; ++d_)
      if (w->count[d_] > w->count[big]) big = d_;
    if (w->count[big] <= 1) break;
    w->count[big] -= 1;
  }
  for (d_ = 0; d_ < 5; ++d_) w->half_width[d_] = hp->gran[d_] * 0.5 * (double)(w->count[d_] - 1);
  w->pad = 0;
  return 1;
}

int orc_hough_seed_windows(const orc_geometry *g, const orc_hough_params *hp, int32_t n_events,
                           const int32_t *ev_off, const int32_t *wire_id, int32_t max_windows,
                           orc_window *out) {
  int64_t nbins = (int64_t)hp->n_xy * hp->n_xy * hp->n_r;
  uint32_t *acc = (uint32_t *)malloc(sizeof(uint32_t) * nbins);
  int64_t *pf = (int64_t *)malloc(sizeof(int64_t) * (hp->max_cand > 0 ? hp->max_cand : 1));
  uint32_t *pc = (uint32_t *)malloc(sizeof(uint32_t) * (hp->max_cand > 0 ? hp->max_cand : 1));
  int32_t e, n = 0;
  if (!hough_geometry_ok(hp)) {
    free(acc); free(pf); free(pc);
    return 0;
  }
  for (e = 0; e < n_events; ++e) {
    int32_t np, j, cand = 0;
    orc_hough_accumulate(g, hp, ev_off[e + 1] - ev_off[e], wire_id + ev_off[e], acc);
    np = orc_hough_peaks(hp, acc, hp->max_cand, pf, pc);
    for (j = 0; j < np; ++j) {
      orc_window w;
      memset(&w, 0, sizeof(w));
      if (!orc_hough_window(hp, acc, pf[j], &w)) continue;
      w.event = e;
      w.candidate = cand++;
      if (n < max_windows) out[n] = w;
      ++n;
    }
  }
  free(acc); free(pf); free(pc);
  return n <= max_windows ? n : -n;
}

/* ------------------------------------------------------------------------- */
/* Refinement (not in the paper, whose refinement is the rescan of finer grids in
 * section 2.2): Gauss-Newton on Phi(s) = sum over the inlier set S of (D_i - d_i)^2,
 * with S fixed by the classification rule (D - d)^2 < lambda at the starting seed.
 * Derivatives are those of the discrete map (differentiate the RKN steps as
 * computed). D_i is the minimum over chords; by the envelope theorem its gradient
 * is that of the minimising chord's distance at its minimising parameters:
 * dD/dx_n = (1 - s*) w and dD/dx_{n+1} = s* w, w the unit closest-approach vector.
 * FP64 forward sensitivities: Y_n = d(x_n, T_n, Lambda)/d(seed) (7 x 5) carried
 * through every stage of the step by the chain rule.                            */

/* Field and its Jacobian dB/dx (row c = component, column k = d/dx_k). */
static void field_jac(const orc_field *f, const double x[3], double B[3], double J[3][3]) {
  int c, k;
  for (c = 0; c < 3; ++c)
    for (k = 0; k < 3; ++k) J[c][k] = 0.0;
  if (f->kind == 0) {
    B[0] = 0.0; B[1] = 0.0; B[2] = f->bz;
    return;
  }
  {
    double r = sqrt(x[0] * x[0] + x[1] * x[1]);
    double dr = (f->r1 - f->r0) / (double)(f->nr - 1), dz = (f->z1 - f->z0) / (double)(f->nz - 1);
    double u = (r - f->r0) / dr, v = (x[2] - f->z0) / dz;
    int i = (int)floor(u), j = (int)floor(v), ui = 1, vi = 1;   /* ui/vi: inside (not clamped) */
    double a, b, q00r, q01r, q10r, q11r, q00z, q01z, q10z, q11z, br, bz, dbr_dr, dbr_dz, dbz_dr, dbz_dz;
    if (i < 0) i = 0;
    if (i > f->nr - 2) i = f->nr - 2;
    if (j < 0) j = 0;
    if (j > f->nz - 2) j = f->nz - 2;
    a = u - i;
    b = v - j;
    if (a < 0.0) { a = 0.0; ui = 0; }
    if (a > 1.0) { a = 1.0; ui = 0; }
    if (b < 0.0) { b = 0.0; vi = 0; }
    if (b > 1.0) { b = 1.0; vi = 0; }
    q00r = f->br[j * f->nr + i]; q01r = f->br[j * f->nr + i + 1];
    q10r = f->br[(j + 1) * f->nr + i]; q11r = f->br[(j + 1) * f->nr + i + 1];
    q00z = f->bzg[j * f->nr + i]; q01z = f->bzg[j * f->nr + i + 1];
    q10z = f->bzg[(j + 1) * f->nr + i]; q11z = f->bzg[(j + 1) * f->nr + i + 1];
    br = (1.0 - b) * ((1.0 - a) * q00r + a * q01r) + b * ((1.0 - a) * q10r + a * q11r);
    bz = (1.0 - b) * ((1.0 - a) * q00z + a * q01z) + b * ((1.0 - a) * q10z + a * q11z);
    dbr_dr = ui ? ((1.0 - b) * (q01r - q00r) + b * (q11r - q10r)) / dr : 0.0;
    dbz_dr = ui ? ((1.0 - b) * (q01z - q00z) + b * (q11z - q10z)) / dr : 0.0;
    dbr_dz = vi ? (((1.0 - a) * q10r + a * q11r) - ((1.0 - a) * q00r + a * q01r)) / dz : 0.0;
    dbz_dz = vi ? (((1.0 - a) * q10z + a * q11z) - ((1.0 - a) * q00z + a * q01z)) / dz : 0.0;
    B[2] = bz;
    if (r < 1e-9) {
      B[0] = 0.0; B[1] = 0.0;
      /* on the axis B_r = r dB_r/dr to first order: B_x = dbr_dr x, B_y = dbr_dr y */
      J[0][0] = dbr_dr; J[1][1] = dbr_dr;
      J[2][2] = dbz_dz;
    } else {
      double cx = x[0] / r, cy = x[1] / r;
      B[0] = br * cx;
      B[1] = br * cy;
      /* d(r)/dx = cx, dr/dy = cy; d(cx)/dx = (1 - cx^2)/r, d(cx)/dy = -cx cy / r, ... */
      J[0][0] = dbr_dr * cx * cx + br * (1.0 - cx * cx) / r;
      J[0][1] = dbr_dr * cx * cy - br * cx * cy / r;
      J[0][2] = dbr_dz * cx;
      J[1][0] = dbr_dr * cy * cx - br * cx * cy / r;
      J[1][1] = dbr_dr * cy * cy + br * (1.0 - cy * cy) / r;
      J[1][2] = dbr_dz * cy;
      J[2][0] = dbz_dr * cx;
      J[2][1] = dbz_dr * cy;
      J[2][2] = dbz_dz;
    }
  }
}

static void cross3(const double a[3], const double b[3], double o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

/* k = Lam T x B(xp) and its tangent for each of the 5 columns: dk = dLam T x B +
 * Lam dT x B + Lam T x (J dxp). */
static void stage_tan(const orc_field *f, double Lam, const double xp[3], const double T[3],
                      double dLam[5], double dxp[3][5], double dT[3][5], double k[3], double dk[3][5]) {
  double B[3], J[3][3], TB[3];
  int c, q;
  field_jac(f, xp, B, J);
  cross3(T, B, TB);
  for (c = 0; c < 3; ++c) k[c] = Lam * TB[c];
  for (q = 0; q < 5; ++q) {
    double dTq[3] = {dT[0][q], dT[1][q], dT[2][q]}, dB[3], t1[3], t2[3];
    for (c = 0; c < 3; ++c) dB[c] = J[c][0] * dxp[0][q] + J[c][1] * dxp[1][q] + J[c][2] * dxp[2][q];
    cross3(dTq, B, t1);
    cross3(T, dB, t2);
    for (c = 0; c < 3; ++c) dk[c][q] = dLam[q] * TB[c] + Lam * (t1[c] + t2[c]);
  }
}

/* One RKN step (the same arithmetic as orc_rkn_step) with the tangents Y of
 * (x, T) and the constant dLam carried along. */
static void rkn_step_tan(const orc_field *f, double Lam, double h, double x[3], double T[3], double Y[6][5],
                         double dLam[5]) {
  double k1[3], k2[3], k3[3], k4[3], xm[3], xe[3], Tt[3];
  double dk1[3][5], dk2[3][5], dk3[3][5], dk4[3][5], dxm[3][5], dxe[3][5], dTt[3][5], dx[3][5], dT[3][5];
  int c, q;
  for (c = 0; c < 3; ++c)
    for (q = 0; q < 5; ++q) {
      dx[c][q] = Y[c][q];
      dT[c][q] = Y[3 + c][q];
    }
  stage_tan(f, Lam, x, T, dLam, dx, dT, k1, dk1);
  for (c = 0; c < 3; ++c) {
    xm[c] = x[c] + 0.5 * h * T[c] + 0.125 * h * h * k1[c];
    Tt[c] = T[c] + 0.5 * h * k1[c];
    for (q = 0; q < 5; ++q) {
      dxm[c][q] = dx[c][q] + 0.5 * h * dT[c][q] + 0.125 * h * h * dk1[c][q];
      dTt[c][q] = dT[c][q] + 0.5 * h * dk1[c][q];
    }
  }
  stage_tan(f, Lam, xm, Tt, dLam, dxm, dTt, k2, dk2);
  for (c = 0; c < 3; ++c) {
    Tt[c] = T[c] + 0.5 * h * k2[c];
    for (q = 0; q < 5; ++q) dTt[c][q] = dT[c][q] + 0.5 * h * dk2[c][q];
  }
  stage_tan(f, Lam, xm, Tt, dLam, dxm, dTt, k3, dk3);
  for (c = 0; c < 3; ++c) {
    xe[c] = x[c] + h * T[c] + 0.5 * h * h * k3[c];
    Tt[c] = T[c] + h * k3[c];
    for (q = 0; q < 5; ++q) {
      dxe[c][q] = dx[c][q] + h * dT[c][q] + 0.5 * h * h * dk3[c][q];
      dTt[c][q] = dT[c][q] + h * dk3[c][q];
    }
  }
  stage_tan(f, Lam, xe, Tt, dLam, dxe, dTt, k4, dk4);
  for (c = 0; c < 3; ++c) {
    x[c] = x[c] + h * T[c] + (h * h / 6.0) * (k1[c] + k2[c] + k3[c]);
    T[c] = T[c] + (h / 6.0) * (k1[c] + 2.0 * k2[c] + 2.0 * k3[c] + k4[c]);
    for (q = 0; q < 5; ++q) {
      Y[c][q] = dx[c][q] + h * dT[c][q] + (h * h / 6.0) * (dk1[c][q] + dk2[c][q] + dk3[c][q]);
      Y[3 + c][q] = dT[c][q] + (h / 6.0) * (dk1[c][q] + 2.0 * dk2[c][q] + 2.0 * dk3[c][q] + dk4[c][q]);
    }
  }
}

/* Residuals r_i = D_i - d_i and their Jacobian J_i = dr_i/d(seed) for the hits
 * with mask[i] != 0 (others: r and J set to 0). Returns 0 if |p| is too small. */
int orc_residual_jacobian(const orc_geometry *g, const orc_field *f, const orc_params *p, const double seed[5],
                          int32_t n_hits, const int32_t *wire_id, const float *drift, const uint8_t *mask,
                          double *resid, double *jac /* [n_hits][5] */) {
  double x[3], T[3], Lam, xo[3], Y[6][5], Yo[6][5], dLam[5], pm;
  double *d2 = (double *)malloc(sizeof(double) * (n_hits > 0 ? n_hits : 1));
  int32_t i, n, c, q;
  for (i = 0; i < n_hits; ++i) {
    d2[i] = INFINITY;
    resid[i] = 0.0;
    for (q = 0; q < 5; ++q) jac[5 * i + q] = 0.0;
  }
  if (!orc_seed_state(p, seed, x, T, &Lam)) {
    free(d2);
    return 0;
  }
  pm = sqrt(seed[2] * seed[2] + seed[3] * seed[3] + seed[4] * seed[4]);
  /* Y0 = d(x0, T0)/d(theta, z0, px, py, pz); dLam/dp_j = -Lam T_j / |p| */
  for (c = 0; c < 6; ++c)
    for (q = 0; q < 5; ++q) Y[c][q] = 0.0;
  Y[0][0] = -p->R0 * sin(seed[0]);
  Y[1][0] = p->R0 * cos(seed[0]);
  Y[2][1] = 1.0;
  for (c = 0; c < 3; ++c)
    for (q = 0; q < 3; ++q) Y[3 + c][2 + q] = ((c == q ? 1.0 : 0.0) - T[c] * T[q]) / pm;
  dLam[0] = 0.0;
  dLam[1] = 0.0;
  for (q = 0; q < 3; ++q) dLam[2 + q] = -Lam * T[q] / pm;
  for (n = 0; n < p->n_steps; ++n) {
    xo[0] = x[0]; xo[1] = x[1]; xo[2] = x[2];
    memcpy(Yo, Y, sizeof(Y));
    rkn_step_tan(f, Lam, p->step_mm, x, T, Y, dLam);
    for (i = 0; i < n_hits; ++i) {
      double m[3], u[3], L, v, sb, tb;
      if (!mask[i]) continue;
      wire_of(g, wire_id[i], m, u, &L);
      v = seg_wire_best(xo, x, m, u, L, &sb, &tb);
      if (v < d2[i]) {
        double w[3], D = sqrt(v);
        d2[i] = v;
        for (c = 0; c < 3; ++c) w[c] = xo[c] + sb * (x[c] - xo[c]) - (m[c] + tb * u[c]);
        resid[i] = D - (double)drift[i];
        for (q = 0; q < 5; ++q) {
          double acc = 0.0;
          if (D > 0.0)
            for (c = 0; c < 3; ++c) acc += (w[c] / D) * ((1.0 - sb) * Yo[c][q] + sb * Y[c][q]);
          jac[5 * i + q] = acc;
        }
      }
    }
    if (turn_ended(p, x)) break;
  }
  free(d2);
  return 1;
}

/* Inlier mask at a seed: (D - d)^2 < lambda (brute-force D). */
int orc_inlier_mask(const orc_geometry *g, const orc_field *f, const orc_params *p, const double seed[5],
                    int32_t n_hits, const int32_t *wire_id, const float *drift, uint8_t *mask) {
  double *d2 = (double *)malloc(sizeof(double) * (n_hits > 0 ? n_hits : 1));
  int32_t i, ok = orc_doca2(g, f, p, seed, n_hits, wire_id, d2);
  for (i = 0; i < n_hits; ++i) {
    double r = sqrt(d2[i]) - (double)drift[i];
    mask[i] = (uint8_t)(ok && r * r < p->lambda_mm2);
  }
  free(d2);
  return ok;
}

static double phi_of(const double *resid, const uint8_t *mask, int32_t n) {
  double s = 0.0;
  int32_t i;
  for (i = 0; i < n; ++i)
    if (mask[i]) s += resid[i] * resid[i];
  return s;
}

/* Solve A x = b for a symmetric positive-definite 5x5 A (Cholesky); returns 0 if A
 * is not positive definite. */
static int chol5(const double A[5][5], const double b[5], double x[5]) {
  double Lm[5][5] = {{0}}, y[5];
  int i, j, k;
  for (i = 0; i < 5; ++i) {
    for (j = 0; j <= i; ++j) {
      double s = A[i][j];
      for (k = 0; k < j; ++k) s -= Lm[i][k] * Lm[j][k];
      if (i == j) {
        if (!(s > 0.0)) return 0;
        Lm[i][i] = sqrt(s);
      } else {
        Lm[i][j] = s / Lm[j][j];
      }
    }
  }
  for (i = 0; i < 5; ++i) {
    double s = b[i];
    for (k = 0; k < i; ++k) s -= Lm[i][k] * y[k];
    y[i] = s / Lm[i][i];
  }
  for (i = 4; i >= 0; --i) {
    double s = y[i];
    for (k = i + 1; k < 5; ++k) s -= Lm[k][i] * x[k];
    x[i] = s / Lm[i][i];
  }
  return 1;
}

/* Gauss-Newton refinement: the normal equations (J^T J) delta = -J^T r in the
 * scaled variables delta' = D delta, D = diag(scale), solved in FP64 by Cholesky
 * (with mu = 1e-12 trace added if not positive definite); a step is accepted at the
 * first of alpha = 1, 1/2, ..., 1/32 that lowers Phi, otherwise the seed stays.
 * Exactly `iters` iterations; phi receives Phi before each and after the last. */
int orc_gn_refine(const orc_geometry *g, const orc_field *f, const orc_params *p, int32_t n_hits,
                  const int32_t *wire_id, const float *drift, const double scale[5], int32_t iters,
                  double seed[5], uint8_t *mask, double *phi) {
  double *r = (double *)malloc(sizeof(double) * (n_hits > 0 ? n_hits : 1));
  double *J = (double *)malloc(sizeof(double) * 5 * (n_hits > 0 ? n_hits : 1));
  double *rt = (double *)malloc(sizeof(double) * (n_hits > 0 ? n_hits : 1));
  double *Jt = (double *)malloc(sizeof(double) * 5 * (n_hits > 0 ? n_hits : 1));
  int32_t it, i, a, b, k;
  double cur;
  orc_inlier_mask(g, f, p, seed, n_hits, wire_id, drift, mask);
  orc_residual_jacobian(g, f, p, seed, n_hits, wire_id, drift, mask, r, J);
  cur = phi_of(r, mask, n_hits);
  for (it = 0; it < iters; ++it) {
    double A[5][5] = {{0}}, rhs[5] = {0}, dlt[5], tr = 0.0;
    phi[it] = cur;
    for (i = 0; i < n_hits; ++i) {
      if (!mask[i]) continue;
      for (a = 0; a < 5; ++a) {
        rhs[a] -= J[5 * i + a] * scale[a] * r[i];
        for (b = 0; b < 5; ++b) A[a][b] += J[5 * i + a] * scale[a] * J[5 * i + b] * scale[b];
      }
    }
    for (a = 0; a < 5; ++a) tr += A[a][a];
    if (!chol5(A, rhs, dlt)) {
      for (a = 0; a < 5; ++a) A[a][a] += 1e-12 * tr;
      if (!chol5(A, rhs, dlt)) continue;
    }
    for (k = 0; k < 6; ++k) {
      double alpha = ldexp(1.0, -k), trial[5], ph;
      for (a = 0; a < 5; ++a) trial[a] = seed[a] + alpha * dlt[a] * scale[a];
      if (!orc_residual_jacobian(g, f, p, trial, n_hits, wire_id, drift, mask, rt, Jt)) continue;
      ph = phi_of(rt, mask, n_hits);
      if (ph < cur) {
        memcpy(seed, trial, sizeof(trial));
        memcpy(r, rt, sizeof(double) * n_hits);
        memcpy(J, Jt, sizeof(double) * 5 * n_hits);
        cur = ph;
        break;
      }
    }
  }
  phi[iters] = cur;
  free(r); free(J); free(rt); free(Jt);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Section 2.3: the seed of the neighbouring turn partition, predicted by
 * extrapolating the fitted track. Reading: the turn partitions of one track meet
 * r = R0 at their entrances and exits; from an entrance seed the next entrance is the
 * second crossing of r = R0 after the first step (exit, then re-entry), and the
 * previous one is the same along the time-reversed track (T and the charge, so
 * Lambda, reversed). The crossing inside the last step is located by bisection on
 * the length of a partial step from the state before it; the momentum keeps |p0|. */
static double radius_minus(const double x[3], double R0) { return sqrt(x[0] * x[0] + x[1] * x[1]) - R0; }

int orc_neighbour_seed(const orc_field *f, const orc_params *p, const double seed[5], int32_t dir,
                       int32_t max_steps, double out[5]) {
  double x[3], T[3], Lam, pm, xo[3], To[3];
  int32_t n, c, side = 0, changes = 0;
  if (!orc_seed_state(p, seed, x, T, &Lam)) return 0;
  pm = sqrt(seed[2] * seed[2] + seed[3] * seed[3] + seed[4] * seed[4]);
  if (dir < 0) {
    for (c = 0; c < 3; ++c) T[c] = -T[c];
    Lam = -Lam;
  }
  for (n = 0; n < max_steps; ++n) {
    int in;
    for (c = 0; c < 3; ++c) { xo[c] = x[c]; To[c] = T[c]; }
    orc_rkn_step(f, Lam, p->step_mm, x, T);
    in = radius_minus(x, p->R0) < 0.0;
    if (n == 0) {
      side = in;
      continue;
    }
    if (in == side) continue;
    side = in;
    if (++changes < 2) continue;
    {
      /* g(s) = r(state after a partial step s from (xo, To)) - R0 changes sign on
       * [0, h]; bisect it */
      double lo = 0.0, hi = p->step_mm, glo = radius_minus(xo, p->R0), xs[3], Ts[3];
      int it;
      for (it = 0; it < 80; ++it) {
        double mid = 0.5 * (lo + hi), g;
        for (c = 0; c < 3; ++c) { xs[c] = xo[c]; Ts[c] = To[c]; }
        orc_rkn_step(f, Lam, mid, xs, Ts);
        g = radius_minus(xs, p->R0);
        if ((g < 0.0) == (glo < 0.0)) {
          lo = mid;
          glo = g;
        } else {
          hi = mid;
        }
      }
      for (c = 0; c < 3; ++c) { xs[c] = xo[c]; Ts[c] = To[c]; }
      orc_rkn_step(f, Lam, 0.5 * (lo + hi), xs, Ts);
      out[0] = atan2(xs[1], xs[0]);
      out[1] = xs[2];
      for (c = 0; c < 3; ++c) out[2 + c] = (dir < 0 ? -pm : pm) * Ts[c];
      return 1;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Adaptive step size. Reading of the error-controlled RKN that section 2.2 cites:
 * the stages of one Nystrom step also give a local error estimate,
 * err = h^2 |k1 - k2 - k3 + k4| (the four stage accelerations agree to O(h^2) for a
 * smooth force, so err is O(h^4)). A trial step is accepted when err <= tol, or when
 * h is already the smallest step; the next step is h times 0.9 (tol/err)^(1/4),
 * clamped to [1/4, 4] and to [h_min, h_max] (a rejected trial retries with the same
 * rule, never growing), and the last step is cut to end the path exactly at length
 * L = n_steps * step_mm. The first trial uses h_max.                            */
void orc_rkn_trial(const orc_field *f, double Lam, double h, const double x[3], const double T[3],
                   double xn[3], double Tn[3], double *err) {
  double k1[3], k2[3], k3[3], k4[3], xm[3], xe[3], Tt[3], e2 = 0.0;
  int c;
  accel(f, Lam, x, T, k1);
  for (c = 0; c < 3; ++c) xm[c] = x[c] + 0.5 * h * T[c] + 0.125 * h * h * k1[c];
  for (c = 0; c < 3; ++c) Tt[c] = T[c] + 0.5 * h * k1[c];
  accel(f, Lam, xm, Tt, k2);
  for (c = 0; c < 3; ++c) Tt[c] = T[c] + 0.5 * h * k2[c];
  accel(f, Lam, xm, Tt, k3);
  for (c = 0; c < 3; ++c) xe[c] = x[c] + h * T[c] + 0.5 * h * h * k3[c];
  for (c = 0; c < 3; ++c) Tt[c] = T[c] + h * k3[c];
  accel(f, Lam, xe, Tt, k4);
  for (c = 0; c < 3; ++c) {
    double d = k1[c] - k2[c] - k3[c] + k4[c];
    xn[c] = x[c] + h * T[c] + (h * h / 6.0) * (k1[c] + k2[c] + k3[c]);
    Tn[c] = T[c] + (h / 6.0) * (k1[c] + 2.0 * k2[c] + 2.0 * k3[c] + k4[c]);
    e2 += d * d;
  }
  *err = h * h * sqrt(e2);
}

static double next_step(const orc_adaptive *a, double h, double err, int accepted) {
  double g = err > 0.0 ? 0.9 * pow(a->tol_mm / err, 0.25) : 4.0;
  if (g > 4.0) g = 4.0;
  if (g < 0.25) g = 0.25;
  if (!accepted && g > 1.0) g = 1.0;
  h *= g;
  if (h > a->h_max_mm) h = a->h_max_mm;
  if (h < a->h_min_mm) h = a->h_min_mm;
  return h;
}

int orc_adaptive_trace(const orc_field *f, const orc_params *p, const orc_adaptive *a, const double seed[5],
                       int32_t max_pts, double *pts, double *s, int32_t *n_rejected) {
  double x[3], T[3], Lam, L = p->n_steps * p->step_mm, arc = 0.0, h = a->h_max_mm;
  int32_t n = 0, rej = 0, c;
  if (n_rejected) *n_rejected = 0;
  if (max_pts < 1 || !orc_seed_state(p, seed, x, T, &Lam)) return 0;
  for (c = 0; c < 3; ++c) pts[c] = x[c];
  s[0] = 0.0;
  n = 1;
  while (arc < L && n < max_pts) {
    double xn[3], Tn[3], err, hs = h < L - arc ? h : L - arc;
    orc_rkn_trial(f, Lam, hs, x, T, xn, Tn, &err);
    if (err <= a->tol_mm || hs <= a->h_min_mm) {
      for (c = 0; c < 3; ++c) { x[c] = xn[c]; T[c] = Tn[c]; pts[3 * n + c] = x[c]; }
      arc += hs;
      s[n] = arc;
      ++n;
      if (hs == h) h = next_step(a, h, err, 1);   /* a cut last step does not set h */
      if (turn_ended(p, x)) break;
    } else {
      ++rej;
      h = next_step(a, hs, err, 0);
    }
  }
  if (n_rejected) *n_rejected = rej;
  return n;
}

double orc_score_adaptive(const orc_geometry *g, const orc_field *f, const orc_params *p, const orc_adaptive *a,
                          const double seed[5], int32_t n_hits, const int32_t *wire_id, const float *drift,
                          int32_t *n_in, int32_t *n_steps_taken) {
  int32_t cap = 4 * (int32_t)ceil(p->n_steps * p->step_mm / a->h_min_mm) + 8, n, i, j, cnt = 0;
  double *pts = (double *)malloc(sizeof(double) * 3 * cap), *s = (double *)malloc(sizeof(double) * cap);
  double E = 0.0;
  n = orc_adaptive_trace(f, p, a, seed, cap, pts, s, NULL);
  if (n_steps_taken) *n_steps_taken = n > 0 ? n - 1 : 0;
  if (n == 0) {
    free(pts); free(s);
    if (n_in) *n_in = 0;
    return INFINITY;
  }
  for (i = 0; i < n_hits; ++i) {
    double m[3], u[3], L, best = INFINITY, r;
    wire_of(g, wire_id[i], m, u, &L);
    for (j = 0; j + 1 < n; ++j) {
      double v = orc_seg_wire_dist2(pts + 3 * j, pts + 3 * (j + 1), m, u, L);
      if (v < best) best = v;
    }
    r = sqrt(best) - (double)drift[i];
    if (r * r < p->lambda_mm2) {
      E += r * r;
      ++cnt;
    } else {
      E += p->lambda_mm2;
    }
  }
  free(pts); free(s);
  if (n_in) *n_in = cnt;
  return E;
}

/* ------------------------------------------------------------------------- */
/* Section 2.2, the paper's refinement of a scan: the several seeds with the
 * lowest E are kept, finer seed sets are built around them and the scan is
 * repeated (ten times in the paper). Readings: a round builds, around each kept
 * seed in the order they were kept, a grid of `grid` points per dimension whose
 * half-width is the grid step the seed came from (a dimension whose step is 0 has
 * one point); every seed of the round's grids is scored (Eq. 1) and the k lowest
 * (E, then position in the round's window order) are kept, each with the step of
 * its own grid, 2 half-width / (grid - 1). An event stops after the round whose
 * lowest E is <= target[e] (never without a target), or after max_rounds. The
 * margin of an event is the smallest relative gap, over its rounds, between
 * consecutive E of the k + 1 lowest (pairs of one seed with one step excepted:
 * they tie exactly in any scorer) and between the lowest E and the target: a
 * scorer whose relative error stays below half of it makes every choice of the
 * loop the same.                                                               */
typedef struct {
  double s;
  int64_t i;
} scored_seed;

static int scored_order(const void *pa, const void *pb) {
  const scored_seed *a = (const scored_seed *)pa, *b = (const scored_seed *)pb;
  if (a->s < b->s) return -1;
  if (a->s > b->s) return 1;
  return a->i < b->i ? -1 : (a->i > b->i ? 1 : 0);
}

static double rel_gap(double a, double b) {
  double d = fabs(a - b), m = fabs(a) > fabs(b) ? fabs(a) : fabs(b);
  if (isinf(a) || isinf(b)) return a == b ? 0.0 : INFINITY;
  return m > 0.0 ? d / m : 0.0;
}

int orc_rescan_refine(const orc_geometry *g, const orc_field *f, const orc_params *p,
                      int32_t n_events, const int32_t *ev_off, const int32_t *wire_id, const float *drift,
                      int32_t k, int32_t grid, int32_t max_rounds, const double *start5, const double *step5,
                      const double *target, int32_t mode, double *out5, double *out_step5, double *out_score,
                      int32_t *rounds, double *margin) {
  int32_t e;
  if (k < 1 || grid < 2 || max_rounds < 0) return -1;
  for (e = 0; e < n_events; ++e) {
    double *cur = out5 + (size_t)e * k * 5, *stp = out_step5 + (size_t)e * k * 5;
    double *sc = out_score + (size_t)e * k;
    const int32_t nh = ev_off[e + 1] - ev_off[e];
    int32_t j, d, r;
    memcpy(cur, start5 + (size_t)e * k * 5, sizeof(double) * 5 * k);
    memcpy(stp, step5 + (size_t)e * k * 5, sizeof(double) * 5 * k);
    for (j = 0; j < k; ++j) sc[j] = NAN;
    rounds[e] = 0;
    if (margin) margin[e] = INFINITY;
    for (r = 0; r < max_rounds; ++r) {
      orc_window *w = (orc_window *)calloc((size_t)k, sizeof(orc_window));
      int64_t *base = (int64_t *)malloc(sizeof(int64_t) * (k + 1));
      int32_t nw = 0, q;
      int64_t total, s;
      scored_seed *all;
      for (j = 0; j < k; ++j) {
        int ok = 1;
        for (d = 0; d < 5; ++d) ok = ok && isfinite(cur[j * 5 + d]) && isfinite(stp[j * 5 + d]);
        if (!ok) continue;
        w[nw].event = e;
        w[nw].candidate = nw;
        for (d = 0; d < 5; ++d) {
          w[nw].center[d] = cur[j * 5 + d];
          w[nw].half_width[d] = stp[j * 5 + d];
          w[nw].count[d] = stp[j * 5 + d] > 0.0 ? grid : 1;
        }
        ++nw;
      }
      if (nw == 0) {
        free(w);
        free(base);
        break;
      }
      base[0] = 0;
      for (q = 0; q < nw; ++q) base[q + 1] = base[q] + window_size(&w[q]);
      total = base[nw];
      all = (scored_seed *)malloc(sizeof(scored_seed) * (size_t)total);
#pragma omp parallel for schedule(static)
      for (s = 0; s < total; ++s) {
        int32_t kw = 0;
        double seed[5];
        while (base[kw + 1] <= s) ++kw;
        orc_window_seed(&w[kw], s - base[kw], seed);
        all[s].s = orc_score(g, f, p, seed, nh, wire_id + ev_off[e], drift + ev_off[e], mode, NULL, NULL);
        all[s].i = s;
      }
      qsort(all, (size_t)total, sizeof(scored_seed), scored_order);
      for (j = 0; j < k; ++j) {
        if (j < total) {
          int32_t kw = 0;
          int64_t gi = all[j].i;
          while (base[kw + 1] <= gi) ++kw;
          orc_window_seed(&w[kw], gi - base[kw], cur + j * 5);
          for (d = 0; d < 5; ++d)
            stp[j * 5 + d] = w[kw].count[d] > 1 ? 2.0 * w[kw].half_width[d] / (double)(w[kw].count[d] - 1) : 0.0;
          sc[j] = all[j].s;
        } else {
          for (d = 0; d < 5; ++d) cur[j * 5 + d] = stp[j * 5 + d] = NAN;
          sc[j] = NAN;
        }
      }
      rounds[e] = r + 1;
      if (margin) {
        /* consecutive pairs of the k + 1 lowest: their order decides the kept set and
         * the next round's window order (equal seeds tie exactly in any scorer) */
        double mg = margin[e];
        for (j = 0; j < k && j + 1 < total; ++j) {
          double sa[5], sb[5];
          int32_t ka = 0, kb = 0;
          while (base[ka + 1] <= all[j].i) ++ka;
          while (base[kb + 1] <= all[j + 1].i) ++kb;
          orc_window_seed(&w[ka], all[j].i - base[ka], sa);
          orc_window_seed(&w[kb], all[j + 1].i - base[kb], sb);
          if (memcmp(sa, sb, sizeof(sa)) != 0 || memcmp(&w[ka].half_width, &w[kb].half_width, sizeof(sa)) != 0) {
            double gk = rel_gap(all[j + 1].s, all[j].s);
            if (gk < mg) mg = gk;
          }
        }
        if (target) {
          double gt = rel_gap(all[0].s, target[e]);
          if (gt < mg) mg = gt;
        }
        margin[e] = mg;
      }
      {
        const double best = all[0].s;
        free(all);
        free(w);
        free(base);
        if (target && best <= target[e]) break;
      }
    }
  }
  return 0;
}
