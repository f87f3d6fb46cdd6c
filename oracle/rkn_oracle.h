/* FP64 CPU oracle of the exhaustive RKN seed scan -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct C: every function computes the definition it
 * cites, with no blocking or fusion. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may call it; the GPU library shares no code with it.
 *
 * Paper: Yeo, Lee, Semertzidis, Kuno, "GPU Tracking in the COMET Phase-I
 * Cylindrical Drift Chamber" (CTD/WIT 2019).
 *
 * Units: mm, MeV/c, tesla, elementary charge. Host pointers only.
 */
#ifndef RKN_ORACLE_H
#define RKN_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_KAPPA 0.299792458   /* (MeV/c) / (T mm e) */

typedef struct {
  int32_t n_wires;
  const double *mx, *my, *mz;        /* wire mid-point */
  const double *ux, *uy, *uz;        /* unit direction */
  const double *half_len;            /* wire = m +- half_len * u */
  const int32_t *layer_of;
  int32_t n_layers;
  const double *layer_rmin, *layer_rmax;   /* radial extent of each layer's wires */
} orc_geometry;

typedef struct {
  int32_t kind;                       /* 0 uniform B_z, 1 (r,z) grid */
  double bz;                          /* uniform value */
  int32_t nr, nz;
  double r0, r1, z0, z1;
  const float *br, *bzg;              /* [nz][nr] row-major */
} orc_field;

typedef struct {
  double R0, charge, step_mm, lambda_mm2;
  int32_t n_steps;
  int32_t turn_stop;                  /* 1: the track ends with the first step inside r < R0 */
} orc_params;

typedef struct {
  int32_t event, candidate;
  double center[5], half_width[5];
  int32_t count[5];
  int32_t pad;
} orc_window;

/* Section 2.2: the field the track is propagated through. */
void orc_field_eval(const orc_field *f, const double x[3], double B[3]);

/* Section 2.1: seed (theta0, z0, px0, py0, pz0) on r = R0 -> (x, T, Lambda).
 * Returns 0 (and leaves outputs untouched) when |p| < 1e-3 MeV/c. */
int orc_seed_state(const orc_params *p, const double seed[5], double x[3], double T[3], double *Lam);

/* Section 2.2 (RKN propagation): one Runge-Kutta-Nystrom step of x'' = Lam x' x B(x). */
void orc_rkn_step(const orc_field *f, double Lam, double h, double x[3], double T[3]);

/* States (x, T) after each of the n_sel step indices (0 = the seed state); with
 * turn_stop, a step index beyond the end of the turn partition gives the last state. */
int orc_trace(const orc_field *f, const orc_params *p, int64_t n_seeds, const double *seeds5,
              int32_t n_sel, const int32_t *step_idx, double *states /* [n][n_sel][6] */);

/* Section 2.2 (DCA): exact squared distance between segment [p0,p1] and wire m +- L u. */
double orc_seg_wire_dist2(const double p0[3], const double p1[3], const double m[3],
                          const double u[3], double L);

/* Per-hit squared DCA, minimum over all chords of the propagated track (brute force). */
int orc_doca2(const orc_geometry *g, const orc_field *f, const orc_params *p, const double seed[5],
              int32_t n_hits, const int32_t *wire_id, double *d2 /* [n_hits] */);

/* Eq. (1): E = sum_i min((D_i - d_i)^2, lambda); n_in = #{(D_i-d_i)^2 < lambda}.
 * mode 0: brute force over every (chord, hit); mode 1: radial-band pruned (exact).
 * pairs (optional) receives the number of (chord, hit) pairs evaluated. */
double orc_score(const orc_geometry *g, const orc_field *f, const orc_params *p, const double seed[5],
                 int32_t n_hits, const int32_t *wire_id, const float *drift, int32_t mode,
                 int32_t *n_in, int64_t *pairs);

/* Seed grid: flat index (theta slowest, pz fastest) -> seed. */
void orc_window_seed(const orc_window *w, int64_t flat, double seed[5]);

/* Scan every seed of every window; scores [sum of counts], best per event. */
int orc_scan_windows(const orc_geometry *g, const orc_field *f, const orc_params *p,
                     int32_t n_events, const int32_t *ev_off, const int32_t *wire_id, const float *drift,
                     int32_t n_windows, const orc_window *w, int32_t mode,
                     double *score, int32_t *n_in, int64_t *best_index, double *best_score,
                     int64_t *pairs_total);

/* Scan an explicit list of seeds (SoA). best_* are per event, indices into the list
 * (lowest E, ties to the lowest index). pairs_total (optional) receives the number
 * of (chord, hit) pairs evaluated over all seeds. */
int orc_scan_seeds(const orc_geometry *g, const orc_field *f, const orc_params *p,
                   int32_t n_events, const int32_t *ev_off, const int32_t *wire_id, const float *drift,
                   int64_t n_seeds, const int32_t *seed_event, const double *theta, const double *z,
                   const double *px, const double *py, const double *pz, int32_t mode,
                   double *score, int32_t *n_in, int64_t *best_index, double *best_score,
                   int64_t *pairs_total);

/* ---- Section 2.2: the coarse-to-fine rescans that refine a scan's best seeds ----
 * Per event, rounds of: a grid of `grid` points per dimension around each of the k
 * kept seeds (half-width = the step of the grid the seed came from; one point where
 * that step is 0), every seed scored (Eq. 1, `mode` as orc_score), the k lowest
 * (E, then position in the round) kept with their own grid step. start5/step5
 * [n_events][k][5] are the first kept seeds and steps (a row with a non-finite
 * value is no seed). Stops after the round whose lowest E <= target[e] (target may
 * be NULL) or after max_rounds. Outputs: out5/out_step5 [n_events][k][5] and
 * out_score [n_events][k] (NaN rows: no seed), rounds [n_events], margin
 * [n_events] (optional): the smallest relative gap between consecutive E of the
 * k + 1 lowest of a round (pairs of one seed with one step excepted) and between
 * the lowest E and the target. Returns 0, or -1 for k < 1, grid < 2, max_rounds < 0. */
int orc_rescan_refine(const orc_geometry *g, const orc_field *f, const orc_params *p,
                      int32_t n_events, const int32_t *ev_off, const int32_t *wire_id, const float *drift,
                      int32_t k, int32_t grid, int32_t max_rounds, const double *start5, const double *step5,
                      const double *target, int32_t mode, double *out5, double *out_step5, double *out_score,
                      int32_t *rounds, double *margin);

/* ---- Section 2.1: circle Hough transform over the wire (x, y) positions ---- */
typedef struct {
  int32_t n_xy, n_r;                  /* accumulator n_xy x n_xy x n_r */
  double xy_half, r_min, r_max;       /* centre range [-xy_half, xy_half]^2, radius [r_min, r_max) */
  int32_t min_votes, max_cand;        /* threshold = max(min_votes, ceil(max/2)); <= max_cand peaks */
  double R0, charge, b_ref;           /* seed radius, charge, field for pT = kappa b_ref R */
  double gran[5];                     /* grid step per seed dimension */
  double center_z, center_pz;         /* longitudinal window centres */
  int32_t count[5];                   /* base points per dimension */
  int32_t grow[5];                    /* extra points per unit of peak half-max extent - 1 */
  int32_t count_max;                  /* per-dimension cap */
  int32_t pad;
  int64_t max_seeds_window;           /* per-window cap on the product of counts */
} orc_hough_params;

/* Exact integer vote: accumulator [n_xy][n_xy][n_r] (uint32) for one event's hits. */
int orc_hough_accumulate(const orc_geometry *g, const orc_hough_params *hp, int32_t n_hits,
                         const int32_t *wire_id, uint32_t *acc);
/* Peaks: flat bin indices ordered by count desc then index asc; returns their number. */
int orc_hough_peaks(const orc_hough_params *hp, const uint32_t *acc, int32_t max_out,
                    int64_t *peak_flat, uint32_t *peak_count);
/* Candidate circle -> seed window; returns 0 if the circle misses r = R0. */
int orc_hough_window(const orc_hough_params *hp, const uint32_t *acc, int64_t peak_flat,
                     orc_window *w);
/* All events: windows ordered by (event, candidate). Returns the number written, or
 * -(required) when max_windows is too small. */
int orc_hough_seed_windows(const orc_geometry *g, const orc_hough_params *hp, int32_t n_events,
                           const int32_t *ev_off, const int32_t *wire_id, int32_t max_windows,
                           orc_window *out);

/* ---- Refinement (Gauss-Newton on the inlier residuals; FP64 forward sensitivities) ---- */
int orc_inlier_mask(const orc_geometry *g, const orc_field *f, const orc_params *p, const double seed[5],
                    int32_t n_hits, const int32_t *wire_id, const float *drift, uint8_t *mask);
int orc_residual_jacobian(const orc_geometry *g, const orc_field *f, const orc_params *p, const double seed[5],
                          int32_t n_hits, const int32_t *wire_id, const float *drift, const uint8_t *mask,
                          double *resid, double *jac /* [n_hits][5] */);
int orc_gn_refine(const orc_geometry *g, const orc_field *f, const orc_params *p, int32_t n_hits,
                  const int32_t *wire_id, const float *drift, const double scale[5], int32_t iters,
                  double seed[5], uint8_t *mask, double *phi /* [iters+1] */);

/* ---- Turn partitions (section 2.3) ---- */
/* Prediction of the neighbouring turn partition's seed by extrapolating a fitted
 * track: dir = +1 forward from the seed (through its exit and the inner region to the
 * next entrance), dir = -1 along the time-reversed track (momentum and charge
 * reversed) back to the previous entrance. The seed is taken where the track crosses
 * r = R0 for the second time after the first step. Returns 1 and out[5], or 0 if the
 * crossing is not reached within max_steps or |p| is too small. */
int orc_neighbour_seed(const orc_field *f, const orc_params *p, const double seed[5], int32_t dir,
                       int32_t max_steps, double out[5]);

/* ---- Adaptive step size (the error-controlled RKN of the propagator section 2.2 cites) ---- */
typedef struct {
  double tol_mm;        /* local error bound per step, mm                           */
  double h_min_mm;      /* smallest step (taken even when the bound is not met)     */
  double h_max_mm;      /* largest step (bounds the chord's sagitta)                */
} orc_adaptive;

/* One trial step of size h from (x, T): the RKN result (xn, Tn) and the error
 * estimate h^2 |k1 - k2 - k3 + k4|. */
void orc_rkn_trial(const orc_field *f, double Lam, double h, const double x[3], const double T[3],
                   double xn[3], double Tn[3], double *err);
/* Accepted positions along a path of length n_steps * step_mm (turn_stop honoured):
 * pts [n][3] (pts[0] = the seed point), s [n] their arc lengths; returns n (at most
 * max_pts; 0 if |p| is too small). n_rejected (optional) counts rejected trials. */
int orc_adaptive_trace(const orc_field *f, const orc_params *p, const orc_adaptive *a, const double seed[5],
                       int32_t max_pts, double *pts, double *s, int32_t *n_rejected);
/* Eq. (1) over the chords between consecutive accepted positions (brute force). */
double orc_score_adaptive(const orc_geometry *g, const orc_field *f, const orc_params *p, const orc_adaptive *a,
                          const double seed[5], int32_t n_hits, const int32_t *wire_id, const float *drift,
                          int32_t *n_in, int32_t *n_steps_taken);

#ifdef __cplusplus
}
#endif
#endif
