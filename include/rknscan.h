/* rknscan: exhaustive Runge-Kutta-Nystrom seed scan for drift-chamber track finding
 * on AMD Instinct MI355X (gfx950).
 *
 * Method: Yeo, Lee, Semertzidis, Kuno, "GPU Tracking in the COMET Phase-I
 * Cylindrical Drift Chamber" (CTD/WIT 2019). Every candidate seed
 * (theta0, z0, px0, py0, pz0) on the cylinder r = R0 is propagated with a fixed-step
 * RKN integrator of the Lorentz force (section 2.2), its distance of closest
 * approach (DCA) to every fired wire is compared with the measured drift distance,
 * and the seed is scored by E of Eq. (1); the lowest-E seed of each event is kept.
 * A circle Hough transform over the hit wires narrows the seed windows (section 2.1).
 *
 * Conventions (all entry points):
 *  - Units: mm, MeV/c, tesla, elementary charge (electrons: charge = -1).
 *  - Status: every call returns rkn_status; 0 is success. On error nothing is
 *    written to the outputs and rkn_last_error() describes the failure. All
 *    arguments are validated before any device work. No exception crosses the ABI.
 *  - Ownership: inputs are caller-owned and copied (uploads) or read during the
 *    call; outputs are caller-owned. The context owns every device copy, its stream
 *    (if it created one), work buffers and captured graphs.
 *  - Pointers: input arrays of upload calls are host pointers. Output arrays are
 *    host pointers unless rkn_scan_params.ptr_flags has RKN_PTR_DEVICE, in which
 *    case they are device pointers on the context's device and the call is
 *    stream-ordered (it returns without waiting). Host outputs make the call
 *    synchronous.
 *  - Threads: one context per host thread; calls on one context are serialised
 *    by the caller.
 */
#ifndef RKNSCAN_H
#define RKNSCAN_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rkn_status;
#define RKN_OK 0
#define RKN_E_ARG (-1)          /* invalid argument (NULL, size, NaN, out of range)   */
#define RKN_E_STATE (-2)        /* missing upload or wrong call order                   */
#define RKN_E_NOMEM (-3)        /* device allocation failed                             */
#define RKN_E_DEVICE (-4)       /* HIP runtime error (text from hipGetErrorString)      */
#define RKN_E_CAPACITY (-5)     /* output capacity too small; required size reported    */
#define RKN_E_UNSUPPORTED (-6)  /* valid but unsupported configuration                  */

#define RKN_PTR_DEVICE 1        /* rkn_scan_params.ptr_flags: outputs are device pointers */

#define RKN_MAX_HITS_PER_EVENT 512
#define RKN_MAX_LAYERS 64
#define RKN_TOPK_MAX 16            /* largest k of the top-k selections */

typedef struct rkn_ctx rkn_ctx;

/* Create a context on HIP device `device`. `hip_stream` is a hipStream_t to run on,
 * or NULL for a context-owned stream. */
rkn_status rkn_create(int32_t device, void *hip_stream, rkn_ctx **out);
/* Release every device resource of the context. NULL-safe. */
void rkn_destroy(rkn_ctx *ctx);
/* Text of the last error on this context; valid until the next call on it. */
const char *rkn_last_error(const rkn_ctx *ctx);
/* Wait for all work queued by the context. */
rkn_status rkn_synchronize(rkn_ctx *ctx);
/* Library version string. */
const char *rkn_version(void);

/* ---- Uploads (section 2.2: the field, hits and seeds are moved to GPU memory
 *      before the scan) ---------------------------------------------------------- */

/* Wire table: wire i is the segment m_i + t u_i, |t| <= half_len_i (u unit), in
 * layer layer_of[i] (0 <= layer_of < n_layers <= RKN_MAX_LAYERS). layer_rmin/rmax
 * bound the radial extent of each layer's wires and must be non-decreasing in the
 * layer index (RKN_E_UNSUPPORTED otherwise). Replaces any previous geometry and
 * invalidates uploaded hits. */
rkn_status rkn_upload_geometry(rkn_ctx *ctx, int32_t n_wires,
                               const double *mx, const double *my, const double *mz,
                               const double *ux, const double *uy, const double *uz,
                               const double *half_len, const int32_t *layer_of,
                               int32_t n_layers, const double *layer_rmin,
                               const double *layer_rmax);

/* Uniform solenoid field B = (0, 0, bz_tesla). Like every field upload, it drops a
 * planned batch (rkn_batch_launch then returns RKN_E_STATE until the batch is
 * planned again) and the refinement state of rkn_refine_setup, both of which were
 * built for the previous field. */
rkn_status rkn_upload_field_uniform(rkn_ctx *ctx, double bz_tesla);

/* Axisymmetric field map: B_r and B_z on nodes r_i = r0 + (r1-r0) i/(nr-1),
 * z_j = z0 + (z1-z0) j/(nz-1), arrays [nz][nr] row-major, FP32 tesla. Evaluated by
 * bilinear interpolation in (r, z), clamped to the edge outside the grid;
 * B_x = B_r x/r, B_y = B_r y/r (0 on the axis). nr, nz >= 2. Drops a planned
 * batch and the refinement state, as rkn_upload_field_uniform does. */
rkn_status rkn_upload_field_rz(rkn_ctx *ctx, int32_t nr, int32_t nz, double r0, double r1,
                               double z0, double z1, const float *br, const float *bz);

/* Hits of n_events events in CSR form: event e owns hits ev_off[e] .. ev_off[e+1]-1
 * (ev_off[0] = 0, non-decreasing, at most RKN_MAX_HITS_PER_EVENT per event);
 * wire_id indexes the uploaded wire table; drift_mm is the measured drift distance
 * (finite, >= 0). Requires the geometry. */
rkn_status rkn_upload_hits(rkn_ctx *ctx, int32_t n_events, const int32_t *ev_off,
                           const int32_t *wire_id, const float *drift_mm);

/* ---- Seed windows ------------------------------------------------------------------ */

/* A 5-D seed grid: per dimension d (theta [rad], z0 [mm], px, py, pz [MeV/c]) an
 * inclusive linspace center-hw .. center+hw of count[d] points (count 1 -> center).
 * Flat index: theta slowest, pz fastest. The global index of a seed is the sum of
 * the sizes of the preceding windows plus its flat index. Windows are grouped by
 * event in non-decreasing event order. */
typedef struct {
  int32_t event, candidate;
  double center[5], half_width[5];
  int32_t count[5];
  int32_t pad;
} rkn_window;

/* Circle Hough transform (section 2.1) and the window built from each peak.
 * Accumulator n_xy x n_xy centre cells over [-xy_half, xy_half]^2 and n_r radius
 * bins over [r_min, r_max); every hit votes with its wire's mid-point (x, y),
 * quantised to 2^-8 mm (half to even), in every centre cell at the radius bin
 * holding its distance to the cell centre. The vote is exact integer arithmetic;
 * xy_half, 2 xy_half/n_xy, r_min and (r_max-r_min)/n_r must be multiples of 2^-8 mm.
 * Peaks: counts >= max(min_votes, ceil(max/2)), >= all 26 neighbours and > the
 * neighbours with a smaller flat index; up to max_cand per event ordered by count
 * desc, then flat index asc. A peak (bin centre xc, yc, R) gives pT = kappa b_ref R
 * and the seed point where the circle crosses r = R0 moving outward (q < 0 turns
 * counter-clockwise seen from +z); peaks whose circle misses r = R0 are dropped.
 * Window: centre (theta0, center_z, px0, py0, center_pz); count[d] + grow[d] (s-1)
 * points capped at count_max, s = the largest half-maximum extent of the peak along
 * its three axes (in bins); while the product exceeds max_seeds_window (a cap per
 * window) the largest
 * count (lowest dimension on ties) is decremented; half width gran[d] (count-1)/2. */
typedef struct {
  int32_t n_xy, n_r;
  double xy_half, r_min, r_max;
  int32_t min_votes, max_cand;
  double R0, charge, b_ref;
  double gran[5];
  double center_z, center_pz;
  int32_t count[5];
  int32_t grow[5];
  int32_t count_max;
  int32_t pad;
  int64_t max_seeds_window;
} rkn_hough_params;

/* Run the Hough stage on every uploaded event; write up to max_windows windows to
 * the host array `out` ordered by (event, candidate) and their number to *n_out.
 * If more are needed, returns RKN_E_CAPACITY with *n_out = the required count. */
rkn_status rkn_hough_seed_windows(rkn_ctx *ctx, const rkn_hough_params *hp, int32_t max_windows,
                                  rkn_window *out, int32_t *n_out);

/* Accumulator of one event (uint32 [n_xy][n_xy][n_r], host or device per ptr_flags);
 * exposed so the integer vote can be checked bit for bit. */
rkn_status rkn_hough_accumulator(rkn_ctx *ctx, const rkn_hough_params *hp, int32_t event,
                                 int32_t ptr_flags, uint32_t *acc);

/* ---- The scan (section 2.2, Eq. 1) ------------------------------------------------- */

typedef struct {
  double R0;          /* seed cylinder radius, mm (the paper fixes 500)            */
  double charge;      /* particle charge, e                                        */
  double step_mm;     /* RKN step h > 0                                            */
  double lambda_mm2;  /* cutoff lambda >= 0 of Eq. (1)                             */
  int32_t n_steps;    /* fixed number of RKN steps per seed, >= 1                  */
  int32_t precision;  /* 32: FP32 propagation and distances, FP64 score; 64: FP64  */
  int32_t ptr_flags;  /* RKN_PTR_DEVICE: outputs are device pointers               */
  int32_t block_steps;/* 0 (= 8), 4, 6 or 8: RKN steps per cull/DCA block; with the  */
                      /* FP32 field map it also sets the workgroup (16/12/8 waves) */
  int32_t turn_stop;  /* 0: all n_steps run; 1: the track ends with its turn       */
                      /* partition (sections 2.3, 4.2): at the first step whose    */
                      /* end point lies inside r < R0, that step's chord the last  */
  int32_t reserved;   /* 0                                                         */
} rkn_scan_params;

/* Score every seed of the windows: E = sum over the event's hits of
 * min((D - d)^2, lambda), D = minimum over the chords of the n_steps RKN steps of
 * the exact chord/wire distance, d = drift (left/right ambiguity: min(d_L^2, d_R^2)
 * = (D - d)^2). n_in[s] = #{hits with (D - d)^2 < lambda} (the classification rule
 * of section 2.2). A seed with |p| < 1e-3 MeV/c scores +inf. score/n_in: arrays of
 * the total seed count, or NULL to skip. best_index/best_score: per uploaded event,
 * the lowest E and its global seed index (ties: lowest index; -1 / +inf when the
 * event has no seed). */
rkn_status rkn_scan_windows(rkn_ctx *ctx, const rkn_scan_params *p, int32_t n_windows,
                            const rkn_window *w, double *score, int32_t *n_in,
                            int64_t *best_index, double *best_score);

/* Allocation-free form of rkn_scan_windows, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that forbid it):
 * the same scan and outputs, which must be device pointers (p->ptr_flags has
 * RKN_PTR_DEVICE; best_index and best_score are required, score and n_in may be
 * NULL). Its work memory (device windows, seed tiles, argmin partials, tile counter,
 * running minima) is one 256 MiB array per GPU, held from the library's load until
 * the process ends and shared by every call on that GPU: calls on one context's
 * stream are ordered, calls that overlap on one GPU from other streams race. The
 * call allocates nothing. RKN_E_CAPACITY when the windows, their tiles and the
 * running minima of one workgroup do not fit the array; when the minima of a full
 * persistent grid do not fit, fewer workgroups run. */
rkn_status rkn_scan_windows_noalloc(rkn_ctx *ctx, const rkn_scan_params *p, int32_t n_windows,
                                    const rkn_window *w, double *score, int32_t *n_in,
                                    int64_t *best_index, double *best_score);

/* The work the scan of rkn_scan_windows does on these windows, counted by an
 * instrumented instance of the same kernel (the timed instances carry no counter):
 * counts[0] = seed-steps taken, counts[1] = sphere tests made by the cull (a wire's
 * line against the sphere around a block's middle point), counts[2] = chord/wire
 * distances evaluated (the DCA update of section 2.2). counts is a host array of 3.
 * Scores are computed but not returned. Fixed steps over the whole path only:
 * RKN_E_UNSUPPORTED with turn_stop. */
rkn_status rkn_scan_work_counts(rkn_ctx *ctx, const rkn_scan_params *p, int32_t n_windows,
                                const rkn_window *w, int64_t *counts);

/* The kernel shape a scan with these parameters uses on the current hits: RKN steps
 * per cull block and seeds per tile (= lanes per workgroup), after the default and
 * the LDS/occupancy fit are resolved (tiles of the batched path and of
 * rkn_scan_windows are built for it). Either output may be NULL. */
rkn_status rkn_scan_shape(rkn_ctx *ctx, const rkn_scan_params *p, int32_t *block_steps, int32_t *seeds_per_tile);

/* The scan of rkn_scan_windows followed by the choice of the k (1..RKN_TOPK_MAX)
 * lowest-score seeds of every event, on the device: the step of the coarse-to-fine
 * refinement that keeps the best seeds of a scan before finer seed sets are built
 * around them (section 2.2). Per event, ordered by (score, global seed index):
 * index [n_events][k] (global seed index as in rkn_scan_windows, -1 when the event
 * has fewer than k seeds), score [n_events][k] (+inf padding) and, unless NULL,
 * seeds5 [n_events][k][5] (the decoded seeds, NaN padding). NaN scores are never
 * chosen. Outputs follow p->ptr_flags; the per-seed scores stay on the device. */
rkn_status rkn_scan_windows_topk(rkn_ctx *ctx, const rkn_scan_params *p, int32_t n_windows,
                                 const rkn_window *w, int32_t k, int64_t *index, double *score,
                                 double *seeds5);

/* Adaptive step size: the error-controlled RKN of the propagator that section 2.2
 * cites, in place of the fixed step. A trial step of size h also gives the error
 * estimate err = h^2 |k1 - k2 - k3 + k4| from its four stage accelerations; it is
 * accepted when err <= tol_mm or h <= h_min_mm, and the next step is h times
 * 0.9 (tol/err)^(1/4) clamped to [1/4, 4] and to [h_min_mm, h_max_mm] (a rejected
 * trial retries shorter). The first trial is h_max_mm; the path has the length of
 * the fixed-step scan, n_steps * step_mm, its last step cut to end there. h_max_mm
 * bounds the chord's sagitta h^2 / 8R (0.006 mm at 4 mm and R = 350 mm). */
typedef struct {
  double tol_mm, h_min_mm, h_max_mm;
} rkn_adaptive_params;

/* rkn_scan_windows with the adaptive step size: the scores use the chords between
 * accepted positions. FP32 or FP64 propagation (p->precision); 4 trial steps per cull
 * block (p->block_steps is ignored); turn_stop is honoured. Outputs as
 * rkn_scan_windows. */
rkn_status rkn_scan_windows_adaptive(rkn_ctx *ctx, const rkn_scan_params *p, const rkn_adaptive_params *ap,
                                     int32_t n_windows, const rkn_window *w, double *score, int32_t *n_in,
                                     int64_t *best_index, double *best_score);

/* The same outputs as rkn_scan_windows, computed by the paper's two-kernel form of
 * the scan (section 4.2), kept as an experiment beside the fused kernel: a record
 * kernel stores every seed's position after each step in HBM (12 bytes per seed and
 * step, in chunks of at most 4 GiB), then a DCA kernel gives each hit of the seed's
 * event its own lane (one wave per seed) and finds its distance from the recorded
 * chords (blocks of 8 chords pruned by the fused kernel's reach test). Same FP32
 * state, step and chord/wire distance as the fused kernel; p->precision must be 32;
 * block_steps is ignored; turn_stop is honoured. Outputs follow p->ptr_flags; any
 * may be NULL. */
rkn_status rkn_scan_windows_two_kernel(rkn_ctx *ctx, const rkn_scan_params *p, int32_t n_windows,
                                       const rkn_window *w, double *score, int32_t *n_in, int64_t *best_index,
                                       double *best_score);

/* Same score for an explicit seed list (SoA, host arrays, FP64). best_index is the
 * position in the list. */
rkn_status rkn_scan_seeds(rkn_ctx *ctx, const rkn_scan_params *p, int64_t n_seeds,
                          const int32_t *seed_event, const double *theta, const double *z,
                          const double *px, const double *py, const double *pz,
                          double *score, int32_t *n_in, int64_t *best_index, double *best_score);

/* Propagated states: for each seed (host [n_seeds][5]) and each of the n_sel
 * non-decreasing step indices (0 = the seed state), write (x, y, z, Tx, Ty, Tz) to
 * states [n_seeds][n_sel][6] (FP64; the FP32 path is widened). */
rkn_status rkn_trace(rkn_ctx *ctx, const rkn_scan_params *p, int64_t n_seeds, const double *seeds5,
                     int32_t n_sel, const int32_t *step_idx, double *states);

/* ---- Batched scan of every uploaded event ---------------------------------------
 * The Hough stage, the expansion of its windows into seed tiles, one persistent
 * scan launch over all tiles (an atomic work queue of tiles of up to 64 seeds per
 * wave of the workgroup, 768 with the default shape, of one window each) and the
 * per-event argmin, captured once as HIP graphs on the
 * context's stream. Re-plan after uploading new hits or geometry. */

/* Validate the parameters, size every buffer for the worst case
 * (n_events x max_cand windows of at most min(max_seeds_window, count_max^5)
 * seeds) and capture the graphs. sp->ptr_flags chooses host or device outputs of
 * rkn_batch_launch. hp and sp must have the same charge and R0 (else RKN_E_ARG). */
rkn_status rkn_batch_plan(rkn_ctx *ctx, const rkn_hough_params *hp, const rkn_scan_params *sp);

/* Autotuner of the batched path: plans the batch with each block size of
 * {4, 6, 8} RKN steps (which with the FP32 field map also sets the workgroup to
 * 16, 12 or 8 waves, i.e. the seeds per tile), times the scan over the tiles of the
 * first sample_events events on the current hits (HIP events, best of reps), and
 * leaves the batch planned with the fastest, as rkn_batch_plan with that
 * block_steps would. chosen (may be NULL): that block size; ms[3] (may be NULL):
 * the sample times of 4, 6 and 8 (+inf where a shape does not fit). sp->block_steps
 * is ignored. */
rkn_status rkn_batch_autotune(rkn_ctx *ctx, const rkn_hough_params *hp, const rkn_scan_params *sp,
                              int32_t sample_events, int32_t reps, int32_t *chosen, float *ms);

/* rkn_batch_plan with the adaptive step size of rkn_scan_windows_adaptive (4 trial
 * steps per cull block; sp->block_steps ignored): later rkn_batch_launch calls replay
 * it, and rkn_batch_topk / rkn_batch_results read its scores. */
rkn_status rkn_batch_plan_adaptive(rkn_ctx *ctx, const rkn_hough_params *hp, const rkn_scan_params *sp,
                                   const rkn_adaptive_params *ap);

/* Replay the graphs on the current hits; best_index/best_score per event (global
 * seed index of the batch, -1/+inf for an event without windows) as in
 * rkn_scan_windows. Either may be NULL. */
rkn_status rkn_batch_launch(rkn_ctx *ctx, int64_t *best_index, double *best_score);

/* After a launch: the k (1..RKN_TOPK_MAX) lowest-score seeds of every event of the
 * batch, chosen on the device, with the same outputs and order as
 * rkn_scan_windows_topk (global seed indices of the batch). Outputs follow the
 * planned sp->ptr_flags. This is how the best seeds of a batch reach the
 * refinement below. */
rkn_status rkn_batch_topk(rkn_ctx *ctx, int32_t k, int64_t *index, double *score, double *seeds5);

/* After a launch (waits for it): number of windows and seeds of the batch, and the
 * HIP-event time of the Hough+expansion graph and of the scan graph, in ms. */
rkn_status rkn_batch_info(rkn_ctx *ctx, int32_t *n_windows, int64_t *n_seeds, float *ms_hough,
                          float *ms_scan);

/* After a launch: the windows (host, ordered by event), per-seed scores and n_in
 * (host, global seed order) and the per-event first seed index ev_seed_off
 * [n_events+1]. Any output may be NULL; RKN_E_CAPACITY if a capacity is short. */
rkn_status rkn_batch_results(rkn_ctx *ctx, int32_t max_windows, rkn_window *windows, int32_t *n_windows,
                             int64_t max_seeds, double *score, int32_t *n_in, int64_t *ev_seed_off);

/* ---- Coarse-to-fine rescans (section 2.2) --------------------------------------------
 * The paper's refinement of a scan: the seeds with the lowest E are kept, finer seed
 * sets are built around them and the scan is repeated (ten times in the paper). Per
 * event and round: around each kept seed, in the order they were kept, a grid of
 * `grid` points per dimension whose half-width is the grid step that seed came from
 * (one point in a dimension whose step is 0); every seed of the event's grids is
 * scored as by rkn_scan_windows (p: precision, steps, lambda, turn_stop); the k
 * lowest (E, then position in the round: grid order, theta slowest within a grid)
 * are kept, each with the step of its own grid, 2 half-width / (grid - 1). An event
 * stops after the round whose lowest E is <= target[e], or after max_rounds. Every
 * round runs on the context's stream with no host synchronisation in between: the
 * grids, the seed tiles and the selection are built on the device. */
typedef struct {
  int32_t k;           /* seeds kept per event, 1..RKN_TOPK_MAX                       */
  int32_t grid;        /* points per dimension of a round's grids, 2..16              */
  int32_t max_rounds;  /* rounds at most, 0..64                                       */
  int32_t reserved;    /* 0                                                           */
} rkn_rescan_params;

/* start5 / step5 [n_events][k][5]: the first kept seeds and the steps of the grids they
 * came from (a row with a non-finite value holds no seed); both NULL: the k lowest
 * seeds of the last rkn_batch_launch with the steps of their windows (RKN_E_STATE if
 * nothing was launched since the last upload). target [n_events] or NULL (every event
 * runs max_rounds rounds). Inputs and outputs are host or device pointers per
 * p->ptr_flags. Outputs (each may be NULL): out5 / out_step5 [n_events][k][5] and
 * out_score [n_events][k] (NaN rows: no seed; NaN scores for an event that ran no
 * round), rounds [n_events] (rounds run). A round scans up to n_events * k * grid^5
 * seeds (RKN_E_CAPACITY above 2^32); its per-seed scores stay in context-owned
 * device memory. RKN_E_UNSUPPORTED for a scan shape that does not fit the device. */
rkn_status rkn_rescan_refine(rkn_ctx *ctx, const rkn_scan_params *p, const rkn_rescan_params *rp,
                             const double *start5, const double *step5, const double *target,
                             double *out5, double *out_step5, double *out_score, int32_t *rounds);

/* ---- Hit classification and the two-direction quality count -----------------------
 * Section 2.2: a hit belongs to a seed's track when (D - d)^2 < lambda; the scan is
 * run independently from seed sets at the chamber entrance and at its exit, and a
 * track is kept when the number N_c of hits both directions classify to it reaches a
 * threshold (20 in the paper). The exit-side scan is the time-reversed track: seeds at
 * the exit crossing with reversed momentum, propagated with the opposite charge
 * (rkn_hough_seed_windows and the scans produce them when given that charge). FP32
 * propagation (p->precision is ignored); masks are [n][H] bytes (H = the largest hit
 * count of an uploaded event; per row the event's hits in upload order, 0 past them);
 * outputs follow p->ptr_flags. */

/* Per seed (any event order): mask [n][H] of the hits classified to its track (may
 * be NULL) and n_in [n] their count (may be NULL; not both). */
rkn_status rkn_classify_hits(rkn_ctx *ctx, const rkn_scan_params *p, int64_t n_seeds, const int32_t *seed_event,
                             const double *seeds5, uint8_t *mask, int32_t *n_in);

/* Per pair (event pair_event[i], entrance seed seeds_entry5[i] propagated with
 * p->charge, exit seed seeds_exit5[i] propagated with -p->charge): the two masks
 * (either may be NULL) and n_common [n] = the number of hits in both. */
rkn_status rkn_bidirectional_common(rkn_ctx *ctx, const rkn_scan_params *p, int64_t n_pairs,
                                    const int32_t *pair_event, const double *seeds_entry5,
                                    const double *seeds_exit5, uint8_t *mask_entry, uint8_t *mask_exit,
                                    int32_t *n_common);

/* ---- Turn partitions (section 2.3, full event reconstruction) ----------------------
 * A turn partition is one pass of a track through the chamber, from its entrance
 * (the outward crossing of r = R0) to the first step inside r < R0 (the turn_stop
 * rule of rkn_scan_params). The seed of the neighbouring partition is predicted by
 * extrapolating a fitted track, and the partitions of an event are found one after
 * the other, each removing the hits it classifies. */

/* Seeds of the neighbouring turn partitions of n_seeds entrance seeds ([n][5] host,
 * FP64): direction +1 the next partition (the track propagated forward through its
 * exit and the inner region to the next outward crossing of r = R0), -1 the previous
 * one (the same along the time-reversed track: direction and charge reversed). The
 * seed is taken at the second crossing of r = R0 after the first step, located by
 * bisection on a partial step's length, with |p| kept. FP64 propagation in the
 * uploaded field. out5 [n][5] (NaN where not found) and found [n] (1/0: reached
 * within max_steps), host or device per p->ptr_flags. */
rkn_status rkn_neighbour_seeds(rkn_ctx *ctx, const rkn_scan_params *p, int64_t n_seeds, const double *seeds5,
                               int32_t direction, int32_t max_steps, double *out5, int32_t *found);

#define RKN_TURNS_MAX 16

typedef struct {
  double half_width[5];       /* window half-widths around a predicted seed             */
  int32_t count[5];           /* its grid counts (at most 4e6 seeds)                    */
  int32_t gn_iters;           /* Gauss-Newton iterations per fit (0: no fits)           */
  double gn_scale[5];         /* Gauss-Newton variable scales (as rkn_gn_refine)        */
  double lambda_classify_mm2; /* the fine cutoff: second fit, choice and classification */
  double fine_half_width[2];  /* first partition: (z0, pz0) rescan half-widths          */
  int32_t fine_count[2];      /* and counts (1, 1: no rescan; at most 1e6 seeds)        */
  int32_t n_candidates;       /* first partition: lowest-E seeds fitted, 1..RKN_TOPK_MAX */
  int32_t min_hits;           /* the loop stops below this many unclassified hits, and  */
                              /* a partition must classify at least this many (10)     */
  int32_t max_turns;          /* partitions per event, 1..RKN_TURNS_MAX                  */
  int32_t max_extrap_steps;   /* step limit of each prediction                           */
} rkn_turn_params;

/* The reconstruction loop over every uploaded event; every scan, fit and
 * classification runs with turn_stop on and sp's other settings (sp->precision must
 * be 32). First partition: the Hough windows of all hits (hp), the n_candidates
 * lowest-E seeds of each event (cutoff sp->lambda_mm2); each is fitted by
 * Gauss-Newton (gn_iters, inlier set at sp's cutoff), unless fine_count is (1, 1)
 * rescanned over a (z0, pz0) grid of fine_count points within fine_half_width of its
 * fitted values with the rest kept (scored at lambda_classify), and fitted again
 * (inlier set at lambda_classify);
 * the event keeps the candidate with the lowest E at lambda_classify and classifies
 * the hits with (D - d)^2 < lambda_classify at it; they are removed. Then, on the side
 * before the earliest and after the latest partition found, the neighbouring
 * partition's seed is predicted from that partition's fitted seed
 * (rkn_neighbour_seeds), a window of count[] seeds with half_width[] around it is
 * scanned over the hits still unclassified (sp's cutoff), and its best seed is
 * fitted at both cutoffs and classifies hits likewise; both sides are classified on
 * the same hits and the side that classifies more keeps them first, the other keeps
 * those left (no hit gets two partitions). A partition is kept when it classifies at
 * least min_hits hits, else that side ends; an event ends when fewer
 * than min_hits hits remain unclassified, both sides have ended or it has max_turns
 * partitions. hp and sp must have the same charge and R0 (else RKN_E_ARG). Outputs
 * (host): hit_turn [total hits] = partition index in the order
 * found, -1 unclassified; n_turns [n_events]; and, unless NULL, per event and
 * partition ([n_events][max_turns]): turn_seed [..][5] the fitted seed, turn_center
 * [..][5] the centre of the window its candidate came from (a Hough window for the
 * first, the prediction otherwise), turn_pos the partition's place along the track
 * relative to the first found (..., -1, 0, +1, ...), turn_nhits the hits it
 * classified. The context's hits are replaced by the unclassified ones during the
 * call and restored at the end (a planned batch or refinement must be set up again). */
rkn_status rkn_find_turns(rkn_ctx *ctx, const rkn_hough_params *hp, const rkn_scan_params *sp,
                          const rkn_turn_params *tp, int32_t *hit_turn, int32_t *n_turns, double *turn_seed,
                          double *turn_center, int32_t *turn_pos, int32_t *turn_nhits);

/* ---- Differentiated refinement of seeds --------------------------------------------
 * The paper refines the best seeds by rescanning finer grids (section 2.2); this is
 * the derivative-based alternative. Per seed the objective is
 *   Phi = sum over the inlier set S of r_i^2,  r_i = D_i - d_i,
 * with S fixed by the classification rule (D - d)^2 < lambda at the seed given to
 * rkn_refine_setup. Derivatives are those of the discrete RKN map; D_i's gradient is
 * that of its minimising chord at the minimising parameters. Propagation is FP32
 * with a checkpoint of the full state every ckpt_every steps; the adjoint sweep
 * recomputes each segment from its checkpoint and accumulates in FP64. Seeds must be
 * grouped by event (non-decreasing seed_event); every array below is in that seed
 * order. Outputs follow p->ptr_flags (host or device pointers). */

/* Upload n_seeds seeds ([n][5] host, FP64) and fix their inlier sets. p->precision
 * must be 32; ckpt_every a multiple of 8 in [8, 4096], or 0 to let the checkpoint
 * tuner pick it: the adjoint sweep (with J^T J) is timed on these seeds for 32, 64,
 * 128 and 256 steps and the fastest is kept (rkn_refine_info reports it). */
rkn_status rkn_refine_setup(rkn_ctx *ctx, const rkn_scan_params *p, int64_t n_seeds, const int32_t *seed_event,
                            const double *seeds5, int32_t ckpt_every);

/* After rkn_refine_setup: the seed count, the checkpoint interval in use and, if it
 * was tuned, tune_ms[4] = the timed sweeps for 32, 64, 128, 256 steps (else zeros).
 * Any output may be NULL. */
rkn_status rkn_refine_info(rkn_ctx *ctx, int64_t *n_seeds, int32_t *ckpt_every, float *tune_ms);

/* Forward pass at seeds5 ([n][5]; NULL keeps the current seeds): resid [n][H]
 * (H = the largest hit count of an uploaded event; per row the event's hits in
 * upload order, NaN for hits outside the inlier set and for unused columns) and
 * phi [n]. An inlier hit that no step block approaches within its drift +
 * sqrt(lambda) + block_steps h / 2 + 0.05 mm (the pruning reach) gets +inf, and so
 * does phi. Records the checkpoints used by rkn_adjoint_bwd. Either output may be NULL. */
rkn_status rkn_residuals_fwd(rkn_ctx *ctx, const double *seeds5, float *resid, double *phi);

/* Adjoint of the last forward pass. d_resid [n][H]: upstream gradient dF/dr (entries
 * of non-inliers ignored), or NULL for F = Phi (dF/dr = 2 r). d_seed [n][5] =
 * dF/d(theta, z0, px, py, pz); JtJ [n][5][5] = J^T J and Jtr [n][5] = J^T r of the
 * inlier residuals (J^T r is grad(Phi)/2, defined for d_resid == NULL). Any output may
 * be NULL; JtJ adds the second-order sweep. */
rkn_status rkn_adjoint_bwd(rkn_ctx *ctx, const float *d_resid, double *d_seed, double *JtJ, double *Jtr);

/* Gauss-Newton from the setup seeds: iters iterations of the normal equations
 * (J^T J) delta = -J^T r solved in FP64 by Cholesky in the scaled variables
 * D delta (D = diag(scale[5]); 1e-12 trace added if not positive definite), a step
 * taken at the first alpha in 1, 1/2, ..., 1/32 that lowers Phi (else the seed
 * stays). seeds_out [n][5]; phi [n][iters+1] (Phi before each iteration and after
 * the last). */
rkn_status rkn_gn_refine(rkn_ctx *ctx, int32_t iters, const double *scale, double *seeds_out, double *phi);

#ifdef __cplusplus
}
#endif
#endif
