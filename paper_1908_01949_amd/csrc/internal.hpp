// Internal host-side declarations of librknscan (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/rknscan.h"
#include "device_math.hpp"

namespace rkn {

// Grow-only device buffer owned by the context.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t n) {
    if (n <= bytes && p) return hipSuccess;
    if (p) {
      (void)hipFree(p);
      p = nullptr;
      bytes = 0;
    }
    hipError_t e = hipMalloc(&p, n > 0 ? n : 16);
    if (e == hipSuccess) bytes = n > 0 ? n : 16;
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <typename T>
  T* as() const {
    return reinterpret_cast<T*>(p);
  }
};

// A tile is up to scan_tile() consecutive seeds of one window (never straddles
// events).
struct Tile {
  int32_t window;
  int32_t event;
  int32_t n;
  int32_t pad;
  int64_t start;   // local flat index of the first seed in the window
  int64_t gbase;   // global seed index of the first seed
};

struct ArgminPart {
  double e;
  int64_t idx;
};

// Device copy of a window: FP64 centres/half-widths and counts.
struct WindowDev {
  double center[5], half_width[5];
  int32_t count[5];
  int32_t event;
};

// Seed k of a window's implicit grid (theta slowest, pz fastest): per dimension
// centre - half_width + 2 half_width i / (count - 1), or the centre when count is 1.
__device__ __forceinline__ void window_seed(const WindowDev& W, int64_t k, double v[5]) {
  int64_t kd[5];
#pragma unroll
  for (int d = 4; d >= 0; --d) {
    const int64_t n = W.count[d];
    kd[d] = k % n;
    k /= n;
  }
#pragma unroll
  for (int d = 0; d < 5; ++d)
    v[d] = W.count[d] <= 1 ? W.center[d]
                           : W.center[d] - W.half_width[d] +
                                 2.0 * W.half_width[d] * (double)kd[d] / (double)(W.count[d] - 1);
}

constexpr int kMaxCand = 64;     // Hough candidates kept per event, upper bound
// Steps per block of the refinement's forward pass; its adjoint recompute folds the
// block-relative sums at the same steps.
constexpr int kRefineBlock = 8;

struct HoughDev {
  int n_xy, n_r;
  int half_q, wxy_q, rmin_q, wr_q;   // in 2^-8 mm
  int min_votes, max_cand;
  double R0, charge, b_ref, xy_half, r_min, wxy, wr;
  double gran[5];
  double center_z, center_pz;
  int count[5], grow[5];
  int count_max;
  long long max_seeds;
};

struct WinSlot {
  WindowDev w;
  int32_t valid;
  int32_t pad;
};

}  // namespace rkn

struct rkn_ctx {
  int device = 0;
  const rkn_adaptive_params* adapt = nullptr;   // set during an adaptive-step scan only
  unsigned long long* count_work = nullptr;     // device counters, set during rkn_scan_work_counts only
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  int n_cu = 0;
  int max_lds_block = 65536;         // bytes of LDS one workgroup may use

  // geometry
  int n_wires = 0, n_layers = 0;
  rkn::DevBuf wire32, wire64;        // HitRec-like rows [n_wires] (drift slot unused)
  rkn::DevBuf wire_layer;            // int32 [n_wires]
  rkn::DevBuf wire_wx, wire_wy;      // FP64 mid-point x, y [n_wires] (Hough votes)
  rkn::DevBuf layer_r;               // float2 (rmin, rmax) [n_layers]
  std::vector<double> h_layer_rmin, h_layer_rmax;
  std::vector<int32_t> h_layer_of;
  std::vector<double> h_wx, h_wy;    // waist (x, y) for host-side checks

  // field
  int field_kind = -1;               // 0 uniform, 1 rz
  double bz = 0.0;
  int nr = 0, nz = 0;
  double r0 = 0, r1 = 0, z0 = 0, z1 = 0;
  rkn::DevBuf field_nodes;           // float2 (B_r, B_z) [nz][nr]

  // hits (prepared: sorted by layer within each event)
  int n_events = 0;
  int64_t total_hits = 0;
  int max_hits_event = 0;
  std::vector<int32_t> h_ev_off;
  std::vector<int32_t> h_wire;    // host copies of the uploaded hits (upload order)
  std::vector<float> h_drift;
  rkn::DevBuf ev_off, hits32, hits64, layer_off, ev_maxdrift;
  rkn::DevBuf hits_wire;             // int32 wire id per hit, upload order
  rkn::DevBuf hits_orig;             // int32 original index within its event, per layer-ordered hit
  rkn::DevBuf hits_phi;              // float twisted azimuth psi of the wire centre, per layer-ordered hit
  rkn::DevBuf layer_ext;             // float2 [n_events][n_layers] (dphi/dz of the layer's wires, psi deviation)
  rkn::DevBuf hough_acc, hough_max, hough_cand_n, hough_cand, hough_slots, hough_nsel;

  // per-call work buffers
  rkn::DevBuf windows, tiles, ev_tiles, parts, counter, mscratch, out_score, out_nin, out_best_i,
      out_best_e, trace_buf, seeds_buf, perm_buf;
  rkn::DevBuf sel_seg, sel_win, sel_idx, sel_sc, sel_seed;   // per-event top-k selection
  rkn::DevBuf work_counts;                                   // rkn_scan_work_counts
  rkn::DevBuf cl_seeds, cl_perm, cl_tiles, cl_resid, cl_argmin, cl_phi, cl_mask, cl_count;   // classification
  std::vector<rkn::DevBuf> extra;

  // batched path (planned once, launched as captured graphs)
  bool batch_ready = false;
  bool batch_launched = false;       // results exist (set by rkn_batch_launch)
  rkn_scan_params batch_scan{};
  rkn::HoughDev batch_hough{};
  int64_t batch_max_tiles = 0, batch_max_seeds = 0;
  hipGraph_t g_hough = nullptr, g_scan = nullptr;
  hipGraphExec_t x_hough = nullptr, x_scan = nullptr;
  hipEvent_t ev_t0 = nullptr, ev_t1 = nullptr, ev_t2 = nullptr;
  rkn::DevBuf b_windows, b_tiles, b_ev_tiles, b_counts, b_ev_seed, b_score, b_nin, b_best_i, b_best_e,
      b_ev_scratch;
  // the scan's scratch of the captured graph is private to it; the Hough buffers are
  // shared with the eager Hough calls, so their addresses are recorded at capture and
  // checked before each replay
  rkn::DevBuf b_slab, b_parts, b_counter;
  void* b_hough_ptrs[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};

  // coarse-to-fine rescans (rescan.hip): kept seeds, per-round windows and scores
  rkn::DevBuf rs_cur, rs_step, rs_score, rs_rounds, rs_active, rs_target, rs_windows, rs_tiles, rs_ev_tiles,
      rs_ev_seed, rs_ev_win, rs_counts, rs_ev_scratch, rs_seed_score, rs_best_i, rs_best_e, rs_sel_idx, rs_sel_sc,
      rs_sel_seed, rs_sel_step, rs_parts, rs_counter, rs_slab;

  // refinement (refine.hip): seeds grouped by event, inlier sets fixed at setup
  bool r_ready = false;
  rkn_scan_params r_params{};
  int64_t r_n = 0, r_ntiles = 0, r_ntiles6 = 0;
  int r_ckpt = 64, r_nckpt = 0;
  float r_tune_ms[4] = {0, 0, 0, 0};   // adjoint sweep times of the checkpoint tuner
  rkn::DevBuf r_seeds, r_seeds0, r_trials, r_event, r_tiles, r_tiles6, r_ident, r_base6, r_mask, r_resid,
      r_argmin, r_resid6, r_argmin6, r_phi, r_phi6, r_phicur, r_tape, r_segbuf, r_list, r_grad, r_jtj, r_cgrad,
      r_slab, r_counter, r_tape6, r_segoff, r_segout, r_accept;

  rkn::DevBuf* refine_buffers_[28] = {&r_seeds,  &r_seeds0, &r_trials, &r_event,  &r_tiles,  &r_tiles6, &r_ident,
                                      &r_base6,  &r_mask,   &r_resid,  &r_argmin, &r_resid6, &r_argmin6, &r_phi,
                                      &r_phi6,   &r_phicur, &r_tape,   &r_segbuf, &r_list,   &r_grad,   &r_jtj,
                                      &r_cgrad,  &r_slab,   &r_counter, &r_tape6, &r_segoff, &r_segout, &r_accept};
  void refine_release() {
    for (rkn::DevBuf* b : refine_buffers_) b->release();
    r_ready = false;
  }

  bool set_err(const std::string& s) {
    err = s;
    return false;
  }
};

namespace rkn {

rkn::FieldDev field_dev(const rkn_ctx* c);

// Launchers (scan.hip). Return a HIP error code; arguments already validated.
hipError_t launch_prep_hits(rkn_ctx* c, const int32_t* d_wire_id, const float* d_drift);
hipError_t launch_scan(rkn_ctx* c, const rkn_scan_params* p, int64_t n_tiles, const Tile* d_tiles,
                       const WindowDev* d_windows, const double* d_seeds5, const int64_t* d_perm,
                       double* d_score, int32_t* d_nin, int64_t* d_best_i, double* d_best_e,
                       const int32_t* d_ev_tiles);
hipError_t launch_trace(rkn_ctx* c, const rkn_scan_params* p, int64_t n_seeds, const double* d_seeds,
                        int32_t n_sel, const int32_t* d_steps, double* d_states);

// Hough (hough.hip): validate parameters; queue the whole stage for every event
// (no host synchronisation, no allocation: capturable once buffers exist).
rkn_status make_hough_dev(rkn_ctx* c, const rkn_hough_params* p, HoughDev& h);
hipError_t ensure_hough_buffers(rkn_ctx* c, const HoughDev& h);
hipError_t queue_hough_all(rkn_ctx* c, const HoughDev& h);

// Refinement forward pass (scan kernel in its second mode) over explicit seeds.
hipError_t launch_refine_fwd(rkn_ctx* c, const rkn_scan_params* p, int64_t n_tiles, const Tile* d_tiles,
                             const double* d_seeds5, const int64_t* d_perm, const int64_t* d_base_of,
                             uint8_t* d_mask, int define_mask, float* d_resid, int32_t* d_argmin, double* d_phi,
                             float* d_tape, int ckpt, int n_ckpt, int64_t n_pos);

// Seeds per tile (= lanes per workgroup) of the scan configuration for p.
int scan_tile(const rkn_ctx* c, const rkn_scan_params* p);
// RKN steps per cull block after resolving the default (0).
int resolve_block_steps(const rkn_ctx* c, const rkn_scan_params* p);

// Release the batched path's graphs, events and buffers (batch.hip).
void batch_release(rkn_ctx* c);

// The k lowest-score seeds of each of n_seg events (select.hip): seeds of event e
// are d_score[d_seg_off[e] .. d_seg_off[e+1]) and come from windows
// d_win_off[e] .. (e + 1 < n_seg ? d_win_off[e+1] : *d_win_total), in order.
// d_seed / d_step (optional): each pick's seed and the grid step of its window.
hipError_t launch_topk(rkn_ctx* c, const double* d_score, const long long* d_seg_off, const WindowDev* d_windows,
                       const int32_t* d_win_off, int n_seg, const int32_t* d_win_total, int k, int64_t* d_idx,
                       double* d_sc, double* d_seed, double* d_step = nullptr);

// Scratch of one user of launch_scan_dev: argmin partials, tile counter, slab.
struct ScanScratch {
  DevBuf* parts;
  DevBuf* counter;
  DevBuf* slab;
};

// Scan launch whose tile count is read from device memory (no host synchronisation;
// capturable once the scratch is sized). The batched path uses its private scratch
// b_slab, b_parts, b_counter; other users pass their own.
hipError_t launch_scan_dev(rkn_ctx* c, const rkn_scan_params* p, int64_t max_tiles, const int32_t* d_n_tiles,
                           const Tile* d_tiles, const WindowDev* d_windows, double* d_score, int32_t* d_nin,
                           int64_t* d_best_i, double* d_best_e, const int32_t* d_ev_tiles, bool alloc_only,
                           const ScanScratch* scratch = nullptr);

// Scan whose work memory the caller provides (no allocation): argmin partials
// [>= n_tiles], the tile counter, and slab_bytes of slab memory for the running
// minima (the persistent grid is capped to the workgroup slabs that fit;
// hipErrorInvalidValue when not even one fits). Tiles and windows already on the
// device.
hipError_t launch_scan_raw(rkn_ctx* c, const rkn_scan_params* p, int64_t n_tiles, const Tile* d_tiles,
                           const WindowDev* d_windows, double* d_score, int32_t* d_nin, int64_t* d_best_i,
                           double* d_best_e, const int32_t* d_ev_tiles, ArgminPart* d_parts, int* d_counter,
                           void* d_slab, size_t slab_bytes);
// Slab bytes one scan workgroup needs for these parameters (block size resolved).
size_t scan_slab_bytes_per_workgroup(const rkn_ctx* c, const rkn_scan_params* p);

// Windows -> device windows, tiles and per-event tile offsets, validated (api.hip).
rkn_status prepare_scan_windows(rkn_ctx* c, const rkn_scan_params* p, int32_t n_windows, const rkn_window* w,
                                std::vector<WindowDev>& wins, std::vector<Tile>& tiles, std::vector<int32_t>& ev_tiles,
                                int64_t& total);

// Device address of the allocation-free scan's work array on `device`, looked up once
// per device (noalloc.hip); called by rkn_create with the device current.
hipError_t noalloc_init(int device);

// Release the rescan loop's buffers (rescan.hip).
void rescan_release(rkn_ctx* c);

// Scan parameters valid and geometry, field and hits uploaded (api.hip); sets the
// error text otherwise.
rkn_status validate_scan(rkn_ctx* c, const rkn_scan_params* p);

}  // namespace rkn
