// Batched seed scan of every uploaded event: Hough windows -> seed tiles -> one
// persistent scan launch -> per-event argmin, captured once as HIP graphs and
// replayed per batch (section 2.1 seeding and section 2.2 scan, many events).
//
// Graph A: the Hough stage for all events and the expansion of its window slots
//          into the compact window list, the seed tiles (at most one workgroup's
//          worth of seeds of one window) and the per-event tile ranges, all on the
//          device.
// Graph B: the persistent scan over the tiles (atomic tile queue, tile count read
//          from device memory) and the per-event argmin.
// HIP events recorded between the two graph launches time each stage.
#include <algorithm>
#include <string>
#include <vector>

#include "internal.hpp"

namespace rkn {

// Single workgroup: per-event sizes, a serial exclusive scan over events, then
// every event writes its windows and tiles. Counts: [0] windows, [1] tiles.
__global__ void __launch_bounds__(256)
batch_expand_kernel(const WinSlot* __restrict__ slots, const int32_t* __restrict__ nsel, int n_events,
                    int32_t* __restrict__ ev_nw, int32_t* __restrict__ ev_nt, long long* __restrict__ ev_ns,
                    WindowDev* __restrict__ windows, Tile* __restrict__ tiles, int32_t* __restrict__ ev_tiles,
                    long long* __restrict__ ev_seed, int32_t* __restrict__ counts, int tile) {
  const int tid = threadIdx.x;
  for (int e = tid; e < n_events; e += 256) {
    int nw = 0, nt = 0;
    long long ns = 0;
    for (int j = 0; j < nsel[e]; ++j) {
      const WinSlot& s = slots[(size_t)e * kMaxCand + j];
      if (!s.valid) continue;
      long long size = 1;
      for (int q = 0; q < 5; ++q) size *= s.w.count[q];
      ++nw;
      nt += (int)((size + tile - 1) / tile);
      ns += size;
    }
    ev_nw[e] = nw;
    ev_nt[e] = nt;
    ev_ns[e] = ns;
  }
  __syncthreads();
  if (tid == 0) {
    int w = 0, t = 0;
    long long s = 0;
    for (int e = 0; e < n_events; ++e) {
      const int nw = ev_nw[e], nt = ev_nt[e];
      const long long ns = ev_ns[e];
      ev_nw[e] = w;
      ev_tiles[e] = t;
      ev_seed[e] = s;
      w += nw;
      t += nt;
      s += ns;
    }
    ev_tiles[n_events] = t;
    ev_seed[n_events] = s;
    counts[0] = w;
    counts[1] = t;
  }
  __syncthreads();
  for (int e = tid; e < n_events; e += 256) {
    int w = ev_nw[e], t = ev_tiles[e];
    long long g = ev_seed[e];
    for (int j = 0; j < nsel[e]; ++j) {
      const WinSlot& s = slots[(size_t)e * kMaxCand + j];
      if (!s.valid) continue;
      long long size = 1;
      for (int q = 0; q < 5; ++q) size *= s.w.count[q];
      windows[w] = s.w;
      for (long long st = 0; st < size; st += tile) {
        Tile tl;
        tl.window = w;
        tl.event = e;
        tl.n = (int32_t)(size - st < tile ? size - st : tile);
        tl.pad = 0;
        tl.start = st;
        tl.gbase = g + st;
        tiles[t++] = tl;
      }
      g += size;
      ++w;
    }
  }
}

}  // namespace rkn

using namespace rkn;

namespace {

rkn_status berr(rkn_ctx* c, hipError_t e, const char* where) {
  c->err = std::string(where) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? RKN_E_NOMEM : RKN_E_DEVICE;
}

void drop_graphs(rkn_ctx* c) {
  if (c->x_hough) (void)hipGraphExecDestroy(c->x_hough);
  if (c->x_scan) (void)hipGraphExecDestroy(c->x_scan);
  if (c->g_hough) (void)hipGraphDestroy(c->g_hough);
  if (c->g_scan) (void)hipGraphDestroy(c->g_scan);
  c->x_hough = c->x_scan = nullptr;
  c->g_hough = c->g_scan = nullptr;
  c->batch_ready = false;
  c->batch_launched = false;
}

// Addresses of the shared Hough buffers that the captured graph A refers to.
void hough_ptrs(const rkn_ctx* c, void* out[6]) {
  out[0] = c->hough_acc.p;
  out[1] = c->hough_max.p;
  out[2] = c->hough_cand_n.p;
  out[3] = c->hough_cand.p;
  out[4] = c->hough_slots.p;
  out[5] = c->hough_nsel.p;
}

}  // namespace

namespace rkn {

void batch_release(rkn_ctx* c) {
  drop_graphs(c);
  if (c->ev_t0) (void)hipEventDestroy(c->ev_t0);
  if (c->ev_t1) (void)hipEventDestroy(c->ev_t1);
  if (c->ev_t2) (void)hipEventDestroy(c->ev_t2);
  c->ev_t0 = c->ev_t1 = c->ev_t2 = nullptr;
  DevBuf* bufs[] = {&c->b_windows, &c->b_tiles, &c->b_ev_tiles, &c->b_counts, &c->b_ev_seed,
                    &c->b_score,   &c->b_nin,   &c->b_best_i,   &c->b_best_e, &c->b_ev_scratch,
                    &c->b_slab,    &c->b_parts, &c->b_counter};
  for (DevBuf* b : bufs) b->release();
}

}  // namespace rkn

extern "C" {

rkn_status rkn_batch_plan(rkn_ctx* c, const rkn_hough_params* hp, const rkn_scan_params* sp) {
  if (!c) return RKN_E_ARG;
  HoughDev h;
  rkn_status st = make_hough_dev(c, hp, h);
  if (st != RKN_OK) return st;
  if (!sp || sp->n_steps < 1 || !(sp->step_mm > 0) || !(sp->lambda_mm2 >= 0) || !(sp->R0 > 0) ||
      !std::isfinite(sp->charge) || sp->charge == 0 || (sp->precision != 32 && sp->precision != 64) ||
      (sp->block_steps != 0 && sp->block_steps != 4 && sp->block_steps != 6 && sp->block_steps != 8) ||
      (sp->ptr_flags & ~RKN_PTR_DEVICE) || (sp->turn_stop != 0 && sp->turn_stop != 1)) {
    c->err = "batch: invalid scan parameters";
    return RKN_E_ARG;
  }
  if (hp->charge != sp->charge || hp->R0 != sp->R0) {
    c->err = "batch: the Hough and scan parameters must have the same charge and R0";
    return RKN_E_ARG;
  }
  if (c->n_wires == 0 || c->field_kind < 0 || c->h_ev_off.empty()) {
    c->err = "batch: upload geometry, field and hits first";
    return RKN_E_STATE;
  }
  hipError_t e;
  if ((e = hipSetDevice(c->device)) != hipSuccess) return berr(c, e, "hipSetDevice");
  drop_graphs(c);
  const int ne = c->n_events;
  const long long per_window = std::min<long long>(h.max_seeds, (long long)h.count_max * h.count_max *
                                                                    h.count_max * h.count_max * h.count_max);
  const int64_t max_windows = (int64_t)ne * h.max_cand;
  c->batch_max_seeds = max_windows * per_window;
  c->batch_scan = *sp;
  c->batch_scan.block_steps = resolve_block_steps(c, &c->batch_scan);
  const int tile = scan_tile(c, &c->batch_scan);
  c->batch_max_tiles = max_windows * ((per_window + tile - 1) / tile);
  if (c->batch_max_tiles > (int64_t(1) << 31) || c->batch_max_seeds > (int64_t(1) << 40)) {
    c->err = "batch: capacity too large; lower max_seeds_window or max_cand";
    return RKN_E_CAPACITY;
  }
  c->batch_scan = *sp;
  c->batch_scan.block_steps = resolve_block_steps(c, &c->batch_scan);
  c->batch_hough = h;
  if ((e = ensure_hough_buffers(c, h)) != hipSuccess) return berr(c, e, "batch alloc");
  if ((e = c->b_windows.ensure(sizeof(WindowDev) * std::max<int64_t>(max_windows, 1))) != hipSuccess ||
      (e = c->b_tiles.ensure(sizeof(Tile) * std::max<int64_t>(c->batch_max_tiles, 1))) != hipSuccess ||
      (e = c->b_ev_tiles.ensure(sizeof(int32_t) * (ne + 1))) != hipSuccess ||
      (e = c->b_counts.ensure(64)) != hipSuccess ||
      (e = c->b_ev_seed.ensure(sizeof(long long) * (ne + 1))) != hipSuccess ||
      (e = c->b_ev_scratch.ensure((sizeof(int32_t) * 2 + sizeof(long long)) * std::max(ne, 1))) != hipSuccess ||
      (e = c->b_score.ensure(sizeof(double) * std::max<int64_t>(c->batch_max_seeds, 1))) != hipSuccess ||
      (e = c->b_nin.ensure(sizeof(int32_t) * std::max<int64_t>(c->batch_max_seeds, 1))) != hipSuccess ||
      (e = c->b_best_i.ensure(sizeof(int64_t) * ne)) != hipSuccess ||
      (e = c->b_best_e.ensure(sizeof(double) * ne)) != hipSuccess)
    return berr(c, e, "batch alloc");
  // size the scan's scratch before capture (no allocation inside a captured stream)
  e = launch_scan_dev(c, &c->batch_scan, c->batch_max_tiles, c->b_counts.as<int32_t>() + 1,
                      c->b_tiles.as<Tile>(), c->b_windows.as<WindowDev>(), c->b_score.as<double>(),
                      c->b_nin.as<int32_t>(), c->b_best_i.as<int64_t>(), c->b_best_e.as<double>(),
                      c->b_ev_tiles.as<int32_t>(), true);
  if (e == hipErrorInvalidConfiguration) {
    c->err = "batch: scan configuration does not fit the device";
    return RKN_E_UNSUPPORTED;
  }
  if (e != hipSuccess) return berr(c, e, "batch scan sizing");
  if (!c->ev_t0) {
    if ((e = hipEventCreate(&c->ev_t0)) != hipSuccess || (e = hipEventCreate(&c->ev_t1)) != hipSuccess ||
        (e = hipEventCreate(&c->ev_t2)) != hipSuccess)
      return berr(c, e, "batch events");
  }
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return berr(c, e, "batch sync");
  // graph A: Hough + expansion
  char* scratch = c->b_ev_scratch.as<char>();
  int32_t* ev_nw = reinterpret_cast<int32_t*>(scratch);
  int32_t* ev_nt = ev_nw + std::max(ne, 1);
  long long* ev_ns = reinterpret_cast<long long*>(ev_nt + std::max(ne, 1));
  if ((e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
    return berr(c, e, "batch capture");
  hipError_t eq = queue_hough_all(c, h);
  if (eq == hipSuccess) {
    hipLaunchKernelGGL(batch_expand_kernel, dim3(1), dim3(256), 0, c->stream, c->hough_slots.as<WinSlot>(),
                       c->hough_nsel.as<int32_t>(), ne, ev_nw, ev_nt, ev_ns, c->b_windows.as<WindowDev>(),
                       c->b_tiles.as<Tile>(), c->b_ev_tiles.as<int32_t>(), c->b_ev_seed.as<long long>(),
                       c->b_counts.as<int32_t>(), tile);
    eq = hipGetLastError();
  }
  e = hipStreamEndCapture(c->stream, &c->g_hough);
  if (eq != hipSuccess) return berr(c, eq, "batch capture (hough)");
  if (e != hipSuccess) return berr(c, e, "batch capture end");
  if ((e = hipGraphInstantiate(&c->x_hough, c->g_hough, nullptr, nullptr, 0)) != hipSuccess)
    return berr(c, e, "batch instantiate");
  // graph B: persistent scan + argmin
  if ((e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
    return berr(c, e, "batch capture");
  eq = launch_scan_dev(c, &c->batch_scan, c->batch_max_tiles, c->b_counts.as<int32_t>() + 1,
                       c->b_tiles.as<Tile>(), c->b_windows.as<WindowDev>(), c->b_score.as<double>(),
                       c->b_nin.as<int32_t>(), c->b_best_i.as<int64_t>(), c->b_best_e.as<double>(),
                       c->b_ev_tiles.as<int32_t>(), false);
  e = hipStreamEndCapture(c->stream, &c->g_scan);
  if (eq != hipSuccess) return berr(c, eq, "batch capture (scan)");
  if (e != hipSuccess) return berr(c, e, "batch capture end");
  if ((e = hipGraphInstantiate(&c->x_scan, c->g_scan, nullptr, nullptr, 0)) != hipSuccess)
    return berr(c, e, "batch instantiate");
  hough_ptrs(c, c->b_hough_ptrs);
  c->batch_ready = true;
  return RKN_OK;
}

rkn_status rkn_batch_plan_adaptive(rkn_ctx* c, const rkn_hough_params* hp, const rkn_scan_params* sp,
                                   const rkn_adaptive_params* ap) {
  if (!c) return RKN_E_ARG;
  if (!sp || !ap || !std::isfinite(ap->tol_mm) || !(ap->tol_mm > 0) ||
      !std::isfinite(ap->h_min_mm) || !(ap->h_min_mm > 0) || !std::isfinite(ap->h_max_mm) ||
      ap->h_max_mm < ap->h_min_mm || sp->n_steps * sp->step_mm / ap->h_min_mm > 1e7) {
    c->err = "batch adaptive: scan parameters, tol > 0, 0 < h_min <= h_max, path / h_min <= 1e7";
    return RKN_E_ARG;
  }
  rkn_scan_params q = *sp;
  q.block_steps = 4;
  // the step-size settings reach the scan's arguments, which the graph captures by value
  c->adapt = ap;
  const rkn_status st = rkn_batch_plan(c, hp, &q);
  c->adapt = nullptr;
  return st;
}

rkn_status rkn_batch_autotune(rkn_ctx* c, const rkn_hough_params* hp, const rkn_scan_params* sp,
                              int32_t sample_events, int32_t reps, int32_t* chosen, float* ms) {
  if (!c) return RKN_E_ARG;
  if (!sp || sample_events < 1 || reps < 1 || reps > 100) {
    c->err = "autotune: need scan parameters, sample_events >= 1 and reps in [1, 100]";
    return RKN_E_ARG;
  }
  const int cand[3] = {4, 6, 8};
  float best_ms = INFINITY;
  int best = 0;
  for (int i = 0; i < 3; ++i) {
    if (ms) ms[i] = INFINITY;
    rkn_scan_params q = *sp;
    q.block_steps = cand[i];
    rkn_status st = rkn_batch_plan(c, hp, &q);
    if (st == RKN_E_UNSUPPORTED) continue;
    if (st != RKN_OK) return st;
    hipError_t e;
    // graph A writes the tiles; the scan then runs over the first events' tiles only
    if ((e = hipGraphLaunch(c->x_hough, c->stream)) != hipSuccess) return berr(c, e, "autotune");
    const int k = std::min(sample_events, c->n_events);
    float t_min = INFINITY;
    for (int r = 0; r < reps; ++r) {
      if ((e = hipEventRecord(c->ev_t1, c->stream)) != hipSuccess) return berr(c, e, "autotune");
      e = launch_scan_dev(c, &c->batch_scan, c->batch_max_tiles, c->b_ev_tiles.as<int32_t>() + k,
                          c->b_tiles.as<Tile>(), c->b_windows.as<WindowDev>(), c->b_score.as<double>(),
                          c->b_nin.as<int32_t>(), c->b_best_i.as<int64_t>(), c->b_best_e.as<double>(),
                          c->b_ev_tiles.as<int32_t>(), false);
      if (e != hipSuccess) return berr(c, e, "autotune scan");
      if ((e = hipEventRecord(c->ev_t2, c->stream)) != hipSuccess || (e = hipEventSynchronize(c->ev_t2)) != hipSuccess)
        return berr(c, e, "autotune");
      float t = 0.0f;
      if ((e = hipEventElapsedTime(&t, c->ev_t1, c->ev_t2)) != hipSuccess) return berr(c, e, "autotune");
      t_min = std::min(t_min, t);
    }
    if (ms) ms[i] = t_min;
    if (t_min < best_ms) {
      best_ms = t_min;
      best = cand[i];
    }
  }
  if (best == 0) {
    c->err = "autotune: no block size fits the device";
    return RKN_E_UNSUPPORTED;
  }
  rkn_scan_params q = *sp;
  q.block_steps = best;
  if (chosen) *chosen = best;
  return rkn_batch_plan(c, hp, &q);
}

rkn_status rkn_batch_launch(rkn_ctx* c, int64_t* best_index, double* best_score) {
  if (!c) return RKN_E_ARG;
  if (!c->batch_ready) {
    c->err = "batch: call rkn_batch_plan first";
    return RKN_E_STATE;
  }
  // an eager Hough call with a larger accumulator since the plan moved a buffer that
  // the captured graph still points at (buffers only grow, so an unchanged address
  // is still large enough)
  void* now[6];
  hough_ptrs(c, now);
  for (int i = 0; i < 6; ++i)
    if (now[i] != c->b_hough_ptrs[i]) {
      drop_graphs(c);
      c->err = "batch: Hough buffers were reallocated since rkn_batch_plan; plan again";
      return RKN_E_STATE;
    }
  hipError_t e;
  if ((e = hipSetDevice(c->device)) != hipSuccess) return berr(c, e, "hipSetDevice");
  if ((e = hipEventRecord(c->ev_t0, c->stream)) != hipSuccess) return berr(c, e, "batch event");
  if ((e = hipGraphLaunch(c->x_hough, c->stream)) != hipSuccess) return berr(c, e, "batch launch");
  if ((e = hipEventRecord(c->ev_t1, c->stream)) != hipSuccess) return berr(c, e, "batch event");
  if ((e = hipGraphLaunch(c->x_scan, c->stream)) != hipSuccess) return berr(c, e, "batch launch");
  if ((e = hipEventRecord(c->ev_t2, c->stream)) != hipSuccess) return berr(c, e, "batch event");
  const bool dev = (c->batch_scan.ptr_flags & RKN_PTR_DEVICE) != 0;
  const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (best_index &&
      (e = hipMemcpyAsync(best_index, c->b_best_i.p, sizeof(int64_t) * c->n_events, kind, c->stream)) != hipSuccess)
    return berr(c, e, "batch copy");
  if (best_score &&
      (e = hipMemcpyAsync(best_score, c->b_best_e.p, sizeof(double) * c->n_events, kind, c->stream)) != hipSuccess)
    return berr(c, e, "batch copy");
  if (!dev && (e = hipStreamSynchronize(c->stream)) != hipSuccess) return berr(c, e, "batch sync");
  c->batch_launched = true;
  return RKN_OK;
}

rkn_status rkn_batch_topk(rkn_ctx* c, int32_t k, int64_t* index, double* score, double* seeds5) {
  if (!c) return RKN_E_ARG;
  if (!c->batch_ready || !c->batch_launched) {
    c->err = "batch: call rkn_batch_plan and rkn_batch_launch first";
    return RKN_E_STATE;
  }
  if (k < 1 || k > RKN_TOPK_MAX || !index || !score) {
    c->err = "batch topk: k in [1, 16] and index/score outputs";
    return RKN_E_ARG;
  }
  hipError_t e;
  if ((e = hipSetDevice(c->device)) != hipSuccess) return berr(c, e, "hipSetDevice");
  const bool dev = (c->batch_scan.ptr_flags & RKN_PTR_DEVICE) != 0;
  const size_t ne = (size_t)c->n_events;
  int64_t* d_idx = index;
  double* d_sc = score;
  double* d_seed = seeds5;
  if (!dev) {
    if ((e = c->sel_idx.ensure(sizeof(int64_t) * ne * k)) != hipSuccess ||
        (e = c->sel_sc.ensure(sizeof(double) * ne * k)) != hipSuccess ||
        (e = c->sel_seed.ensure(sizeof(double) * ne * k * 5)) != hipSuccess)
      return berr(c, e, "batch topk alloc");
    d_idx = c->sel_idx.as<int64_t>();
    d_sc = c->sel_sc.as<double>();
    d_seed = seeds5 ? c->sel_seed.as<double>() : nullptr;
  }
  // after the expansion, the first n_events entries of the scratch hold each event's
  // first window; counts[0] is the window total
  e = launch_topk(c, c->b_score.as<double>(), c->b_ev_seed.as<long long>(), c->b_windows.as<WindowDev>(),
                  c->b_ev_scratch.as<int32_t>(), c->n_events, c->b_counts.as<int32_t>(), k, d_idx, d_sc, d_seed);
  if (e != hipSuccess) return berr(c, e, "batch topk");
  if (!dev) {
    if ((e = hipMemcpyAsync(index, d_idx, sizeof(int64_t) * ne * k, hipMemcpyDeviceToHost, c->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(score, d_sc, sizeof(double) * ne * k, hipMemcpyDeviceToHost, c->stream)) != hipSuccess ||
        (seeds5 && (e = hipMemcpyAsync(seeds5, d_seed, sizeof(double) * ne * k * 5, hipMemcpyDeviceToHost,
                                       c->stream)) != hipSuccess) ||
        (e = hipStreamSynchronize(c->stream)) != hipSuccess)
      return berr(c, e, "batch topk copy");
  }
  return RKN_OK;
}

rkn_status rkn_batch_info(rkn_ctx* c, int32_t* n_windows, int64_t* n_seeds, float* ms_hough, float* ms_scan) {
  if (!c) return RKN_E_ARG;
  if (!c->batch_ready || !c->batch_launched) {
    c->err = "batch: nothing launched";
    return RKN_E_STATE;
  }
  hipError_t e;
  if ((e = hipSetDevice(c->device)) != hipSuccess) return berr(c, e, "hipSetDevice");
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return berr(c, e, "batch sync");
  int32_t counts[2] = {0, 0};
  long long total = 0;
  if ((e = hipMemcpy(counts, c->b_counts.p, sizeof(counts), hipMemcpyDeviceToHost)) != hipSuccess ||
      (e = hipMemcpy(&total, c->b_ev_seed.as<long long>() + c->n_events, sizeof(long long),
                     hipMemcpyDeviceToHost)) != hipSuccess)
    return berr(c, e, "batch info");
  if (n_windows) *n_windows = counts[0];
  if (n_seeds) *n_seeds = total;
  float t1 = 0.f, t2 = 0.f;
  if (ms_hough && (e = hipEventElapsedTime(&t1, c->ev_t0, c->ev_t1)) == hipSuccess) *ms_hough = t1;
  if (ms_scan && (e = hipEventElapsedTime(&t2, c->ev_t1, c->ev_t2)) == hipSuccess) *ms_scan = t2;
  return RKN_OK;
}

rkn_status rkn_batch_results(rkn_ctx* c, int32_t max_windows, rkn_window* windows, int32_t* n_windows,
                             int64_t max_seeds, double* score, int32_t* n_in, int64_t* ev_seed_off) {
  if (!c) return RKN_E_ARG;
  int32_t nw = 0;
  int64_t ns = 0;
  rkn_status st = rkn_batch_info(c, &nw, &ns, nullptr, nullptr);
  if (st != RKN_OK) return st;
  if (n_windows) *n_windows = nw;
  if ((windows && nw > max_windows) || ((score || n_in) && ns > max_seeds)) {
    c->err = "batch: output capacity too small";
    return RKN_E_CAPACITY;
  }
  hipError_t e = hipSuccess;
  if (windows && nw > 0) {
    std::vector<WindowDev> w(nw);
    e = hipMemcpy(w.data(), c->b_windows.p, sizeof(WindowDev) * nw, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return berr(c, e, "batch results");
    std::vector<int32_t> cand_of_event(c->n_events, 0);
    for (int i = 0; i < nw; ++i) {
      rkn_window& o = windows[i];
      o.event = w[i].event;
      o.candidate = cand_of_event[w[i].event]++;
      for (int q = 0; q < 5; ++q) {
        o.center[q] = w[i].center[q];
        o.half_width[q] = w[i].half_width[q];
        o.count[q] = w[i].count[q];
      }
      o.pad = 0;
    }
  }
  if (score && ns > 0 && (e = hipMemcpy(score, c->b_score.p, sizeof(double) * ns, hipMemcpyDeviceToHost)) != hipSuccess)
    return berr(c, e, "batch results");
  if (n_in && ns > 0 && (e = hipMemcpy(n_in, c->b_nin.p, sizeof(int32_t) * ns, hipMemcpyDeviceToHost)) != hipSuccess)
    return berr(c, e, "batch results");
  if (ev_seed_off &&
      (e = hipMemcpy(ev_seed_off, c->b_ev_seed.p, sizeof(int64_t) * (c->n_events + 1), hipMemcpyDeviceToHost)) != hipSuccess)
    return berr(c, e, "batch results");
  return RKN_OK;
}

}  // extern "C"
