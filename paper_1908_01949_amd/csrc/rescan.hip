// The paper's coarse-to-fine rescans on the device (section 2.2): the seeds with the
// lowest E are kept, finer grids are built around them and the scan is repeated.
//
// Per round, on the context's stream and with no host synchronisation:
//   rescan_expand_kernel  the grids of every still-running event (one window per kept
//                         seed, half-width = the step that seed came from), the seed
//                         tiles and the per-event window/tile/seed offsets;
//   launch_scan_dev       the persistent scan over those tiles (tile count read from
//                         device memory) with scores per seed;
//   launch_topk           the k lowest (E, index) per event, decoded with the step of
//                         each pick's own grid;
//   rescan_update_kernel  the picks become the kept seeds; the round count and the
//                         per-event stop (lowest E <= target).
// An event that stopped contributes no window to later rounds, so its seeds cost
// nothing there.
#include <math.h>

#include <algorithm>
#include <string>

#include "internal.hpp"

namespace rkn {

namespace {

__device__ __forceinline__ bool row_ok(const double* cur, const double* step) {
  bool ok = true;
#pragma unroll
  for (int d = 0; d < 5; ++d) ok = ok && isfinite(cur[d]) && isfinite(step[d]);
  return ok;
}

// One thread per event: the kept seeds and steps from the start rows, the target,
// scores NaN, no round run, running while the event has a seed.
__global__ void rescan_init_kernel(int ne, int k, const double* __restrict__ start5,
                                   const double* __restrict__ step5, const double* __restrict__ target,
                                   double* __restrict__ cur, double* __restrict__ step, double* __restrict__ score,
                                   int32_t* __restrict__ rounds, int32_t* __restrict__ active,
                                   double* __restrict__ tgt) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  bool any = false;
  for (int j = 0; j < k; ++j) {
    const size_t o = ((size_t)e * k + j) * 5;
    for (int d = 0; d < 5; ++d) {
      cur[o + d] = start5[o + d];
      step[o + d] = step5[o + d];
    }
    any = any || row_ok(cur + o, step + o);
    score[(size_t)e * k + j] = NAN;
  }
  rounds[e] = 0;
  active[e] = any ? 1 : 0;
  // no target: a lowest E is never <= -inf (scores are >= 0 or +inf)
  tgt[e] = target ? target[e] : -INFINITY;
}

__device__ __forceinline__ long long window_points(const double* step, int grid, int32_t count[5]) {
  long long size = 1;
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    count[d] = step[d] > 0.0 ? grid : 1;
    size *= count[d];
  }
  return size;
}

// Single workgroup: per-event window, tile and seed counts of the running events, a
// serial exclusive scan over events, then the windows and tiles. counts[0] = windows,
// counts[1] = tiles.
__global__ void __launch_bounds__(256)
rescan_expand_kernel(int ne, int k, int grid, int tile, const double* __restrict__ cur,
                     const double* __restrict__ step, const int32_t* __restrict__ active, int32_t* __restrict__ ev_nw,
                     int32_t* __restrict__ ev_nt, long long* __restrict__ ev_ns, WindowDev* __restrict__ windows,
                     Tile* __restrict__ tiles, int32_t* __restrict__ ev_win, int32_t* __restrict__ ev_tiles,
                     long long* __restrict__ ev_seed, int32_t* __restrict__ counts) {
  const int tid = threadIdx.x;
  for (int e = tid; e < ne; e += 256) {
    int nw = 0, nt = 0;
    long long ns = 0;
    if (active[e]) {
      for (int j = 0; j < k; ++j) {
        const size_t o = ((size_t)e * k + j) * 5;
        if (!row_ok(cur + o, step + o)) continue;
        int32_t cnt[5];
        const long long size = window_points(step + o, grid, cnt);
        ++nw;
        nt += (int)((size + tile - 1) / tile);
        ns += size;
      }
    }
    ev_nw[e] = nw;
    ev_nt[e] = nt;
    ev_ns[e] = ns;
  }
  __syncthreads();
  if (tid == 0) {
    int w = 0, t = 0;
    long long s = 0;
    for (int e = 0; e < ne; ++e) {
      const int nw = ev_nw[e], nt = ev_nt[e];
      const long long ns = ev_ns[e];
      ev_win[e] = w;
      ev_tiles[e] = t;
      ev_seed[e] = s;
      w += nw;
      t += nt;
      s += ns;
    }
    ev_win[ne] = w;
    ev_tiles[ne] = t;
    ev_seed[ne] = s;
    counts[0] = w;
    counts[1] = t;
  }
  __syncthreads();
  for (int e = tid; e < ne; e += 256) {
    if (!active[e]) continue;
    int w = ev_win[e], t = ev_tiles[e];
    long long g = ev_seed[e];
    for (int j = 0; j < k; ++j) {
      const size_t o = ((size_t)e * k + j) * 5;
      if (!row_ok(cur + o, step + o)) continue;
      WindowDev W;
      const long long size = window_points(step + o, grid, W.count);
      for (int d = 0; d < 5; ++d) {
        W.center[d] = cur[o + d];
        W.half_width[d] = step[o + d];
      }
      W.event = e;
      windows[w] = W;
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

// One thread per event: a running event takes the round's picks as its kept seeds
// (NaN rows and scores past the round's seed count), counts the round and stops
// when its lowest E reached the target.
__global__ void rescan_update_kernel(int ne, int k, const int64_t* __restrict__ sel_idx,
                                     const double* __restrict__ sel_sc, const double* __restrict__ sel_seed,
                                     const double* __restrict__ sel_step, const double* __restrict__ tgt,
                                     double* __restrict__ cur, double* __restrict__ step, double* __restrict__ score,
                                     int32_t* __restrict__ rounds, int32_t* __restrict__ active) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne || !active[e]) return;
  for (int j = 0; j < k; ++j) {
    const size_t r = (size_t)e * k + j, o = r * 5;
    const bool has = sel_idx[r] >= 0;
    for (int d = 0; d < 5; ++d) {
      cur[o + d] = has ? sel_seed[o + d] : NAN;
      step[o + d] = has ? sel_step[o + d] : NAN;
    }
    score[r] = has ? sel_sc[r] : NAN;
  }
  rounds[e] += 1;
  const size_t r0 = (size_t)e * k;
  if (sel_idx[r0] < 0 || sel_sc[r0] <= tgt[e]) active[e] = 0;
}

rkn_status rerr(rkn_ctx* c, hipError_t e, const char* where) {
  c->err = std::string(where) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? RKN_E_NOMEM : RKN_E_DEVICE;
}

rkn_status aerr(rkn_ctx* c, const char* s) {
  c->err = s;
  return RKN_E_ARG;
}

}  // namespace

void rescan_release(rkn_ctx* c) {
  DevBuf* bufs[] = {&c->rs_cur,       &c->rs_step,    &c->rs_score,    &c->rs_rounds,    &c->rs_active,
                    &c->rs_target,    &c->rs_windows, &c->rs_tiles,    &c->rs_ev_tiles,  &c->rs_ev_seed,
                    &c->rs_ev_win,    &c->rs_counts,  &c->rs_ev_scratch, &c->rs_seed_score, &c->rs_best_i,
                    &c->rs_best_e,    &c->rs_sel_idx, &c->rs_sel_sc,   &c->rs_sel_seed,  &c->rs_sel_step,
                    &c->rs_parts,     &c->rs_counter, &c->rs_slab};
  for (DevBuf* b : bufs) b->release();
}

}  // namespace rkn

using namespace rkn;

extern "C" {

rkn_status rkn_rescan_refine(rkn_ctx* c, const rkn_scan_params* p, const rkn_rescan_params* rp,
                             const double* start5, const double* step5, const double* target, double* out5,
                             double* out_step5, double* out_score, int32_t* rounds) {
  if (!c) return RKN_E_ARG;
  rkn_status st = validate_scan(c, p);
  if (st != RKN_OK) return st;
  if (!rp) return aerr(c, "rescan: params is NULL");
  if (rp->k < 1 || rp->k > RKN_TOPK_MAX || rp->grid < 2 || rp->grid > 16 || rp->max_rounds < 0 ||
      rp->max_rounds > 64 || rp->reserved != 0)
    return aerr(c, "rescan: k in [1, 16], grid in [2, 16], max_rounds in [0, 64], reserved 0");
  if ((start5 == nullptr) != (step5 == nullptr)) return aerr(c, "rescan: start5 and step5 are both given or both NULL");
  const bool from_batch = start5 == nullptr;
  if (from_batch && !(c->batch_ready && c->batch_launched)) {
    c->err = "rescan: no batch launched to start from; pass start5 and step5";
    return RKN_E_STATE;
  }
  const int ne = c->n_events, k = rp->k, G = rp->grid;
  rkn_scan_params q = *p;
  q.block_steps = resolve_block_steps(c, &q);
  const int tile = scan_tile(c, &q);
  const long long per_window = (long long)G * G * G * G * G;
  const long long max_seeds = (long long)ne * k * per_window;
  const long long max_tiles = (long long)ne * k * ((per_window + tile - 1) / tile);
  if (max_seeds > (1LL << 32) || max_tiles > (1LL << 31)) {
    c->err = "rescan: a round could scan more than 2^32 seeds; lower k or grid";
    return RKN_E_CAPACITY;
  }
  const bool dev = (p->ptr_flags & RKN_PTR_DEVICE) != 0;
  const size_t nk = (size_t)ne * k;
  hipError_t e;
  if ((e = hipSetDevice(c->device)) != hipSuccess) return rerr(c, e, "hipSetDevice");
  if ((e = c->rs_cur.ensure(sizeof(double) * nk * 5)) != hipSuccess ||
      (e = c->rs_step.ensure(sizeof(double) * nk * 5)) != hipSuccess ||
      (e = c->rs_score.ensure(sizeof(double) * nk)) != hipSuccess ||
      (e = c->rs_rounds.ensure(sizeof(int32_t) * ne)) != hipSuccess ||
      (e = c->rs_active.ensure(sizeof(int32_t) * ne)) != hipSuccess ||
      (e = c->rs_target.ensure(sizeof(double) * ne)) != hipSuccess ||
      (e = c->rs_windows.ensure(sizeof(WindowDev) * nk)) != hipSuccess ||
      (e = c->rs_tiles.ensure(sizeof(Tile) * (size_t)std::max<long long>(max_tiles, 1))) != hipSuccess ||
      (e = c->rs_ev_tiles.ensure(sizeof(int32_t) * (ne + 1))) != hipSuccess ||
      (e = c->rs_ev_win.ensure(sizeof(int32_t) * (ne + 1))) != hipSuccess ||
      (e = c->rs_ev_seed.ensure(sizeof(long long) * (ne + 1))) != hipSuccess ||
      (e = c->rs_counts.ensure(64)) != hipSuccess ||
      (e = c->rs_ev_scratch.ensure((sizeof(int32_t) * 2 + sizeof(long long)) * ne)) != hipSuccess ||
      (e = c->rs_seed_score.ensure(sizeof(double) * (size_t)std::max<long long>(max_seeds, 1))) != hipSuccess ||
      (e = c->rs_best_i.ensure(sizeof(int64_t) * ne)) != hipSuccess ||
      (e = c->rs_best_e.ensure(sizeof(double) * ne)) != hipSuccess ||
      (e = c->rs_sel_idx.ensure(sizeof(int64_t) * nk)) != hipSuccess ||
      (e = c->rs_sel_sc.ensure(sizeof(double) * nk)) != hipSuccess ||
      (e = c->rs_sel_seed.ensure(sizeof(double) * nk * 5)) != hipSuccess ||
      (e = c->rs_sel_step.ensure(sizeof(double) * nk * 5)) != hipSuccess)
    return rerr(c, e, "rescan alloc");
  const ScanScratch scratch{&c->rs_parts, &c->rs_counter, &c->rs_slab};
  // size the scan's scratch before the first round (the launches then allocate nothing)
  e = launch_scan_dev(c, &q, max_tiles, c->rs_counts.as<int32_t>() + 1, c->rs_tiles.as<Tile>(),
                      c->rs_windows.as<WindowDev>(), c->rs_seed_score.as<double>(), nullptr,
                      c->rs_best_i.as<int64_t>(), c->rs_best_e.as<double>(), c->rs_ev_tiles.as<int32_t>(), true,
                      &scratch);
  if (e == hipErrorInvalidConfiguration) {
    c->err = "rescan: scan configuration does not fit the device";
    return RKN_E_UNSUPPORTED;
  }
  if (e != hipSuccess) return rerr(c, e, "rescan scan sizing");

  // ---- the first kept seeds -------------------------------------------------------
  const double* d_start = start5;
  const double* d_step = step5;
  const double* d_target = target;
  if (from_batch) {
    // the batch's k best with the steps of their windows (the batch's expansion left
    // each event's first window in the first n_events entries of its scratch)
    e = launch_topk(c, c->b_score.as<double>(), c->b_ev_seed.as<long long>(), c->b_windows.as<WindowDev>(),
                    c->b_ev_scratch.as<int32_t>(), ne, c->b_counts.as<int32_t>(), k, c->rs_sel_idx.as<int64_t>(),
                    c->rs_sel_sc.as<double>(), c->rs_sel_seed.as<double>(), c->rs_sel_step.as<double>());
    if (e != hipSuccess) return rerr(c, e, "rescan start (batch top-k)");
    d_start = c->rs_sel_seed.as<double>();
    d_step = c->rs_sel_step.as<double>();
  } else if (!dev) {
    if ((e = hipMemcpyAsync(c->rs_cur.p, start5, sizeof(double) * nk * 5, hipMemcpyHostToDevice, c->stream)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(c->rs_step.p, step5, sizeof(double) * nk * 5, hipMemcpyHostToDevice, c->stream)) !=
            hipSuccess)
      return rerr(c, e, "rescan upload");
    d_start = c->rs_cur.as<double>();
    d_step = c->rs_step.as<double>();
  }
  if (target && !dev) {
    if ((e = hipMemcpyAsync(c->rs_target.p, target, sizeof(double) * ne, hipMemcpyHostToDevice, c->stream)) !=
        hipSuccess)
      return rerr(c, e, "rescan upload");
    d_target = c->rs_target.as<double>();
  }
  const dim3 eb(256), eg((unsigned)((ne + 255) / 256));
  hipLaunchKernelGGL(rescan_init_kernel, eg, eb, 0, c->stream, ne, k, d_start, d_step, d_target,
                     c->rs_cur.as<double>(), c->rs_step.as<double>(), c->rs_score.as<double>(),
                     c->rs_rounds.as<int32_t>(), c->rs_active.as<int32_t>(), c->rs_target.as<double>());
  if ((e = hipGetLastError()) != hipSuccess) return rerr(c, e, "rescan init");

  // ---- rounds -----------------------------------------------------------------------
  char* scr = c->rs_ev_scratch.as<char>();
  int32_t* ev_nw = reinterpret_cast<int32_t*>(scr);
  int32_t* ev_nt = ev_nw + ne;
  long long* ev_ns = reinterpret_cast<long long*>(ev_nt + ne);
  for (int r = 0; r < rp->max_rounds; ++r) {
    hipLaunchKernelGGL(rescan_expand_kernel, dim3(1), dim3(256), 0, c->stream, ne, k, G, tile,
                       c->rs_cur.as<double>(), c->rs_step.as<double>(), c->rs_active.as<int32_t>(), ev_nw, ev_nt,
                       ev_ns, c->rs_windows.as<WindowDev>(), c->rs_tiles.as<Tile>(), c->rs_ev_win.as<int32_t>(),
                       c->rs_ev_tiles.as<int32_t>(), c->rs_ev_seed.as<long long>(), c->rs_counts.as<int32_t>());
    if ((e = hipGetLastError()) != hipSuccess) return rerr(c, e, "rescan expand");
    e = launch_scan_dev(c, &q, max_tiles, c->rs_counts.as<int32_t>() + 1, c->rs_tiles.as<Tile>(),
                        c->rs_windows.as<WindowDev>(), c->rs_seed_score.as<double>(), nullptr,
                        c->rs_best_i.as<int64_t>(), c->rs_best_e.as<double>(), c->rs_ev_tiles.as<int32_t>(), false,
                        &scratch);
    if (e != hipSuccess) return rerr(c, e, "rescan scan");
    e = launch_topk(c, c->rs_seed_score.as<double>(), c->rs_ev_seed.as<long long>(), c->rs_windows.as<WindowDev>(),
                    c->rs_ev_win.as<int32_t>(), ne, c->rs_counts.as<int32_t>(), k, c->rs_sel_idx.as<int64_t>(),
                    c->rs_sel_sc.as<double>(), c->rs_sel_seed.as<double>(), c->rs_sel_step.as<double>());
    if (e != hipSuccess) return rerr(c, e, "rescan top-k");
    hipLaunchKernelGGL(rescan_update_kernel, eg, eb, 0, c->stream, ne, k, c->rs_sel_idx.as<int64_t>(),
                       c->rs_sel_sc.as<double>(), c->rs_sel_seed.as<double>(), c->rs_sel_step.as<double>(),
                       c->rs_target.as<double>(), c->rs_cur.as<double>(), c->rs_step.as<double>(),
                       c->rs_score.as<double>(), c->rs_rounds.as<int32_t>(), c->rs_active.as<int32_t>());
    if ((e = hipGetLastError()) != hipSuccess) return rerr(c, e, "rescan update");
  }

  // ---- outputs ------------------------------------------------------------------------
  const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if ((out5 && (e = hipMemcpyAsync(out5, c->rs_cur.p, sizeof(double) * nk * 5, kind, c->stream)) != hipSuccess) ||
      (out_step5 &&
       (e = hipMemcpyAsync(out_step5, c->rs_step.p, sizeof(double) * nk * 5, kind, c->stream)) != hipSuccess) ||
      (out_score &&
       (e = hipMemcpyAsync(out_score, c->rs_score.p, sizeof(double) * nk, kind, c->stream)) != hipSuccess) ||
      (rounds && (e = hipMemcpyAsync(rounds, c->rs_rounds.p, sizeof(int32_t) * ne, kind, c->stream)) != hipSuccess))
    return rerr(c, e, "rescan copy");
  if (!dev && (e = hipStreamSynchronize(c->stream)) != hipSuccess) return rerr(c, e, "rescan sync");
  return RKN_OK;
}

}  // extern "C"
