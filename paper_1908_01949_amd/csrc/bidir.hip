// Hit classification of explicit seeds and the two-direction quality count
// (section 2.2: the scan is run independently from seed sets at the chamber
// entrance and at its exit, and the number of hits that both directions classify
// to the track must reach a threshold).
//
// The exit-side scan is the time-reversed track: a seed at the exit crossing with
// the momentum reversed, propagated forward with the opposite charge (the circle
// Hough stage and the scan give such seeds when run with that charge). A hit is
// classified to a seed's track when (D - d)^2 < lambda; the classification uses the
// refinement's forward pass (same pruning, same LDS staging) without checkpoints.
#include <algorithm>
#include <numeric>
#include <string>
#include <vector>

#include "internal.hpp"

namespace rkn {

// Per row: the number of hits flagged in mask_a (and in mask_b when given).
__global__ void __launch_bounds__(256) count_common_kernel(int64_t n, int H, const uint8_t* __restrict__ mask_a,
                                                           const uint8_t* __restrict__ mask_b,
                                                           int32_t* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint8_t* a = mask_a + (size_t)p * H;
  const uint8_t* b = mask_b ? mask_b + (size_t)p * H : nullptr;
  int cnt = 0;
  for (int o = 0; o < H; ++o) cnt += (a[o] != 0) && (!b || b[o] != 0);
  out[p] = cnt;
}

}  // namespace rkn

using namespace rkn;

namespace {

rkn_status cerr(rkn_ctx* c, hipError_t e, const char* where) {
  c->err = std::string(where) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? RKN_E_NOMEM : RKN_E_DEVICE;
}

rkn_status check_params(rkn_ctx* c, const rkn_scan_params* p) {
  if (!p || p->n_steps < 1 || !(p->step_mm > 0) || !(p->lambda_mm2 >= 0) || !(p->R0 > 0) ||
      !std::isfinite(p->charge) || p->charge == 0 || (p->ptr_flags & ~RKN_PTR_DEVICE) ||
      (p->turn_stop != 0 && p->turn_stop != 1)) {
    c->err = "classify: invalid scan parameters";
    return RKN_E_ARG;
  }
  if (c->n_wires == 0 || c->field_kind < 0 || c->h_ev_off.empty()) {
    c->err = "classify: upload geometry, field and hits first";
    return RKN_E_STATE;
  }
  return RKN_OK;
}

// Classification of n seeds (any event order) into the inlier masks at dmask
// ([n][H], caller order); q->charge gives the propagation direction.
rkn_status classify(rkn_ctx* c, const rkn_scan_params* q, int64_t n, const int32_t* seed_event,
                    const double* seeds5, uint8_t* dmask) {
  for (int64_t s = 0; s < n; ++s) {
    if (seed_event[s] < 0 || seed_event[s] >= c->n_events) {
      c->err = "classify: seed event out of range";
      return RKN_E_ARG;
    }
    for (int d = 0; d < 5; ++d)
      if (!std::isfinite(seeds5[5 * s + d])) {
        c->err = "classify: non-finite seed";
        return RKN_E_ARG;
      }
  }
  rkn_scan_params p = *q;
  p.precision = 32;
  p.block_steps = 8;
  const int T = scan_tile(c, &p);
  std::vector<int64_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return seed_event[a] < seed_event[b]; });
  std::vector<double> sorted((size_t)n * 5);
  for (int64_t i = 0; i < n; ++i)
    for (int d = 0; d < 5; ++d) sorted[5 * i + d] = seeds5[5 * order[i] + d];
  std::vector<Tile> tiles;
  for (int64_t i = 0; i < n;) {
    const int ev = seed_event[order[i]];
    int64_t j = i;
    while (j < n && seed_event[order[j]] == ev) ++j;
    for (int64_t s = i; s < j; s += T) {
      Tile t{};
      t.event = ev;
      t.n = (int32_t)std::min<int64_t>(T, j - s);
      t.start = s;
      t.gbase = s;
      tiles.push_back(t);
    }
    i = j;
  }
  const size_t H = (size_t)(c->max_hits_event > 0 ? c->max_hits_event : 1);
  hipError_t e;
  if ((e = c->cl_seeds.ensure(sizeof(double) * 5 * (size_t)n)) != hipSuccess ||
      (e = c->cl_perm.ensure(sizeof(int64_t) * (size_t)n)) != hipSuccess ||
      (e = c->cl_tiles.ensure(sizeof(Tile) * std::max<size_t>(tiles.size(), 1))) != hipSuccess ||
      (e = c->cl_resid.ensure(sizeof(float) * (size_t)n * H)) != hipSuccess ||
      (e = c->cl_argmin.ensure(sizeof(int32_t) * (size_t)n * H)) != hipSuccess ||
      (e = c->cl_phi.ensure(sizeof(double) * (size_t)n)) != hipSuccess)
    return cerr(c, e, "classify alloc");
  e = hipMemcpyAsync(c->cl_seeds.p, sorted.data(), sizeof(double) * 5 * (size_t)n, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->cl_perm.p, order.data(), sizeof(int64_t) * (size_t)n, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && !tiles.empty())
    e = hipMemcpyAsync(c->cl_tiles.p, tiles.data(), sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = launch_refine_fwd(c, &p, (int64_t)tiles.size(), c->cl_tiles.as<Tile>(), c->cl_seeds.as<double>(),
                          c->cl_perm.as<int64_t>(), nullptr, dmask, 1, c->cl_resid.as<float>(),
                          c->cl_argmin.as<int32_t>(), c->cl_phi.as<double>(), nullptr, 64, 0, n);
  if (e == hipErrorInvalidConfiguration) {
    c->err = "classify: scan configuration does not fit the device";
    return RKN_E_UNSUPPORTED;
  }
  if (e != hipSuccess) return cerr(c, e, "classify");
  return RKN_OK;
}

rkn_status deliver_out(rkn_ctx* c, bool dev, void* dst, const void* src, size_t bytes) {
  if (!dst) return RKN_OK;
  hipError_t e = hipMemcpyAsync(dst, src, bytes, dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream);
  return e == hipSuccess ? RKN_OK : cerr(c, e, "classify copy");
}

}  // namespace

extern "C" {

rkn_status rkn_classify_hits(rkn_ctx* c, const rkn_scan_params* p, int64_t n_seeds, const int32_t* seed_event,
                             const double* seeds5, uint8_t* mask, int32_t* n_in) {
  if (!c) return RKN_E_ARG;
  rkn_status st = check_params(c, p);
  if (st != RKN_OK) return st;
  if (n_seeds < 1 || n_seeds > (int64_t(1) << 24) || !seed_event || !seeds5 || (!mask && !n_in)) {
    c->err = "classify: need 1..2^24 seeds with events and an output";
    return RKN_E_ARG;
  }
  hipError_t e;
  if ((e = hipSetDevice(c->device)) != hipSuccess) return cerr(c, e, "hipSetDevice");
  const size_t n = (size_t)n_seeds, H = (size_t)(c->max_hits_event > 0 ? c->max_hits_event : 1);
  if ((e = c->cl_mask.ensure(n * H)) != hipSuccess || (e = c->cl_count.ensure(sizeof(int32_t) * n)) != hipSuccess)
    return cerr(c, e, "classify alloc");
  if ((st = classify(c, p, n_seeds, seed_event, seeds5, c->cl_mask.as<uint8_t>())) != RKN_OK) return st;
  hipLaunchKernelGGL(count_common_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, n_seeds,
                     (int)H, c->cl_mask.as<uint8_t>(), (const uint8_t*)nullptr, c->cl_count.as<int32_t>());
  if ((e = hipGetLastError()) != hipSuccess) return cerr(c, e, "classify count");
  const bool dev = (p->ptr_flags & RKN_PTR_DEVICE) != 0;
  if ((st = deliver_out(c, dev, mask, c->cl_mask.p, n * H)) != RKN_OK) return st;
  if ((st = deliver_out(c, dev, n_in, c->cl_count.p, sizeof(int32_t) * n)) != RKN_OK) return st;
  if (!dev && (e = hipStreamSynchronize(c->stream)) != hipSuccess) return cerr(c, e, "classify sync");
  return RKN_OK;
}

rkn_status rkn_bidirectional_common(rkn_ctx* c, const rkn_scan_params* p, int64_t n_pairs, const int32_t* pair_event,
                                    const double* seeds_entry5, const double* seeds_exit5, uint8_t* mask_entry,
                                    uint8_t* mask_exit, int32_t* n_common) {
  if (!c) return RKN_E_ARG;
  rkn_status st = check_params(c, p);
  if (st != RKN_OK) return st;
  if (n_pairs < 1 || n_pairs > (int64_t(1) << 24) || !pair_event || !seeds_entry5 || !seeds_exit5 || !n_common) {
    c->err = "bidirectional: need 1..2^24 seed pairs with events and n_common";
    return RKN_E_ARG;
  }
  hipError_t e;
  if ((e = hipSetDevice(c->device)) != hipSuccess) return cerr(c, e, "hipSetDevice");
  const size_t n = (size_t)n_pairs, H = (size_t)(c->max_hits_event > 0 ? c->max_hits_event : 1);
  if ((e = c->cl_mask.ensure(2 * n * H)) != hipSuccess || (e = c->cl_count.ensure(sizeof(int32_t) * n)) != hipSuccess)
    return cerr(c, e, "bidirectional alloc");
  uint8_t* m_in = c->cl_mask.as<uint8_t>();
  uint8_t* m_out = m_in + n * H;
  rkn_scan_params back = *p;
  back.charge = -p->charge;   // the time-reversed track
  if ((st = classify(c, p, n_pairs, pair_event, seeds_entry5, m_in)) != RKN_OK) return st;
  if ((st = classify(c, &back, n_pairs, pair_event, seeds_exit5, m_out)) != RKN_OK) return st;
  hipLaunchKernelGGL(count_common_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, n_pairs,
                     (int)H, (const uint8_t*)m_in, (const uint8_t*)m_out, c->cl_count.as<int32_t>());
  if ((e = hipGetLastError()) != hipSuccess) return cerr(c, e, "bidirectional count");
  const bool dev = (p->ptr_flags & RKN_PTR_DEVICE) != 0;
  if ((st = deliver_out(c, dev, mask_entry, m_in, n * H)) != RKN_OK) return st;
  if ((st = deliver_out(c, dev, mask_exit, m_out, n * H)) != RKN_OK) return st;
  if ((st = deliver_out(c, dev, n_common, c->cl_count.p, sizeof(int32_t) * n)) != RKN_OK) return st;
  if (!dev && (e = hipStreamSynchronize(c->stream)) != hipSuccess) return cerr(c, e, "bidirectional sync");
  return RKN_OK;
}

}  // extern "C"
