// C-ABI entry points of librknscan: context, validated uploads, and dispatch of the
// scan and trace kernels. See include/rknscan.h for the contract of each call.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <string>
#include <vector>

#include "internal.hpp"

using rkn::DevBuf;

namespace {

const char* kVersion = "rknscan 0.1 (gfx950)";

rkn_status dev_err(rkn_ctx* c, hipError_t e, const char* where) {
  c->err = std::string(where) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? RKN_E_NOMEM : RKN_E_DEVICE;
}

rkn_status arg_err(rkn_ctx* c, const std::string& s) {
  c->err = s;
  return RKN_E_ARG;
}

#define RKN_HIP(call, where)                   \
  do {                                         \
    hipError_t e_ = (call);                    \
    if (e_ != hipSuccess) return dev_err(c, e_, where); \
  } while (0)

bool is_fin(double v) { return std::isfinite(v); }

template <typename T>
hipError_t upload(DevBuf& b, const T* src, size_t n, hipStream_t s) {
  hipError_t e = b.ensure(sizeof(T) * n);
  if (e != hipSuccess) return e;
  if (n == 0) return hipSuccess;
  return hipMemcpyAsync(b.p, src, sizeof(T) * n, hipMemcpyHostToDevice, s);
}

rkn_status check_scan_params(rkn_ctx* c, const rkn_scan_params* p) {
  if (!p) return arg_err(c, "params is NULL");
  if (!is_fin(p->R0) || p->R0 <= 0) return arg_err(c, "R0 must be finite and > 0");
  if (!is_fin(p->charge) || p->charge == 0) return arg_err(c, "charge must be finite and non-zero");
  if (!is_fin(p->step_mm) || p->step_mm <= 0) return arg_err(c, "step_mm must be finite and > 0");
  if (!is_fin(p->lambda_mm2) || p->lambda_mm2 < 0) return arg_err(c, "lambda_mm2 must be finite and >= 0");
  if (p->n_steps < 1) return arg_err(c, "n_steps must be >= 1");
  if (p->precision != 32 && p->precision != 64) return arg_err(c, "precision must be 32 or 64");
  if (p->block_steps != 0 && p->block_steps != 4 && p->block_steps != 6 && p->block_steps != 8)
    return arg_err(c, "block_steps must be 0, 4, 6 or 8");
  if (p->ptr_flags & ~RKN_PTR_DEVICE) return arg_err(c, "unknown ptr_flags bits");
  if (p->turn_stop != 0 && p->turn_stop != 1) return arg_err(c, "turn_stop must be 0 or 1");
  return RKN_OK;
}

rkn_status check_state(rkn_ctx* c) {
  if (c->n_wires == 0) {
    c->err = "no geometry uploaded";
    return RKN_E_STATE;
  }
  if (c->field_kind < 0) {
    c->err = "no field uploaded";
    return RKN_E_STATE;
  }
  if (c->h_ev_off.empty()) {
    c->err = "no hits uploaded";
    return RKN_E_STATE;
  }
  return RKN_OK;
}

}  // namespace

namespace rkn {

rkn_status validate_scan(rkn_ctx* c, const rkn_scan_params* p) {
  const rkn_status st = check_scan_params(c, p);
  return st != RKN_OK ? st : check_state(c);
}

}  // namespace rkn

namespace {

// Copy a device result to caller memory (host or device per ptr_flags).
template <typename T>
hipError_t deliver(rkn_ctx* c, T* dst, const T* dsrc, size_t n, bool dev) {
  if (!dst || n == 0 || dst == dsrc) return hipSuccess;
  return hipMemcpyAsync(dst, dsrc, sizeof(T) * n, dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                        c->stream);
}

}  // namespace

extern "C" {

const char* rkn_version(void) { return kVersion; }

rkn_status rkn_create(int32_t device, void* hip_stream, rkn_ctx** out) {
  if (!out) return RKN_E_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return RKN_E_ARG;
  rkn_ctx* c = new (std::nothrow) rkn_ctx();
  if (!c) return RKN_E_NOMEM;
  c->device = device;
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return RKN_E_DEVICE;
  }
  if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      c->n_cu <= 0) {
    delete c;
    return RKN_E_DEVICE;
  }
  int lds = 0, lds_optin = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
    c->max_lds_block = lds;
  if (hipDeviceGetAttribute(&lds_optin, hipDeviceAttributeSharedMemPerBlockOptin, device) == hipSuccess &&
      lds_optin > c->max_lds_block)
    c->max_lds_block = lds_optin;
  // the allocation-free scan's work memory on this device (its absence only disables
  // that entry point, which then reports the error)
  (void)rkn::noalloc_init(device);
  if (hip_stream) {
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return RKN_E_DEVICE;
    }
    c->own_stream = true;
  }
  *out = c;
  return RKN_OK;
}

void rkn_destroy(rkn_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  rkn::batch_release(c);
  c->refine_release();
  rkn::rescan_release(c);
  DevBuf* bufs[] = {&c->wire32, &c->wire64, &c->wire_layer, &c->layer_r, &c->field_nodes, &c->ev_off,
                    &c->hits32, &c->hits64, &c->layer_off, &c->ev_maxdrift, &c->windows, &c->tiles,
                    &c->ev_tiles, &c->parts, &c->counter, &c->mscratch, &c->out_score, &c->out_nin,
                    &c->out_best_i, &c->out_best_e, &c->trace_buf, &c->seeds_buf, &c->perm_buf,
                    &c->wire_wx, &c->wire_wy, &c->hits_wire, &c->hough_acc, &c->hough_max,
                    &c->hough_cand_n, &c->hough_cand, &c->hough_slots, &c->hough_nsel, &c->hits_orig, &c->hits_phi, &c->layer_ext,
                    &c->sel_seg, &c->sel_win, &c->sel_idx, &c->sel_sc, &c->sel_seed, &c->cl_seeds,
                    &c->cl_perm, &c->cl_tiles, &c->cl_resid, &c->cl_argmin, &c->cl_phi, &c->cl_mask,
                    &c->cl_count, &c->work_counts};
  for (DevBuf* b : bufs) b->release();
  for (DevBuf& b : c->extra) b.release();
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* rkn_last_error(const rkn_ctx* c) { return c ? c->err.c_str() : "NULL context"; }

rkn_status rkn_synchronize(rkn_ctx* c) {
  if (!c) return RKN_E_ARG;
  RKN_HIP(hipSetDevice(c->device), "hipSetDevice");
  RKN_HIP(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  return RKN_OK;
}

rkn_status rkn_upload_geometry(rkn_ctx* c, int32_t n_wires, const double* mx, const double* my,
                               const double* mz, const double* ux, const double* uy, const double* uz,
                               const double* half_len, const int32_t* layer_of, int32_t n_layers,
                               const double* layer_rmin, const double* layer_rmax) {
  if (!c) return RKN_E_ARG;
  if (n_wires < 1) return arg_err(c, "n_wires must be >= 1");
  if (n_layers < 1 || n_layers > RKN_MAX_LAYERS) return arg_err(c, "n_layers out of range");
  if (!mx || !my || !mz || !ux || !uy || !uz || !half_len || !layer_of || !layer_rmin || !layer_rmax)
    return arg_err(c, "NULL geometry array");
  for (int i = 0; i < n_wires; ++i) {
    if (!is_fin(mx[i]) || !is_fin(my[i]) || !is_fin(mz[i]) || !is_fin(half_len[i]) || half_len[i] <= 0)
      return arg_err(c, "wire " + std::to_string(i) + ": non-finite point or half_len <= 0");
    const double un = sqrt(ux[i] * ux[i] + uy[i] * uy[i] + uz[i] * uz[i]);
    if (!is_fin(un) || fabs(un - 1.0) > 1e-9)
      return arg_err(c, "wire " + std::to_string(i) + ": direction is not a unit vector");
    if (layer_of[i] < 0 || layer_of[i] >= n_layers)
      return arg_err(c, "wire " + std::to_string(i) + ": layer out of range");
  }
  for (int l = 0; l < n_layers; ++l) {
    if (!is_fin(layer_rmin[l]) || !is_fin(layer_rmax[l]) || layer_rmin[l] < 0 ||
        layer_rmax[l] < layer_rmin[l])
      return arg_err(c, "layer " + std::to_string(l) + ": bad radial extent");
    if (l > 0 && (layer_rmin[l] < layer_rmin[l - 1] || layer_rmax[l] < layer_rmax[l - 1])) {
      c->err = "layer radial extents must be non-decreasing in the layer index";
      return RKN_E_UNSUPPORTED;
    }
  }
  RKN_HIP(hipSetDevice(c->device), "hipSetDevice");
  std::vector<rkn::HitRec<float>> w32(n_wires);
  std::vector<rkn::HitRec<double>> w64(n_wires);
  for (int i = 0; i < n_wires; ++i) {
    w64[i] = {mx[i], my[i], mz[i], ux[i], uy[i], uz[i], half_len[i], 0.0};
    w32[i] = {(float)mx[i], (float)my[i], (float)mz[i], (float)ux[i], (float)uy[i], (float)uz[i],
              (float)half_len[i], 0.0f};
  }
  std::vector<float2> lr(n_layers);
  for (int l = 0; l < n_layers; ++l) lr[l] = make_float2((float)layer_rmin[l], (float)layer_rmax[l]);
  RKN_HIP(upload(c->wire32, w32.data(), w32.size(), c->stream), "geometry upload");
  RKN_HIP(upload(c->wire64, w64.data(), w64.size(), c->stream), "geometry upload");
  RKN_HIP(upload(c->wire_layer, layer_of, (size_t)n_wires, c->stream), "geometry upload");
  RKN_HIP(upload(c->layer_r, lr.data(), lr.size(), c->stream), "geometry upload");
  RKN_HIP(upload(c->wire_wx, mx, (size_t)n_wires, c->stream), "geometry upload");
  RKN_HIP(upload(c->wire_wy, my, (size_t)n_wires, c->stream), "geometry upload");
  RKN_HIP(hipStreamSynchronize(c->stream), "geometry upload");
  c->n_wires = n_wires;
  c->n_layers = n_layers;
  c->h_layer_rmin.assign(layer_rmin, layer_rmin + n_layers);
  c->h_layer_rmax.assign(layer_rmax, layer_rmax + n_layers);
  c->h_layer_of.assign(layer_of, layer_of + n_wires);
  c->h_wx.assign(mx, mx + n_wires);
  c->h_wy.assign(my, my + n_wires);
  c->h_ev_off.clear();       // hits refer to the old wire table
  c->n_events = 0;
  rkn::batch_release(c);
  c->refine_release();
  return RKN_OK;
}

rkn_status rkn_upload_field_uniform(rkn_ctx* c, double bz) {
  if (!c) return RKN_E_ARG;
  if (!is_fin(bz)) return arg_err(c, "bz must be finite");
  c->field_kind = 0;
  c->bz = bz;
  rkn::batch_release(c);   // captured graphs hold the previous field's kind and nodes
  c->refine_release();     // checkpoints were propagated in the previous field
  return RKN_OK;
}

rkn_status rkn_upload_field_rz(rkn_ctx* c, int32_t nr, int32_t nz, double r0, double r1, double z0,
                               double z1, const float* br, const float* bz) {
  if (!c) return RKN_E_ARG;
  if (nr < 2 || nz < 2) return arg_err(c, "nr and nz must be >= 2");
  if ((int64_t)nr * nz > (1 << 22)) return arg_err(c, "field grid too large");
  if (!is_fin(r0) || !is_fin(r1) || !is_fin(z0) || !is_fin(z1) || r1 <= r0 || z1 <= z0 || r0 < 0)
    return arg_err(c, "bad field grid extent");
  if (!br || !bz) return arg_err(c, "NULL field array");
  for (size_t i = 0; i < (size_t)nr * nz; ++i)
    if (!std::isfinite(br[i]) || !std::isfinite(bz[i])) return arg_err(c, "non-finite field node");
  // device layout: [nz + 1][nr + 1], the extra column and row repeating the edge
  std::vector<float2> nodes(rkn::padded_field_nodes(nr, nz));
  for (int j = 0; j <= nz; ++j)
    for (int i = 0; i <= nr; ++i) {
      const size_t src = (size_t)std::min(j, nz - 1) * nr + std::min(i, nr - 1);
      nodes[(size_t)j * (nr + 1) + i] = make_float2(br[src], bz[src]);
    }
  RKN_HIP(hipSetDevice(c->device), "hipSetDevice");
  RKN_HIP(upload(c->field_nodes, nodes.data(), nodes.size(), c->stream), "field upload");
  RKN_HIP(hipStreamSynchronize(c->stream), "field upload");
  c->field_kind = 1;
  c->nr = nr;
  c->nz = nz;
  c->r0 = r0;
  c->r1 = r1;
  c->z0 = z0;
  c->z1 = z1;
  c->bz = 0.0;
  rkn::batch_release(c);   // captured graphs hold the previous field's kind and nodes
  c->refine_release();     // checkpoints were propagated in the previous field
  return RKN_OK;
}

rkn_status rkn_upload_hits(rkn_ctx* c, int32_t n_events, const int32_t* ev_off, const int32_t* wire_id,
                           const float* drift) {
  if (!c) return RKN_E_ARG;
  if (c->n_wires == 0) {
    c->err = "upload the geometry before the hits";
    return RKN_E_STATE;
  }
  if (n_events < 1) return arg_err(c, "n_events must be >= 1");
  if (!ev_off) return arg_err(c, "ev_off is NULL");
  if (ev_off[0] != 0) return arg_err(c, "ev_off[0] must be 0");
  int maxh = 0;
  for (int e = 0; e < n_events; ++e) {
    const int n = ev_off[e + 1] - ev_off[e];
    if (n < 0) return arg_err(c, "ev_off must be non-decreasing");
    if (n > RKN_MAX_HITS_PER_EVENT) {
      c->err = "event " + std::to_string(e) + " has " + std::to_string(n) + " hits (max " +
               std::to_string(RKN_MAX_HITS_PER_EVENT) + ")";
      return RKN_E_CAPACITY;
    }
    maxh = std::max(maxh, n);
  }
  const int64_t H = ev_off[n_events];
  if (H > 0 && (!wire_id || !drift)) return arg_err(c, "NULL hit array");
  for (int64_t i = 0; i < H; ++i) {
    if (wire_id[i] < 0 || wire_id[i] >= c->n_wires) return arg_err(c, "wire id out of range at hit " + std::to_string(i));
    if (!std::isfinite(drift[i]) || drift[i] < 0) return arg_err(c, "drift must be finite and >= 0 at hit " + std::to_string(i));
  }
  RKN_HIP(hipSetDevice(c->device), "hipSetDevice");
  rkn::batch_release(c);   // a planned batch refers to the previous events
  c->refine_release();     // so do refinement seeds and their inlier sets
  DevBuf d_drift;
  DevBuf& d_wid = c->hits_wire;
  hipError_t e = upload(c->ev_off, ev_off, (size_t)n_events + 1, c->stream);
  if (e == hipSuccess) e = upload(d_wid, wire_id, (size_t)H, c->stream);
  if (e == hipSuccess) e = upload(d_drift, drift, (size_t)H, c->stream);
  if (e == hipSuccess) e = c->hits32.ensure(sizeof(rkn::HitRec<float>) * (size_t)std::max<int64_t>(H, 1));
  if (e == hipSuccess) e = c->hits64.ensure(sizeof(rkn::HitRec<double>) * (size_t)std::max<int64_t>(H, 1));
  if (e == hipSuccess) e = c->layer_off.ensure(sizeof(int32_t) * (size_t)n_events * (c->n_layers + 1));
  if (e == hipSuccess) e = c->ev_maxdrift.ensure(sizeof(float) * (size_t)n_events);
  if (e == hipSuccess) e = c->hits_orig.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(H, 1));
  if (e == hipSuccess) e = c->hits_phi.ensure(sizeof(float) * (size_t)std::max<int64_t>(H, 1));
  if (e == hipSuccess)
    e = c->layer_ext.ensure(sizeof(float2) * (size_t)std::max(n_events, 1) * (size_t)std::max(c->n_layers, 1));
  if (e == hipSuccess) {
    c->n_events = n_events;
    e = rkn::launch_prep_hits(c, d_wid.as<int32_t>(), d_drift.as<float>());
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  d_drift.release();
  if (e != hipSuccess) {
    c->n_events = 0;
    c->h_ev_off.clear();
    return dev_err(c, e, "hit upload");
  }
  c->total_hits = H;
  c->max_hits_event = maxh;
  c->h_ev_off.assign(ev_off, ev_off + n_events + 1);
  c->h_wire.assign(wire_id, wire_id + H);
  c->h_drift.assign(drift, drift + H);
  return RKN_OK;
}

// ---------------------------------------------------------------------------------
static rkn_status run_scan(rkn_ctx* c, const rkn_scan_params* p, std::vector<rkn::WindowDev>& wins,
                           std::vector<rkn::Tile>& tiles, std::vector<int32_t>& ev_tiles,
                           int64_t total, double* score, int32_t* n_in, int64_t* best_index,
                           double* best_score, const double* d_seeds5 = nullptr,
                           const int64_t* d_perm = nullptr) {
  const bool dev = (p->ptr_flags & RKN_PTR_DEVICE) != 0;
  RKN_HIP(upload(c->windows, wins.data(), wins.size(), c->stream), "window upload");
  RKN_HIP(upload(c->tiles, tiles.data(), tiles.size(), c->stream), "tile upload");
  RKN_HIP(upload(c->ev_tiles, ev_tiles.data(), ev_tiles.size(), c->stream), "tile upload");
  double* d_score = nullptr;
  int32_t* d_nin = nullptr;
  int64_t* d_bi;
  double* d_be;
  if (score) {
    if (dev) {
      d_score = score;
    } else {
      RKN_HIP(c->out_score.ensure(sizeof(double) * (size_t)std::max<int64_t>(total, 1)), "alloc");
      d_score = c->out_score.as<double>();
    }
  }
  if (n_in) {
    if (dev) {
      d_nin = n_in;
    } else {
      RKN_HIP(c->out_nin.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(total, 1)), "alloc");
      d_nin = c->out_nin.as<int32_t>();
    }
  }
  if (dev) {
    d_bi = best_index;
    d_be = best_score;
  } else {
    RKN_HIP(c->out_best_i.ensure(sizeof(int64_t) * c->n_events), "alloc");
    RKN_HIP(c->out_best_e.ensure(sizeof(double) * c->n_events), "alloc");
    d_bi = c->out_best_i.as<int64_t>();
    d_be = c->out_best_e.as<double>();
  }
  rkn_scan_params q = *p;
  q.block_steps = rkn::resolve_block_steps(c, &q);
  hipError_t e = rkn::launch_scan(c, &q, (int64_t)tiles.size(), c->tiles.as<rkn::Tile>(),
                                  c->windows.as<rkn::WindowDev>(), d_seeds5, d_perm, d_score, d_nin,
                                  d_bi, d_be, c->ev_tiles.as<int32_t>());
  if (e == hipErrorInvalidConfiguration) {
    c->err = "scan configuration does not fit the device (LDS per workgroup); use FP32 or fewer hits per event";
    return RKN_E_UNSUPPORTED;
  }
  if (e != hipSuccess) return dev_err(c, e, "scan launch");
  if (!dev) {
    RKN_HIP(deliver(c, score, d_score, (size_t)total, false), "copy scores");
    RKN_HIP(deliver(c, n_in, d_nin, (size_t)total, false), "copy n_in");
    RKN_HIP(deliver(c, best_index, d_bi, (size_t)c->n_events, false), "copy best");
    RKN_HIP(deliver(c, best_score, d_be, (size_t)c->n_events, false), "copy best");
    RKN_HIP(hipStreamSynchronize(c->stream), "scan");
  }
  return RKN_OK;
}

// Windows -> device windows, tiles and per-event tile, seed and window offsets
// (windows must be ordered by event; an event's seeds are contiguous).
static rkn_status prepare_windows(rkn_ctx* c, const rkn_scan_params* p, int32_t n_windows, const rkn_window* w,
                                  std::vector<rkn::WindowDev>& wins, std::vector<rkn::Tile>& tiles,
                                  std::vector<int32_t>& ev_tiles, int64_t& total, std::vector<long long>* ev_seed,
                                  std::vector<int32_t>* ev_win) {
  if (n_windows < 0 || (n_windows > 0 && !w)) return arg_err(c, "bad window array");
  wins.assign(std::max(n_windows, 1), rkn::WindowDev{});
  tiles.clear();
  ev_tiles.assign(c->n_events + 1, 0);
  if (ev_seed) ev_seed->assign(c->n_events + 1, 0);
  if (ev_win) ev_win->assign(c->n_events + 1, 0);
  const int T = rkn::scan_tile(c, p);
  total = 0;
  int last_ev = -1;
  for (int k = 0; k < n_windows; ++k) {
    const rkn_window& x = w[k];
    if (x.event < 0 || x.event >= c->n_events) return arg_err(c, "window " + std::to_string(k) + ": event out of range");
    if (x.event < last_ev) return arg_err(c, "windows must be ordered by event");
    int64_t size = 1;
    for (int d = 0; d < 5; ++d) {
      if (x.count[d] < 1) return arg_err(c, "window " + std::to_string(k) + ": count must be >= 1");
      if (!is_fin(x.center[d]) || !is_fin(x.half_width[d]) || x.half_width[d] < 0)
        return arg_err(c, "window " + std::to_string(k) + ": bad centre or half width");
      size *= x.count[d];
      if (size > (int64_t(1) << 40)) return arg_err(c, "window too large");
    }
    for (int e = last_ev + 1; e <= x.event; ++e) {
      ev_tiles[e] = (int32_t)tiles.size();
      if (ev_seed) (*ev_seed)[e] = total;
      if (ev_win) (*ev_win)[e] = k;
    }
    last_ev = x.event;
    rkn::WindowDev& d = wins[k];
    for (int j = 0; j < 5; ++j) {
      d.center[j] = x.center[j];
      d.half_width[j] = x.half_width[j];
      d.count[j] = x.count[j];
    }
    d.event = x.event;
    for (int64_t s = 0; s < size; s += T) {
      rkn::Tile t{};
      t.window = k;
      t.event = x.event;
      t.n = (int32_t)std::min<int64_t>(T, size - s);
      t.start = s;
      t.gbase = total + s;
      tiles.push_back(t);
    }
    total += size;
  }
  for (int e = last_ev + 1; e <= c->n_events; ++e) {
    ev_tiles[e] = (int32_t)tiles.size();
    if (ev_seed) (*ev_seed)[e] = total;
    if (ev_win) (*ev_win)[e] = n_windows;
  }
  return RKN_OK;
}

}  // extern "C"

namespace rkn {

rkn_status prepare_scan_windows(rkn_ctx* c, const rkn_scan_params* p, int32_t n_windows, const rkn_window* w,
                                std::vector<WindowDev>& wins, std::vector<Tile>& tiles, std::vector<int32_t>& ev_tiles,
                                int64_t& total) {
  return prepare_windows(c, p, n_windows, w, wins, tiles, ev_tiles, total, nullptr, nullptr);
}

}  // namespace rkn

extern "C" {

rkn_status rkn_scan_shape(rkn_ctx* c, const rkn_scan_params* p, int32_t* block_steps, int32_t* seeds_per_tile) {
  if (!c) return RKN_E_ARG;
  rkn_status st = check_scan_params(c, p);
  if (st != RKN_OK) return st;
  if ((st = check_state(c)) != RKN_OK) return st;
  RKN_HIP(hipSetDevice(c->device), "hipSetDevice");
  if (block_steps) *block_steps = p->precision == 64 ? 4 : rkn::resolve_block_steps(c, p);
  if (seeds_per_tile) *seeds_per_tile = rkn::scan_tile(c, p);
  return RKN_OK;
}

rkn_status rkn_scan_windows(rkn_ctx* c, const rkn_scan_params* p, int32_t n_windows, const rkn_window* w,
                            double* score, int32_t* n_in, int64_t* best_index, double* best_score) {
  if (!c) return RKN_E_ARG;
  rkn_status st = check_scan_params(c, p);
  if (st != RKN_OK) return st;
  if ((st = check_state(c)) != RKN_OK) return st;
  if (!best_index || !best_score) return arg_err(c, "best_index/best_score must not be NULL");
  std::vector<rkn::WindowDev> wins;
  std::vector<rkn::Tile> tiles;
  std::vector<int32_t> ev_tiles;
  int64_t total = 0;
  if ((st = prepare_windows(c, p, n_windows, w, wins, tiles, ev_tiles, total, nullptr, nullptr)) != RKN_OK)
    return st;
  RKN_HIP(hipSetDevice(c->device), "hipSetDevice");
  return run_scan(c, p, wins, tiles, ev_tiles, total, score, n_in, best_index, best_score);
}

rkn_status rkn_scan_work_counts(rkn_ctx* c, const rkn_scan_params* p, int32_t n_windows, const rkn_window* w,
                                int64_t* counts) {
  if (!c) return RKN_E_ARG;
  rkn_status st = check_scan_params(c, p);
  if (st != RKN_OK) return st;
  if ((st = check_state(c)) != RKN_OK) return st;
  if (!counts) return arg_err(c, "counts must not be NULL");
  if (p->turn_stop) {
    c->err = "work counts: fixed steps over the whole path only (turn_stop = 0)";
    return RKN_E_UNSUPPORTED;
  }
  std::vector<rkn::WindowDev> wins;
  std::vector<rkn::Tile> tiles;
  std::vector<int32_t> ev_tiles;
  int64_t total = 0;
  if ((st = prepare_windows(c, p, n_windows, w, wins, tiles, ev_tiles, total, nullptr, nullptr)) != RKN_OK)
    return st;
  RKN_HIP(hipSetDevice(c->device), "hipSetDevice");
  RKN_HIP(c->work_counts.ensure(4 * sizeof(unsigned long long)), "alloc");
  const unsigned long long zero[4] = {0, 0, 0, 0};
  RKN_HIP(hipMemcpyAsync(c->work_counts.p, zero, sizeof(zero), hipMemcpyHostToDevice, c->stream), "counter reset");
  std::vector<int64_t> bi((size_t)std::max(c->n_events, 1));
  std::vector<double> bs((size_t)std::max(c->n_events, 1));
  rkn_scan_params q = *p;
  q.ptr_flags = 0;
  c->count_work = c->work_counts.as<unsigned long long>();
  st = run_scan(c, &q, wins, tiles, ev_tiles, total, nullptr, nullptr, bi.data(), bs.data());
  c->count_work = nullptr;
  if (st != RKN_OK) return st;
  unsigned long long h[4];
  RKN_HIP(hipMemcpy(h, c->work_counts.p, sizeof(h), hipMemcpyDeviceToHost), "counter copy");
  for (int k = 0; k < 3; ++k) counts[k] = (int64_t)h[k];
  return RKN_OK;
}

rkn_status rkn_scan_windows_adaptive(rkn_ctx* c, const rkn_scan_params* p, const rkn_adaptive_params* ap,
                                     int32_t n_windows, const rkn_window* w, double* score, int32_t* n_in,
                                     int64_t* best_index, double* best_score) {
  if (!c) return RKN_E_ARG;
  rkn_status st = check_scan_params(c, p);
  if (st != RKN_OK) return st;
  if ((st = check_state(c)) != RKN_OK) return st;
  if (!ap || !is_fin(ap->tol_mm) || !(ap->tol_mm > 0) || !is_fin(ap->h_min_mm) || !(ap->h_min_mm > 0) ||
      !is_fin(ap->h_max_mm) || ap->h_max_mm < ap->h_min_mm ||
      p->n_steps * p->step_mm / ap->h_min_mm > 1e7)
    return arg_err(c, "adaptive scan: tol > 0, 0 < h_min <= h_max, path / h_min <= 1e7");
  rkn_scan_params q = *p;
  q.block_steps = 4;
  std::vector<rkn::WindowDev> wins;
  std::vector<rkn::Tile> tiles;
  std::vector<int32_t> ev_tiles;
  int64_t total = 0;
  if ((st = prepare_windows(c, &q, n_windows, w, wins, tiles, ev_tiles, total, nullptr, nullptr)) != RKN_OK)
    return st;
  RKN_HIP(hipSetDevice(c->device), "hipSetDevice");
  c->adapt = ap;
  st = run_scan(c, &q, wins, tiles, ev_tiles, total, score, n_in, best_index, best_score);
  c->adapt = nullptr;
  return st;
}

rkn_status rkn_scan_windows_topk(rkn_ctx* c, const rkn_scan_params* p, int32_t n_windows, const rkn_window* w,
                                 int32_t k, int64_t* index, double* score, double* seeds5) {
  if (!c) return RKN_E_ARG;
  rkn_status st = check_scan_params(c, p);
  if (st != RKN_OK) return st;
  if ((st = check_state(c)) != RKN_OK) return st;
  if (k < 1 || k > RKN_TOPK_MAX || !index || !score) return arg_err(c, "topk: k in [1, 16] and index/score outputs");
  std::vector<rkn::WindowDev> wins;
  std::vector<rkn::Tile> tiles;
  std::vector<int32_t> ev_tiles, ev_win;
  std::vector<long long> ev_seed;
  int64_t total = 0;
  if ((st = prepare_windows(c, p, n_windows, w, wins, tiles, ev_tiles, total, &ev_seed, &ev_win)) != RKN_OK)
    return st;
  RKN_HIP(hipSetDevice(c->device), "hipSetDevice");
  const bool dev = (p->ptr_flags & RKN_PTR_DEVICE) != 0;
  const size_t ne = (size_t)c->n_events;
  RKN_HIP(upload(c->windows, wins.data(), wins.size(), c->stream), "window upload");
  RKN_HIP(upload(c->tiles, tiles.data(), std::max<size_t>(tiles.size(), 1), c->stream), "tile upload");
  RKN_HIP(upload(c->ev_tiles, ev_tiles.data(), ev_tiles.size(), c->stream), "tile upload");
  RKN_HIP(upload(c->sel_seg, ev_seed.data(), ev_seed.size(), c->stream), "offset upload");
  RKN_HIP(upload(c->sel_win, ev_win.data(), ev_win.size(), c->stream), "offset upload");
  RKN_HIP(c->out_score.ensure(sizeof(double) * (size_t)std::max<int64_t>(total, 1)), "alloc");
  RKN_HIP(c->out_best_i.ensure(sizeof(int64_t) * ne), "alloc");
  RKN_HIP(c->out_best_e.ensure(sizeof(double) * ne), "alloc");
  int64_t* d_idx = index;
  double* d_sc = score;
  double* d_seed = seeds5;
  if (!dev) {
    RKN_HIP(c->sel_idx.ensure(sizeof(int64_t) * ne * k), "alloc");
    RKN_HIP(c->sel_sc.ensure(sizeof(double) * ne * k), "alloc");
    RKN_HIP(c->sel_seed.ensure(sizeof(double) * ne * k * 5), "alloc");
    d_idx = c->sel_idx.as<int64_t>();
    d_sc = c->sel_sc.as<double>();
    d_seed = seeds5 ? c->sel_seed.as<double>() : nullptr;
  }
  rkn_scan_params q = *p;
  q.block_steps = rkn::resolve_block_steps(c, &q);
  hipError_t e = rkn::launch_scan(c, &q, (int64_t)tiles.size(), c->tiles.as<rkn::Tile>(),
                                  c->windows.as<rkn::WindowDev>(), nullptr, nullptr, c->out_score.as<double>(),
                                  nullptr, c->out_best_i.as<int64_t>(), c->out_best_e.as<double>(),
                                  c->ev_tiles.as<int32_t>());
  if (e == hipErrorInvalidConfiguration) {
    c->err = "scan configuration does not fit the device (LDS per workgroup); use FP32 or fewer hits per event";
    return RKN_E_UNSUPPORTED;
  }
  if (e != hipSuccess) return dev_err(c, e, "scan launch");
  e = rkn::launch_topk(c, c->out_score.as<double>(), c->sel_seg.as<long long>(), c->windows.as<rkn::WindowDev>(),
                       c->sel_win.as<int32_t>(), c->n_events, c->sel_win.as<int32_t>() + c->n_events, k, d_idx,
                       d_sc, d_seed);
  if (e != hipSuccess) return dev_err(c, e, "topk launch");
  if (!dev) {
    RKN_HIP(deliver(c, index, d_idx, ne * k, false), "copy topk");
    RKN_HIP(deliver(c, score, d_sc, ne * k, false), "copy topk");
    if (seeds5) RKN_HIP(deliver(c, seeds5, d_seed, ne * k * 5, false), "copy topk");
    RKN_HIP(hipStreamSynchronize(c->stream), "topk");
  }
  return RKN_OK;
}

rkn_status rkn_scan_seeds(rkn_ctx* c, const rkn_scan_params* p, int64_t n_seeds, const int32_t* seed_event,
                          const double* theta, const double* z, const double* px, const double* py,
                          const double* pz, double* score, int32_t* n_in, int64_t* best_index,
                          double* best_score) {
  if (!c) return RKN_E_ARG;
  rkn_status st = check_scan_params(c, p);
  if (st != RKN_OK) return st;
  if ((st = check_state(c)) != RKN_OK) return st;
  if (n_seeds < 0 || (n_seeds > 0 && (!seed_event || !theta || !z || !px || !py || !pz)))
    return arg_err(c, "bad seed arrays");
  if (!best_index || !best_score) return arg_err(c, "best_index/best_score must not be NULL");
  if (n_seeds > (int64_t(1) << 31)) return arg_err(c, "too many seeds");
  // Each explicit seed becomes a one-point window; seeds are grouped by event (stable)
  // and a permutation maps scan order back to the caller's order.
  std::vector<int64_t> order(n_seeds);
  std::iota(order.begin(), order.end(), 0);
  for (int64_t s = 0; s < n_seeds; ++s) {
    if (seed_event[s] < 0 || seed_event[s] >= c->n_events) return arg_err(c, "seed event out of range");
    if (!is_fin(theta[s]) || !is_fin(z[s]) || !is_fin(px[s]) || !is_fin(py[s]) || !is_fin(pz[s]))
      return arg_err(c, "non-finite seed " + std::to_string(s));
  }
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t a, int64_t b) { return seed_event[a] < seed_event[b]; });
  std::vector<double> sorted((size_t)std::max<int64_t>(n_seeds, 1) * 5);
  for (int64_t i = 0; i < n_seeds; ++i) {
    const int64_t s = order[i];
    sorted[5 * i + 0] = theta[s];
    sorted[5 * i + 1] = z[s];
    sorted[5 * i + 2] = px[s];
    sorted[5 * i + 3] = py[s];
    sorted[5 * i + 4] = pz[s];
  }
  std::vector<rkn::WindowDev> wins(1);
  std::vector<rkn::Tile> tiles;
  std::vector<int32_t> ev_tiles(c->n_events + 1, 0);
  const int T = rkn::scan_tile(c, p);
  int last_ev = -1;
  for (int64_t i = 0; i < n_seeds;) {
    const int ev = seed_event[order[i]];
    int64_t j = i;
    while (j < n_seeds && seed_event[order[j]] == ev) ++j;
    for (int e = last_ev + 1; e <= ev; ++e) ev_tiles[e] = (int32_t)tiles.size();
    last_ev = ev;
    for (int64_t s = i; s < j; s += T) {
      rkn::Tile t{};
      t.window = 0;
      t.event = ev;
      t.n = (int32_t)std::min<int64_t>(T, j - s);
      t.start = s;
      t.gbase = s;
      tiles.push_back(t);
    }
    i = j;
  }
  for (int e = last_ev + 1; e <= c->n_events; ++e) ev_tiles[e] = (int32_t)tiles.size();
  RKN_HIP(hipSetDevice(c->device), "hipSetDevice");
  RKN_HIP(upload(c->seeds_buf, sorted.data(), sorted.size(), c->stream), "seed upload");
  RKN_HIP(upload(c->perm_buf, order.data(), (size_t)std::max<int64_t>(n_seeds, 1), c->stream), "seed upload");
  return run_scan(c, p, wins, tiles, ev_tiles, n_seeds, score, n_in, best_index, best_score,
                  c->seeds_buf.as<double>(), c->perm_buf.as<int64_t>());
}

rkn_status rkn_trace(rkn_ctx* c, const rkn_scan_params* p, int64_t n_seeds, const double* seeds5,
                     int32_t n_sel, const int32_t* step_idx, double* states) {
  if (!c) return RKN_E_ARG;
  rkn_status st = check_scan_params(c, p);
  if (st != RKN_OK) return st;
  if (c->field_kind < 0) {
    c->err = "no field uploaded";
    return RKN_E_STATE;
  }
  if (n_seeds < 0 || n_sel < 0 || (n_seeds > 0 && !seeds5) || (n_sel > 0 && !step_idx) ||
      (n_seeds > 0 && n_sel > 0 && !states))
    return arg_err(c, "bad trace arrays");
  for (int k = 0; k < n_sel; ++k)
    if (step_idx[k] < 0 || (k > 0 && step_idx[k] < step_idx[k - 1]))
      return arg_err(c, "step_idx must be non-negative and non-decreasing");
  for (int64_t i = 0; i < 5 * n_seeds; ++i)
    if (!is_fin(seeds5[i])) return arg_err(c, "non-finite seed");
  if (n_seeds == 0 || n_sel == 0) return RKN_OK;
  const bool dev = (p->ptr_flags & RKN_PTR_DEVICE) != 0;
  RKN_HIP(hipSetDevice(c->device), "hipSetDevice");
  DevBuf d_steps;
  RKN_HIP(upload(c->seeds_buf, seeds5, (size_t)n_seeds * 5, c->stream), "trace upload");
  RKN_HIP(upload(d_steps, step_idx, (size_t)n_sel, c->stream), "trace upload");
  double* d_out = states;
  if (!dev) {
    RKN_HIP(c->trace_buf.ensure(sizeof(double) * (size_t)n_seeds * n_sel * 6), "alloc");
    d_out = c->trace_buf.as<double>();
  }
  RKN_HIP(rkn::launch_trace(c, p, n_seeds, c->seeds_buf.as<double>(), n_sel, d_steps.as<int32_t>(), d_out),
          "trace launch");
  if (!dev) RKN_HIP(deliver(c, states, (const double*)d_out, (size_t)n_seeds * n_sel * 6, false), "copy states");
  RKN_HIP(hipStreamSynchronize(c->stream), "trace");
  d_steps.release();
  return RKN_OK;
}

}  // extern "C"
