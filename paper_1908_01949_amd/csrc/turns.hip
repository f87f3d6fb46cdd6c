// Turn partitions of a track (section 2.3, full event reconstruction): the seed of a
// neighbouring turn partition predicted by extrapolating a fitted track, and the
// reconstruction loop that finds an event's partitions one after the other.
//
// A turn partition is one pass of the track through the chamber: it starts where
// the track crosses the seed cylinder r = R0 outwards (its entrance) and ends at the
// first step inside r < R0 (every scan of the loop runs with that stop rule). The
// loop starts from the Hough windows of all hits, keeps a few lowest-E seeds, fits
// them by Gauss-Newton (standing in for the Kalman fit), classifies the hits (D -
// d)^2 < lambda_c of the best fit and removes them; then, on both sides of the
// partitions found so far, it predicts the neighbouring partition's seed from the
// outermost fitted seed, scans a window around the prediction, fits and classifies
// again (the side that classifies more hits keeps them first), until fewer than
// min_hits hits are left unclassified or no side finds a partition.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "internal.hpp"

namespace rkn {

// One thread per seed, FP64. From an entrance seed the track (dir = +1) or the
// time-reversed track (dir = -1: direction and charge reversed, so Lambda changes
// sign) is propagated until it crosses r = R0 for the second time after its first
// step: first it leaves the side the first step reached, then it comes back. The
// crossing inside that step is located by bisection on the length of a partial step
// from the state before it; the seed there keeps |p0| and, for dir = -1, the
// direction of the original (not the reversed) track.
template <int FIELD>
__global__ void __launch_bounds__(256)
neighbour_kernel(FieldDev f, double R0, double charge, double hstep, int dir, int max_steps, int64_t n,
                 const double* __restrict__ seeds, double* __restrict__ out, int32_t* __restrict__ found) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const double* v = seeds + 5 * s;
  double* o = out + 5 * s;
  found[s] = 0;
  for (int d = 0; d < 5; ++d) o[d] = NAN;
  const double pm = sqrt(v[2] * v[2] + v[3] * v[3] + v[4] * v[4]);
  if (!(pm >= 1e-3) || !(fabs(v[0]) < 1e3) || !(fabs(v[1]) < 1e7)) return;
  const double sg = dir < 0 ? -1.0 : 1.0;
  State<double> st;
  st.x = R0 * cos(v[0]);
  st.y = R0 * sin(v[0]);
  st.z = v[1];
  st.tx = sg * v[2] / pm;
  st.ty = sg * v[3] / pm;
  st.tz = sg * v[4] / pm;
  st.lam = sg * kKappa * charge / pm;
  st.cx = st.cy = st.cz = 0.0;
  st.ctx = st.cty = st.ctz = 0.0;
  const double r0sq = R0 * R0;
  bool side = false;
  int changes = 0;
  for (int k = 0; k < max_steps; ++k) {
    const State<double> prev = st;
    rkn_step<double, FIELD>(st, f, f.nodes, hstep);
    const bool in = st.x * st.x + st.y * st.y < r0sq;
    if (k == 0) {
      side = in;
      continue;
    }
    if (in == side) continue;
    side = in;
    if (++changes < 2) continue;
    const bool in_lo = prev.x * prev.x + prev.y * prev.y < r0sq;
    double lo = 0.0, hi = hstep;
    State<double> q;
    for (int it = 0; it < 64; ++it) {
      const double mid = 0.5 * (lo + hi);
      q = prev;
      rkn_step<double, FIELD>(q, f, f.nodes, mid);
      if ((q.x * q.x + q.y * q.y < r0sq) == in_lo)
        lo = mid;
      else
        hi = mid;
    }
    q = prev;
    rkn_step<double, FIELD>(q, f, f.nodes, 0.5 * (lo + hi));
    o[0] = atan2(q.y, q.x);
    o[1] = q.z;
    o[2] = sg * pm * q.tx;
    o[3] = sg * pm * q.ty;
    o[4] = sg * pm * q.tz;
    found[s] = 1;
    return;
  }
}

hipError_t launch_neighbour(rkn_ctx* c, const rkn_scan_params* p, int dir, int max_steps, int64_t n,
                            const double* d_seeds, double* d_out, int32_t* d_found) {
  if (n == 0) return hipSuccess;
  const FieldDev f = field_dev(c);
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  if (c->field_kind == 0)
    hipLaunchKernelGGL((neighbour_kernel<0>), grid, block, 0, c->stream, f, p->R0, p->charge, p->step_mm, dir,
                       max_steps, n, d_seeds, d_out, d_found);
  else
    hipLaunchKernelGGL((neighbour_kernel<1>), grid, block, 0, c->stream, f, p->R0, p->charge, p->step_mm, dir,
                       max_steps, n, d_seeds, d_out, d_found);
  return hipGetLastError();
}

}  // namespace rkn

using namespace rkn;

namespace {

rkn_status herr(rkn_ctx* c, hipError_t e, const char* where) {
  c->err = std::string(where) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? RKN_E_NOMEM : RKN_E_DEVICE;
}

bool scan_params_ok(const rkn_scan_params* p) {
  return p && p->n_steps >= 1 && p->step_mm > 0 && p->lambda_mm2 >= 0 && p->R0 > 0 && std::isfinite(p->charge) &&
         p->charge != 0 && !(p->ptr_flags & ~RKN_PTR_DEVICE) && (p->turn_stop == 0 || p->turn_stop == 1) &&
         (p->precision == 32 || p->precision == 64);
}

// Predictions for n host seeds through the device (one small launch).
rkn_status predict(rkn_ctx* c, const rkn_scan_params* p, int dir, int max_steps, const std::vector<double>& seeds,
                   std::vector<double>& out, std::vector<int32_t>& found) {
  const size_t n = seeds.size() / 5;
  out.assign(5 * n, NAN);
  found.assign(n, 0);
  if (n == 0) return RKN_OK;
  DevBuf d_in, d_out, d_found;
  hipError_t e;
  if ((e = d_in.ensure(sizeof(double) * 5 * n)) != hipSuccess || (e = d_out.ensure(sizeof(double) * 5 * n)) != hipSuccess ||
      (e = d_found.ensure(sizeof(int32_t) * n)) != hipSuccess)
    return herr(c, e, "neighbour alloc");
  e = hipMemcpyAsync(d_in.p, seeds.data(), sizeof(double) * 5 * n, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = launch_neighbour(c, p, dir, max_steps, (int64_t)n, d_in.as<double>(), d_out.as<double>(),
                         d_found.as<int32_t>());
  if (e == hipSuccess)
    e = hipMemcpyAsync(out.data(), d_out.p, sizeof(double) * 5 * n, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(found.data(), d_found.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return herr(c, e, "neighbour");
  return RKN_OK;
}

// One side of the loop's state per event.
struct Side {
  bool alive = false;
  int pos = 0;
  double seed[5];
};

struct EventState {
  bool done = false;
  int n_turns = 0;
  int remaining = 0;
  Side lo, hi;   // the earliest and the latest partition found along the track
};

// Partition candidates, grouped by event: the event, the centre of the window each
// came from and the current seed.
struct Cands {
  std::vector<int32_t> ev;
  std::vector<double> center, seed;
  size_t size() const { return ev.size(); }
  void add(int e, const double* c5, const double* s5) {
    ev.push_back(e);
    center.insert(center.end(), c5, c5 + 5);
    seed.insert(seed.end(), s5, s5 + 5);
  }
};

}  // namespace

extern "C" {

rkn_status rkn_neighbour_seeds(rkn_ctx* c, const rkn_scan_params* p, int64_t n_seeds, const double* seeds5,
                               int32_t direction, int32_t max_steps, double* out5, int32_t* found) {
  if (!c) return RKN_E_ARG;
  if (!scan_params_ok(p) || (direction != 1 && direction != -1) || max_steps < 1 || n_seeds < 0 ||
      n_seeds > (int64_t(1) << 24) || (n_seeds > 0 && (!seeds5 || !out5 || !found))) {
    c->err = "neighbour seeds: invalid arguments";
    return RKN_E_ARG;
  }
  if (c->field_kind < 0) {
    c->err = "neighbour seeds: upload the field first";
    return RKN_E_STATE;
  }
  if (n_seeds == 0) return RKN_OK;
  hipError_t e;
  if ((e = hipSetDevice(c->device)) != hipSuccess) return herr(c, e, "hipSetDevice");
  const size_t n = (size_t)n_seeds;
  const bool dev = (p->ptr_flags & RKN_PTR_DEVICE) != 0;
  DevBuf d_in, d_out, d_found;
  if ((e = d_in.ensure(sizeof(double) * 5 * n)) != hipSuccess) return herr(c, e, "neighbour alloc");
  if (!dev && ((e = d_out.ensure(sizeof(double) * 5 * n)) != hipSuccess ||
               (e = d_found.ensure(sizeof(int32_t) * n)) != hipSuccess))
    return herr(c, e, "neighbour alloc");
  double* o = dev ? out5 : d_out.as<double>();
  int32_t* fo = dev ? found : d_found.as<int32_t>();
  e = hipMemcpyAsync(d_in.p, seeds5, sizeof(double) * 5 * n, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = launch_neighbour(c, p, direction, max_steps, n_seeds, d_in.as<double>(), o, fo);
  if (e == hipSuccess && !dev) {
    e = hipMemcpyAsync(out5, o, sizeof(double) * 5 * n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(found, fo, sizeof(int32_t) * n, hipMemcpyDeviceToHost, c->stream);
  }
  // the staging buffers are freed on return: wait for the launch either way
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return herr(c, e, "neighbour seeds");
  return RKN_OK;
}

rkn_status rkn_find_turns(rkn_ctx* c, const rkn_hough_params* hp, const rkn_scan_params* sp,
                          const rkn_turn_params* tp, int32_t* hit_turn, int32_t* n_turns, double* turn_seed,
                          double* turn_center, int32_t* turn_pos, int32_t* turn_nhits) {
  if (!c) return RKN_E_ARG;
  if (!hp || !tp || !scan_params_ok(sp) || sp->precision != 32 || !hit_turn || !n_turns) {
    c->err = "find turns: need hough, FP32 scan and turn parameters and the hit_turn/n_turns outputs";
    return RKN_E_ARG;
  }
  if (hp->charge != sp->charge || hp->R0 != sp->R0) {
    c->err = "find turns: the Hough and scan parameters must have the same charge and R0";
    return RKN_E_ARG;
  }
  int64_t wsize = 1;
  for (int d = 0; d < 5; ++d) {
    if (tp->count[d] < 1 || !(tp->half_width[d] >= 0) || !std::isfinite(tp->half_width[d]) ||
        !(tp->gn_scale[d] > 0) || !std::isfinite(tp->gn_scale[d])) {
      c->err = "find turns: window counts >= 1, finite half-widths >= 0, scales > 0";
      return RKN_E_ARG;
    }
    wsize *= tp->count[d];
  }
  int64_t fsize = 1;
  for (int d = 0; d < 2; ++d) {
    if (tp->fine_count[d] < 1 || !(tp->fine_half_width[d] >= 0) || !std::isfinite(tp->fine_half_width[d])) {
      c->err = "find turns: fine counts >= 1 and finite fine half-widths >= 0";
      return RKN_E_ARG;
    }
    fsize *= tp->fine_count[d];
  }
  if (wsize > 4000000 || fsize > 1000000 || tp->max_turns < 1 || tp->max_turns > RKN_TURNS_MAX ||
      tp->min_hits < 1 || tp->gn_iters < 0 || tp->gn_iters > 100 || !(tp->lambda_classify_mm2 > 0) ||
      tp->max_extrap_steps < 1 || tp->n_candidates < 1 || tp->n_candidates > RKN_TOPK_MAX) {
    c->err = "find turns: windows of at most 4e6 (fine: 1e6) seeds, 1 <= max_turns <= RKN_TURNS_MAX, "
             "min_hits >= 1, 0 <= gn_iters <= 100, lambda_classify > 0, max_extrap_steps >= 1, "
             "1 <= n_candidates <= RKN_TOPK_MAX";
    return RKN_E_ARG;
  }
  if (c->n_wires == 0 || c->field_kind < 0 || c->h_ev_off.empty()) {
    c->err = "find turns: upload geometry, field and hits first";
    return RKN_E_STATE;
  }
  hipError_t e;
  if ((e = hipSetDevice(c->device)) != hipSuccess) return herr(c, e, "hipSetDevice");

  // the event set the caller uploaded; the loop replaces the context's hits by the
  // unclassified ones before each neighbour scan and restores these at the end
  const int ne = c->n_events;
  const std::vector<int32_t> off0 = c->h_ev_off;
  const std::vector<int32_t> wire0 = c->h_wire;
  const std::vector<float> drift0 = c->h_drift;
  const int T = tp->max_turns;
  const int K = tp->n_candidates;
  std::vector<int32_t> label(wire0.size(), -1);
  std::vector<EventState> evs(ne);
  for (int e2 = 0; e2 < ne; ++e2) evs[e2].remaining = off0[e2 + 1] - off0[e2];
  std::vector<double> seeds_out((size_t)ne * T * 5, NAN), centers_out((size_t)ne * T * 5, NAN);
  std::vector<int32_t> pos_out((size_t)ne * T, 0), nhits_out((size_t)ne * T, 0);
  std::vector<std::vector<int32_t>> cur(ne);   // per event: global indices of the uploaded hits

  rkn_scan_params s1 = *sp;                    // the scan: lambda of sp, stop at the turn's end
  s1.turn_stop = 1;
  s1.ptr_flags = 0;
  rkn_scan_params sc = s1;                     // classification and the fine stages
  sc.lambda_mm2 = tp->lambda_classify_mm2;

  auto upload_remaining = [&]() -> rkn_status {
    std::vector<int32_t> off(ne + 1, 0), wid;
    std::vector<float> dr;
    for (int e2 = 0; e2 < ne; ++e2) {
      cur[e2].clear();
      for (int i = off0[e2]; i < off0[e2 + 1]; ++i)
        if (label[i] < 0) {
          cur[e2].push_back(i);
          wid.push_back(wire0[i]);
          dr.push_back(drift0[i]);
        }
      off[e2 + 1] = off[e2] + (int32_t)cur[e2].size();
    }
    return rkn_upload_hits(c, ne, off.data(), wid.data(), dr.data());
  };
  auto restore = [&]() { rkn_upload_hits(c, ne, off0.data(), wire0.data(), drift0.data()); };

  // Gauss-Newton of every candidate with its inlier set fixed by the cutoff q
  auto fit = [&](Cands& cd, const rkn_scan_params& q) -> rkn_status {
    if (tp->gn_iters == 0 || cd.size() == 0) return RKN_OK;
    rkn_status st2 = rkn_refine_setup(c, &q, (int64_t)cd.size(), cd.ev.data(), cd.seed.data(), 64);
    if (st2 != RKN_OK) return st2;
    std::vector<double> out(cd.seed.size());
    st2 = rkn_gn_refine(c, tp->gn_iters, tp->gn_scale, out.data(), nullptr);
    if (st2 == RKN_OK) cd.seed.swap(out);
    return st2;
  };

  // per event, the best seed of the windows (-1 when the event has none)
  auto scan_best = [&](const rkn_scan_params& q, const std::vector<rkn_window>& w, int k,
                       std::vector<int64_t>& idx, std::vector<double>& best5) -> rkn_status {
    idx.assign((size_t)ne * k, -1);
    best5.assign((size_t)ne * k * 5, NAN);
    std::vector<double> scores((size_t)ne * k);
    return rkn_scan_windows_topk(c, &q, (int32_t)w.size(), w.data(), k, idx.data(), scores.data(), best5.data());
  };

  // classify the fitted candidates (any rows, any events) at the fine cutoff
  auto classify_rows = [&](const Cands& cd, std::vector<uint8_t>& mask, std::vector<int32_t>& nin,
                           int& H) -> rkn_status {
    const int64_t n = (int64_t)cd.size();
    H = c->max_hits_event > 0 ? c->max_hits_event : 1;
    mask.assign((size_t)n * H, 0);
    nin.assign(n, 0);
    if (n == 0) return RKN_OK;
    return rkn_classify_hits(c, &sc, n, cd.ev.data(), cd.seed.data(), mask.data(), nin.data());
  };

  // keep or not the classified candidates, in the given row order: a row's partition is
  // the hits of its mask still unclassified when its turn comes, kept when there are
  // at least min_hits of them; dirs[i] 0 is the first partition of an event, -1/+1
  // extend its earlier/later side
  auto keep = [&](const Cands& cd, const std::vector<int>& dirs, const std::vector<int64_t>& order,
                  const std::vector<uint8_t>& mask, int H) {
    for (int64_t i : order) {
      const int e2 = cd.ev[i];
      const int dir = dirs[i];
      EventState& es = evs[e2];
      if (es.done) continue;
      const uint8_t* m = mask.data() + (size_t)i * H;
      int k = 0;
      for (size_t o = 0; o < cur[e2].size(); ++o) k += (m[o] && label[cur[e2][o]] < 0) ? 1 : 0;
      if (k < tp->min_hits) {
        if (dir == 0) es.done = true;
        if (dir < 0) es.lo.alive = false;
        if (dir > 0) es.hi.alive = false;
        continue;
      }
      const int t = es.n_turns++;
      for (size_t o = 0; o < cur[e2].size(); ++o)
        if (m[o] && label[cur[e2][o]] < 0) label[cur[e2][o]] = t;
      es.remaining -= k;
      const int pos = dir == 0 ? 0 : (dir < 0 ? es.lo.pos - 1 : es.hi.pos + 1);
      const size_t b = (size_t)e2 * T + t;
      const double* f5 = &cd.seed[5 * i];
      std::copy(f5, f5 + 5, &seeds_out[5 * b]);
      std::copy(&cd.center[5 * i], &cd.center[5 * i] + 5, &centers_out[5 * b]);
      pos_out[b] = pos;
      nhits_out[b] = k;
      if (dir <= 0) {
        es.lo.alive = true;
        es.lo.pos = pos;
        std::copy(f5, f5 + 5, es.lo.seed);
      }
      if (dir >= 0) {
        es.hi.alive = true;
        es.hi.pos = pos;
        std::copy(f5, f5 + 5, es.hi.seed);
      }
      if (es.remaining < tp->min_hits || es.n_turns >= T) es.done = true;
    }
  };

  auto accept = [&](const Cands& cd, int dir) -> rkn_status {
    std::vector<uint8_t> mask;
    std::vector<int32_t> nin;
    int H = 1;
    rkn_status st2 = classify_rows(cd, mask, nin, H);
    if (st2 != RKN_OK) return st2;
    std::vector<int64_t> order(cd.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int64_t)i;
    keep(cd, std::vector<int>(cd.size(), dir), order, mask, H);
    return RKN_OK;
  };

  rkn_status st = RKN_OK;
  // ---- first partition: the K lowest-E seeds of the Hough windows of every hit;
  // each is fitted at the scan's cutoff, rescanned over a fine (z0, pz0) grid and
  // fitted again at the classification cutoff; per event the fitted candidate with
  // the lowest E at that cutoff is kept
  for (int e2 = 0; e2 < ne; ++e2) {
    cur[e2].clear();
    for (int i = off0[e2]; i < off0[e2 + 1]; ++i) cur[e2].push_back(i);
    if (evs[e2].remaining < tp->min_hits) evs[e2].done = true;
  }
  {
    int32_t nw = 0;
    std::vector<rkn_window> w;
    st = rkn_hough_seed_windows(c, hp, 0, nullptr, &nw);   // the count first
    if (st == RKN_E_CAPACITY && nw > 0) {
      w.resize(nw);
      st = rkn_hough_seed_windows(c, hp, nw, w.data(), &nw);
    }
    if (st != RKN_OK) return st;
    Cands cd;
    if (nw > 0) {
      std::vector<int64_t> idx;
      std::vector<double> best5;
      if ((st = scan_best(s1, w, K, idx, best5)) != RKN_OK) return st;
      std::vector<int64_t> base(nw + 1, 0);   // the window that holds a seed gives its centre
      for (int k = 0; k < nw; ++k) {
        int64_t sz = 1;
        for (int d = 0; d < 5; ++d) sz *= w[k].count[d];
        base[k + 1] = base[k] + sz;
      }
      for (int e2 = 0; e2 < ne; ++e2)
        for (int j = 0; j < K; ++j) {
          const int64_t g = idx[(size_t)e2 * K + j];
          if (evs[e2].done || g < 0) continue;
          const int k = (int)(std::upper_bound(base.begin(), base.end(), g) - base.begin()) - 1;
          cd.add(e2, w[k].center, &best5[((size_t)e2 * K + j) * 5]);
        }
    }
    for (int e2 = 0; e2 < ne; ++e2)
      if (std::find(cd.ev.begin(), cd.ev.end(), e2) == cd.ev.end()) evs[e2].done = true;
    if ((st = fit(cd, s1)) != RKN_OK) return st;
    if (fsize > 1 && cd.size() > 0) {
      // candidates of one rank form one window per event, so each gets its own best
      std::vector<int> rank(cd.size());
      for (size_t i = 0; i < cd.size(); ++i) rank[i] = (i > 0 && cd.ev[i] == cd.ev[i - 1]) ? rank[i - 1] + 1 : 0;
      for (int j = 0; j < K; ++j) {
        std::vector<rkn_window> fw;
        std::vector<size_t> who;
        for (size_t i = 0; i < cd.size(); ++i) {
          if (rank[i] != j) continue;
          rkn_window wi{};
          wi.event = cd.ev[i];
          for (int d = 0; d < 5; ++d) {
            wi.center[d] = cd.seed[5 * i + d];
            wi.count[d] = 1;
          }
          wi.half_width[1] = tp->fine_half_width[0];
          wi.half_width[4] = tp->fine_half_width[1];
          wi.count[1] = tp->fine_count[0];
          wi.count[4] = tp->fine_count[1];
          fw.push_back(wi);
          who.push_back(i);
        }
        if (fw.empty()) continue;
        std::vector<int64_t> idx;
        std::vector<double> best5;
        if ((st = scan_best(sc, fw, 1, idx, best5)) != RKN_OK) return st;
        for (size_t q = 0; q < who.size(); ++q) {
          const int e2 = fw[q].event;
          if (idx[e2] >= 0) std::copy(&best5[5 * (size_t)e2], &best5[5 * (size_t)e2] + 5, &cd.seed[5 * who[q]]);
        }
      }
    }
    if ((st = fit(cd, sc)) != RKN_OK) return st;
    Cands chosen;
    if (cd.size() > 0) {
      const size_t n = cd.size();
      std::vector<double> th(n), z(n), px(n), py(n), pz(n), score(n);
      for (size_t i = 0; i < n; ++i) {
        th[i] = cd.seed[5 * i];
        z[i] = cd.seed[5 * i + 1];
        px[i] = cd.seed[5 * i + 2];
        py[i] = cd.seed[5 * i + 3];
        pz[i] = cd.seed[5 * i + 4];
      }
      std::vector<int64_t> bi(ne);
      std::vector<double> bs(ne);
      if ((st = rkn_scan_seeds(c, &sc, (int64_t)n, cd.ev.data(), th.data(), z.data(), px.data(), py.data(),
                               pz.data(), score.data(), nullptr, bi.data(), bs.data())) != RKN_OK)
        return st;
      for (int e2 = 0; e2 < ne; ++e2)
        if (bi[e2] >= 0) chosen.add(e2, &cd.center[5 * bi[e2]], &cd.seed[5 * bi[e2]]);
    }
    if ((st = accept(chosen, 0)) != RKN_OK) {
      restore();
      return st;
    }
  }
  // ---- neighbouring partitions: on both sides, the predicted seed, a window scan over
  // the unclassified hits and fits at the scan's and the classification cutoffs; both
  // sides' candidates are classified on the same hits and, per event, the one that
  // classifies more of them is kept first, the other keeps what is left (a hit gets
  // one partition)
  for (int round = 1; round < T; ++round) {
    bool any = false;
    Cands all;
    std::vector<int> dirs;
    bool uploaded = false;
    for (int dir = -1; dir <= 1; dir += 2) {
      std::vector<int> evl;
      std::vector<double> from;
      for (int e2 = 0; e2 < ne; ++e2) {
        const EventState& es = evs[e2];
        const Side& sd = dir < 0 ? es.lo : es.hi;
        if (es.done || !sd.alive) continue;
        evl.push_back(e2);
        from.insert(from.end(), sd.seed, sd.seed + 5);
      }
      if (evl.empty()) continue;
      any = true;
      std::vector<double> pred;
      std::vector<int32_t> found;
      if ((st = predict(c, &s1, dir, tp->max_extrap_steps, from, pred, found)) != RKN_OK) break;
      if (!uploaded) {
        if ((st = upload_remaining()) != RKN_OK) break;
        uploaded = true;
      }
      std::vector<rkn_window> w;
      for (size_t i = 0; i < evl.size(); ++i) {
        EventState& es = evs[evl[i]];
        if (!found[i]) {
          (dir < 0 ? es.lo : es.hi).alive = false;
          continue;
        }
        rkn_window wi{};
        wi.event = evl[i];
        for (int d = 0; d < 5; ++d) {
          wi.center[d] = pred[5 * i + d];
          wi.half_width[d] = tp->half_width[d];
          wi.count[d] = tp->count[d];
        }
        w.push_back(wi);
      }
      if (w.empty()) continue;
      std::vector<int64_t> idx;
      std::vector<double> best5;
      if ((st = scan_best(s1, w, 1, idx, best5)) != RKN_OK) break;
      Cands cd;
      for (const auto& wi : w) {
        const int e2 = wi.event;
        if (idx[e2] < 0) {
          (dir < 0 ? evs[e2].lo : evs[e2].hi).alive = false;
          continue;
        }
        cd.add(e2, wi.center, &best5[5 * (size_t)e2]);
      }
      if ((st = fit(cd, s1)) != RKN_OK || (st = fit(cd, sc)) != RKN_OK) break;
      for (size_t i = 0; i < cd.size(); ++i) {
        all.add(cd.ev[i], &cd.center[5 * i], &cd.seed[5 * i]);
        dirs.push_back(dir);
      }
    }
    if (st != RKN_OK || !any) break;
    std::vector<uint8_t> mask;
    std::vector<int32_t> nin;
    int H = 1;
    if ((st = classify_rows(all, mask, nin, H)) != RKN_OK) break;
    std::vector<int64_t> order(all.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int64_t)i;
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
      if (all.ev[a] != all.ev[b]) return all.ev[a] < all.ev[b];
      return nin[a] > nin[b];
    });
    keep(all, dirs, order, mask, H);
  }
  restore();
  if (st != RKN_OK) return st;
  std::copy(label.begin(), label.end(), hit_turn);
  for (int e2 = 0; e2 < ne; ++e2) n_turns[e2] = evs[e2].n_turns;
  if (turn_seed) std::copy(seeds_out.begin(), seeds_out.end(), turn_seed);
  if (turn_center) std::copy(centers_out.begin(), centers_out.end(), turn_center);
  if (turn_pos) std::copy(pos_out.begin(), pos_out.end(), turn_pos);
  if (turn_nhits) std::copy(nhits_out.begin(), nhits_out.end(), turn_nhits);
  return RKN_OK;
}

}  // extern "C"
