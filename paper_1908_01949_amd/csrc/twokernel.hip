// The paper's two-kernel form of the scan (section 4.2), kept beside the fused scan
// kernel as an experiment: a record kernel propagates every seed and stores its
// position after each RKN step, and a DCA kernel gives each fired wire of the seed's
// event its own lane (one wave per seed, as the paper gives one thread per wire),
// which finds the wire's distance of closest approach from the recorded chords.
// Both use the fused kernel's FP32 state, step and chord/wire distance, so the
// scores agree with it to rounding; what differs is the work layout: the trajectory
// goes through HBM (12 bytes per seed and step) and the lanes of a wave diverge on
// the blocks where their wires are reached.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "internal.hpp"

namespace rkn {

constexpr int kRecBlock = 8;          // steps per pruning block of the DCA kernel
constexpr size_t kTrajBudget = size_t(4) << 30;   // bytes of recorded trajectories per chunk

// One lane per seed: the seed of global index s0 + k decoded from its window, then
// n_steps RKN steps; traj[k][j][3] = position after step j (j = 0: the seed point).
// With turn_stop the state freezes at the first step inside r < R0. seed_win[k] = the
// window, or -1 for a seed with |p| < 1e-3 MeV/c.
template <int FIELD>
__global__ void __launch_bounds__(256)
record_kernel(FieldDev f, const WindowDev* __restrict__ wins, const int64_t* __restrict__ win_base, int n_windows,
              int64_t s0, int64_t n, double R0, double charge, double hstep, int n_steps, int turn_stop,
              int fold, float* __restrict__ traj, int32_t* __restrict__ seed_win) {
  extern __shared__ float2 s_field[];
  const float2* nodes = f.nodes;
  if constexpr (FIELD == 1) {
    const int nn = (int)padded_field_nodes(f.nr, f.nz);
    for (int i = threadIdx.x; i < nn; i += blockDim.x) s_field[i] = f.nodes[i];
    __syncthreads();
    nodes = s_field;
  }
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t g = s0 + k;
  int lo = 0, hi = n_windows;   // the window with win_base[w] <= g < win_base[w + 1]
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (win_base[mid] <= g)
      lo = mid;
    else
      hi = mid;
  }
  double v[5];
  window_seed(wins[lo], g - win_base[lo], v);
  const double pm = sqrt(v[2] * v[2] + v[3] * v[3] + v[4] * v[4]);
  const bool valid = pm >= 1e-3;
  const double ipm = valid ? 1.0 / pm : 0.0;
  State<float> st;
  st.x = (float)(R0 * cos(v[0]));
  st.y = (float)(R0 * sin(v[0]));
  st.z = (float)v[1];
  st.tx = valid ? (float)(v[2] * ipm) : 1.0f;
  st.ty = valid ? (float)(v[3] * ipm) : 0.0f;
  st.tz = valid ? (float)(v[4] * ipm) : 0.0f;
  st.lam = valid ? (float)(kKappa * charge * ipm) : 0.0f;
  st.cx = st.cy = st.cz = 0.0f;
  st.ctx = st.cty = st.ctz = 0.0f;
  seed_win[k] = valid ? lo : -1;
  const float h = (float)hstep;
  const float r0sq = (float)(R0 * R0);
  float* out = traj + (size_t)k * (size_t)(n_steps + 1) * 3;
  out[0] = st.x;
  out[1] = st.y;
  out[2] = st.z;
  // the fused scan's propagation: block-relative sums folded at the ends of its
  // blocks of `fold` steps (while the track was live at the block's start)
  Prop<float, FIELD> pr;
  pr.start(st);
  pr.init_field(st, f, nodes);
  bool live = true, live_blk = true;
  for (int j = 1; j <= n_steps; ++j) {
    if (live) {
      pr.step(st, f, nodes, h);
      live = !(turn_stop && inside_r0(pr.px, pr.py, r0sq));
    }
    if (j % fold == 0 || j == n_steps) {
      if (live_blk) pr.fold(st);
      live_blk = live;
    }
    out[3 * j + 0] = pr.px;
    out[3 * j + 1] = pr.py;
    out[3 * j + 2] = pr.pz;
  }
}

// One wave per seed, one lane per hit of its event (64 at a time). Per hit: every
// block of kRecBlock recorded chords whose middle point lies within the block's
// reach (kRecBlock h / 2 + sqrt(lambda) + 0.05 mm + d) of the wire's line is
// searched chord by chord; then E (Eq. 1, FP64) and n_in summed over the wave.
__global__ void __launch_bounds__(256)
dca_kernel(const HitRec<float>* __restrict__ hits, const int32_t* __restrict__ ev_off,
           const WindowDev* __restrict__ wins, const float* __restrict__ traj, const int32_t* __restrict__ seed_win,
           int64_t s0, int64_t n, int n_steps, double hstep, double lambda, double* __restrict__ score,
           int32_t* __restrict__ nin) {
  const int lane = threadIdx.x & 63;
  const int64_t k = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  if (k >= n) return;   // whole waves leave together; no barrier follows
  const int w = seed_win[k];
  if (w < 0) {
    if (lane == 0) {
      score[s0 + k] = INFINITY;
      if (nin) nin[s0 + k] = 0;
    }
    return;
  }
  const int ev = wins[w].event;
  const int hbase = ev_off[ev], nh = ev_off[ev + 1] - hbase;
  const float* T = traj + (size_t)k * (size_t)(n_steps + 1) * 3;
  const float kc = (float)(0.5 * kRecBlock * hstep + sqrt(lambda) + 0.05);
  double E = 0.0;
  int cnt = 0;
  for (int i = lane; i < nh; i += 64) {
    const HitRec<float> hr = hits[hbase + i];
    const float thr = kc + hr.drift;
    float best = INFINITY;
    for (int b0 = 0; b0 < n_steps; b0 += kRecBlock) {
      const int nb = min(kRecBlock, n_steps - b0);
      const float* c = T + 3 * (b0 + nb / 2);
      const float rx = c[0] - hr.mx, ry = c[1] - hr.my, rz = c[2] - hr.mz;
      const float t = rx * hr.ux + ry * hr.uy + rz * hr.uz;
      const float d2 = rx * rx + ry * ry + rz * rz - t * t;
      if (d2 > thr * thr) continue;
      for (int j = b0; j < b0 + nb; ++j) {
        const float* p = T + 3 * j;
        const float v = seg_wire_d2<float>(p[0], p[1], p[2], p[3], p[4], p[5], hr.mx, hr.my, hr.mz, hr.ux, hr.uy,
                                           hr.uz, hr.L);
        best = v < best ? v : best;
      }
    }
    const double r = sqrt((double)best) - (double)hr.drift;
    const double q = r * r;
    if (q < lambda) {
      E += q;
      ++cnt;
    } else {
      E += lambda;
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    E += __shfl_xor(E, o, 64);
    cnt += __shfl_xor(cnt, o, 64);
  }
  if (lane == 0) {
    score[s0 + k] = E;
    if (nin) nin[s0 + k] = cnt;
  }
}

// Per event: the lowest score of its seed range and its global index (ties: lowest
// index; -1 and +inf for an event without seeds).
__global__ void __launch_bounds__(256)
range_argmin_kernel(const double* __restrict__ score, const int64_t* __restrict__ ev_seed, int64_t* __restrict__ bi,
                    double* __restrict__ be) {
  __shared__ double s_e[256];
  __shared__ int64_t s_i[256];
  const int e = blockIdx.x;
  const int64_t lo = ev_seed[e], hi = ev_seed[e + 1];
  double m = INFINITY;
  int64_t mi = -1;
  for (int64_t s = lo + threadIdx.x; s < hi; s += blockDim.x) {
    const double v = score[s];
    if (v < m || (mi < 0 && !(v != v))) {
      m = v;
      mi = s;
    }
  }
  s_e[threadIdx.x] = m;
  s_i[threadIdx.x] = mi;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if ((int)threadIdx.x < o) {
      const double e2 = s_e[threadIdx.x + o];
      const int64_t i2 = s_i[threadIdx.x + o];
      const bool take = i2 >= 0 && (s_i[threadIdx.x] < 0 || e2 < s_e[threadIdx.x] ||
                                    (e2 == s_e[threadIdx.x] && i2 < s_i[threadIdx.x]));
      if (take) {
        s_e[threadIdx.x] = e2;
        s_i[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    bi[e] = s_i[0];
    be[e] = s_i[0] >= 0 ? s_e[0] : INFINITY;
  }
}

}  // namespace rkn

using namespace rkn;

namespace {

rkn_status terr(rkn_ctx* c, hipError_t e, const char* where) {
  c->err = std::string(where) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? RKN_E_NOMEM : RKN_E_DEVICE;
}

}  // namespace

extern "C" {

rkn_status rkn_scan_windows_two_kernel(rkn_ctx* c, const rkn_scan_params* p, int32_t n_windows, const rkn_window* w,
                                       double* score, int32_t* n_in, int64_t* best_index, double* best_score) {
  if (!c) return RKN_E_ARG;
  if (!p || p->precision != 32 || p->n_steps < 1 || !(p->step_mm > 0) || !(p->lambda_mm2 >= 0) || !(p->R0 > 0) ||
      !std::isfinite(p->charge) || p->charge == 0 || (p->ptr_flags & ~RKN_PTR_DEVICE) ||
      (p->turn_stop != 0 && p->turn_stop != 1) || n_windows < 0 || (n_windows > 0 && !w)) {
    c->err = "two-kernel scan: FP32 scan parameters and a window array";
    return RKN_E_ARG;
  }
  if (c->n_wires == 0 || c->field_kind < 0 || c->h_ev_off.empty()) {
    c->err = "two-kernel scan: upload geometry, field and hits first";
    return RKN_E_STATE;
  }
  const int ne = c->n_events;
  std::vector<WindowDev> wins(std::max(n_windows, 1));
  std::vector<int64_t> base(n_windows + 1, 0), ev_seed(ne + 1, 0);
  int last = -1;
  for (int k = 0; k < n_windows; ++k) {
    const rkn_window& x = w[k];
    if (x.event < 0 || x.event >= ne || x.event < last) {
      c->err = "two-kernel scan: window events must be in range and non-decreasing";
      return RKN_E_ARG;
    }
    int64_t size = 1;
    for (int d = 0; d < 5; ++d) {
      if (x.count[d] < 1 || !std::isfinite(x.center[d]) || !std::isfinite(x.half_width[d]) || x.half_width[d] < 0) {
        c->err = "two-kernel scan: window counts >= 1, finite centres and half-widths >= 0";
        return RKN_E_ARG;
      }
      size *= x.count[d];
      if (size > (int64_t(1) << 40)) {
        c->err = "two-kernel scan: window too large";
        return RKN_E_ARG;
      }
    }
    for (int e2 = last + 1; e2 <= x.event; ++e2) ev_seed[e2] = base[k];
    last = x.event;
    for (int d = 0; d < 5; ++d) {
      wins[k].center[d] = x.center[d];
      wins[k].half_width[d] = x.half_width[d];
      wins[k].count[d] = x.count[d];
    }
    wins[k].event = x.event;
    base[k + 1] = base[k] + size;
  }
  const int64_t total = base[n_windows];
  for (int e2 = last + 1; e2 <= ne; ++e2) ev_seed[e2] = total;
  hipError_t e;
  if ((e = hipSetDevice(c->device)) != hipSuccess) return terr(c, e, "hipSetDevice");
  const bool dev = (p->ptr_flags & RKN_PTR_DEVICE) != 0;
  const size_t per_seed = (size_t)(p->n_steps + 1) * 3 * sizeof(float);
  const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(total, (int64_t)(kTrajBudget / per_seed)));
  DevBuf d_wins, d_base, d_evs, d_traj, d_swin, d_score, d_nin, d_bi, d_be;
  if ((e = d_wins.ensure(sizeof(WindowDev) * wins.size())) != hipSuccess ||
      (e = d_base.ensure(sizeof(int64_t) * base.size())) != hipSuccess ||
      (e = d_evs.ensure(sizeof(int64_t) * ev_seed.size())) != hipSuccess ||
      (e = d_traj.ensure(per_seed * (size_t)chunk)) != hipSuccess ||
      (e = d_swin.ensure(sizeof(int32_t) * (size_t)chunk)) != hipSuccess ||
      (e = d_bi.ensure(sizeof(int64_t) * ne)) != hipSuccess || (e = d_be.ensure(sizeof(double) * ne)) != hipSuccess)
    return terr(c, e, "two-kernel alloc");
  double* o_score = score;
  int32_t* o_nin = n_in;
  if (!dev || !score) {
    if ((e = d_score.ensure(sizeof(double) * (size_t)std::max<int64_t>(total, 1))) != hipSuccess)
      return terr(c, e, "two-kernel alloc");
    o_score = d_score.as<double>();
  }
  if (n_in && !dev) {
    if ((e = d_nin.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(total, 1))) != hipSuccess)
      return terr(c, e, "two-kernel alloc");
    o_nin = d_nin.as<int32_t>();
  }
  e = hipMemcpyAsync(d_wins.p, wins.data(), sizeof(WindowDev) * wins.size(), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_base.p, base.data(), sizeof(int64_t) * base.size(), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_evs.p, ev_seed.data(), sizeof(int64_t) * ev_seed.size(), hipMemcpyHostToDevice, c->stream);
  const FieldDev f = field_dev(c);
  const int fold = resolve_block_steps(c, p);   // the fused scan's block: the same trajectories
  const size_t smem = c->field_kind == 1 ? sizeof(float2) * padded_field_nodes(c->nr, c->nz) : 0;
  if (e == hipSuccess && c->field_kind == 1)
    e = hipFuncSetAttribute((const void*)record_kernel<1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  for (int64_t s0 = 0; e == hipSuccess && s0 < total; s0 += chunk) {
    const int64_t m = std::min(chunk, total - s0);
    const dim3 g1((unsigned)((m + 255) / 256)), b1(256);
    if (c->field_kind == 0)
      hipLaunchKernelGGL(record_kernel<0>, g1, b1, 0, c->stream, f, d_wins.as<WindowDev>(), d_base.as<int64_t>(),
                         n_windows, s0, m, p->R0, p->charge, p->step_mm, p->n_steps, p->turn_stop, fold,
                         d_traj.as<float>(), d_swin.as<int32_t>());
    else
      hipLaunchKernelGGL(record_kernel<1>, g1, b1, smem, c->stream, f, d_wins.as<WindowDev>(), d_base.as<int64_t>(),
                         n_windows, s0, m, p->R0, p->charge, p->step_mm, p->n_steps, p->turn_stop, fold,
                         d_traj.as<float>(), d_swin.as<int32_t>());
    if ((e = hipGetLastError()) != hipSuccess) break;
    hipLaunchKernelGGL(dca_kernel, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, c->stream, c->hits32.as<HitRec<float>>(),
                       c->ev_off.as<int32_t>(), d_wins.as<WindowDev>(), d_traj.as<float>(), d_swin.as<int32_t>(), s0,
                       m, p->n_steps, p->step_mm, p->lambda_mm2, o_score, o_nin);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(range_argmin_kernel, dim3((unsigned)ne), dim3(256), 0, c->stream, o_score,
                       d_evs.as<int64_t>(), d_bi.as<int64_t>(), d_be.as<double>());
    e = hipGetLastError();
  }
  const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (e == hipSuccess && score && !dev && total > 0)
    e = hipMemcpyAsync(score, o_score, sizeof(double) * (size_t)total, kind, c->stream);
  if (e == hipSuccess && n_in && !dev && total > 0)
    e = hipMemcpyAsync(n_in, o_nin, sizeof(int32_t) * (size_t)total, kind, c->stream);
  if (e == hipSuccess && best_index) e = hipMemcpyAsync(best_index, d_bi.p, sizeof(int64_t) * ne, kind, c->stream);
  if (e == hipSuccess && best_score) e = hipMemcpyAsync(best_score, d_be.p, sizeof(double) * ne, kind, c->stream);
  // the staging buffers are freed on return: wait for the work either way
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return terr(c, e, "two-kernel scan");
  return RKN_OK;
}

}  // extern "C"
