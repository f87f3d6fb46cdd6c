// Circle Hough transform over the hit wires and the seed window of each peak
// (Yeo et al., CTD/WIT 2019, section 2.1 and Fig. 4), for gfx950.
//
//  vote:   one lane per centre cell, 256 cells per workgroup; the event's hits
//          (wire waists quantised to 2^-8 mm) sit in LDS; every lane computes the
//          squared distance to each hit exactly (FP64 on integers < 2^53), picks the
//          radius bin with an FP32 estimate corrected by exact edge comparisons, and
//          counts into its private LDS column (no atomics); the column block is then
//          written out coalesced and the workgroup's maximum folded into the
//          event maximum with an integer atomic max (order-free).
//  peaks:  one lane per bin; bins at or above max(min_votes, ceil(max/2)) test their
//          26 neighbours and survivors are appended to a per-event list (4096
//          entries; an event with more peaks is resolved by the select stage).
//  select: one workgroup per event keeps the max_cand best (count desc, flat asc)
//          and turns each into a window (FP64 geometry, integer counts); when the
//          list overflowed it walks the whole accumulator with the peak rule, so the
//          choice never depends on the order of the list's appends.
#include <math.h>

#include <algorithm>
#include <string>
#include <vector>

#include "internal.hpp"

namespace rkn {

constexpr int kHoughCells = 256;
constexpr int kMaxNr = 64;
constexpr int kCandCap = 4096;
constexpr int kEventChunk = 32;

__global__ void __launch_bounds__(kHoughCells)
hough_vote_kernel(HoughDev hp, const int32_t* __restrict__ ev_off, const int32_t* __restrict__ wire_id,
                  const double* __restrict__ wx, const double* __restrict__ wy, int ev0,
                  uint32_t* __restrict__ acc, uint32_t* __restrict__ ev_max) {
  __shared__ int s_x[RKN_MAX_HITS_PER_EVENT], s_y[RKN_MAX_HITS_PER_EVENT];
  __shared__ unsigned short s_cnt[kMaxNr][kHoughCells];
  __shared__ double s_edge[kMaxNr + 1];
  __shared__ unsigned int s_max;
  const int e = ev0 + blockIdx.y, tid = threadIdx.x;
  const int base = ev_off[e], nh = ev_off[e + 1] - base;
  for (int i = tid; i < nh; i += kHoughCells) {
    const int w = wire_id[base + i];
    s_x[i] = (int)rint(wx[w] * 256.0);   // round half to even
    s_y[i] = (int)rint(wy[w] * 256.0);
  }
  for (int k = tid; k <= hp.n_r; k += kHoughCells) {
    const double rk = (double)hp.rmin_q + (double)hp.wr_q * k;
    s_edge[k] = 4.0 * rk * rk;
  }
  for (int k = 0; k < hp.n_r; ++k) s_cnt[k][tid] = 0;
  if (tid == 0) s_max = 0u;
  __syncthreads();
  const long long ncell = (long long)hp.n_xy * hp.n_xy;
  const long long cell = (long long)blockIdx.x * kHoughCells + tid;
  if (cell < ncell) {
    const int a = (int)(cell / hp.n_xy), b = (int)(cell % hp.n_xy);
    const int xc2 = -2 * hp.half_q + hp.wxy_q * (2 * a + 1);   // twice the centre, exact
    const int yc2 = -2 * hp.half_q + hp.wxy_q * (2 * b + 1);
    const double e0 = s_edge[0], en = s_edge[hp.n_r];
    const float inv2w = 1.0f / (2.0f * (float)hp.wr_q);
    const float r2min = 2.0f * (float)hp.rmin_q;
    for (int i = 0; i < nh; ++i) {
      const double dx = (double)(2 * s_x[i] - xc2), dy = (double)(2 * s_y[i] - yc2);
      const double rho2 = dx * dx + dy * dy;      // 4 rho^2, exact
      if (rho2 < e0 || rho2 >= en) continue;
      int k = (int)((sqrtf((float)rho2) - r2min) * inv2w);
      k = k < 0 ? 0 : (k > hp.n_r - 1 ? hp.n_r - 1 : k);
      while (k > 0 && rho2 < s_edge[k]) --k;
      while (k < hp.n_r - 1 && rho2 >= s_edge[k + 1]) ++k;
      s_cnt[k][tid] += 1;
    }
  }
  __syncthreads();
  // coalesced write of this block of cells: acc[e][cell][k]
  uint32_t* out = acc + (size_t)blockIdx.y * ncell * hp.n_r + (size_t)blockIdx.x * kHoughCells * hp.n_r;
  const long long ncells_here = min((long long)kHoughCells, ncell - (long long)blockIdx.x * kHoughCells);
  unsigned int mymax = 0u;
  for (long long i = tid; i < ncells_here * hp.n_r; i += kHoughCells) {
    const int cl = (int)(i / hp.n_r), k = (int)(i % hp.n_r);
    const unsigned int v = s_cnt[k][cl];
    out[i] = v;
    mymax = v > mymax ? v : mymax;
  }
  atomicMax(&s_max, mymax);
  __syncthreads();
  if (tid == 0) atomicMax(ev_max + e, s_max);
}

__global__ void hough_zero_kernel(uint32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Peak rule: the bin's count reaches the event's threshold, is >= all 26
// neighbours and > the neighbours with a smaller flat index.
__device__ __forceinline__ uint32_t peak_threshold(const HoughDev& hp, uint32_t ev_max) {
  uint32_t thr = (ev_max + 1u) / 2u;
  if (thr < (uint32_t)hp.min_votes) thr = (uint32_t)hp.min_votes;
  return thr < 1u ? 1u : thr;
}

__device__ __forceinline__ bool beats_neighbours(const HoughDev& hp, const uint32_t* A, long long v, uint32_t c) {
  const int a = (int)(v / ((long long)hp.n_xy * hp.n_r));
  const int b = (int)((v / hp.n_r) % hp.n_xy);
  const int k = (int)(v % hp.n_r);
  for (int da = -1; da <= 1; ++da)
    for (int db = -1; db <= 1; ++db)
      for (int dk = -1; dk <= 1; ++dk) {
        if (!da && !db && !dk) continue;
        const int aa = a + da, bb = b + db, kk = k + dk;
        if (aa < 0 || bb < 0 || kk < 0 || aa >= hp.n_xy || bb >= hp.n_xy || kk >= hp.n_r) continue;
        const long long nv = ((long long)aa * hp.n_xy + bb) * hp.n_r + kk;
        const uint32_t o = A[nv];
        if (o > c || (o == c && nv < v)) return false;
      }
  return true;
}

__global__ void __launch_bounds__(256)
hough_peaks_kernel(HoughDev hp, const uint32_t* __restrict__ acc, const uint32_t* __restrict__ ev_max,
                   int ev0, uint32_t* __restrict__ cand_n, uint2* __restrict__ cand) {
  const int e = ev0 + blockIdx.y;
  const long long nb = (long long)hp.n_xy * hp.n_xy * hp.n_r;
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nb) return;
  const uint32_t* A = acc + (size_t)blockIdx.y * nb;
  const uint32_t c = A[v];
  if (c < peak_threshold(hp, ev_max[e])) return;
  if (!beats_neighbours(hp, A, v, c)) return;
  const uint32_t slot = atomicAdd(cand_n + e, 1u);
  if (slot < (uint32_t)kCandCap) cand[(size_t)e * kCandCap + slot] = make_uint2(c, (uint32_t)v);
}

__device__ int half_max_extent(const HoughDev& hp, const uint32_t* A, int a, int b, int k, int axis) {
  const uint32_t c = A[((long long)a * hp.n_xy + b) * hp.n_r + k];
  const int lim = axis == 2 ? hp.n_r : hp.n_xy;
  int n = 1;
  for (int dir = -1; dir <= 1; dir += 2) {
    for (int step = 1;; ++step) {
      int aa = a, bb = b, kk = k;
      if (axis == 0) aa += dir * step;
      if (axis == 1) bb += dir * step;
      if (axis == 2) kk += dir * step;
      const int pos = axis == 0 ? aa : (axis == 1 ? bb : kk);
      if (pos < 0 || pos >= lim) break;
      if (2u * A[((long long)aa * hp.n_xy + bb) * hp.n_r + kk] < c) break;
      ++n;
    }
  }
  return n;
}

__global__ void __launch_bounds__(256)
hough_select_kernel(HoughDev hp, const uint32_t* __restrict__ acc, const uint32_t* __restrict__ ev_max, int ev0,
                    const uint32_t* __restrict__ cand_n, const uint2* __restrict__ cand,
                    WinSlot* __restrict__ slots, int32_t* __restrict__ n_valid) {
  __shared__ uint2 s_best[kMaxCand];
  __shared__ uint2 s_red[256];
  __shared__ int s_nsel;
  const int e = ev0 + blockIdx.x, tid = threadIdx.x;
  const long long nbins = (long long)hp.n_xy * hp.n_xy * hp.n_r;
  const uint32_t* A = acc + (size_t)blockIdx.x * nbins;
  // More peaks than the list holds: which ones the list kept depends on the order
  // of the appends, so the selection then walks the whole accumulator with the
  // peak rule instead (slower, same result as an unbounded list).
  const bool overflow = cand_n[e] > (uint32_t)kCandCap;
  const uint32_t thr = peak_threshold(hp, ev_max[e]);
  const int n = (int)min(cand_n[e], (uint32_t)kCandCap);
  const uint2* L = cand + (size_t)e * kCandCap;
  // repeated selection of the best remaining (count desc, flat asc)
  uint2 prev = make_uint2(0xffffffffu, 0u);   // strictly "worse than" this bound
  int nsel = 0;
  for (int j = 0; j < hp.max_cand && (overflow || j < n); ++j) {
    uint2 best = make_uint2(0u, 0xffffffffu);
    bool have = false;
    if (!overflow) {
      for (int i = tid; i < n; i += 256) {
        const uint2 x = L[i];
        const bool after_prev = x.x < prev.x || (x.x == prev.x && x.y > prev.y);
        if (!after_prev) continue;
        if (!have || x.x > best.x || (x.x == best.x && x.y < best.y)) {
          best = x;
          have = true;
        }
      }
    } else {
      for (long long v = tid; v < nbins; v += 256) {
        const uint32_t cnt = A[v];
        if (cnt < thr) continue;
        const uint2 x = make_uint2(cnt, (uint32_t)v);
        const bool after_prev = x.x < prev.x || (x.x == prev.x && x.y > prev.y);
        if (!after_prev) continue;
        if (have && !(x.x > best.x || (x.x == best.x && x.y < best.y))) continue;
        if (!beats_neighbours(hp, A, v, cnt)) continue;
        best = x;
        have = true;
      }
    }
    s_red[tid] = have ? best : make_uint2(0u, 0xffffffffu);
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) {
        const uint2 o = s_red[tid + s], m = s_red[tid];
        if (o.x > m.x || (o.x == m.x && o.y < m.y)) s_red[tid] = o;
      }
      __syncthreads();
    }
    const uint2 w = s_red[0];
    __syncthreads();
    if (w.y == 0xffffffffu && w.x == 0u) break;
    if (tid == 0) s_best[nsel] = w;
    prev = w;
    ++nsel;
  }
  if (tid == 0) s_nsel = nsel;
  __syncthreads();
  nsel = s_nsel;
  if (tid < nsel) {
    const long long flat = s_best[tid].y;
    const int a = (int)(flat / ((long long)hp.n_xy * hp.n_r));
    const int b = (int)((flat / hp.n_r) % hp.n_xy);
    const int k = (int)(flat % hp.n_r);
    const double xc = -hp.xy_half + hp.wxy * (a + 0.5), yc = -hp.xy_half + hp.wxy * (b + 0.5);
    const double R = hp.r_min + hp.wr * (k + 0.5);
    const double d = sqrt(xc * xc + yc * yc), R0 = hp.R0;
    WinSlot out{};
    out.valid = 0;
    if (d > 0.0 && d <= R + R0 && d >= fabs(R - R0)) {
      const double al = (R0 * R0 - R * R + d * d) / (2.0 * d);
      double hh = R0 * R0 - al * al;
      hh = hh > 0.0 ? sqrt(hh) : 0.0;
      const double cx = xc / d, cy = yc / d;
      const double P[2][2] = {{al * cx - hh * cy, al * cy + hh * cx}, {al * cx + hh * cy, al * cy - hh * cx}};
      const double pt = kKappa * hp.b_ref * R;
      double best_dot = 0.0;
      int pick = -1;
      for (int j = 0; j < 2; ++j) {
        double vx = -(P[j][1] - yc) / R, vy = (P[j][0] - xc) / R;
        if (hp.charge > 0.0) {
          vx = -vx;
          vy = -vy;
        }
        const double dot = vx * P[j][0] + vy * P[j][1];
        if (dot > best_dot) {
          best_dot = dot;
          pick = j;
          out.w.center[2] = pt * vx;
          out.w.center[3] = pt * vy;
        }
      }
      if (pick >= 0) {
        out.valid = 1;
        out.w.center[0] = atan2(P[pick][1], P[pick][0]);
        out.w.center[1] = hp.center_z;
        out.w.center[4] = hp.center_pz;
        const int e1 = half_max_extent(hp, A, a, b, k, 0);
        const int e2 = half_max_extent(hp, A, a, b, k, 1);
        const int e3 = half_max_extent(hp, A, a, b, k, 2);
        int s = e1 > e2 ? e1 : e2;
        s = e3 > s ? e3 : s;
        for (int q = 0; q < 5; ++q) {
          int nn = hp.count[q] + hp.grow[q] * (s - 1);
          nn = nn > hp.count_max ? hp.count_max : nn;
          nn = nn < 1 ? 1 : nn;
          out.w.count[q] = nn;
        }
        for (;;) {
          const long long prod = (long long)out.w.count[0] * out.w.count[1] * out.w.count[2] *
                                 out.w.count[3] * out.w.count[4];
          if (prod <= hp.max_seeds) break;
          int big = 0;
          for (int q = 1; q < 5; ++q)
            if (out.w.count[q] > out.w.count[big]) big = q;
          if (out.w.count[big] <= 1) break;
          out.w.count[big] -= 1;
        }
        for (int q = 0; q < 5; ++q) out.w.half_width[q] = hp.gran[q] * 0.5 * (double)(out.w.count[q] - 1);
        out.w.event = e;
      }
    }
    slots[(size_t)e * kMaxCand + tid] = out;
  }
  if (tid == 0) n_valid[e] = nsel;
}

}  // namespace rkn

namespace rkn {

static rkn_status herr(rkn_ctx* c, hipError_t e, const char* where) {
  c->err = std::string(where) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? RKN_E_NOMEM : RKN_E_DEVICE;
}

static bool dyadic(double v) { return std::isfinite(v) && v * 256.0 == std::floor(v * 256.0) && std::fabs(v) < 1e6; }

rkn_status make_hough_dev(rkn_ctx* c, const rkn_hough_params* p, HoughDev& h) {
  if (!p) {
    c->err = "hough params is NULL";
    return RKN_E_ARG;
  }
  const double wxy = 2.0 * p->xy_half / (p->n_xy > 0 ? p->n_xy : 1);
  const double wr = (p->r_max - p->r_min) / (p->n_r > 0 ? p->n_r : 1);
  if (p->n_xy < 1 || p->n_xy > 2048 || p->n_r < 1 || p->n_r > kMaxNr) {
    c->err = "hough: n_xy must be in [1, 2048] and n_r in [1, 64]";
    return RKN_E_ARG;
  }
  if (!(p->xy_half > 0) || !(p->r_max > p->r_min) || !(p->r_min >= 0) || !dyadic(p->xy_half) ||
      !dyadic(wxy) || !dyadic(p->r_min) || !dyadic(wr) || p->r_max > 4096.0 || p->xy_half > 4096.0) {
    c->err = "hough: xy_half, 2 xy_half/n_xy, r_min and (r_max-r_min)/n_r must be positive multiples of 2^-8 mm (<= 4096 mm)";
    return RKN_E_ARG;
  }
  if (p->max_cand < 1 || p->max_cand > kMaxCand || p->min_votes < 0 || p->count_max < 1 || p->max_seeds_window < 1) {
    c->err = "hough: max_cand in [1, 64], min_votes >= 0, count_max >= 1, max_seeds_window >= 1";
    return RKN_E_ARG;
  }
  if (!std::isfinite(p->R0) || p->R0 <= 0 || !std::isfinite(p->charge) || p->charge == 0 ||
      !std::isfinite(p->b_ref) || p->b_ref == 0 || !std::isfinite(p->center_z) || !std::isfinite(p->center_pz)) {
    c->err = "hough: R0 > 0, charge != 0, b_ref != 0, finite centres";
    return RKN_E_ARG;
  }
  for (int q = 0; q < 5; ++q) {
    if (!std::isfinite(p->gran[q]) || p->gran[q] < 0 || p->count[q] < 1 || p->grow[q] < 0) {
      c->err = "hough: gran >= 0, count >= 1, grow >= 0";
      return RKN_E_ARG;
    }
  }
  h.n_xy = p->n_xy;
  h.n_r = p->n_r;
  h.half_q = (int)std::llround(p->xy_half * 256.0);
  h.wxy_q = (int)std::llround(wxy * 256.0);
  h.rmin_q = (int)std::llround(p->r_min * 256.0);
  h.wr_q = (int)std::llround(wr * 256.0);
  h.min_votes = p->min_votes;
  h.max_cand = p->max_cand;
  h.R0 = p->R0;
  h.charge = p->charge;
  h.b_ref = p->b_ref;
  h.xy_half = p->xy_half;
  h.r_min = p->r_min;
  h.wxy = wxy;
  h.wr = wr;
  for (int q = 0; q < 5; ++q) {
    h.gran[q] = p->gran[q];
    h.count[q] = p->count[q];
    h.grow[q] = p->grow[q];
  }
  h.center_z = p->center_z;
  h.center_pz = p->center_pz;
  h.count_max = p->count_max;
  h.max_seeds = p->max_seeds_window;
  return RKN_OK;
}

// Accumulate, find peaks and build windows for events [ev0, ev0+n); device slots.
static hipError_t run_hough_chunk(rkn_ctx* c, const HoughDev& h, int ev0, int n, bool windows) {
  const size_t nb = (size_t)h.n_xy * h.n_xy * h.n_r;
  hipError_t e;
  DevBuf& acc = c->hough_acc;
  hipLaunchKernelGGL(hough_zero_kernel, dim3((n + 255) / 256), dim3(256), 0, c->stream,
                     c->hough_max.as<uint32_t>() + ev0, n);
  hipLaunchKernelGGL(hough_zero_kernel, dim3((n + 255) / 256), dim3(256), 0, c->stream,
                     c->hough_cand_n.as<uint32_t>() + ev0, n);
  const long long ncell = (long long)h.n_xy * h.n_xy;
  hipLaunchKernelGGL(hough_vote_kernel, dim3((unsigned)((ncell + kHoughCells - 1) / kHoughCells), n),
                     dim3(kHoughCells), 0, c->stream, h, c->ev_off.as<int32_t>(), c->hits_wire.as<int32_t>(),
                     c->wire_wx.as<double>(), c->wire_wy.as<double>(), ev0, acc.as<uint32_t>(),
                     c->hough_max.as<uint32_t>());
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (!windows) return hipSuccess;
  hipLaunchKernelGGL(hough_peaks_kernel, dim3((unsigned)((nb + 255) / 256), n), dim3(256), 0, c->stream, h,
                     acc.as<uint32_t>(), c->hough_max.as<uint32_t>(), ev0, c->hough_cand_n.as<uint32_t>(),
                     c->hough_cand.as<uint2>());
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(hough_select_kernel, dim3(n), dim3(256), 0, c->stream, h, acc.as<uint32_t>(),
                     c->hough_max.as<uint32_t>(), ev0,
                     c->hough_cand_n.as<uint32_t>(), c->hough_cand.as<uint2>(), c->hough_slots.as<WinSlot>(),
                     c->hough_nsel.as<int32_t>());
  return hipGetLastError();
}

hipError_t ensure_hough_buffers(rkn_ctx* c, const HoughDev& h) {
  hipError_t e;
  const int ne = c->n_events;
  const size_t nb = (size_t)h.n_xy * h.n_xy * h.n_r;
  if ((e = c->hough_acc.ensure(sizeof(uint32_t) * nb * std::min(kEventChunk, std::max(ne, 1)))) != hipSuccess)
    return e;
  if ((e = c->hough_max.ensure(sizeof(uint32_t) * ne)) != hipSuccess) return e;
  if ((e = c->hough_cand_n.ensure(sizeof(uint32_t) * ne)) != hipSuccess) return e;
  if ((e = c->hough_cand.ensure(sizeof(uint2) * (size_t)kCandCap * ne)) != hipSuccess) return e;
  if ((e = c->hough_slots.ensure(sizeof(WinSlot) * (size_t)kMaxCand * ne)) != hipSuccess) return e;
  if ((e = c->hough_nsel.ensure(sizeof(int32_t) * ne)) != hipSuccess) return e;
  return hipSuccess;
}

hipError_t queue_hough_all(rkn_ctx* c, const HoughDev& h) {
  for (int ev0 = 0; ev0 < c->n_events; ev0 += kEventChunk) {
    const int n = std::min(kEventChunk, c->n_events - ev0);
    hipError_t e = run_hough_chunk(c, h, ev0, n, true);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rkn

using namespace rkn;

extern "C" {

rkn_status rkn_hough_accumulator(rkn_ctx* c, const rkn_hough_params* hp, int32_t event, int32_t ptr_flags,
                                 uint32_t* acc) {
  if (!c) return RKN_E_ARG;
  HoughDev h;
  rkn_status st = make_hough_dev(c, hp, h);
  if (st != RKN_OK) return st;
  if (c->h_ev_off.empty()) {
    c->err = "no hits uploaded";
    return RKN_E_STATE;
  }
  if (event < 0 || event >= c->n_events || !acc || (ptr_flags & ~RKN_PTR_DEVICE)) {
    c->err = "bad event, output pointer or flags";
    return RKN_E_ARG;
  }
  hipError_t e;
  if ((e = hipSetDevice(c->device)) != hipSuccess) return herr(c, e, "hipSetDevice");
  if ((e = ensure_hough_buffers(c, h)) != hipSuccess) return herr(c, e, "hough alloc");
  if ((e = run_hough_chunk(c, h, event, 1, false)) != hipSuccess) return herr(c, e, "hough vote");
  const size_t nb = (size_t)h.n_xy * h.n_xy * h.n_r;
  e = hipMemcpyAsync(acc, c->hough_acc.p, nb * sizeof(uint32_t),
                     (ptr_flags & RKN_PTR_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess && !(ptr_flags & RKN_PTR_DEVICE)) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return herr(c, e, "hough copy");
  return RKN_OK;
}

rkn_status rkn_hough_seed_windows(rkn_ctx* c, const rkn_hough_params* hp, int32_t max_windows, rkn_window* out,
                                  int32_t* n_out) {
  if (!c) return RKN_E_ARG;
  HoughDev h;
  rkn_status st = make_hough_dev(c, hp, h);
  if (st != RKN_OK) return st;
  if (c->h_ev_off.empty()) {
    c->err = "no hits uploaded";
    return RKN_E_STATE;
  }
  if (max_windows < 0 || (max_windows > 0 && !out) || !n_out) {
    c->err = "bad output arrays";
    return RKN_E_ARG;
  }
  hipError_t e;
  if ((e = hipSetDevice(c->device)) != hipSuccess) return herr(c, e, "hipSetDevice");
  if ((e = ensure_hough_buffers(c, h)) != hipSuccess) return herr(c, e, "hough alloc");
  const int ne = c->n_events;
  std::vector<WinSlot> slots((size_t)kMaxCand * ne);
  std::vector<int32_t> nsel(ne);
  if ((e = queue_hough_all(c, h)) != hipSuccess) return herr(c, e, "hough");
  e = hipMemcpyAsync(slots.data(), c->hough_slots.p, sizeof(WinSlot) * slots.size(), hipMemcpyDeviceToHost,
                     c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(nsel.data(), c->hough_nsel.p, sizeof(int32_t) * ne, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return herr(c, e, "hough copy");
  int32_t n = 0;
  for (int ev = 0; ev < ne; ++ev) {
    int cand = 0;
    for (int j = 0; j < nsel[ev]; ++j) {
      const WinSlot& s = slots[(size_t)ev * kMaxCand + j];
      if (!s.valid) continue;
      if (n < max_windows) {
        rkn_window& w = out[n];
        w.event = ev;
        w.candidate = cand;
        for (int q = 0; q < 5; ++q) {
          w.center[q] = s.w.center[q];
          w.half_width[q] = s.w.half_width[q];
          w.count[q] = s.w.count[q];
        }
        w.pad = 0;
      }
      ++cand;
      ++n;
    }
  }
  *n_out = n;
  if (n > max_windows) {
    c->err = "hough: " + std::to_string(n) + " windows do not fit in max_windows";
    return RKN_E_CAPACITY;
  }
  return RKN_OK;
}

}  // extern "C"
