// Selection of the k lowest-score seeds of every event, on the device: the host step
// of the paper's coarse-to-fine refinement that picks the best seeds of a scan
// before finer seed sets are built around them (section 2.2), and the input of the
// derivative-based refinement (the best seeds per event of a batched scan).
#include <algorithm>
#include <string>
#include <vector>

#include "internal.hpp"

namespace rkn {

constexpr int kTopMax = 16;

__device__ __forceinline__ bool key_less(double a, long long ia, double b, long long ib) {
  return a < b || (a == b && ia < ib);
}

// One workgroup per event. Each thread keeps a sorted list of its kTopMax best
// (score, index) pairs over a strided pass of the event's seeds; k rounds of a
// workgroup argmin over the list heads then merge them. Order: score, then index
// (NaN scores are never selected). Seeds are decoded from the event's windows, whose
// seeds are contiguous from seg_off[e] in window order.
__global__ void __launch_bounds__(256)
topk_kernel(const double* __restrict__ score, const long long* __restrict__ seg_off,
            const WindowDev* __restrict__ windows, const int32_t* __restrict__ win_off, int n_seg,
            const int32_t* __restrict__ win_total, int k, int64_t* __restrict__ out_idx,
            double* __restrict__ out_score, double* __restrict__ out_seed, double* __restrict__ out_step) {
  const int e = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long long lo = seg_off[e], hi = seg_off[e + 1];
  double bs[kTopMax];
  long long bi[kTopMax];
#pragma unroll
  for (int j = 0; j < kTopMax; ++j) {
    bs[j] = INFINITY;
    bi[j] = 0x7fffffffffffffffLL;
  }
  for (long long g = lo + tid; g < hi; g += 256) {
    double s = score[g];
    long long i = g;
    if (!(s == s)) continue;
#pragma unroll
    for (int j = 0; j < kTopMax; ++j) {
      const bool lt = key_less(s, i, bs[j], bi[j]);
      const double ts = lt ? bs[j] : s;
      const long long ti = lt ? bi[j] : i;
      bs[j] = lt ? s : bs[j];
      bi[j] = lt ? i : bi[j];
      s = ts;
      i = ti;
    }
  }
  __shared__ double s_e[4];
  __shared__ long long s_i[4];
  __shared__ long long s_sel[kTopMax];
  __shared__ double s_sc[kTopMax];
  for (int r = 0; r < k; ++r) {
    double be = bs[0];
    long long bx = bi[0];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const double oe = __shfl_xor(be, o, 64);
      const long long ox = __shfl_xor(bx, o, 64);
      if (key_less(oe, ox, be, bx)) {
        be = oe;
        bx = ox;
      }
    }
    if (lane == 0) {
      s_e[wave] = be;
      s_i[wave] = bx;
    }
    __syncthreads();
    be = s_e[0];
    bx = s_i[0];
    for (int w = 1; w < 4; ++w)
      if (key_less(s_e[w], s_i[w], be, bx)) {
        be = s_e[w];
        bx = s_i[w];
      }
    const bool none = bx == 0x7fffffffffffffffLL;
    if (tid == 0) {
      s_sel[r] = none ? -1 : bx;
      s_sc[r] = none ? INFINITY : be;
    }
    // the owner of the winning head (indices are unique) pops it
    if (!none && bi[0] == bx) {
#pragma unroll
      for (int j = 0; j + 1 < kTopMax; ++j) {
        bs[j] = bs[j + 1];
        bi[j] = bi[j + 1];
      }
      bs[kTopMax - 1] = INFINITY;
      bi[kTopMax - 1] = 0x7fffffffffffffffLL;
    }
    __syncthreads();
  }
  if (tid < k) {
    const long long g = s_sel[tid];
    const size_t o = (size_t)e * k + tid;
    out_idx[o] = g;
    out_score[o] = s_sc[tid];
    double v[5] = {NAN, NAN, NAN, NAN, NAN}, st[5] = {NAN, NAN, NAN, NAN, NAN};
    if (g >= 0 && (out_seed || out_step)) {
      const int w0 = win_off[e];
      const int w1 = e + 1 < n_seg ? win_off[e + 1] : *win_total;
      long long local = g - lo;
      for (int w = w0; w < w1; ++w) {
        long long size = 1;
        for (int d = 0; d < 5; ++d) size *= windows[w].count[d];
        if (local < size) {
          window_seed(windows[w], local, v);
          // the step of the grid the seed came from (0 where the window has one point)
          for (int d = 0; d < 5; ++d)
            st[d] = windows[w].count[d] > 1 ? 2.0 * windows[w].half_width[d] / (double)(windows[w].count[d] - 1)
                                            : 0.0;
          break;
        }
        local -= size;
      }
    }
    if (out_seed)
      for (int d = 0; d < 5; ++d) out_seed[o * 5 + d] = v[d];
    if (out_step)
      for (int d = 0; d < 5; ++d) out_step[o * 5 + d] = st[d];
  }
}

hipError_t launch_topk(rkn_ctx* c, const double* d_score, const long long* d_seg_off, const WindowDev* d_windows,
                       const int32_t* d_win_off, int n_seg, const int32_t* d_win_total, int k, int64_t* d_idx,
                       double* d_sc, double* d_seed, double* d_step) {
  if (n_seg <= 0) return hipSuccess;
  if (k < 1 || k > kTopMax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(topk_kernel, dim3(n_seg), dim3(256), 0, c->stream, d_score, d_seg_off, d_windows, d_win_off,
                     n_seg, d_win_total, k, d_idx, d_sc, d_seed, d_step);
  return hipGetLastError();
}

}  // namespace rkn
