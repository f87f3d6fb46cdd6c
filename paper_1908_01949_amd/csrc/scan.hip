// The seed-scan kernels for gfx950 (Yeo et al., CTD/WIT 2019, section 2.2, Eq. 1).
//
// Work decomposition (one MI355X):
//   * one lane per seed; a workgroup of 64*WAVES lanes takes tiles of up to 64*WAVES
//     seeds of one event from an atomic queue (persistent grid sized to the resident
//     capacity); with a field map, the 65x129 (B_r, B_z) nodes are staged in LDS once
//     per workgroup and shared by all its waves;
//   * the event's hits are staged in LDS, ordered by layer and, within a layer, by
//     the twisted azimuth psi = phi - s_l z of the wire centre; a 1 mm radial table
//     maps a radius range to the layers whose band (widened by the largest drift +
//     sqrt(lambda) + 1 mm) it can meet, and a layer x psi-sector table gives the
//     circular run of a layer's hits that a block in that sector can reach;
//   * each lane runs B RKN steps in registers and writes the B+1 points to an LDS
//     column; it then walks the runs of its block's layers and sector (records
//     gathered from LDS), tests each hit with a sphere bound (all B chords lie within
//     B h / 2 of the block's middle point) and the wave appends the survivors to an
//     LDS work list (ballot + mbcnt compaction);
//   * the list is processed densely (one item per lane, the tail spread over lane
//     groups): exact chord/wire distance of the B chords, the minimum folded into the
//     seed's running minimum (a per-workgroup slab [hit][lane] in HBM, updated with an
//     integer atomic min on the non-negative float bit pattern: order-free and
//     deterministic); a per-wave LDS bitmap marks the (wave, hit) rows that received
//     a minimum in the current tile;
//   * after the last block each lane forms E = sum min((D - d)^2, lambda) in FP64,
//     reading only the marked rows (the others still hold +inf) and resetting them to
//     +inf, so the slab is written once per workgroup at launch and afterwards only
//     where a tile touched it.
// Every filter is exact: a pair it drops can only have a distance above
// d + sqrt(lambda), where the term is lambda whatever the distance is.
#include <type_traits>

#include <algorithm>

#include "internal.hpp"

namespace rkn {

constexpr int kCap = 176;          // work-list entries per wave
constexpr int kTabBins = 1024;     // 1 mm radial bins, the last one open-ended
constexpr float kBandMargin = 1.0f;   // radial band table
constexpr float kCullMargin = 0.05f;  // sphere test: covers FP32 rounding of the test (~1e-2 mm)
constexpr int kSectors = 256;         // twisted-azimuth sectors of the candidate table (finer
                                      // sectors stage fewer pairs; 256 fill the workgroup's LDS)
// A sector entry: the run's first hit (bits 0-8) and length (bits 9-15); kSectAll
// stands for the whole layer (a run longer than 127 hits, or a reach past pi).
constexpr uint32_t kSectAll = 0xffffu;
constexpr int kTraceFold = 8;   // rkn_trace: steps between folds of the block-relative sums
constexpr float kPi = 3.14159265358979f;

struct ScanArgs {
  FieldDev field;
  const HitRec<float>* hits32;
  const HitRec<double>* hits64;
  const int32_t* ev_off;
  const int32_t* layer_off;   // [n_events][n_layers+1]
  const float2* layer_r;      // (rmin, rmax) per layer
  const float* ev_maxdrift;
  const float* hits_phi;      // twisted azimuth psi of each layer-ordered hit's wire centre
  const float2* layer_twist;  // [n_events][n_layers] (dphi/dz of the layer's wires, psi deviation)
  int n_layers;
  int sect_bytes;             // LDS bytes reserved for the layer x sector table
  int hits_bytes;             // LDS bytes reserved for hit records
  int field_bytes;            // LDS bytes reserved for the field map (0: uniform)
  int touch_words;            // 32-bit words of a wave's row bitmap (>= max hits / 32)
  const Tile* tiles;
  int64_t n_tiles;
  const int32_t* n_tiles_dev;   // if set, the tile count is read here (captured launches)
  const WindowDev* windows;
  const double* seeds5;       // explicit seeds [n][5] in scan order (NULL: windows)
  const int64_t* perm;        // scan order -> caller index (explicit seeds)
  int* tile_counter;
  void* mscratch;
  int64_t slab_stride;        // elements per workgroup slab
  double R0, charge, h, lambda;
  int n_steps;
  int turn_stop;              // 1: a lane's track ends with the first step inside r < R0
  double* score;
  int32_t* nin;
  ArgminPart* parts;
  // refinement forward mode (MODE 1): per output slot = scan position
  const int32_t* hits_orig;   // original index (within its event) of each layer-ordered hit
  const int64_t* base_of;     // scan position -> refinement seed whose inlier set applies
  uint8_t* mask;              // [n_base][max_hits] inlier flags (original hit order)
  int define_mask;            // 1: set mask from (D - d)^2 < lambda, 0: read it
  float* resid;               // [n_pos][max_hits] residual D - d of inliers, NaN otherwise
  int32_t* argmin_step;       // [n_pos][max_hits] chord index of the minimum (inliers), -1 otherwise
  double* phi;                // [n_pos] sum of squared inlier residuals
  float* tape;                // [n_ckpt][13][n_pos] FP32 states every ckpt steps (NULL: none)
  int ckpt, n_ckpt;
  int64_t n_pos;
  int max_hits;
  // adaptive step size (scan_kernel variant 2): path length, error bound, step range
  double path_len;
  float tol, h_min, h_max;
  // work counters of the counting instance (COUNT): seed-steps taken, sphere tests
  // made, chord/wire distances evaluated
  unsigned long long* work;
};

// ---------------------------------------------------------------------------------
// Upload-time preparation: per event, order the hits by layer and, within a layer,
// by the twisted azimuth psi = phi(m) - s_l m_z of the wire centre m (ties by upload
// order), where s_l = dphi/dz of the layer's stereo wires (taken from the layer's
// first hit). Along a wire, phi - s_l z stays within dev_l of psi; the kernel uses
// (s_l, dev_l) per layer to turn a block's middle point into a psi window. Also
// builds the FP32/FP64 hit records, the per-layer offsets and the event's largest
// drift.
// Azimuth for the sector lookup: octant reduction and an odd degree-7 polynomial
// for atan on [0, 1] (our least-squares fit; |error| < 1e-4 rad, far inside the
// table's 2e-3 rad margin).
__device__ __forceinline__ float sector_atan2(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float hi = fmaxf(ax, ay), lo = fminf(ax, ay);
  const float t = hi > 0.0f ? lo * __builtin_amdgcn_rcpf(hi) : 0.0f;
  const float u = t * t;
  float r = t * fmaf(fmaf(fmaf(-0.03898633f, u, 0.14626420f), u, -0.32117486f), u, 0.99921381f);
  r = ay > ax ? 0.5f * kPi - r : r;
  r = x < 0.0f ? kPi - r : r;
  return y < 0.0f ? -r : r;
}

__device__ __forceinline__ float wrap_pi(float d) {
  return d >= kPi ? d - 2.0f * kPi : (d < -kPi ? d + 2.0f * kPi : d);
}

__global__ void __launch_bounds__(256)
prep_hits_kernel(const int32_t* __restrict__ ev_off, const int32_t* __restrict__ wire_id,
                 const float* __restrict__ drift, const HitRec<float>* __restrict__ wire32,
                 const HitRec<double>* __restrict__ wire64, const int32_t* __restrict__ wire_layer,
                 int n_layers, HitRec<float>* __restrict__ out32, HitRec<double>* __restrict__ out64,
                 int32_t* __restrict__ layer_off, float* __restrict__ ev_maxdrift, int32_t* __restrict__ orig,
                 float* __restrict__ out_psi, float2* __restrict__ layer_twist) {
  __shared__ int s_layer[RKN_MAX_HITS_PER_EVENT];
  __shared__ float s_psi[RKN_MAX_HITS_PER_EVENT];
  __shared__ int s_count[RKN_MAX_LAYERS + 1];
  __shared__ int s_first[RKN_MAX_LAYERS];
  __shared__ unsigned int s_dev[RKN_MAX_LAYERS];
  __shared__ float s_slope[RKN_MAX_LAYERS];
  __shared__ unsigned int s_max;
  const int e = blockIdx.x, tid = threadIdx.x;
  const int base = ev_off[e], n = ev_off[e + 1] - base;
  for (int l = tid; l <= n_layers; l += blockDim.x) s_count[l] = 0;
  for (int l = tid; l < n_layers; l += blockDim.x) {
    s_dev[l] = 0u;
    s_first[l] = 0x7fffffff;
  }
  if (tid == 0) s_max = 0u;
  __syncthreads();
  unsigned int mymax = 0u;
  for (int i = tid; i < n; i += blockDim.x) {
    const int l = wire_layer[wire_id[base + i]];
    s_layer[i] = l;
    atomicAdd(&s_count[l], 1);
    atomicMin(&s_first[l], i);
    const unsigned int bits = __float_as_uint(drift[base + i]);
    mymax = bits > mymax ? bits : mymax;
  }
  atomicMax(&s_max, mymax);
  __syncthreads();
  for (int l = tid; l < n_layers; l += blockDim.x) {
    float sl = 0.0f;
    if (s_first[l] < n) {
      const HitRec<float> r = wire32[wire_id[base + s_first[l]]];
      const float r2 = r.mx * r.mx + r.my * r.my;
      sl = (fabsf(r.uz) > 1e-6f && r2 > 0.0f) ? (r.mx * r.uy - r.my * r.ux) / (r2 * r.uz) : 0.0f;
    }
    s_slope[l] = sl;
  }
  __syncthreads();
  for (int i = tid; i < n; i += blockDim.x) {
    const int l = s_layer[i];
    const float sl = s_slope[l];
    const HitRec<float> r = wire32[wire_id[base + i]];
    const float phi = atan2f(r.my, r.mx);
    s_psi[i] = wrap_pi(phi - sl * r.mz);
    float dev = 0.0f;
    for (int q = -2; q <= 2; ++q) {
      if (q == 0) continue;
      const float t = 0.5f * (float)q * r.L;
      const float d = wrap_pi(atan2f(r.my + t * r.uy, r.mx + t * r.ux) - phi) - sl * r.uz * t;
      dev = fmaxf(dev, fabsf(d));
    }
    atomicMax(&s_dev[l], __float_as_uint(dev));
  }
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int l = 0; l < n_layers; ++l) {
      const int c = s_count[l];
      s_count[l] = acc;
      acc += c;
    }
    s_count[n_layers] = acc;
    for (int l = 0; l <= n_layers; ++l) layer_off[(size_t)e * (n_layers + 1) + l] = s_count[l];
    // the deviation is sampled at t = +-L/2, +-L; its curvature term is bounded by
    // doubling the sampled maximum
    for (int l = 0; l < n_layers; ++l)
      layer_twist[(size_t)e * n_layers + l] = make_float2(s_slope[l], 2.0f * __uint_as_float(s_dev[l]));
    ev_maxdrift[e] = __uint_as_float(s_max);
  }
  __syncthreads();
  for (int i = tid; i < n; i += blockDim.x) {
    const int l = s_layer[i];
    const float psi = s_psi[i];
    int rank = s_count[l];
    for (int j = 0; j < n; ++j)
      rank += (s_layer[j] == l) && (s_psi[j] < psi || (s_psi[j] == psi && j < i));
    const int w = wire_id[base + i];
    HitRec<float> r32 = wire32[w];
    HitRec<double> r64 = wire64[w];
    r32.drift = drift[base + i];
    r64.drift = (double)drift[base + i];
    out32[base + rank] = r32;
    out64[base + rank] = r64;
    orig[base + rank] = i;
    out_psi[base + rank] = psi;
  }
}

hipError_t launch_prep_hits(rkn_ctx* c, const int32_t* d_wire_id, const float* d_drift) {
  if (c->n_events == 0) return hipSuccess;
  hipLaunchKernelGGL(prep_hits_kernel, dim3(c->n_events), dim3(256), 0, c->stream,
                     c->ev_off.as<int32_t>(), d_wire_id, d_drift, c->wire32.as<HitRec<float>>(),
                     c->wire64.as<HitRec<double>>(), c->wire_layer.as<int32_t>(), c->n_layers,
                     c->hits32.as<HitRec<float>>(), c->hits64.as<HitRec<double>>(),
                     c->layer_off.as<int32_t>(), c->ev_maxdrift.as<float>(), c->hits_orig.as<int32_t>(),
                     c->hits_phi.as<float>(), c->layer_ext.as<float2>());
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
__global__ void reset_counter_kernel(int* counter) { *counter = 0; }

template <typename R>
__device__ __forceinline__ const HitRec<R>* hits_of(const ScanArgs& a);
template <>
__device__ __forceinline__ const HitRec<float>* hits_of<float>(const ScanArgs& a) { return a.hits32; }
template <>
__device__ __forceinline__ const HitRec<double>* hits_of<double>(const ScanArgs& a) { return a.hits64; }

template <typename R>
__device__ __forceinline__ void atomic_min_nonneg(R* p, R v) {
  if constexpr (sizeof(R) == 4) {
    atomicMin(reinterpret_cast<unsigned int*>(p), __float_as_uint(v));
  } else {
    atomicMin(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v));
  }
}

template <typename R>
__device__ __forceinline__ R load_coherent(const R* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Fold one item's block minimum into the seed's running minimum for the hit. In
// the scan, a block whose minimum is not below (d + sqrt(lambda))^2 cannot change
// the hit's term (it stays lambda unless another block comes closer), so it is not
// written. The refinement pass writes every block (its inlier set is fixed).
// The wave's row of the hit is marked in its LDS bitmap.
template <typename R, int TILE, int MODE, typename S>
__device__ __forceinline__ void fold_min(S* slab, uint32_t* touch, int hh, int wave, int s, R d2, int chord,
                                         R lim2) {
  if constexpr (MODE == 0) {
    if (!(d2 < lim2)) return;
    atomic_min_nonneg(slab + (size_t)hh * TILE + wave * 64 + s, d2);
  } else {
    // (distance bits, chord index): the minimum distance, then the lowest chord
    const unsigned long long key =
        ((unsigned long long)__float_as_uint((float)d2) << 32) | (unsigned long long)(unsigned)chord;
    atomicMin(reinterpret_cast<unsigned long long*>(slab + (size_t)hh * TILE + wave * 64 + s), key);
  }
  atomicOr(touch + (hh >> 5), 1u << (hh & 31));
}

// Dense pass over a wave's work list: item = (lane << 16) | hit. Full groups of 64
// items take one item per lane and all chords of the block; the remaining n < 64
// items take G lanes each (G = 8, 4 or 2 with G n <= 64), the chords of an item
// strided over its lanes, so the tail pass costs about B / G chords instead of B.
// The fold is an atomic minimum of (distance[, chord]) and so order-free: lanes of an
// item may fold separately and the seed's running minimum ends as after a full
// reduction over the G lanes. In the scan, adjacent lanes first merge their minima
// with one row shift (half the atomics, and half their L2 write-backs, for three
// instructions); the refinement pass folds every lane's (distance, chord) key.
template <typename R, int B, int TILE, int MODE, typename S>
__device__ __forceinline__ void flush_items(const uint32_t* items, int n_items, const R* pts,
                                            const HitRec<R>* s_hits, S* slab, uint32_t* touch, int wave,
                                            int lane, int nb, int step0, R sqrt_lam) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  int done = 0;
  for (; n_items - done >= 64; done += 64) {
    const uint32_t it = items[done + lane];
    const int s = (int)(it >> 16), hh = (int)(it & 0xffffu);
    const HitRec<R> w = s_hits[hh];
    R px = pts[0 * 64 + s], py = pts[1 * 64 + s], pz = pts[2 * 64 + s];
    R dmin = (R)INFINITY;
    int jmin = 0;
#pragma unroll
    for (int j = 1; j <= B; ++j) {
      if (j <= nb) {
        const R qx = pts[(j * 3 + 0) * 64 + s], qy = pts[(j * 3 + 1) * 64 + s],
                qz = pts[(j * 3 + 2) * 64 + s];
        const R d2 = seg_wire_d2<R>(px, py, pz, qx, qy, qz, w.mx, w.my, w.mz, w.ux, w.uy, w.uz, w.L);
        if (d2 < dmin) {
          dmin = d2;
          jmin = j - 1;
        }
        px = qx;
        py = qy;
        pz = qz;
      }
    }
    const R lim = w.drift + sqrt_lam;
    fold_min<R, TILE, MODE>(slab, touch, hh, wave, s, dmin, step0 + jmin, lim * lim);
  }
  const int n_rem = n_items - done;
  if (n_rem > 0) {
    const int G = n_rem <= 8 ? 8 : (n_rem <= 16 ? 4 : (n_rem <= 32 ? 2 : 1));
    const int k = lane / G, sub = lane - k * G;
    const bool act = k < n_rem;
    const uint32_t it = items[done + (act ? k : 0)];
    const int s = (int)(it >> 16), hh = (int)(it & 0xffffu);
    const HitRec<R> w = s_hits[hh];
    R dmin = (R)INFINITY;
    int jmin = 0;
    for (int j = sub; j < nb; j += G) {
      const R d2 = seg_wire_d2<R>(pts[(j * 3 + 0) * 64 + s], pts[(j * 3 + 1) * 64 + s], pts[(j * 3 + 2) * 64 + s],
                                  pts[(j * 3 + 3) * 64 + s], pts[(j * 3 + 4) * 64 + s], pts[(j * 3 + 5) * 64 + s],
                                  w.mx, w.my, w.mz, w.ux, w.uy, w.uz, w.L);
      if (d2 < dmin) {   // the lane's chords in increasing order: keeps the lowest on ties
        dmin = d2;
        jmin = j;
      }
    }
    bool folds = act && sub < nb;
    if constexpr (MODE == 0 && sizeof(R) == 4) {
      if (G > 1) {
        // pairs of an item's lanes (aligned inside rows of 16) merge their minima first:
        // non-negative floats order as their bit patterns
        const unsigned bits = __float_as_uint(dmin);
        const unsigned o = (unsigned)__builtin_amdgcn_update_dpp((int)bits, (int)bits, 0x101, 0xf, 0xf, false);
        dmin = __uint_as_float(o < bits ? o : bits);
        folds = folds && (sub & 1) == 0;
      }
    }
    if (folds) {
      const R lim = w.drift + sqrt_lam;
      fold_min<R, TILE, MODE>(slab, touch, hh, wave, s, dmin, step0 + jmin, lim * lim);
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS writes of the wave's lanes visible to all its lanes (list handoffs within a wave).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Dense sphere test of the staged candidates items[lo, hi) (item = (lane << 16) | hit),
// one per lane: the wire's line against the sphere of radius Kcull + d around the
// middle point of the owner lane's block (column jc of its points). Survivors are
// compacted in place from items[lo] on (every lane reads its chunk before any lane
// writes, and survivors never pass the chunk being read); returns their end.
template <typename R, bool COUNT>
__device__ __forceinline__ int test_staged(uint32_t* items, int lo, int hi, const R* pts, const HitRec<R>* s_hits,
                                           int jc, R Kcull, int lane, int nb, unsigned long long& w_tests,
                                           unsigned long long& w_chords) {
  wave_sync();
  int out = lo;
  for (int base = lo; base < hi; base += 64) {
    const bool act = base + lane < hi;
    const uint32_t it = items[act ? base + lane : lo];
    wave_sync();
    const int s = (int)(it >> 16), hh = (int)(it & 0xffffu);
    const HitRec<R> w = s_hits[hh];
    const R cx = pts[(jc * 3 + 0) * 64 + s], cy = pts[(jc * 3 + 1) * 64 + s], cz = pts[(jc * 3 + 2) * 64 + s];
    const R rx = cx - w.mx, ry = cy - w.my, rz = cz - w.mz;
    const R tt = rx * w.ux + ry * w.uy + rz * w.uz;
    const R d2 = rx * rx + ry * ry + rz * rz - tt * tt;
    const R thr = Kcull + w.drift;
    const bool pass = act & (d2 <= thr * thr);   // every lane's loads are in bounds
    if constexpr (COUNT) {
      w_tests += act ? 1 : 0;
      w_chords += pass ? nb : 0;
    }
    const uint64_t m = __ballot(pass);
    if (pass) items[out + lane_rank(m)] = it;
    out += (int)__popcll(m);
    wave_sync();
  }
  return out;
}

// VAR 0: fixed steps over the whole path; 1: fixed steps, the track ends with its
// turn partition; 2: adaptive step size (scan mode only), turn_stop as given.
// COUNT: the instance that also counts its work (seed-steps, sphere tests, chord
// distances) into a.work; the timed instances leave it out.
template <typename R, int FIELD, int B, int WAVES, int MODE, int VAR, bool COUNT = false>
__global__ void __launch_bounds__(64 * WAVES) scan_kernel(ScanArgs a) {
  constexpr int TILE = 64 * WAVES;
  // MODE 0: the scan (score E). MODE 1: the refinement forward pass (FP32 only):
  // argmin chords, checkpoints and inlier residuals.
  using Slab = typename std::conditional<MODE == 0, R, unsigned long long>::type;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  float2* s_field = reinterpret_cast<float2*>(smem);
  HitRec<R>* s_hits = reinterpret_cast<HitRec<R>*>(smem + a.field_bytes);
  uint16_t* s_ltab = reinterpret_cast<uint16_t*>(smem + a.field_bytes + a.hits_bytes);
  uint16_t* s_sect = reinterpret_cast<uint16_t*>(smem + a.field_bytes + a.hits_bytes + kTabBins * 2);
  R* s_pts = reinterpret_cast<R*>(smem + a.field_bytes + a.hits_bytes + kTabBins * 2 + a.sect_bytes);
  uint32_t* s_items = reinterpret_cast<uint32_t*>(s_pts + WAVES * (B + 1) * 3 * 64);
  // small tables sized by the uploaded event set: layer offsets and twist slopes of
  // the current event, the per-wave row bitmaps
  int* s_loff = reinterpret_cast<int*>(s_items + WAVES * kCap);
  float* s_slope = reinterpret_cast<float*>(s_loff + a.n_layers + 1);
  uint32_t* s_touch = reinterpret_cast<uint32_t*>(s_slope + a.n_layers);
  __shared__ int s_tile;
  __shared__ double s_red_e[WAVES];
  __shared__ long long s_red_i[WAVES];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t n_tiles = a.n_tiles_dev ? (int64_t)*a.n_tiles_dev : a.n_tiles;
  // longest chord: every point of a block's chords lies within B hmax / 2 of its
  // middle point, and every point of a chord within hmax / 2 of one of its ends
  const double hmax = VAR == 2 ? (double)a.h_max : a.h;
  R* pts = s_pts + wave * (B + 1) * 3 * 64;
  uint32_t* items = s_items + wave * kCap;
  Slab* slab = reinterpret_cast<Slab*>(a.mscratch) + (size_t)blockIdx.x * a.slab_stride;
  uint32_t* touch = s_touch + wave * a.touch_words;
  unsigned long long w_steps = 0, w_tests = 0, w_chords = 0;   // COUNT only
  // every slab entry holds "no minimum yet" between tiles: written here once, then
  // reset by the tile that read it
  for (int64_t i = tid; i < a.slab_stride; i += TILE) {
    if constexpr (MODE == 0)
      slab[i] = (R)INFINITY;
    else
      slab[i] = 0xffffffffffffffffULL;
  }
  __threadfence_block();
  const R h = (R)a.h;
  const double lam = a.lambda;
  int cur_event = -1;
  const float2* nodes = nullptr;
  if constexpr (FIELD == 1) {
    const int nn = (int)padded_field_nodes(a.field.nr, a.field.nz);
    for (int i = tid; i < nn; i += TILE) s_field[i] = a.field.nodes[i];
    nodes = s_field;   // made visible by the first tile's barrier
  }

  for (;;) {
    if (tid == 0) s_tile = atomicAdd(a.tile_counter, 1);
    __syncthreads();
    const int64_t ti = __builtin_amdgcn_readfirstlane(s_tile);
    if (ti >= n_tiles) break;
    const Tile t = a.tiles[ti];
    const int ev = t.event;
    const int hbase = a.ev_off[ev];
    const int nh = a.ev_off[ev + 1] - hbase;
    const HitRec<R>* ghits = hits_of<R>(a) + hbase;

    if (ev != cur_event) {
      for (int i = tid; i < nh; i += TILE) s_hits[i] = ghits[i];
      const int32_t* loff = a.layer_off + (size_t)ev * (a.n_layers + 1);
      for (int l = tid; l <= a.n_layers; l += TILE) s_loff[l] = loff[l];
      // radial bins: the layers whose band, widened by the event's largest drift +
      // sqrt(lambda) + 1 mm, meets the bin: [l0, l1p) packed as l0 | l1p << 8
      const float D = a.ev_maxdrift[ev] + (float)sqrt(lam) + kBandMargin;
      for (int b = tid; b < kTabBins; b += TILE) {
        const float lo_r = (float)b, hi_r = b == kTabBins - 1 ? INFINITY : (float)(b + 1);
        int l0 = 0;
        while (l0 < a.n_layers && a.layer_r[l0].y + D < lo_r) ++l0;
        int l1 = a.n_layers - 1;
        while (l1 >= 0 && a.layer_r[l1].x - D > hi_r) --l1;
        s_ltab[b] = (uint16_t)(l0 | ((l1 + 1) << 8));
      }
      // layer x twisted-azimuth sector: the circular run of a layer's hits (sorted by
      // psi) that a block whose middle point c has psi_c = phi_c - s_l z_c in the
      // sector can reach. A kept pair needs a wire point w within
      // rho = d + sqrt(lambda) + margin + B h / 2 of c; then |phi_w - phi_c| <=
      // 2 asin(rho / (2 (r_l - rho))) (radii >= r_l - rho and r_l),
      // |z_w - z_c| <= rho, and phi_w - s_l z_w is within dev_l of the hit's psi.
      const float rho = a.ev_maxdrift[ev] + (float)sqrt(lam) + kCullMargin + 0.5f * (float)(B * hmax);
      const float* gpsi = a.hits_phi + hbase;
      for (int l = tid; l < a.n_layers; l += TILE) s_slope[l] = a.layer_twist[(size_t)ev * a.n_layers + l].x;
      for (int q = tid; q < a.n_layers * kSectors; q += TILE) {
        const int l = q / kSectors, k = q - l * kSectors;
        const int lb = loff[l], nl = loff[l + 1] - lb;
        uint32_t ent = 0u;
        if (nl > 0) {
          const float2 tw = a.layer_twist[(size_t)ev * a.n_layers + l];
          const float rl = a.layer_r[l].x - rho;
          const float ratio = rl > 0.0f ? rho / (2.0f * rl) : 2.0f;
          const float dphi = ratio < 1.0f ? 2.0f * asinf(ratio) : kPi;
          const float W = dphi + fabsf(tw.x) * rho + tw.y + 2e-3f;
          if (W >= kPi) {
            ent = kSectAll;
          } else {
            const float a0 = -kPi + (2.0f * kPi / kSectors) * k, a1 = a0 + 2.0f * kPi / kSectors;
            auto inside = [&](int j) {
              const float ps = gpsi[lb + j];
              if (ps >= a0 && ps <= a1) return true;
              float d1 = a0 - ps, d2 = ps - a1;
              d1 -= 2.0f * kPi * floorf(d1 / (2.0f * kPi));
              d2 -= 2.0f * kPi * floorf(d2 / (2.0f * kPi));
              return fminf(d1, d2) <= W;
            };
            int cnt = 0, start = -1;
            bool prev = inside(nl - 1);
            for (int j = 0; j < nl; ++j) {
              const bool in = inside(j);
              cnt += in;
              if (in && !prev && start < 0) start = j;
              prev = in;
            }
            if (cnt == nl) start = 0;
            ent = cnt > 127 ? kSectAll : (cnt > 0 ? ((uint32_t)start | ((uint32_t)cnt << 9)) : 0u);
          }
        }
        s_sect[q] = (uint16_t)ent;
      }
      cur_event = ev;
    }

    // ---- seed of this lane ------------------------------------------------------
    const bool in_tile = tid < t.n;
    bool valid = in_tile;
    int64_t gidx = t.gbase + tid;
    State<R> st;
    {
      double v[5];
      if (a.seeds5) {
        const int64_t pos = t.start + (in_tile ? tid : 0);
#pragma unroll
        for (int d = 0; d < 5; ++d) v[d] = a.seeds5[pos * 5 + d];
        gidx = a.perm[pos];
      } else {
        window_seed(a.windows[t.window], t.start + (in_tile ? tid : 0), v);
      }
      const double pm = sqrt(v[2] * v[2] + v[3] * v[3] + v[4] * v[4]);
      valid = valid && (pm >= 1e-3);
      const double ipm = valid ? 1.0 / pm : 0.0;
      st.x = (R)(a.R0 * cos(v[0]));
      st.y = (R)(a.R0 * sin(v[0]));
      st.z = (R)v[1];
      st.tx = valid ? (R)(v[2] * ipm) : (R)1;
      st.ty = valid ? (R)(v[3] * ipm) : (R)0;
      st.tz = valid ? (R)(v[4] * ipm) : (R)0;
      st.lam = valid ? (R)(kKappa * a.charge * ipm) : (R)0;
      st.cx = st.cy = st.cz = (R)0;
      st.ctx = st.cty = st.ctz = (R)0;
    }
    Prop<R, FIELD> pr;   // fixed steps: current point and the block's increments
    pr.start(st);
    pr.init_field(st, a.field, nodes);
    if (lane < a.touch_words) touch[lane] = 0u;
    __syncthreads();

    constexpr bool STOP = VAR != 0;    // lanes can end before the last block
    constexpr bool ADAPT = VAR == 2;
    // adaptive: at most 4 L / h_min + 8 trial steps per lane (every rejection at
    // least shortens the step, and h_min steps are always taken)
    const int nblocks = ADAPT ? (int)((4.0 * a.path_len / a.h_min + 8.0 + B - 1) / B) : (a.n_steps + B - 1) / B;
    const R Kcull = (R)(0.5 * B * hmax + sqrt(lam) + (double)kCullMargin);
    const R sqrt_lam = (R)sqrt(lam);
    // STOP (a lane's track can end early: at the end of its turn partition, the first
    // step inside r < R0, or with adaptive steps at the end of the path): from then on
    // the lane's state is frozen, so its later chords have zero length at that end
    // point and cannot lower any distance; a block that starts frozen is not culled at
    // all, and a wave whose lanes are all frozen leaves the loop (after writing the
    // frozen state into the checkpoints still ahead, when a tape is recorded)
    const R r0sq = (R)(a.R0 * a.R0);
    const bool may_exit = STOP;
    const bool stop_turn = VAR == 1 || (ADAPT && a.turn_stop);
    bool live = valid;                          // lanes without a seed have no track to end
    R hl = (R)a.h_max, arc = (R)0;              // adaptive: next step and path so far
    const R path = (R)a.path_len;
    for (int blk = 0; blk < nblocks; ++blk) {
      if constexpr (STOP) {
        if (may_exit && __ballot(live) == 0) {
          if constexpr (MODE == 1) {
            // the remaining checkpoints hold the frozen state (as if stepped on)
            if (a.tape && in_tile) {
              const float v13[13] = {(float)st.x, (float)st.y, (float)st.z, (float)st.cx, (float)st.cy, (float)st.cz,
                                     (float)st.tx, (float)st.ty, (float)st.tz, (float)st.ctx, (float)st.cty,
                                     (float)st.ctz, (float)st.lam};
              for (int step = blk * B; step < a.n_steps; step += B) {
                if (step % a.ckpt != 0) continue;
                float* tp = a.tape + (size_t)(step / a.ckpt) * 13 * a.n_pos + gidx;
#pragma unroll
                for (int q = 0; q < 13; ++q) tp[(size_t)q * a.n_pos] = v13[q];
              }
            }
          }
          break;
        }
      }
      const bool live0 = live;
      const int nb = ADAPT ? B : min(B, a.n_steps - blk * B);
      const int jc = nb / 2;
      if constexpr (MODE == 1) {
        const int step = blk * B;
        // a checkpoint restarts the adjoint's recompute: the field there is evaluated
        // at the stored state, as the recompute does
        if (a.ckpt > 0 && step % a.ckpt == 0) pr.init_field(st, a.field, nodes);
        if (a.tape && in_tile && step % a.ckpt == 0) {
          float* tp = a.tape + (size_t)(step / a.ckpt) * 13 * a.n_pos + gidx;
          const float v13[13] = {(float)st.x, (float)st.y, (float)st.z, (float)st.cx, (float)st.cy, (float)st.cz,
                                 (float)st.tx, (float)st.ty, (float)st.tz, (float)st.ctx, (float)st.cty,
                                 (float)st.ctz, (float)st.lam};
#pragma unroll
          for (int q = 0; q < 13; ++q) tp[(size_t)q * a.n_pos] = v13[q];
        }
      }
      pts[0 * 64 + lane] = st.x;
      pts[1 * 64 + lane] = st.y;
      pts[2 * 64 + lane] = st.z;
      R r2min, r2max;
      if constexpr (ADAPT) {
        r2min = r2max = radius2(st.x, st.y);
#pragma unroll
        for (int j = 1; j <= B; ++j) {
          // one trial step; accepted when its error estimate is within the bound
          // (or it is the smallest step), else the lane stays and retries shorter
          if (live) {
            const R hs = hl < path - arc ? hl : path - arc;
            State<R> tr = st;
            R err;
            rkn_step_err<R, FIELD>(tr, a.field, nodes, hs, err);
            const bool acc = err <= (R)a.tol || hs <= (R)a.h_min;
            R g = err > (R)0 ? (R)0.9 * fsqrt(fsqrt((R)a.tol / err)) : (R)4;
            g = g > (R)4 ? (R)4 : (g < (R)0.25 ? (R)0.25 : g);
            if (acc) {
              st = tr;
              arc += hs;
              if (hs == hl) hl *= g;   // a cut last step leaves the step size
              live = arc < path && !(stop_turn && inside_r0(st.x, st.y, r0sq));
            } else {
              hl = hs * (g < (R)1 ? g : (R)1);
            }
            hl = hl > (R)a.h_max ? (R)a.h_max : (hl < (R)a.h_min ? (R)a.h_min : hl);
          }
          pts[(j * 3 + 0) * 64 + lane] = st.x;
          pts[(j * 3 + 1) * 64 + lane] = st.y;
          pts[(j * 3 + 2) * 64 + lane] = st.z;
          const R r2 = radius2(st.x, st.y);
          r2min = vmin(r2min, r2);
          r2max = vmax(r2max, r2);
        }
      } else {
        r2min = r2max = pr.r2;
        auto take = [&](int j, bool go) {
          if (go) pr.step(st, a.field, nodes, h);
          pts[(j * 3 + 0) * 64 + lane] = pr.px;
          pts[(j * 3 + 1) * 64 + lane] = pr.py;
          pts[(j * 3 + 2) * 64 + lane] = pr.pz;
          if constexpr (VAR == 1) live = live && !inside_r0(pr.px, pr.py, r0sq);
          r2min = vmin(r2min, pr.r2);
          r2max = vmax(r2max, pr.r2);
        };
        if (nb == B) {   // every block but a short last one: straight-line steps
#pragma unroll
          for (int j = 1; j <= B; ++j) take(j, !STOP || live);
        } else {
          for (int j = 1; j <= B; ++j) take(j, j <= nb && (!STOP || live));
        }
        // the block's increments go into the origin; the folded position (within an
        // ulp of the last one) ends the block's last chord and starts the next block
        if (!STOP || live0) {
          pr.fold(st);
          pts[(nb * 3 + 0) * 64 + lane] = pr.px;
          pts[(nb * 3 + 1) * 64 + lane] = pr.py;
          pts[(nb * 3 + 2) * 64 + lane] = pr.pz;
          r2min = vmin(r2min, pr.r2);
          r2max = vmax(r2max, pr.r2);
        }
      }
      // the block's middle point, from this lane's own column
      const R cx = pts[(jc * 3 + 0) * 64 + lane], cy = pts[(jc * 3 + 1) * 64 + lane],
              cz = pts[(jc * 3 + 2) * 64 + lane];
      // radial range of the block's chords (a chord point is within hmax/2 of an endpoint)
      const float rmin = fmaxf((float)fsqrt(r2min) - 0.5f * (float)hmax, 0.0f);
      const float rmax = (float)fsqrt(r2max);
      // clamp in float first: fminf/fmaxf map NaN to the bound, so the index is in range
      const int b_lo = (int)fminf(fmaxf(rmin, 0.0f), (float)(kTabBins - 1));
      const int b_hi = (int)fminf(fmaxf(rmax, 0.0f), (float)(kTabBins - 1));
      // candidates: per layer whose band meets the block's radial range, the run of
      // hits that can reach the azimuth sector of the block's middle point. Each lane
      // walks its own runs and stages (lane, hit) pairs in the wave's list (cheap
      // steps, as many as the longest run in the wave); the staged pairs are then
      // sphere-tested densely, one per lane, and the survivors kept at the list's
      // front for the distance pass
      const int L0 = s_ltab[b_lo] & 0xff, L1p = s_ltab[b_hi] >> 8;
      const int n_lay = (valid && (!STOP || live0)) ? max(L1p - L0, 0) : 0;
      const float phic = sector_atan2((float)cy, (float)cx);
      int n_items = 0;   // survivors: items[0, n_items)
      int n_stage = 0;   // staged candidates: items[n_items, n_items + n_stage)
      for (int dl = 0; __ballot(dl < n_lay) != 0; ++dl) {
        const bool has = dl < n_lay;
        const int l = has ? L0 + dl : 0;
        const float psic = wrap_pi(phic - s_slope[l] * (float)cz);
        int sect = (int)((psic + kPi) * (kSectors / (2.0f * kPi)));
        sect = sect < 0 ? 0 : (sect > kSectors - 1 ? kSectors - 1 : sect);
        const uint32_t ent = has ? (uint32_t)s_sect[l * kSectors + sect] : 0u;
        const int lb = s_loff[l], nl = s_loff[l + 1] - lb;
        const bool all = ent == kSectAll;
        const int start = all ? 0 : (int)(ent & 511u), cnt = all ? nl : (int)(ent >> 9);
        // the run's first item and the step at which it wraps to the layer's first hit,
        // formed before the loop (so the loop waits on none of the table reads)
        const uint32_t first = ((uint32_t)lane << 16) | (uint32_t)(lb + start);
        const int wrap = nl - start;
        for (int k = 0;; ++k) {
          const bool act = k < cnt;
          const uint64_t m = __ballot(act);
          if (m == 0) break;
          const int off = k < wrap ? k : k - nl;
          if (act) items[n_items + n_stage + lane_rank(m)] = first + (uint32_t)off;
          n_stage += (int)__popcll(m);
          if (n_items + n_stage > kCap - 64) {
            n_items = test_staged<R, COUNT>(items, n_items, n_items + n_stage, pts, s_hits, jc, Kcull, lane, nb,
                                            w_tests, w_chords);
            n_stage = 0;
            if (n_items > kCap - 64) {
              flush_items<R, B, TILE, MODE>(items, n_items, pts, s_hits, slab, touch, wave, lane, nb, blk * B,
                                            sqrt_lam);
              n_items = 0;
            }
          }
        }
      }
      if (n_stage)
        n_items = test_staged<R, COUNT>(items, n_items, n_items + n_stage, pts, s_hits, jc, Kcull, lane, nb, w_tests,
                                        w_chords);
      if (n_items)
        flush_items<R, B, TILE, MODE>(items, n_items, pts, s_hits, slab, touch, wave, lane, nb, blk * B, sqrt_lam);
      if constexpr (COUNT) w_steps += (valid && (!STOP || live0)) ? nb : 0;
    }
    // The minima of a seed were folded by lanes of its own wave, and the slab is this
    // workgroup's alone: a workgroup-scope release/acquire (the atomics complete at L2;
    // the reads below bypass L1) orders them before the reads. An agent-scope fence
    // here would write the whole L2's dirty lines back to memory at every tile.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");

    if constexpr (MODE == 1) {
      // ---- refinement outputs: inlier residuals (original hit order), argmin chords
      if (in_tile) {
        const int64_t base = a.base_of ? a.base_of[gidx] : gidx;
        uint8_t* mrow = a.mask + (size_t)base * a.max_hits;
        float* rrow = a.resid + (size_t)gidx * a.max_hits;
        int32_t* arow = a.argmin_step + (size_t)gidx * a.max_hits;
        double ph = 0.0;
        for (int i = 0; i < nh; ++i) {
          unsigned long long key = 0xffffffffffffffffULL;
          if ((touch[i >> 5] >> (i & 31)) & 1u) {
            key = load_coherent(slab + (size_t)i * TILE + tid);
            slab[(size_t)i * TILE + tid] = 0xffffffffffffffffULL;
          }
          // no block came within the cull reach: the distance is beyond it (+inf here)
          const float d2 = key == 0xffffffffffffffffULL ? INFINITY : __uint_as_float((unsigned)(key >> 32));
          const double r = sqrt((double)d2) - (double)s_hits[i].drift;
          const int o = a.hits_orig[hbase + i];
          bool in;
          if (a.define_mask) {
            in = valid && (r * r < lam);
            mrow[o] = in ? 1 : 0;
          } else {
            in = valid && mrow[o] != 0;
          }
          rrow[o] = in ? (float)r : NAN;
          arow[o] = (in && key != 0xffffffffffffffffULL) ? (int32_t)(unsigned)(key & 0xffffffffu) : -1;
          if (in) ph += r * r;
        }
        for (int i = nh; i < a.max_hits; ++i) {
          if (a.define_mask) mrow[i] = 0;   // the whole row is defined, unused columns 0
          rrow[i] = NAN;
          arow[i] = -1;
        }
        a.phi[gidx] = valid ? ph : INFINITY;
      } else {
        for (int i = 0; i < nh; ++i)
          if ((touch[i >> 5] >> (i & 31)) & 1u) slab[(size_t)i * TILE + tid] = 0xffffffffffffffffULL;
      }
      __threadfence_block();
      __syncthreads();
      continue;
    }
    // ---- score (Eq. 1), in FP64 ---------------------------------------------------
    double E = 0.0;
    int cnt = 0;
    for (int i = 0; i < nh; ++i) {
      // rows without a mark were not written in this tile: +inf, nothing to reset
      R m2 = (R)INFINITY;
      if ((touch[i >> 5] >> (i & 31)) & 1u) {
        m2 = load_coherent(slab + (size_t)i * TILE + tid);
        slab[(size_t)i * TILE + tid] = (R)INFINITY;
      }
      if (valid) {
        const double r = sqrt((double)m2) - (double)s_hits[i].drift;
        const double tq = r * r;
        if (tq < lam) {
          E += tq;
          ++cnt;
        } else {
          E += lam;
        }
      }
    }
    if (!valid) E = INFINITY;
    __threadfence_block();   // the resets land before the next tile's minima
    long long idx = in_tile ? (long long)gidx : (long long)0x7fffffffffffffffLL;
    if (in_tile) {
      if (a.score) a.score[gidx] = E;
      if (a.nin) a.nin[gidx] = cnt;
    }
    // ---- argmin of the tile (E, then index) -------------------------------------
    double be = in_tile ? E : INFINITY;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const double oe = __shfl_xor(be, o, 64);
      const long long oi = __shfl_xor(idx, o, 64);
      if (oe < be || (oe == be && oi < idx)) {
        be = oe;
        idx = oi;
      }
    }
    if (lane == 0) {
      s_red_e[wave] = be;
      s_red_i[wave] = idx;
    }
    __syncthreads();
    if (tid == 0) {
      for (int k = 1; k < WAVES; ++k)
        if (s_red_e[k] < be || (s_red_e[k] == be && s_red_i[k] < idx)) {
          be = s_red_e[k];
          idx = s_red_i[k];
        }
      a.parts[ti].e = be;
      a.parts[ti].idx = idx;
    }
    __syncthreads();
  }
  if constexpr (COUNT) {
    atomicAdd(a.work + 0, w_steps);
    atomicAdd(a.work + 1, w_tests);
    atomicAdd(a.work + 2, w_chords);
  }
}

__global__ void __launch_bounds__(256)
event_argmin_kernel(const ArgminPart* __restrict__ parts, const int32_t* __restrict__ ev_tiles,
                    int64_t* best_i, double* best_e) {
  const int e = blockIdx.x, tid = threadIdx.x;
  const int t0 = ev_tiles[e], t1 = ev_tiles[e + 1];
  double be = INFINITY;
  long long bi = 0x7fffffffffffffffLL;
  for (int t = t0 + tid; t < t1; t += 256) {
    const ArgminPart p = parts[t];
    if (p.e < be || (p.e == be && p.idx < bi)) {
      be = p.e;
      bi = p.idx;
    }
  }
  __shared__ double se[256];
  __shared__ long long si[256];
  se[tid] = be;
  si[tid] = bi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) {
      const double oe = se[tid + s];
      const long long oi = si[tid + s];
      if (oe < se[tid] || (oe == se[tid] && oi < si[tid])) {
        se[tid] = oe;
        si[tid] = oi;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    const bool none = t1 <= t0;
    best_i[e] = none ? -1 : si[0];
    best_e[e] = none ? INFINITY : se[0];
  }
}

// LDS bytes of the layer x sector candidate table (uint16 entries, 256-byte rounded).
static size_t align64(size_t n) { return (n + 63) & ~(size_t)63; }

static size_t sect_table_bytes(const rkn_ctx* c) {
  return align64((size_t)std::max(c->n_layers, 1) * kSectors * sizeof(uint16_t));
}

static int touch_words(const rkn_ctx* c) { return std::max((c->max_hits_event + 31) / 32, 1); }

// LDS regions of one workgroup of scan_kernel<R, FIELD, B, WAVES, ...>, in order:
// field map, hit records, radial table, sector table, points, work lists, layer
// offsets and slopes, row bitmaps.
static size_t field_lds_bytes(const rkn_ctx* c, int field) {
  return field == 1 ? align64(padded_field_nodes(c->nr, c->nz) * sizeof(float2)) : 0;
}
static size_t hits_lds_bytes(const rkn_ctx* c, size_t rsize) {
  return align64((size_t)c->max_hits_event * (rsize == 4 ? sizeof(HitRec<float>) : sizeof(HitRec<double>)));
}
static size_t scan_lds_bytes(const rkn_ctx* c, size_t rsize, int field, int B, int waves) {
  return field_lds_bytes(c, field) + hits_lds_bytes(c, rsize) + kTabBins * 2 + sect_table_bytes(c) +
         (size_t)waves * (B + 1) * 3 * 64 * rsize + (size_t)waves * kCap * 4 +
         (size_t)(2 * std::max(c->n_layers, 1) + 1) * 4 + (size_t)waves * touch_words(c) * 4;
}

// Steps per block; 0 picks the default: 6 for the FP32 field-map path (12-wave
// workgroups, the fastest shape measured on the 512-event batch), else 8.
int resolve_block_steps(const rkn_ctx* c, const rkn_scan_params* p) {
  if (p->block_steps != 0) return p->block_steps;
  return (p->precision == 32 && c->field_kind == 1) ? 6 : 8;
}

// Workgroups of a kernel that one CU holds, from the kernel's register and LDS
// needs (code-object metadata) and the CU's resources on gfx950: 4 SIMDs of 512
// VGPRs per lane (allocated in granules of 8) and at most 8 waves each, and the
// LDS of the device. (This does not use the runtime's occupancy query, whose
// answer for wide workgroups differs between HIP runtime versions.)
static int resident_per_cu(const rkn_ctx* c, const void* kern, int threads, size_t smem) {
  hipFuncAttributes at{};
  if (hipFuncGetAttributes(&at, kern) != hipSuccess) return 0;
  const int waves = (threads + 63) / 64;
  const size_t lds = smem + at.sharedSizeBytes;
  if (lds > (size_t)c->max_lds_block) return 0;
  const int by_lds = lds > 0 ? (int)((size_t)c->max_lds_block / lds) : 32;
  const int regs = at.numRegs > 0 ? ((at.numRegs + 7) / 8) * 8 : 8;
  const int per_simd = std::min(512 / regs, 8);
  const int by_regs = (4 * per_simd) / waves;
  return std::min(by_lds, by_regs);
}

template <typename R, int FIELD, int B, int WAVES>
static bool shape_fits(const rkn_ctx* c) {
  const size_t smem = scan_lds_bytes(c, sizeof(R), FIELD, B, WAVES);
  if (smem + 256 > (size_t)c->max_lds_block) return false;
  // every variant (fixed steps, turn-partition stop, adaptive) must fit the shape
  bool ok = resident_per_cu(c, (const void*)scan_kernel<R, FIELD, B, WAVES, 0, 0>, 64 * WAVES, smem) >= 1 &&
            resident_per_cu(c, (const void*)scan_kernel<R, FIELD, B, WAVES, 0, 1>, 64 * WAVES, smem) >= 1;
  if constexpr (std::is_same<R, float>::value)
    ok = ok && resident_per_cu(c, (const void*)scan_kernel<R, FIELD, B, WAVES, 0, 2>, 64 * WAVES, smem) >= 1;
  return ok;
}

// Waves per workgroup. The FP32 field-map path stages the map in LDS once per
// workgroup, so it uses the widest workgroup that fits: 16 waves with 4-step
// blocks, 12 with 6-step blocks, 8 with 8-step blocks (falling back to 8 waves when
// an event has too many hits, or the runtime reserves too much LDS, for the wider
// shape). Tiles are built for the shape chosen here, and the launch uses the same.
static int scan_waves(const rkn_ctx* c, int precision, int B) {
  if (precision == 64 || c->field_kind == 0) return 4;
  if (B == 4 && shape_fits<float, 1, 4, 16>(c)) return 16;
  if (B == 6 && shape_fits<float, 1, 6, 12>(c)) return 12;
  return 8;
}

template <typename R, int FIELD, int B, int WAVES, int MODE = 0>
static hipError_t launch_scan_t(rkn_ctx* c, ScanArgs& a, int64_t max_tiles, bool alloc_only, DevBuf* slab_buf,
                                void* raw_slab = nullptr, size_t raw_bytes = 0) {
  constexpr int TILE = 64 * WAVES;
  a.hits_bytes = (int)hits_lds_bytes(c, sizeof(R));
  a.field_bytes = (int)field_lds_bytes(c, FIELD);
  a.sect_bytes = (int)sect_table_bytes(c);
  a.touch_words = touch_words(c);
  const size_t smem = scan_lds_bytes(c, sizeof(R), FIELD, B, WAVES);
  if (smem + 256 > (size_t)c->max_lds_block) return hipErrorInvalidConfiguration;
  auto kern = a.turn_stop ? scan_kernel<R, FIELD, B, WAVES, MODE, 1> : scan_kernel<R, FIELD, B, WAVES, MODE, 0>;
  if constexpr (MODE == 0) {
    if (a.h_max > 0) kern = scan_kernel<R, FIELD, B, WAVES, MODE, 2>;
    if (a.work) kern = scan_kernel<R, FIELD, B, WAVES, MODE, 0, true>;   // fixed steps only (checked by the caller)
  }
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  const int per_cu = resident_per_cu(c, (const void*)kern, TILE, smem);
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  int64_t grid = (int64_t)per_cu * c->n_cu;
  if (grid > max_tiles) grid = max_tiles;
  if (grid < 1) grid = 1;
  a.slab_stride = (int64_t)(c->max_hits_event > 0 ? c->max_hits_event : 1) * TILE;
  const size_t per_wg = (size_t)a.slab_stride * (MODE == 0 ? sizeof(R) : sizeof(unsigned long long));
  if (raw_slab) {
    // caller-provided memory: the persistent grid shrinks to the slabs that fit
    const int64_t fit = (int64_t)(raw_bytes / per_wg);
    if (fit < 1) return hipErrorInvalidValue;
    if (grid > fit) grid = fit;
    a.mscratch = raw_slab;
  } else {
    e = slab_buf->ensure((size_t)grid * per_wg);
    if (e != hipSuccess) return e;
    a.mscratch = slab_buf->p;
  }
  if (alloc_only) return hipSuccess;
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, c->stream, a.tile_counter);
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(TILE), smem, c->stream, a);
  return hipGetLastError();
}

int scan_tile(const rkn_ctx* c, const rkn_scan_params* p) {
  return 64 * scan_waves(c, p->precision, p->precision == 64 ? 4 : resolve_block_steps(c, p));
}

static hipError_t dispatch_scan(rkn_ctx* c, const rkn_scan_params* p, ScanArgs& a, int64_t max_tiles,
                                bool alloc_only, DevBuf* slab, void* raw_slab = nullptr, size_t raw_bytes = 0) {
  const int B = resolve_block_steps(c, p);
  if (p->precision == 64)
    return c->field_kind == 0 ? launch_scan_t<double, 0, 4, 4>(c, a, max_tiles, alloc_only, slab, raw_slab, raw_bytes)
                              : launch_scan_t<double, 1, 4, 4>(c, a, max_tiles, alloc_only, slab, raw_slab, raw_bytes);
  if (c->field_kind == 0) {
    if (B == 4) return launch_scan_t<float, 0, 4, 4>(c, a, max_tiles, alloc_only, slab, raw_slab, raw_bytes);
    if (B == 6) return launch_scan_t<float, 0, 6, 4>(c, a, max_tiles, alloc_only, slab, raw_slab, raw_bytes);
    return launch_scan_t<float, 0, 8, 4>(c, a, max_tiles, alloc_only, slab, raw_slab, raw_bytes);
  }
  const int W = scan_waves(c, 32, B);
  if (B == 4)
    return W == 16 ? launch_scan_t<float, 1, 4, 16>(c, a, max_tiles, alloc_only, slab, raw_slab, raw_bytes)
                   : launch_scan_t<float, 1, 4, 8>(c, a, max_tiles, alloc_only, slab, raw_slab, raw_bytes);
  if (B == 6)
    return W == 12 ? launch_scan_t<float, 1, 6, 12>(c, a, max_tiles, alloc_only, slab, raw_slab, raw_bytes)
                   : launch_scan_t<float, 1, 6, 8>(c, a, max_tiles, alloc_only, slab, raw_slab, raw_bytes);
  return launch_scan_t<float, 1, 8, 8>(c, a, max_tiles, alloc_only, slab, raw_slab, raw_bytes);
}

FieldDev field_dev(const rkn_ctx* c) {
  FieldDev f{};
  f.bz = c->bz;
  if (c->field_kind == 1) {
    f.nodes = c->field_nodes.as<float2>();
    f.nr = c->nr;
    f.nz = c->nz;
    f.stride = c->nr + 1;
    f.r0 = c->r0;
    f.z0 = c->z0;
    f.inv_dr = (double)(c->nr - 1) / (c->r1 - c->r0);
    f.inv_dz = (double)(c->nz - 1) / (c->z1 - c->z0);
  }
  return f;
}

// Refinement forward pass over explicit seeds (FP32, block of 8 steps).
hipError_t launch_refine_fwd(rkn_ctx* c, const rkn_scan_params* p, int64_t n_tiles, const Tile* d_tiles,
                             const double* d_seeds5, const int64_t* d_perm, const int64_t* d_base_of,
                             uint8_t* d_mask, int define_mask, float* d_resid, int32_t* d_argmin, double* d_phi,
                             float* d_tape, int ckpt, int n_ckpt, int64_t n_pos) {
  hipError_t e = c->r_counter.ensure(64);
  if (e != hipSuccess) return e;
  ScanArgs a{};
  a.field = field_dev(c);
  a.hits32 = c->hits32.as<HitRec<float>>();
  a.hits64 = c->hits64.as<HitRec<double>>();
  a.ev_off = c->ev_off.as<int32_t>();
  a.layer_off = c->layer_off.as<int32_t>();
  a.layer_r = c->layer_r.as<float2>();
  a.ev_maxdrift = c->ev_maxdrift.as<float>();
  a.hits_phi = c->hits_phi.as<float>();
  a.layer_twist = c->layer_ext.as<float2>();
  a.n_layers = c->n_layers;
  a.tiles = d_tiles;
  a.n_tiles = n_tiles;
  a.seeds5 = d_seeds5;
  a.perm = d_perm;
  a.tile_counter = c->r_counter.as<int>();
  a.R0 = p->R0;
  a.charge = p->charge;
  a.h = p->step_mm;
  a.lambda = p->lambda_mm2;
  a.n_steps = p->n_steps;
  a.turn_stop = p->turn_stop;
  a.hits_orig = c->hits_orig.as<int32_t>();
  a.base_of = d_base_of;
  a.mask = d_mask;
  a.define_mask = define_mask;
  a.resid = d_resid;
  a.argmin_step = d_argmin;
  a.phi = d_phi;
  a.tape = d_tape;
  a.ckpt = ckpt;
  a.n_ckpt = n_ckpt;
  a.n_pos = n_pos;
  a.max_hits = c->max_hits_event > 0 ? c->max_hits_event : 1;
  if (n_tiles == 0) return hipSuccess;
  static_assert(kRefineBlock == 8, "the refinement pass runs 8-step blocks");
  return c->field_kind == 0 ? launch_scan_t<float, 0, 8, 4, 1>(c, a, n_tiles, false, &c->r_slab)
                            : launch_scan_t<float, 1, 8, 8, 1>(c, a, n_tiles, false, &c->r_slab);
}

static ScanArgs scan_args(rkn_ctx* c, const rkn_scan_params* p, const Tile* d_tiles, const WindowDev* d_windows,
                          double* d_score, int32_t* d_nin, ArgminPart* parts, int* counter) {
  ScanArgs a{};
  a.field = field_dev(c);
  a.hits32 = c->hits32.as<HitRec<float>>();
  a.hits64 = c->hits64.as<HitRec<double>>();
  a.ev_off = c->ev_off.as<int32_t>();
  a.layer_off = c->layer_off.as<int32_t>();
  a.layer_r = c->layer_r.as<float2>();
  a.ev_maxdrift = c->ev_maxdrift.as<float>();
  a.hits_phi = c->hits_phi.as<float>();
  a.layer_twist = c->layer_ext.as<float2>();
  a.n_layers = c->n_layers;
  a.tiles = d_tiles;
  a.windows = d_windows;
  a.tile_counter = counter;
  a.R0 = p->R0;
  a.charge = p->charge;
  a.h = p->step_mm;
  a.lambda = p->lambda_mm2;
  a.n_steps = p->n_steps;
  a.turn_stop = p->turn_stop;
  a.score = d_score;
  if (c->adapt) {   // set only for the adaptive scan entry point's call
    a.path_len = p->n_steps * p->step_mm;
    a.tol = (float)c->adapt->tol_mm;
    a.h_min = (float)c->adapt->h_min_mm;
    a.h_max = (float)c->adapt->h_max_mm;
  }
  a.nin = d_nin;
  a.parts = parts;
  a.work = c->count_work;
  return a;
}

hipError_t launch_scan(rkn_ctx* c, const rkn_scan_params* p, int64_t n_tiles, const Tile* d_tiles,
                       const WindowDev* d_windows, const double* d_seeds5, const int64_t* d_perm,
                       double* d_score, int32_t* d_nin, int64_t* d_best_i, double* d_best_e,
                       const int32_t* d_ev_tiles) {
  hipError_t e = c->parts.ensure(sizeof(ArgminPart) * (size_t)(n_tiles > 0 ? n_tiles : 1));
  if (e != hipSuccess) return e;
  e = c->counter.ensure(64);
  if (e != hipSuccess) return e;
  ScanArgs a = scan_args(c, p, d_tiles, d_windows, d_score, d_nin, c->parts.as<ArgminPart>(), c->counter.as<int>());
  a.n_tiles = n_tiles;
  a.seeds5 = d_seeds5;
  a.perm = d_perm;
  if (n_tiles > 0) {
    e = dispatch_scan(c, p, a, n_tiles, false, &c->mscratch);
    if (e != hipSuccess) return e;
  }
  if (c->n_events > 0) {
    hipLaunchKernelGGL(event_argmin_kernel, dim3(c->n_events), dim3(256), 0, c->stream,
                       c->parts.as<ArgminPart>(), d_ev_tiles, d_best_i, d_best_e);
  }
  return hipGetLastError();
}

hipError_t launch_scan_dev(rkn_ctx* c, const rkn_scan_params* p, int64_t max_tiles, const int32_t* d_n_tiles,
                           const Tile* d_tiles, const WindowDev* d_windows, double* d_score, int32_t* d_nin,
                           int64_t* d_best_i, double* d_best_e, const int32_t* d_ev_tiles, bool alloc_only,
                           const ScanScratch* scratch) {
  const ScanScratch own{&c->b_parts, &c->b_counter, &c->b_slab};
  const ScanScratch& s = scratch ? *scratch : own;
  hipError_t e = s.parts->ensure(sizeof(ArgminPart) * (size_t)(max_tiles > 0 ? max_tiles : 1));
  if (e != hipSuccess) return e;
  e = s.counter->ensure(64);
  if (e != hipSuccess) return e;
  ScanArgs a = scan_args(c, p, d_tiles, d_windows, d_score, d_nin, s.parts->as<ArgminPart>(), s.counter->as<int>());
  a.n_tiles = max_tiles;
  a.n_tiles_dev = d_n_tiles;
  e = dispatch_scan(c, p, a, max_tiles, alloc_only, s.slab);
  if (e != hipSuccess || alloc_only) return e;
  hipLaunchKernelGGL(event_argmin_kernel, dim3(c->n_events), dim3(256), 0, c->stream,
                     s.parts->as<ArgminPart>(), d_ev_tiles, d_best_i, d_best_e);
  return hipGetLastError();
}

hipError_t launch_scan_raw(rkn_ctx* c, const rkn_scan_params* p, int64_t n_tiles, const Tile* d_tiles,
                           const WindowDev* d_windows, double* d_score, int32_t* d_nin, int64_t* d_best_i,
                           double* d_best_e, const int32_t* d_ev_tiles, ArgminPart* d_parts, int* d_counter,
                           void* d_slab, size_t slab_bytes) {
  ScanArgs a = scan_args(c, p, d_tiles, d_windows, d_score, d_nin, d_parts, d_counter);
  a.n_tiles = n_tiles;
  if (n_tiles > 0) {
    const hipError_t e = dispatch_scan(c, p, a, n_tiles, false, nullptr, d_slab, slab_bytes);
    if (e != hipSuccess) return e;
  }
  if (c->n_events > 0)
    hipLaunchKernelGGL(event_argmin_kernel, dim3(c->n_events), dim3(256), 0, c->stream, d_parts, d_ev_tiles,
                       d_best_i, d_best_e);
  return hipGetLastError();
}

size_t scan_slab_bytes_per_workgroup(const rkn_ctx* c, const rkn_scan_params* p) {
  const size_t elem = p->precision == 64 ? sizeof(double) : sizeof(float);
  return (size_t)(c->max_hits_event > 0 ? c->max_hits_event : 1) * (size_t)scan_tile(c, p) * elem;
}

// ---------------------------------------------------------------------------------
template <typename R, int FIELD>
__global__ void __launch_bounds__(256)
trace_kernel(FieldDev f, double R0, double charge, double hstep, int turn_stop, int64_t n_seeds,
             const double* __restrict__ seeds, int n_sel, const int32_t* __restrict__ steps,
             double* __restrict__ out) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_seeds) return;
  const double* v = seeds + 5 * s;
  const double pm = sqrt(v[2] * v[2] + v[3] * v[3] + v[4] * v[4]);
  double* o = out + (size_t)s * n_sel * 6;
  if (!(pm >= 1e-3)) {
    for (int k = 0; k < 6 * n_sel; ++k) o[k] = NAN;
    return;
  }
  State<R> st;
  st.x = (R)(R0 * cos(v[0]));
  st.y = (R)(R0 * sin(v[0]));
  st.z = (R)v[1];
  st.tx = (R)(v[2] / pm);
  st.ty = (R)(v[3] / pm);
  st.tz = (R)(v[4] / pm);
  st.lam = (R)(kKappa * charge / pm);
  st.cx = st.cy = st.cz = (R)0;
      st.ctx = st.cty = st.ctz = (R)0;
  const R h = (R)hstep;
  const R r0sq = (R)(R0 * R0);
  int n = 0;
  bool live = true;   // with turn_stop, states after the end of the turn partition stay
  Prop<R, FIELD> pr;  // the scan's propagation, folded every kTraceFold steps
  pr.start(st);
  pr.init_field(st, f, f.nodes);
  for (int k = 0; k < n_sel; ++k) {
    const int target = steps[k];
    for (; n < target && live; ++n) {
      pr.step(st, f, f.nodes, h);
      live = !(turn_stop && inside_r0(pr.px, pr.py, r0sq));
      if ((n + 1) % kTraceFold == 0) pr.fold(st);
    }
    o[6 * k + 0] = (double)pr.px;
    o[6 * k + 1] = (double)pr.py;
    o[6 * k + 2] = (double)pr.pz;
    o[6 * k + 3] = (double)pr.tx;
    o[6 * k + 4] = (double)pr.ty;
    o[6 * k + 5] = (double)pr.tz;
  }
}

hipError_t launch_trace(rkn_ctx* c, const rkn_scan_params* p, int64_t n_seeds, const double* d_seeds,
                        int32_t n_sel, const int32_t* d_steps, double* d_states) {
  const FieldDev f = field_dev(c);
  const dim3 grid((unsigned)((n_seeds + 255) / 256)), block(256);
  if (n_seeds == 0) return hipSuccess;
  if (p->precision == 64) {
    if (c->field_kind == 0)
      hipLaunchKernelGGL((trace_kernel<double, 0>), grid, block, 0, c->stream, f, p->R0, p->charge,
                         p->step_mm, p->turn_stop, n_seeds, d_seeds, n_sel, d_steps, d_states);
    else
      hipLaunchKernelGGL((trace_kernel<double, 1>), grid, block, 0, c->stream, f, p->R0, p->charge,
                         p->step_mm, p->turn_stop, n_seeds, d_seeds, n_sel, d_steps, d_states);
  } else {
    if (c->field_kind == 0)
      hipLaunchKernelGGL((trace_kernel<float, 0>), grid, block, 0, c->stream, f, p->R0, p->charge,
                         p->step_mm, p->turn_stop, n_seeds, d_seeds, n_sel, d_steps, d_states);
    else
      hipLaunchKernelGGL((trace_kernel<float, 1>), grid, block, 0, c->stream, f, p->R0, p->charge,
                         p->step_mm, p->turn_stop, n_seeds, d_seeds, n_sel, d_steps, d_states);
  }
  return hipGetLastError();
}

}  // namespace rkn
