// Device-side arithmetic of the seed scan for gfx950: field evaluation, one RKN
// step, the exact chord/wire distance, and wave-level helpers.
//
// Method (Yeo et al., CTD/WIT 2019, section 2.2): tracks are propagated with a
// fixed-step Runge-Kutta-Nystrom integrator of the Lorentz force and compared
// with the wires by their distance of closest approach.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rkn {

constexpr double kKappa = 0.299792458;  // (MeV/c) / (T mm e)

// Hit record staged per event, ordered by layer: wire segment m +- L u and drift.
template <typename R>
struct alignas(sizeof(R) * 8) HitRec {
  R mx, my, mz, ux, uy, uz, L, drift;
};

// Axisymmetric field: uniform B_z, or FP32 (B_r, B_z) nodes interleaved
// [nz + 1][stride = nr + 1]: the extra column and row repeat the edge nodes, so a
// coordinate clamped to the upper edge selects a cell whose far nodes carry weight 0
// and no index clamp is needed.
struct FieldDev {
  const float2* nodes;
  int nr, nz;
  int stride;
  double r0, z0, inv_dr, inv_dz;
  double bz;
};

// Nodes of the padded table (the layout FieldDev describes).
__host__ __device__ inline size_t padded_field_nodes(int nr, int nz) { return (size_t)(nr + 1) * (nz + 1); }

template <typename R>
__device__ __forceinline__ R clampv(R v, R lo, R hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

// Square root and reciprocal: the hardware instructions (about 1 ulp) in FP32, the
// correctly rounded ones in FP64.
template <typename R>
__device__ __forceinline__ R fsqrt(R x) {
  if constexpr (sizeof(R) == 4) {
    return __builtin_amdgcn_sqrtf(x);
  } else {
    return sqrt(x);
  }
}

template <typename R>
__device__ __forceinline__ R frcp(R x) {
  if constexpr (sizeof(R) == 4) {
    return __builtin_amdgcn_rcpf(x);
  } else {
    return (R)1 / x;
  }
}

// Bilinear (r, z) interpolation clamped to the grid edge, scaled by sc:
// (bx, by, bz) = sc B with B_x,y = B_r (x, y)/r. `nodes` is the padded map in LDS
// (staged by the caller) or in global memory; r2 = x^2 + y^2 is passed in.
template <typename R>
__device__ __forceinline__ void field_rz_r2(const FieldDev& f, const float2* nodes, R x, R y, R z, R r2, R sc,
                                            R& bx, R& by, R& bz) {
  if constexpr (sizeof(R) == 4) {
    // FP32: one rsq, clamps by med3; the clamped coordinate is >= 0, so truncation
    // is the floor and fract the cell offset; at the upper edge the cell is the
    // padding one (offset 0)
    // + 1e-30 keeps rsq finite on the axis (r = 0 there) and vanishes against any
    // r^2 above 1e-22 mm^2
    const float inv_r = __builtin_amdgcn_rsqf(r2 + 1e-30f);
    const float r = r2 * inv_r;
    const float u = __builtin_amdgcn_fmed3f(fmaf(r, (float)f.inv_dr, (float)(-f.r0 * f.inv_dr)), 0.0f,
                                            (float)(f.nr - 1));
    const float v = __builtin_amdgcn_fmed3f(fmaf(z, (float)f.inv_dz, (float)(-f.z0 * f.inv_dz)), 0.0f,
                                            (float)(f.nz - 1));
    const float a = __builtin_amdgcn_fractf(u), b = __builtin_amdgcn_fractf(v);
    unsigned idx = __umul24((unsigned)(int)v, (unsigned)f.stride) + (unsigned)(int)u;
    // keep the node index as one value (one multiply-add, then one shift-add into the
    // address) rather than two shifted terms
    asm volatile("" : "+v"(idx));
    const float2* row0 = nodes + idx;
    const float2* row1 = row0 + f.stride;
    const float2 n00 = row0[0], n01 = row0[1], n10 = row1[0], n11 = row1[1];
    const float br0 = fmaf(a, n01.x - n00.x, n00.x);
    const float br1 = fmaf(a, n11.x - n10.x, n10.x);
    const float bz0 = fmaf(a, n01.y - n00.y, n00.y);
    const float bz1 = fmaf(a, n11.y - n10.y, n10.y);
    const float br = fmaf(b, br1 - br0, br0);
    bz = sc * fmaf(b, bz1 - bz0, bz0);
    // on the axis x = y = 0, so B_x = B_y = 0 whatever inv_r is (finite here)
    const float s = br * (sc * inv_r);
    bx = s * x;
    by = s * y;
  } else {
    const R r = sqrt(r2);
    const R inv_r = r > (R)1e-9 ? (R)1 / r : (R)0;
    const R u = clampv((r - (R)f.r0) * (R)f.inv_dr, (R)0, (R)(f.nr - 1));
    const R v = clampv((z - (R)f.z0) * (R)f.inv_dz, (R)0, (R)(f.nz - 1));
    const int iu = (int)u, jv = (int)v;
    const int i = iu < f.nr - 2 ? iu : f.nr - 2;
    const int j = jv < f.nz - 2 ? jv : f.nz - 2;
    const R a = u - (R)i;
    const R b = v - (R)j;
    const float2* row0 = nodes + j * f.stride + i;
    const float2* row1 = row0 + f.stride;
    const float2 n00 = row0[0], n01 = row0[1], n10 = row1[0], n11 = row1[1];
    const R br0 = (R)n00.x + a * ((R)n01.x - (R)n00.x);
    const R br1 = (R)n10.x + a * ((R)n11.x - (R)n10.x);
    const R bz0 = (R)n00.y + a * ((R)n01.y - (R)n00.y);
    const R bz1 = (R)n10.y + a * ((R)n11.y - (R)n10.y);
    const R br = br0 + b * (br1 - br0);
    bz = sc * (bz0 + b * (bz1 - bz0));
    const R s = sc * (br * inv_r);
    bx = s * x;
    by = s * y;
  }
}

template <typename R>
__device__ __forceinline__ R vmin(R a, R b) {
  if constexpr (sizeof(R) == 4) {
    return fminf(a, b);
  } else {
    return fmin(a, b);
  }
}

template <typename R>
__device__ __forceinline__ R vmax(R a, R b) {
  if constexpr (sizeof(R) == 4) {
    return fmaxf(a, b);
  } else {
    return fmax(a, b);
  }
}

template <typename R>
__device__ __forceinline__ R radius2(R x, R y) {
  if constexpr (sizeof(R) == 4) {
    return __builtin_fmaf(x, x, y * y);
  } else {
    return __builtin_fma(x, x, y * y);
  }
}

template <typename R>
__device__ __forceinline__ void field_rz(const FieldDev& f, const float2* nodes, R x, R y, R z, R& bx, R& by,
                                         R& bz) {
  field_rz_r2<R>(f, nodes, x, y, z, radius2(x, y), (R)1, bx, by, bz);
}

// Whether (x, y) lies strictly inside the seed cylinder r < R0 (r0sq = R0^2 in the
// state's precision): the end of a turn partition. One explicitly fused form, so
// that every kernel (scan, trace, adjoint recompute) takes the same decision on the
// same state.
template <typename R>
__device__ __forceinline__ bool inside_r0(R x, R y, R r0sq) {
  return radius2(x, y) < r0sq;
}

// Propagation state. For FP32 the position and the direction carry Kahan
// compensation terms (the sums of 1 mm increments into ~800 mm positions and of
// ~3e-3 increments into unit directions would otherwise drift).
template <typename R>
struct State {
  R x, y, z, tx, ty, tz, lam;
  R cx, cy, cz;
  R ctx, cty, ctz;
};

template <typename R>
__device__ __forceinline__ void kahan_add(R& s, R& c, R d) {
  const R y = d - c;
  const R t = s + y;
  c = (t - s) - y;
  s = t;
}

template <typename R>
__device__ __forceinline__ void turn(R& t, R& c, R d) {
  if constexpr (sizeof(R) == 4) {
    kahan_add(t, c, d);
  } else {
    t += d;
  }
}

template <typename R>
__device__ __forceinline__ void advance(State<R>& st, R dx, R dy, R dz) {
  if constexpr (sizeof(R) == 4) {
    kahan_add(st.x, st.cx, dx);
    kahan_add(st.y, st.cy, dy);
    kahan_add(st.z, st.cz, dz);
  } else {
    st.x += dx;
    st.y += dy;
    st.z += dz;
  }
}

// One RKN4 step (Nystrom formula for x'' = lam x' x B(x), three field evaluations:
// start, middle, end) as increments: from the position p and unit direction t, the
// changes d[0..2] of the position and d[3..5] of the direction over a step h.
// FIELD 0: uniform B_z; FIELD 1: (r, z) map, where the field is evaluated already
// scaled by lam (k = t x (lam B)) and r2 = px^2 + py^2 comes from the caller.
// With the map, b1 (if not NULL) is lam B at p, taken as given instead of evaluated,
// and b4 (if not NULL) receives lam B at the last stage's point
// p + h t + h^2/2 k3, r2_4 (if not NULL) that point's x^2 + y^2.
// RAW_W (FP32): d[0..2] = k1 + k2 + k3 and d[3..5] = k1 + 2 (k2 + k3) + k4, left for
// the caller to form the increments h t + h^2/6 d[0..2] and h/6 d[3..5] as
// multiply-adds into its sums (with the map; the uniform field returns them scaled).
template <typename R, int FIELD, bool RAW_W = false>
__device__ __forceinline__ void rkn_delta(const FieldDev& f, const float2* nodes, R lam, R h, R px, R py, R pz,
                                          R tx, R ty, R tz, R r2, R d[6], const R* b1 = nullptr,
                                          R* b4 = nullptr, R* r2_4 = nullptr) {
  const R h2 = (R)0.5 * h, hh6 = h * h / (R)6, h6 = RAW_W ? (R)1 : h / (R)6;
  if constexpr (FIELD == 0) {
    const R a = lam * (R)f.bz;
    const R k1x = a * ty, k1y = -a * tx;
    const R t2x = tx + h2 * k1x, t2y = ty + h2 * k1y;
    const R k2x = a * t2y, k2y = -a * t2x;
    const R t3x = tx + h2 * k2x, t3y = ty + h2 * k2y;
    const R k3x = a * t3y, k3y = -a * t3x;
    const R t4x = tx + h * k3x, t4y = ty + h * k3y;
    const R k4x = a * t4y, k4y = -a * t4x;
    d[0] = h * tx + hh6 * (k1x + k2x + k3x);
    d[1] = h * ty + hh6 * (k1y + k2y + k3y);
    d[2] = h * tz;
    d[3] = h6 * (k1x + (R)2 * (k2x + k3x) + k4x);
    d[4] = h6 * (k1y + (R)2 * (k2y + k3y) + k4y);
    d[5] = (R)0;
  } else {
    R bx, by, bz;   // lam B
    if (b1) {
      bx = b1[0];
      by = b1[1];
      bz = b1[2];
    } else {
      field_rz_r2(f, nodes, px, py, pz, r2, lam, bx, by, bz);
    }
    const R k1x = ty * bz - tz * by;
    const R k1y = tz * bx - tx * bz;
    const R k1z = tx * by - ty * bx;
    const R hh8 = h * h * (R)0.125;
    {
      const R qx = px + h2 * tx + hh8 * k1x, qy = py + h2 * ty + hh8 * k1y;
      field_rz_r2(f, nodes, qx, qy, pz + h2 * tz + hh8 * k1z, radius2(qx, qy), lam, bx, by, bz);
    }
    // stages 2 and 3 share the middle field
    const R t2x = tx + h2 * k1x, t2y = ty + h2 * k1y, t2z = tz + h2 * k1z;
    const R k2x = t2y * bz - t2z * by;
    const R k2y = t2z * bx - t2x * bz;
    const R k2z = t2x * by - t2y * bx;
    const R t3x = tx + h2 * k2x, t3y = ty + h2 * k2y, t3z = tz + h2 * k2z;
    const R k3x = t3y * bz - t3z * by;
    const R k3y = t3z * bx - t3x * bz;
    const R k3z = t3x * by - t3y * bx;
    const R hh2 = h * h * (R)0.5;
    {
      const R qx = px + h * tx + hh2 * k3x, qy = py + h * ty + hh2 * k3y;
      const R r2e = radius2(qx, qy);
      field_rz_r2(f, nodes, qx, qy, pz + h * tz + hh2 * k3z, r2e, lam, bx, by, bz);
      if (r2_4) *r2_4 = r2e;
    }
    const R t4x = tx + h * k3x, t4y = ty + h * k3y, t4z = tz + h * k3z;
    const R k4x = t4y * bz - t4z * by;
    const R k4y = t4z * bx - t4x * bz;
    const R k4z = t4x * by - t4y * bx;
    if (b4) {
      b4[0] = bx;
      b4[1] = by;
      b4[2] = bz;
    }
    if constexpr (sizeof(R) == 4 && RAW_W) {
      // d[0..2] = k1 + (k2 + k3), for the caller's q += h t + h^2/6 d (two multiply-adds)
      const R sx = k2x + k3x, sy = k2y + k3y, sz = k2z + k3z;
      d[0] = k1x + sx;
      d[1] = k1y + sy;
      d[2] = k1z + sz;
      d[3] = k1x + (R)2 * sx + k4x;
      d[4] = k1y + (R)2 * sy + k4y;
      d[5] = k1z + (R)2 * sz + k4z;
    } else if constexpr (sizeof(R) == 4) {
      const R sx = k2x + k3x, sy = k2y + k3y, sz = k2z + k3z;
      d[0] = h * tx + hh6 * (k1x + sx);
      d[1] = h * ty + hh6 * (k1y + sy);
      d[2] = h * tz + hh6 * (k1z + sz);
      d[3] = h6 * (k1x + (R)2 * sx + k4x);
      d[4] = h6 * (k1y + (R)2 * sy + k4y);
      d[5] = h6 * (k1z + (R)2 * sz + k4z);
    } else {
      d[0] = h * tx + hh6 * (k1x + k2x + k3x);
      d[1] = h * ty + hh6 * (k1y + k2y + k3y);
      d[2] = h * tz + hh6 * (k1z + k2z + k3z);
      d[3] = h6 * (k1x + (R)2 * (k2x + k3x) + k4x);
      d[4] = h6 * (k1y + (R)2 * (k2y + k3y) + k4y);
      d[5] = h6 * (k1z + (R)2 * (k2z + k3z) + k4z);
    }
  }
}

// One step applied to a State: FP32 with Kahan-compensated position and direction
// at every step (the adaptive path, whose trial steps can be rejected), FP64 plain.
template <typename R, int FIELD>
__device__ __forceinline__ void rkn_step(State<R>& st, const FieldDev& f, const float2* nodes, R h) {
  R d[6];
  rkn_delta<R, FIELD>(f, nodes, st.lam, h, st.x, st.y, st.z, st.tx, st.ty, st.tz,
                      FIELD == 1 ? radius2(st.x, st.y) : (R)0, d);
  turn(st.tx, st.ctx, d[3]);
  turn(st.ty, st.cty, d[4]);
  if (FIELD == 1) turn(st.tz, st.ctz, d[5]);
  advance(st, d[0], d[1], d[2]);
}

// Fixed-step propagation with block-relative sums. The State holds the origin of the
// current block (position and direction with their Kahan compensation terms); the
// current position p and direction t are that origin plus the plain sum q, u of the
// increments since the block started. fold() adds q and u into the origin with
// compensation and starts a new block at the result. In FP32 this keeps the origin's
// compensation (the sums of ~1 mm increments into ~800 mm positions, and of ~3e-3
// increments into unit directions, would otherwise drift by up to ~0.2 mm over 6000
// steps) while each step makes only plain adds; callers fold at the same step
// indices (the ends of the scan's cull blocks), so every kernel that recomputes a
// trajectory reproduces it exactly. In FP64 every step is a plain add into p and t
// (the oracle's sums) and fold() stores them.
//
// FP32 with the field map: the first stage of a step takes the field of the previous
// step's last stage, whose point p_n + h t_n + h^2/2 k3 lies (h^2/6) |2 k3 - k1 - k2|
// ~ h^3 |lam B|^2 / 6 ~ 1e-6 mm from p_{n+1}: below the FP32 spacing of positions
// there (3e-5 mm at 500 mm), so both points are mostly the same FP32 point, and the
// field's change over that distance (< 2e-10 relative in the solenoid map) is far
// below the FP32 rounding of the field itself. The field is evaluated at the seed
// (init_field) and wherever a caller restarts a trajectory from a stored state (the
// checkpoints of the refinement pass); fold() keeps it.
template <typename R, int FIELD>
struct Prop {
  static constexpr bool kReuse = sizeof(R) == 4 && FIELD == 1;
  R px, py, pz, tx, ty, tz;   // current position and direction
  R qx, qy, qz, ux, uy, uz;   // increments since the block started (FP32)
  R r2;                       // px^2 + py^2 (FP32 map: of the last stage's point, within
                              // ~1e-6 mm of p, for the cull's radial range)
  R fb[3];                    // lam B at the current point (FP32 map)
  __device__ __forceinline__ void start(const State<R>& s) {
    px = s.x;
    py = s.y;
    pz = s.z;
    tx = s.tx;
    ty = s.ty;
    tz = s.tz;
    qx = qy = qz = ux = uy = uz = (R)0;
    r2 = radius2(px, py);
  }
  // lam B evaluated at the current point (FP32 map; nothing otherwise)
  __device__ __forceinline__ void init_field(const State<R>& s, const FieldDev& f, const float2* nodes) {
    if constexpr (kReuse) field_rz_r2(f, nodes, px, py, pz, r2, s.lam, fb[0], fb[1], fb[2]);
  }
  __device__ __forceinline__ void step(const State<R>& s, const FieldDev& f, const float2* nodes, R h) {
    R d[6];
    constexpr bool kRawW = kReuse;   // FP32 map: the increments as multiply-adds into q, u
    rkn_delta<R, FIELD, kRawW>(f, nodes, s.lam, h, px, py, pz, tx, ty, tz, r2, d, kReuse ? fb : nullptr,
                               kReuse ? fb : nullptr, kReuse ? &r2 : nullptr);
    if constexpr (sizeof(R) == 4) {
      const R h6 = h / (R)6, hh6 = h * h / (R)6;
      if constexpr (FIELD == 1) {
        qx = __builtin_fmaf(hh6, d[0], __builtin_fmaf(h, tx, qx));
        qy = __builtin_fmaf(hh6, d[1], __builtin_fmaf(h, ty, qy));
        qz = __builtin_fmaf(hh6, d[2], __builtin_fmaf(h, tz, qz));
        ux = __builtin_fmaf(h6, d[3], ux);
        uy = __builtin_fmaf(h6, d[4], uy);
      } else {
        qx += d[0];
        qy += d[1];
        qz += d[2];
        ux += d[3];
        uy += d[4];
      }
      px = s.x + qx;
      py = s.y + qy;
      pz = s.z + qz;
      tx = s.tx + ux;
      ty = s.ty + uy;
      if constexpr (FIELD == 1) {
        uz = __builtin_fmaf(h6, d[5], uz);
        tz = s.tz + uz;
      }
      (void)h6;
      (void)hh6;
    } else {
      px += d[0];
      py += d[1];
      pz += d[2];
      tx += d[3];
      ty += d[4];
      if constexpr (FIELD == 1) tz += d[5];
    }
    if constexpr (!kReuse) r2 = radius2(px, py);
  }
  __device__ __forceinline__ void fold(State<R>& s) {
    if constexpr (sizeof(R) == 4) {
      kahan_add(s.x, s.cx, qx);
      kahan_add(s.y, s.cy, qy);
      kahan_add(s.z, s.cz, qz);
      kahan_add(s.tx, s.ctx, ux);
      kahan_add(s.ty, s.cty, uy);
      if constexpr (FIELD == 1) kahan_add(s.tz, s.ctz, uz);
    } else {
      s.x = px;
      s.y = py;
      s.z = pz;
      s.tx = tx;
      s.ty = ty;
      s.tz = tz;
    }
    start(s);
  }
};

// The same step with the local error estimate of the adaptive step size: err =
// h^2 |k1 - k2 - k3 + k4| (the stage accelerations agree to O(h^2) for a smooth
// force). Kept apart from rkn_step so that the fixed-step path carries none of it.
template <typename R, int FIELD>
__device__ __forceinline__ void rkn_step_err(State<R>& st, const FieldDev& f, const float2* nodes, R h, R& err) {
  const R h2 = (R)0.5 * h, hh6 = h * h / (R)6, h6 = h / (R)6;
  if constexpr (FIELD == 0) {
    const R a = st.lam * (R)f.bz;
    const R k1x = a * st.ty, k1y = -a * st.tx;
    const R t2x = st.tx + h2 * k1x, t2y = st.ty + h2 * k1y;
    const R k2x = a * t2y, k2y = -a * t2x;
    const R t3x = st.tx + h2 * k2x, t3y = st.ty + h2 * k2y;
    const R k3x = a * t3y, k3y = -a * t3x;
    const R t4x = st.tx + h * k3x, t4y = st.ty + h * k3y;
    const R k4x = a * t4y, k4y = -a * t4x;
    const R ex = k1x - k2x - k3x + k4x, ey = k1y - k2y - k3y + k4y;
    err = h * h * fsqrt(ex * ex + ey * ey);
    const R dx = h * st.tx + hh6 * (k1x + k2x + k3x);
    const R dy = h * st.ty + hh6 * (k1y + k2y + k3y);
    const R dz = h * st.tz;
    turn(st.tx, st.ctx, h6 * (k1x + (R)2 * (k2x + k3x) + k4x));
    turn(st.ty, st.cty, h6 * (k1y + (R)2 * (k2y + k3y) + k4y));
    advance(st, dx, dy, dz);
  } else {
    const R l = st.lam;
    R bx, by, bz;
    field_rz(f, nodes, st.x, st.y, st.z, bx, by, bz);
    const R k1x = l * (st.ty * bz - st.tz * by);
    const R k1y = l * (st.tz * bx - st.tx * bz);
    const R k1z = l * (st.tx * by - st.ty * bx);
    const R hh8 = h * h * (R)0.125;
    field_rz(f, nodes, st.x + h2 * st.tx + hh8 * k1x, st.y + h2 * st.ty + hh8 * k1y,
             st.z + h2 * st.tz + hh8 * k1z, bx, by, bz);
    const R t2x = st.tx + h2 * k1x, t2y = st.ty + h2 * k1y, t2z = st.tz + h2 * k1z;
    const R lbx = l * bx, lby = l * by, lbz = l * bz;
    const R k2x = t2y * lbz - t2z * lby;
    const R k2y = t2z * lbx - t2x * lbz;
    const R k2z = t2x * lby - t2y * lbx;
    const R t3x = st.tx + h2 * k2x, t3y = st.ty + h2 * k2y, t3z = st.tz + h2 * k2z;
    const R k3x = t3y * lbz - t3z * lby;
    const R k3y = t3z * lbx - t3x * lbz;
    const R k3z = t3x * lby - t3y * lbx;
    const R hh2 = h * h * (R)0.5;
    field_rz(f, nodes, st.x + h * st.tx + hh2 * k3x, st.y + h * st.ty + hh2 * k3y,
             st.z + h * st.tz + hh2 * k3z, bx, by, bz);
    const R t4x = st.tx + h * k3x, t4y = st.ty + h * k3y, t4z = st.tz + h * k3z;
    const R k4x = l * (t4y * bz - t4z * by);
    const R k4y = l * (t4z * bx - t4x * bz);
    const R k4z = l * (t4x * by - t4y * bx);
    const R ex = k1x - k2x - k3x + k4x, ey = k1y - k2y - k3y + k4y, ez = k1z - k2z - k3z + k4z;
    err = h * h * fsqrt(ex * ex + ey * ey + ez * ez);
    const R dx = h * st.tx + hh6 * (k1x + k2x + k3x);
    const R dy = h * st.ty + hh6 * (k1y + k2y + k3y);
    const R dz = h * st.tz + hh6 * (k1z + k2z + k3z);
    turn(st.tx, st.ctx, h6 * (k1x + (R)2 * (k2x + k3x) + k4x));
    turn(st.ty, st.cty, h6 * (k1y + (R)2 * (k2y + k3y) + k4y));
    turn(st.tz, st.ctz, h6 * (k1z + (R)2 * (k2z + k3z) + k4z));
    advance(st, dx, dy, dz);
  }
}

// Exact squared distance between the chord p0 + s d (s in [0,1]) and the wire
// m + t u (|t| <= L, |u| = 1): clamp the chord parameter of the line-line optimum,
// take the wire's closest parameter for it, and if that leaves [-L, L] clamp it and
// re-optimise the chord parameter (convexity makes this the global minimum).
template <typename R>
__device__ __forceinline__ R seg_wire_d2(R p0x, R p0y, R p0z, R p1x, R p1y, R p1z, R mx, R my,
                                         R mz, R ux, R uy, R uz, R L) {
  const R dx = p1x - p0x, dy = p1y - p0y, dz = p1z - p0z;
  const R rx = p0x - mx, ry = p0y - my, rz = p0z - mz;
  const R a = dx * dx + dy * dy + dz * dz;
  const R b = dx * ux + dy * uy + dz * uz;
  const R e = dx * rx + dy * ry + dz * rz;
  const R f = ux * rx + uy * ry + uz * rz;
  const R den = a - b * b;
  R s = den > (R)1e-6 * a ? (b * f - e) * frcp(den) : (R)0;
  s = clampv(s, (R)0, (R)1);
  const R t = b * s + f;
  const R tc = clampv(t, -L, L);
  if (tc != t) s = a > (R)0 ? clampv((tc * b - e) * frcp(a), (R)0, (R)1) : (R)0;
  const R vx = rx + s * dx - tc * ux;
  const R vy = ry + s * dy - tc * uy;
  const R vz = rz + s * dz - tc * uz;
  return vx * vx + vy * vy + vz * vz;
}

__device__ __forceinline__ int wave_min_i32(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const int w = __shfl_xor(v, o, 64);
    v = w < v ? w : v;
  }
  return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ int wave_max_i32(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const int w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ uint32_t lane_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

}  // namespace rkn
