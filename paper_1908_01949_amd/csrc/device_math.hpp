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

// Axisymmetric field: uniform B_z, or FP32 (B_r, B_z) nodes interleaved [nz][nr].
struct FieldDev {
  const float2* nodes;
  int nr, nz;
  double r0, z0, inv_dr, inv_dz;
  double bz;
};

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

// Bilinear (r, z) interpolation clamped to the grid edge; B_x,y = B_r (x, y)/r.
// `nodes` is the map in LDS (staged by the caller) or in global memory. The cell
// index is truncated from the clamped coordinate, which equals the floor there.
template <typename R>
__device__ __forceinline__ void field_rz(const FieldDev& f, const float2* nodes, R x, R y, R z, R& bx, R& by,
                                         R& bz) {
  if constexpr (sizeof(R) == 4) {
    // FP32: one rsq, clamps by med3, the cell from floor in float (exact for the
    // small integers involved), and the node index from one fma.
    const float r2 = fmaf(x, x, y * y);
    const float inv_r = __builtin_amdgcn_rsqf(fmaxf(r2, 1e-30f));
    const float r = r2 * inv_r;
    const float fnr = (float)f.nr, fnz = (float)f.nz;
    const float u = __builtin_amdgcn_fmed3f(fmaf(r, (float)f.inv_dr, (float)(-f.r0 * f.inv_dr)), 0.0f, fnr - 1.0f);
    const float v = __builtin_amdgcn_fmed3f(fmaf(z, (float)f.inv_dz, (float)(-f.z0 * f.inv_dz)), 0.0f, fnz - 1.0f);
    const float fi = fminf(floorf(u), fnr - 2.0f);
    const float fj = fminf(floorf(v), fnz - 2.0f);
    const float a = u - fi, b = v - fj;
    const float2* row0 = nodes + (int)fmaf(fj, fnr, fi);
    const float2* row1 = row0 + f.nr;
    const float2 n00 = row0[0], n01 = row0[1], n10 = row1[0], n11 = row1[1];
    const float br0 = fmaf(a, n01.x - n00.x, n00.x);
    const float br1 = fmaf(a, n11.x - n10.x, n10.x);
    const float bz0 = fmaf(a, n01.y - n00.y, n00.y);
    const float bz1 = fmaf(a, n11.y - n10.y, n10.y);
    const float br = fmaf(b, br1 - br0, br0);
    bz = fmaf(b, bz1 - bz0, bz0);
    // on the axis x = y = 0, so B_x = B_y = 0 whatever inv_r is (finite here)
    const float s = br * inv_r;
    bx = s * x;
    by = s * y;
  } else {
    const R r2 = x * x + y * y;
    const R r = sqrt(r2);
    const R inv_r = r > (R)1e-9 ? (R)1 / r : (R)0;
    const R u = clampv((r - (R)f.r0) * (R)f.inv_dr, (R)0, (R)(f.nr - 1));
    const R v = clampv((z - (R)f.z0) * (R)f.inv_dz, (R)0, (R)(f.nz - 1));
    const int iu = (int)u, jv = (int)v;
    const int i = iu < f.nr - 2 ? iu : f.nr - 2;
    const int j = jv < f.nz - 2 ? jv : f.nz - 2;
    const R a = u - (R)i;
    const R b = v - (R)j;
    const float2* row0 = nodes + j * f.nr + i;
    const float2* row1 = row0 + f.nr;
    const float2 n00 = row0[0], n01 = row0[1], n10 = row1[0], n11 = row1[1];
    const R br0 = (R)n00.x + a * ((R)n01.x - (R)n00.x);
    const R br1 = (R)n10.x + a * ((R)n11.x - (R)n10.x);
    const R bz0 = (R)n00.y + a * ((R)n01.y - (R)n00.y);
    const R bz1 = (R)n10.y + a * ((R)n11.y - (R)n10.y);
    const R br = br0 + b * (br1 - br0);
    bz = bz0 + b * (bz1 - bz0);
    const R s = br * inv_r;
    bx = s * x;
    by = s * y;
  }
}

// Whether (x, y) lies strictly inside the seed cylinder r < R0 (r0sq = R0^2 in the
// state's precision): the end of a turn partition. One explicitly fused form, so
// that every kernel (scan, trace, adjoint recompute) takes the same decision on the
// same state.
template <typename R>
__device__ __forceinline__ bool inside_r0(R x, R y, R r0sq) {
  if constexpr (sizeof(R) == 4) {
    return __builtin_fmaf(x, x, y * y) < r0sq;
  } else {
    return __builtin_fma(x, x, y * y) < r0sq;
  }
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
// start, middle, end). FIELD 0: uniform B_z; FIELD 1: (r, z) map.
template <typename R, int FIELD>
__device__ __forceinline__ void rkn_step(State<R>& st, const FieldDev& f, const float2* nodes, R h) {
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
    // stages 2 and 3 share the middle field: scale it by Lambda once
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
    const R dx = h * st.tx + hh6 * (k1x + k2x + k3x);
    const R dy = h * st.ty + hh6 * (k1y + k2y + k3y);
    const R dz = h * st.tz + hh6 * (k1z + k2z + k3z);
    turn(st.tx, st.ctx, h6 * (k1x + (R)2 * (k2x + k3x) + k4x));
    turn(st.ty, st.cty, h6 * (k1y + (R)2 * (k2y + k3y) + k4y));
    turn(st.tz, st.ctz, h6 * (k1z + (R)2 * (k2z + k3z) + k4z));
    advance(st, dx, dy, dz);
  }
}

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
