// Differentiated refinement of seeds: a checkpointed FP32 forward pass, a
// hand-written adjoint backward sweep and a Gauss-Newton update in FP64.
//
// The paper refines the best seeds by rescanning finer grids ten times (section
// 2.2); this is the derivative-based alternative. Objective per seed:
//   Phi(s) = sum over the inlier set S of r_i^2,  r_i = D_i(s) - d_i,
// S fixed by the classification rule (D - d)^2 < lambda at the starting seed.
// Derivatives are those of the discrete map (the RKN steps as computed). D_i is a
// minimum over chords; at its minimising chord n with parameters (s*, t*) and unit
// closest-approach vector w, dD/dx_n = (1 - s*) w and dD/dx_{n+1} = s* w.
//
// State y = (x, T, Lambda) in R^7; M_n = dy_{n+1}/dy_n. The backward sweep runs, for
// n = N-1 .. 0, with e_i = [(1 - s*) w; 0] + M_n^T [s* w; 0] for the hits whose
// minimum is on chord n:
//   lambda_n = M_n^T lambda_{n+1} + sum c_i e_i        (gradient, c_i = dF/dr_i)
//   S_n      = M_n^T S_{n+1} M_n + sum e_i e_i^T       (Gauss-Newton matrix)
// so that with P = dy_0/ds: grad = P^T lambda_0, J^T J = P^T S_0 P, and with
// c_i = 2 r_i, J^T r = grad / 2. States are recomputed segment by segment from the
// checkpoints written by the forward pass every `ckpt` steps. lambda and S are
// accumulated in FP64; M_n comes from forward-mode tangents through the FP32 step.
#include <math.h>

#include <algorithm>
#include <string>
#include <vector>

#include "internal.hpp"

namespace rkn {

// Field map and its Jacobian dB/dx (row = component, column = d/dx_k), FP32.
__device__ __forceinline__ void field_rz_jac(const FieldDev& f, float x, float y, float z, float B[3],
                                             float J[3][3]) {
  const float r2 = x * x + y * y;
  const float inv_r = __builtin_amdgcn_rsqf(r2 > 1e-30f ? r2 : 1e-30f);
  const float r = r2 * inv_r;
  const float uraw = (r - (float)f.r0) * (float)f.inv_dr;
  const float vraw = (z - (float)f.z0) * (float)f.inv_dz;
  const float u = clampv(uraw, 0.0f, (float)(f.nr - 1));
  const float v = clampv(vraw, 0.0f, (float)(f.nz - 1));
  const bool in_r = uraw == u, in_z = vraw == v;
  const int iu = (int)u, jv = (int)v;
  const int i = iu < f.nr - 2 ? iu : f.nr - 2;
  const int j = jv < f.nz - 2 ? jv : f.nz - 2;
  const float a = u - (float)i, b = v - (float)j;
  const float2* row0 = f.nodes + j * f.stride + i;
  const float2* row1 = row0 + f.stride;
  const float2 n00 = row0[0], n01 = row0[1], n10 = row1[0], n11 = row1[1];
  const float r0r = n00.x + a * (n01.x - n00.x), r1r = n10.x + a * (n11.x - n10.x);
  const float r0z = n00.y + a * (n01.y - n00.y), r1z = n10.y + a * (n11.y - n10.y);
  const float br = r0r + b * (r1r - r0r);
  const float bz = r0z + b * (r1z - r0z);
  const float dbr_dr = in_r ? ((n01.x - n00.x) + b * ((n11.x - n10.x) - (n01.x - n00.x))) * (float)f.inv_dr : 0.0f;
  const float dbz_dr = in_r ? ((n01.y - n00.y) + b * ((n11.y - n10.y) - (n01.y - n00.y))) * (float)f.inv_dr : 0.0f;
  const float dbr_dz = in_z ? (r1r - r0r) * (float)f.inv_dz : 0.0f;
  const float dbz_dz = in_z ? (r1z - r0z) * (float)f.inv_dz : 0.0f;
  const float cx = x * inv_r, cy = y * inv_r;
  const float q = br * inv_r;   // B_r / r
  B[0] = q * x;
  B[1] = q * y;
  B[2] = bz;
  J[0][0] = dbr_dr * cx * cx + q * (1.0f - cx * cx);
  J[0][1] = (dbr_dr - q) * cx * cy;
  J[0][2] = dbr_dz * cx;
  J[1][0] = (dbr_dr - q) * cx * cy;
  J[1][1] = dbr_dr * cy * cy + q * (1.0f - cy * cy);
  J[1][2] = dbr_dz * cy;
  J[2][0] = dbz_dr * cx;
  J[2][1] = dbz_dr * cy;
  J[2][2] = dbz_dz;
}

template <int FIELD>
__device__ __forceinline__ void field_and_jac(const FieldDev& f, const float p[3], float B[3], float J[3][3]) {
  if constexpr (FIELD == 0) {
    B[0] = 0.0f;
    B[1] = 0.0f;
    B[2] = (float)f.bz;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int k = 0; k < 3; ++k) J[c][k] = 0.0f;
  } else {
    field_rz_jac(f, p[0], p[1], p[2], B, J);
  }
}

__device__ __forceinline__ void cross(const float a[3], const float b[3], float o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

// M = d(x', T', Lambda)/d(x, T, Lambda) of one FP32 RKN step at state st: the seven
// tangent columns carried through the step's stages (the same stage arithmetic as
// the forward step; the compensation terms are rounding corrections, not state).
template <int FIELD>
__device__ void step_jacobian(const State<float>& st, const FieldDev& f, float h, float M[7][7]) {
  const float L = st.lam;
  const float T[3] = {st.tx, st.ty, st.tz};
  const float X[3] = {st.x, st.y, st.z};
  const float h2 = 0.5f * h, hh8 = h * h * 0.125f, hh2 = h * h * 0.5f, hh6 = h * h / 6.0f, h6 = h / 6.0f;
  float B1[3], J1[3][3], B2[3], J2[3][3], B3[3], J3[3][3], TB[3];
  float k1[3], k2[3], k3[3], T2[3], T3[3], T4[3], xm[3], xe[3];
  field_and_jac<FIELD>(f, X, B1, J1);
  cross(T, B1, TB);
#pragma unroll
  for (int c = 0; c < 3; ++c) k1[c] = L * TB[c];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    xm[c] = X[c] + h2 * T[c] + hh8 * k1[c];
    T2[c] = T[c] + h2 * k1[c];
  }
  field_and_jac<FIELD>(f, xm, B2, J2);
  cross(T2, B2, TB);
#pragma unroll
  for (int c = 0; c < 3; ++c) k2[c] = L * TB[c];
#pragma unroll
  for (int c = 0; c < 3; ++c) T3[c] = T[c] + h2 * k2[c];
  cross(T3, B2, TB);
#pragma unroll
  for (int c = 0; c < 3; ++c) k3[c] = L * TB[c];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    xe[c] = X[c] + h * T[c] + hh2 * k3[c];
    T4[c] = T[c] + h * k3[c];
  }
  field_and_jac<FIELD>(f, xe, B3, J3);
#pragma unroll
  for (int q = 0; q < 7; ++q) {
    float dx[3] = {q == 0 ? 1.0f : 0.0f, q == 1 ? 1.0f : 0.0f, q == 2 ? 1.0f : 0.0f};
    float dT[3] = {q == 3 ? 1.0f : 0.0f, q == 4 ? 1.0f : 0.0f, q == 5 ? 1.0f : 0.0f};
    const float dL = q == 6 ? 1.0f : 0.0f;
    float dk1[3], dk2[3], dk3[3], dk4[3], dxm[3], dxe[3], dTt[3], dB[3], t1[3], t2[3], tb[3];
    // stage 1
#pragma unroll
    for (int c = 0; c < 3; ++c) dB[c] = J1[c][0] * dx[0] + J1[c][1] * dx[1] + J1[c][2] * dx[2];
    cross(T, B1, tb);
    cross(dT, B1, t1);
    cross(T, dB, t2);
#pragma unroll
    for (int c = 0; c < 3; ++c) dk1[c] = dL * tb[c] + L * (t1[c] + t2[c]);
    // stage 2
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      dxm[c] = dx[c] + h2 * dT[c] + hh8 * dk1[c];
      dTt[c] = dT[c] + h2 * dk1[c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) dB[c] = J2[c][0] * dxm[0] + J2[c][1] * dxm[1] + J2[c][2] * dxm[2];
    cross(T2, B2, tb);
    cross(dTt, B2, t1);
    cross(T2, dB, t2);
#pragma unroll
    for (int c = 0; c < 3; ++c) dk2[c] = dL * tb[c] + L * (t1[c] + t2[c]);
    // stage 3 (shares the middle field)
#pragma unroll
    for (int c = 0; c < 3; ++c) dTt[c] = dT[c] + h2 * dk2[c];
    cross(T3, B2, tb);
    cross(dTt, B2, t1);
    cross(T3, dB, t2);
#pragma unroll
    for (int c = 0; c < 3; ++c) dk3[c] = dL * tb[c] + L * (t1[c] + t2[c]);
    // stage 4
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      dxe[c] = dx[c] + h * dT[c] + hh2 * dk3[c];
      dTt[c] = dT[c] + h * dk3[c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) dB[c] = J3[c][0] * dxe[0] + J3[c][1] * dxe[1] + J3[c][2] * dxe[2];
    cross(T4, B3, tb);
    cross(dTt, B3, t1);
    cross(T4, dB, t2);
#pragma unroll
    for (int c = 0; c < 3; ++c) dk4[c] = dL * tb[c] + L * (t1[c] + t2[c]);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      M[c][q] = dx[c] + h * dT[c] + hh6 * (dk1[c] + dk2[c] + dk3[c]);
      M[3 + c][q] = dT[c] + h6 * (dk1[c] + 2.0f * (dk2[c] + dk3[c]) + dk4[c]);
    }
    M[6][q] = dL;
  }
}

// Closest points of chord [p0, p1] and wire m + t u (|t| <= Lw): same rule as the
// scan's distance, also returning s* and the closest-approach vector.
__device__ __forceinline__ float seg_wire_closest(const float p0[3], const float p1[3], const float m[3],
                                                  const float u[3], float Lw, float& s, float w[3]) {
  const float d[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
  const float r[3] = {p0[0] - m[0], p0[1] - m[1], p0[2] - m[2]};
  const float a = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  const float b = d[0] * u[0] + d[1] * u[1] + d[2] * u[2];
  const float e = d[0] * r[0] + d[1] * r[1] + d[2] * r[2];
  const float g = u[0] * r[0] + u[1] * r[1] + u[2] * r[2];
  const float den = a - b * b;
  s = den > 1e-6f * a ? (b * g - e) / den : 0.0f;
  s = clampv(s, 0.0f, 1.0f);
  const float t = b * s + g;
  const float tc = clampv(t, -Lw, Lw);
  if (tc != t) s = a > 0.0f ? clampv((tc * b - e) / a, 0.0f, 1.0f) : 0.0f;
#pragma unroll
  for (int c = 0; c < 3; ++c) w[c] = r[c] + s * d[c] - tc * u[c];
  return w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
}

__device__ __forceinline__ State<float> load_state(const float* base, int64_t stride) {
  State<float> s;
  s.x = base[0 * stride];
  s.y = base[1 * stride];
  s.z = base[2 * stride];
  s.cx = base[3 * stride];
  s.cy = base[4 * stride];
  s.cz = base[5 * stride];
  s.tx = base[6 * stride];
  s.ty = base[7 * stride];
  s.tz = base[8 * stride];
  s.ctx = base[9 * stride];
  s.cty = base[10 * stride];
  s.ctz = base[11 * stride];
  s.lam = base[12 * stride];
  return s;
}

struct BwdArgs {
  FieldDev field;
  int64_t n;                  // seeds (slots)
  int n_steps, ckpt, n_ckpt;
  int turn_stop;              // 1: the forward pass froze the state at the end of the turn partition
  float h;
  double R0, charge;
  const double* seeds5;       // [n][5]
  const int32_t* seed_event;  // [n]
  const int32_t* ev_off;
  const int32_t* hits_wire;   // wire id per hit, original order
  const HitRec<float>* wire32;
  const float* tape;          // [n_ckpt][13][n] checkpoints
  const float* resid;         // [n][max_hits]
  const int32_t* argmin;      // [n][max_hits] chord index, -1 outside the inlier set
  const float* cgrad;         // [n][max_hits] upstream dF/dr, or NULL: c = 2 r
  int max_hits;
  float* segbuf;              // [n_ckpt][ckpt+1][6][n] recomputed (x, T) per step
  int32_t* segoff;            // [n_ckpt+1][n] list offsets of each segment's hits
  int2* list;                 // [max_hits][n] (chord, hit) grouped by segment
  double* segout;             // [n_ckpt][kSegVals][n] per segment: Phi, a, A
  double* grad;               // [n][5]
  double* jtj;                // [n][25] or NULL
};

// Per segment: the transfer matrix Phi (7x7, row-major), the accumulated adjoint
// source a (7) and the Gauss-Newton source A (7x7 symmetric, 28 upper entries).
constexpr int kSegVals = 49 + 7 + 28;

__device__ __forceinline__ int upper_index(int r, int c) {   // r <= c
  return r * 7 - r * (r - 1) / 2 + (c - r);
}

// Group each seed's inlier hits by the segment of their minimising chord (counting
// sort over segments; the order within a segment does not matter).
__global__ void __launch_bounds__(64) adj_prep_kernel(BwdArgs a) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.n) return;
  const int64_t n = a.n;
  const int e = a.seed_event[p];
  const int nh = a.ev_off[e + 1] - a.ev_off[e];
  for (int k = 0; k <= a.n_ckpt; ++k) a.segoff[(size_t)k * n + p] = 0;
  for (int o = 0; o < nh; ++o) {
    const int st = a.argmin[p * a.max_hits + o];
    if (st >= 0) a.segoff[(size_t)(st / a.ckpt + 1) * n + p] += 1;
  }
  int acc = 0;
  for (int k = 0; k <= a.n_ckpt; ++k) {
    acc += a.segoff[(size_t)k * n + p];
    a.segoff[(size_t)k * n + p] = acc;     // segoff[k] = first list slot of segment k
  }
  for (int o = 0; o < nh; ++o) {
    const int st = a.argmin[p * a.max_hits + o];
    if (st < 0) continue;
    const size_t cs = (size_t)(st / a.ckpt) * n + p;
    const int pos = a.segoff[cs];
    a.segoff[cs] = pos + 1;
    a.list[(size_t)pos * n + p] = make_int2(st, o);
  }
  // the scatter advanced each offset to the next segment's start: shift back
  for (int k = a.n_ckpt; k >= 1; --k) a.segoff[(size_t)k * n + p] = a.segoff[(size_t)(k - 1) * n + p];
  a.segoff[p] = 0;
}

// One (segment, seed) work item: recompute the segment's states from its checkpoint,
// then walk its steps backwards from lambda = 0, S = 0 at the segment end:
//   Phi <- M_n^T Phi,  a <- M_n^T a + sum c e,  A <- M_n^T A M_n + sum e e^T,
// so that lambda(start) = Phi lambda(end) + a and S(start) = Phi S(end) Phi^T + A.
template <int FIELD, bool WANT_S>
__global__ void __launch_bounds__(64) adj_seg_kernel(BwdArgs a) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = a.n;
  if (idx >= n * a.n_ckpt) return;
  const int k = (int)(idx / n);
  const int64_t p = idx - (int64_t)k * n;
  const int n0 = k * a.ckpt;
  const int n1 = min(n0 + a.ckpt, a.n_steps);
  float* sb = a.segbuf + (size_t)k * (a.ckpt + 1) * 6 * n + p;
  State<float> s = load_state(a.tape + (size_t)k * 13 * n + p, n);
  const float lam = s.lam;
  auto put = [&](int j, const State<float>& q) {
    float* b = sb + (size_t)j * 6 * n;
    b[0] = q.x;
    b[n] = q.y;
    b[2 * n] = q.z;
    b[3 * n] = q.tx;
    b[4 * n] = q.ty;
    b[5 * n] = q.tz;
  };
  auto get = [&](int j) {
    const float* b = sb + (size_t)j * 6 * n;
    State<float> q{};
    q.x = b[0];
    q.y = b[n];
    q.z = b[2 * n];
    q.tx = b[3 * n];
    q.ty = b[4 * n];
    q.tz = b[5 * n];
    q.lam = lam;
    return q;
  };
  // The forward pass's propagation: block-relative sums folded at the ends of its
  // kRefineBlock-step blocks (and at the last step) when the track was live at the
  // block's start; the checkpoint is taken right after a fold. With the
  // turn-partition stop the forward pass took a step only while every earlier step
  // ended outside r < R0 (the seed itself is not tested) and froze the state after
  // that; steps from first_frozen on leave the state as it is (M = I).
  const float r0sq = (float)(a.R0 * a.R0);
  bool live = !(a.turn_stop && k > 0 && inside_r0(s.x, s.y, r0sq));
  bool live_blk = live;
  int first_frozen = live ? n1 : n0;
  Prop<float, FIELD> pr;
  pr.start(s);
  pr.init_field(s, a.field, a.field.nodes);
  auto cur = [&]() {
    State<float> q = s;
    q.x = pr.px;
    q.y = pr.py;
    q.z = pr.pz;
    q.tx = pr.tx;
    q.ty = pr.ty;
    q.tz = pr.tz;
    return q;
  };
  put(0, cur());
  for (int j = 1; j <= n1 - n0; ++j) {
    if (live) {
      pr.step(s, a.field, a.field.nodes, a.h);
      if (a.turn_stop && inside_r0(pr.px, pr.py, r0sq)) {
        live = false;
        first_frozen = n0 + j;
      }
    }
    if ((n0 + j) % kRefineBlock == 0 || n0 + j == a.n_steps) {
      if (live_blk) pr.fold(s);
      live_blk = live;
    }
    put(j, cur());
  }
  const int e = a.seed_event[p];
  const int hb = a.ev_off[e];
  const int l0 = a.segoff[(size_t)k * n + p], l1 = a.segoff[(size_t)(k + 1) * n + p];
  double Phi[7][7], av[7], A[28];
#pragma unroll
  for (int r = 0; r < 7; ++r) {
    av[r] = 0.0;
#pragma unroll
    for (int c = 0; c < 7; ++c) Phi[r][c] = r == c ? 1.0 : 0.0;
  }
#pragma unroll
  for (int q = 0; q < 28; ++q) A[q] = 0.0;
  for (int st = n1 - 1; st >= n0; --st) {
    const State<float> sn = get(st - n0);
    const bool frozen = st >= first_frozen;
    float M[7][7];
    if (frozen) {
#pragma unroll
      for (int r = 0; r < 7; ++r)
#pragma unroll
        for (int c = 0; c < 7; ++c) M[r][c] = r == c ? 1.0f : 0.0f;
    } else {
      step_jacobian<FIELD>(sn, a.field, a.h, M);
    }
    // Phi <- M^T Phi, a <- M^T a (column by column, in place); nothing when frozen
    if (!frozen) {
#pragma unroll
      for (int c = 0; c < 7; ++c) {
        double col[7];
#pragma unroll
        for (int r = 0; r < 7; ++r) {
          double acc = 0.0;
#pragma unroll
          for (int q = 0; q < 7; ++q) acc += (double)M[q][r] * Phi[q][c];
          col[r] = acc;
        }
#pragma unroll
        for (int r = 0; r < 7; ++r) Phi[r][c] = col[r];
      }
      {
        double col[7];
#pragma unroll
        for (int r = 0; r < 7; ++r) {
          double acc = 0.0;
#pragma unroll
          for (int q = 0; q < 7; ++q) acc += (double)M[q][r] * av[q];
          col[r] = acc;
        }
#pragma unroll
        for (int r = 0; r < 7; ++r) av[r] = col[r];
      }
      if constexpr (WANT_S) {
        // A <- M^T A M over the upper triangle: B = A M by columns, then (M^T B)
        double nA[28];
#pragma unroll
        for (int c = 0; c < 7; ++c) {
          double b[7];
#pragma unroll
          for (int r = 0; r < 7; ++r) {
            double acc = 0.0;
#pragma unroll
            for (int q = 0; q < 7; ++q) acc += A[r <= q ? upper_index(r, q) : upper_index(q, r)] * (double)M[q][c];
            b[r] = acc;
          }
#pragma unroll
          for (int r = 0; r <= c; ++r) {
            double acc = 0.0;
#pragma unroll
            for (int q = 0; q < 7; ++q) acc += (double)M[q][r] * b[q];
            nA[upper_index(r, c)] = acc;
          }
        }
#pragma unroll
        for (int q = 0; q < 28; ++q) A[q] = nA[q];
      }
    }
    // sources of the hits whose minimum lies on chord st
    for (int li = l0; li < l1; ++li) {
      const int2 it = a.list[(size_t)li * n + p];
      if (it.x != st) continue;
      const int o = it.y;
      const State<float> sn1 = get(st - n0 + 1);
      const HitRec<float> w = a.wire32[a.hits_wire[hb + o]];
      const float p0[3] = {sn.x, sn.y, sn.z}, p1[3] = {sn1.x, sn1.y, sn1.z};
      const float m[3] = {w.mx, w.my, w.mz}, u[3] = {w.ux, w.uy, w.uz};
      float sstar, v[3];
      const float d2 = seg_wire_closest(p0, p1, m, u, w.L, sstar, v);
      const float D = sqrtf(d2);
      if (!(D > 0.0f)) continue;   // D = 0: the derivative is taken as 0
      const float iv = 1.0f / D;
      const float aa[3] = {(1.0f - sstar) * v[0] * iv, (1.0f - sstar) * v[1] * iv, (1.0f - sstar) * v[2] * iv};
      const float bb[3] = {sstar * v[0] * iv, sstar * v[1] * iv, sstar * v[2] * iv};
      double ev[7];
#pragma unroll
      for (int c = 0; c < 7; ++c) {
        double acc = c < 3 ? (double)aa[c] : 0.0;
#pragma unroll
        for (int q = 0; q < 3; ++q) acc += (double)M[q][c] * (double)bb[q];
        ev[c] = acc;
      }
      const float r = a.resid[p * a.max_hits + o];
      const double cg = a.cgrad ? (double)a.cgrad[p * a.max_hits + o] : 2.0 * (double)r;
#pragma unroll
      for (int c = 0; c < 7; ++c) av[c] += cg * ev[c];
      if constexpr (WANT_S) {
#pragma unroll
        for (int r2 = 0; r2 < 7; ++r2)
#pragma unroll
          for (int c = r2; c < 7; ++c) A[upper_index(r2, c)] += ev[r2] * ev[c];
      }
    }
  }
  double* out = a.segout + (size_t)k * kSegVals * n + p;
#pragma unroll
  for (int r = 0; r < 7; ++r)
#pragma unroll
    for (int c = 0; c < 7; ++c) out[(size_t)(r * 7 + c) * n] = Phi[r][c];
#pragma unroll
  for (int r = 0; r < 7; ++r) out[(size_t)(49 + r) * n] = av[r];
  if constexpr (WANT_S) {
#pragma unroll
    for (int q = 0; q < 28; ++q) out[(size_t)(56 + q) * n] = A[q];
  }
}

// Per seed: lambda_0 and S_0 from the segments, last to first, then the seed
// derivatives through P = dy0/dseed: grad = P^T lambda_0, J^T J = P^T S_0 P.
template <bool WANT_S>
__global__ void __launch_bounds__(64) adj_combine_kernel(BwdArgs a) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.n) return;
  const int64_t n = a.n;
  double lam[7] = {0, 0, 0, 0, 0, 0, 0};
  double S[28];
#pragma unroll
  for (int q = 0; q < 28; ++q) S[q] = 0.0;
  for (int k = a.n_ckpt - 1; k >= 0; --k) {
    const double* in = a.segout + (size_t)k * kSegVals * n + p;
    double Phi[7][7];
#pragma unroll
    for (int r = 0; r < 7; ++r)
#pragma unroll
      for (int c = 0; c < 7; ++c) Phi[r][c] = in[(size_t)(r * 7 + c) * n];
    double nl[7];
#pragma unroll
    for (int r = 0; r < 7; ++r) {
      double acc = in[(size_t)(49 + r) * n];
#pragma unroll
      for (int c = 0; c < 7; ++c) acc += Phi[r][c] * lam[c];
      nl[r] = acc;
    }
#pragma unroll
    for (int r = 0; r < 7; ++r) lam[r] = nl[r];
    if constexpr (WANT_S) {
      // S <- Phi S Phi^T + A
      double B[7][7];   // B = Phi S
#pragma unroll
      for (int r = 0; r < 7; ++r)
#pragma unroll
        for (int c = 0; c < 7; ++c) {
          double acc = 0.0;
#pragma unroll
          for (int q = 0; q < 7; ++q) acc += Phi[r][q] * S[q <= c ? upper_index(q, c) : upper_index(c, q)];
          B[r][c] = acc;
        }
#pragma unroll
      for (int r = 0; r < 7; ++r)
#pragma unroll
        for (int c = r; c < 7; ++c) {
          double acc = in[(size_t)(56 + upper_index(r, c)) * n];
#pragma unroll
          for (int q = 0; q < 7; ++q) acc += B[r][q] * Phi[c][q];
          S[upper_index(r, c)] = acc;
        }
    }
  }
  const double* sd = a.seeds5 + 5 * p;
  const double pm = sqrt(sd[2] * sd[2] + sd[3] * sd[3] + sd[4] * sd[4]);
  double P[7][5];
#pragma unroll
  for (int i = 0; i < 7; ++i)
#pragma unroll
    for (int j = 0; j < 5; ++j) P[i][j] = 0.0;
  if (pm >= 1e-3) {
    const double T0[3] = {sd[2] / pm, sd[3] / pm, sd[4] / pm};
    P[0][0] = -a.R0 * sin(sd[0]);
    P[1][0] = a.R0 * cos(sd[0]);
    P[2][1] = 1.0;
    for (int c = 0; c < 3; ++c)
      for (int q = 0; q < 3; ++q) P[3 + c][2 + q] = ((c == q ? 1.0 : 0.0) - T0[c] * T0[q]) / pm;
    const double lam0 = kKappa * a.charge / pm;   // dLambda/dp_j = -Lambda T_j / |p|
    for (int q = 0; q < 3; ++q) P[6][2 + q] = -lam0 * T0[q] / pm;
  }
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < 7; ++i) acc += P[i][j] * lam[i];
    a.grad[p * 5 + j] = acc;
  }
  if constexpr (WANT_S) {
    if (a.jtj) {
#pragma unroll
      for (int r = 0; r < 5; ++r)
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          double acc = 0.0;
#pragma unroll
          for (int i = 0; i < 7; ++i) {
            double sp = 0.0;
#pragma unroll
            for (int j = 0; j < 7; ++j) sp += S[i <= j ? upper_index(i, j) : upper_index(j, i)] * P[j][c];
            acc += P[i][r] * sp;
          }
          a.jtj[p * 25 + r * 5 + c] = acc;
        }
    }
  }
}

// Gauss-Newton step per seed: (D A D) x = -D g/2 with D = diag(scale), A = J^T J,
// g = grad Phi = 2 J^T r; Cholesky in FP64 (mu = 1e-12 trace added if needed);
// trial seeds seed + alpha delta for alpha = 1, 1/2, ..., 1/32.
__global__ void gn_solve_kernel(int64_t n, const double* __restrict__ jtj, const double* __restrict__ grad,
                                const double* __restrict__ seeds, double s0, double s1, double s2, double s3,
                                double s4, double* __restrict__ trials) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const double sc[5] = {s0, s1, s2, s3, s4};
  double A[5][5], b[5], x[5] = {0, 0, 0, 0, 0};
  double tr = 0.0;
  for (int r = 0; r < 5; ++r) {
    b[r] = -0.5 * grad[p * 5 + r] * sc[r];
    for (int c = 0; c < 5; ++c) A[r][c] = jtj[p * 25 + r * 5 + c] * sc[r] * sc[c];
    tr += A[r][r];
  }
  bool ok = false;
  for (int attempt = 0; attempt < 2 && !ok; ++attempt) {
    double Lm[5][5] = {{0}};
    ok = true;
    for (int i = 0; i < 5 && ok; ++i) {
      for (int j = 0; j <= i; ++j) {
        double s = A[i][j] + (attempt && i == j ? 1e-12 * tr : 0.0);
        for (int k = 0; k < j; ++k) s -= Lm[i][k] * Lm[j][k];
        if (i == j) {
          if (!(s > 0.0)) {
            ok = false;
            break;
          }
          Lm[i][i] = sqrt(s);
        } else {
          Lm[i][j] = s / Lm[j][j];
        }
      }
    }
    if (ok) {
      double y[5];
      for (int i = 0; i < 5; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= Lm[i][k] * y[k];
        y[i] = s / Lm[i][i];
      }
      for (int i = 4; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < 5; ++k) s -= Lm[k][i] * x[k];
        x[i] = s / Lm[i][i];
      }
    }
  }
  for (int k = 0; k < 6; ++k) {
    const double alpha = ldexp(1.0, -k);
    for (int d = 0; d < 5; ++d)
      trials[((size_t)p * 6 + k) * 5 + d] = seeds[p * 5 + d] + (ok ? alpha * x[d] * sc[d] : 0.0);
  }
}

// Take the first trial (alpha = 1, 1/2, ...) that lowers Phi; its forward outputs
// (checkpoints, residuals, argmin chords) become the current ones, so the next
// iteration's adjoint needs no forward pass of its own.
__global__ void gn_accept_kernel(int64_t n, int n_ckpt, int max_hits, const double* __restrict__ trials,
                                 const double* __restrict__ phi_trial, const float* __restrict__ tape6,
                                 const float* __restrict__ resid6, const int32_t* __restrict__ argmin6,
                                 double* __restrict__ seeds, double* __restrict__ phi_cur, float* __restrict__ tape,
                                 float* __restrict__ resid, int32_t* __restrict__ argmin) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  for (int k = 0; k < 6; ++k) {
    const int64_t g = p * 6 + k;   // trials of a seed are adjacent
    const double ph = phi_trial[g];
    if (ph < phi_cur[p]) {
      phi_cur[p] = ph;
      for (int d = 0; d < 5; ++d) seeds[p * 5 + d] = trials[g * 5 + d];
      for (int c = 0; c < n_ckpt; ++c)
        for (int q = 0; q < 13; ++q) tape[((size_t)c * 13 + q) * n + p] = tape6[((size_t)c * 13 + q) * 6 * n + g];
      for (int o = 0; o < max_hits; ++o) {
        resid[p * max_hits + o] = resid6[g * max_hits + o];
        argmin[p * max_hits + o] = argmin6[g * max_hits + o];
      }
      break;
    }
  }
}

__global__ void copy_phi_kernel(int64_t n, const double* __restrict__ src, double* __restrict__ dst, int stride,
                                int col) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) dst[p * stride + col] = src[p];
}

}  // namespace rkn

using namespace rkn;

namespace {

rkn_status rerr(rkn_ctx* c, hipError_t e, const char* where) {
  c->err = std::string(where) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? RKN_E_NOMEM : RKN_E_DEVICE;
}

// Tiles over runs of equal events of a slot list (slots grouped by event).
std::vector<Tile> slot_tiles(const std::vector<int32_t>& ev, int T) {
  std::vector<Tile> tiles;
  const int64_t n = (int64_t)ev.size();
  for (int64_t i = 0; i < n;) {
    int64_t j = i;
    while (j < n && ev[j] == ev[i]) ++j;
    for (int64_t s = i; s < j; s += T) {
      Tile t{};
      t.window = 0;
      t.event = ev[i];
      t.n = (int32_t)std::min<int64_t>(T, j - s);
      t.start = s;
      t.gbase = s;
      tiles.push_back(t);
    }
    i = j;
  }
  return tiles;
}

// Sets the checkpoint interval and sizes the buffers that depend on it.
hipError_t refine_ckpt_buffers(rkn_ctx* c, int ckpt) {
  c->r_ckpt = ckpt;
  c->r_nckpt = (c->r_params.n_steps + ckpt - 1) / ckpt;
  const size_t n = (size_t)c->r_n, nk = (size_t)c->r_nckpt;
  hipError_t e;
  if ((e = c->r_tape.ensure(sizeof(float) * 13 * n * nk)) != hipSuccess ||
      (e = c->r_tape6.ensure(sizeof(float) * 13 * 6 * n * nk)) != hipSuccess ||
      (e = c->r_segbuf.ensure(sizeof(float) * 6 * n * (size_t)(ckpt + 1) * nk)) != hipSuccess ||
      (e = c->r_segoff.ensure(sizeof(int32_t) * n * (nk + 1))) != hipSuccess ||
      (e = c->r_segout.ensure(sizeof(double) * kSegVals * n * nk)) != hipSuccess)
    return e;
  return hipSuccess;
}

hipError_t refine_forward(rkn_ctx* c, bool trials, int define_mask, bool tape) {
  const int64_t n = c->r_n;
  const int copies = trials ? 6 : 1;
  const int64_t npos = n * copies;
  Tile* tl = trials ? c->r_tiles6.as<Tile>() : c->r_tiles.as<Tile>();
  const int64_t nt = trials ? c->r_ntiles6 : c->r_ntiles;
  const double* seeds = trials ? c->r_trials.as<double>() : c->r_seeds.as<double>();
  return launch_refine_fwd(c, &c->r_params, nt, tl, seeds, c->r_ident.as<int64_t>(),
                           trials ? c->r_base6.as<int64_t>() : nullptr, c->r_mask.as<uint8_t>(), define_mask,
                           trials ? c->r_resid6.as<float>() : c->r_resid.as<float>(),
                           trials ? c->r_argmin6.as<int32_t>() : c->r_argmin.as<int32_t>(),
                           trials ? c->r_phi6.as<double>() : c->r_phi.as<double>(),
                           tape ? (trials ? c->r_tape6.as<float>() : c->r_tape.as<float>()) : nullptr, c->r_ckpt,
                           c->r_nckpt, npos);
}

hipError_t refine_backward(rkn_ctx* c, const float* cgrad, bool want_S) {
  BwdArgs b{};
  b.field = field_dev(c);
  b.n = c->r_n;
  b.n_steps = c->r_params.n_steps;
  b.ckpt = c->r_ckpt;
  b.n_ckpt = c->r_nckpt;
  b.h = (float)c->r_params.step_mm;
  b.R0 = c->r_params.R0;
  b.turn_stop = c->r_params.turn_stop;
  b.charge = c->r_params.charge;
  b.seeds5 = c->r_seeds.as<double>();
  b.seed_event = c->r_event.as<int32_t>();
  b.ev_off = c->ev_off.as<int32_t>();
  b.hits_wire = c->hits_wire.as<int32_t>();
  b.wire32 = c->wire32.as<HitRec<float>>();
  b.tape = c->r_tape.as<float>();
  b.resid = c->r_resid.as<float>();
  b.argmin = c->r_argmin.as<int32_t>();
  b.cgrad = cgrad;
  b.max_hits = c->max_hits_event > 0 ? c->max_hits_event : 1;
  b.segbuf = c->r_segbuf.as<float>();
  b.segoff = c->r_segoff.as<int32_t>();
  b.list = c->r_list.as<int2>();
  b.segout = c->r_segout.as<double>();
  b.grad = c->r_grad.as<double>();
  b.jtj = want_S ? c->r_jtj.as<double>() : nullptr;
  const dim3 blk(64);
  const dim3 g1((unsigned)((b.n + 63) / 64));
  const dim3 gs((unsigned)((b.n * b.n_ckpt + 63) / 64));
  hipLaunchKernelGGL(adj_prep_kernel, g1, blk, 0, c->stream, b);
  if (want_S) {
    if (c->field_kind == 0)
      hipLaunchKernelGGL((adj_seg_kernel<0, true>), gs, blk, 0, c->stream, b);
    else
      hipLaunchKernelGGL((adj_seg_kernel<1, true>), gs, blk, 0, c->stream, b);
    hipLaunchKernelGGL(adj_combine_kernel<true>, g1, blk, 0, c->stream, b);
  } else {
    if (c->field_kind == 0)
      hipLaunchKernelGGL((adj_seg_kernel<0, false>), gs, blk, 0, c->stream, b);
    else
      hipLaunchKernelGGL((adj_seg_kernel<1, false>), gs, blk, 0, c->stream, b);
    hipLaunchKernelGGL(adj_combine_kernel<false>, g1, blk, 0, c->stream, b);
  }
  return hipGetLastError();
}

}  // namespace

extern "C" {

rkn_status rkn_refine_setup(rkn_ctx* c, const rkn_scan_params* p, int64_t n_seeds, const int32_t* seed_event,
                            const double* seeds5, int32_t ckpt_every) {
  if (!c) return RKN_E_ARG;
  if (!p || p->precision != 32 || p->n_steps < 1 || !(p->step_mm > 0) || !(p->lambda_mm2 >= 0) || !(p->R0 > 0) ||
      !std::isfinite(p->charge) || p->charge == 0 || (p->ptr_flags & ~RKN_PTR_DEVICE) ||
      (p->turn_stop != 0 && p->turn_stop != 1)) {
    c->err = "refine: parameters must be valid with precision 32";
    return RKN_E_ARG;
  }
  if (c->n_wires == 0 || c->field_kind < 0 || c->h_ev_off.empty()) {
    c->err = "refine: upload geometry, field and hits first";
    return RKN_E_STATE;
  }
  if (n_seeds < 1 || n_seeds > (int64_t(1) << 24) || !seed_event || !seeds5) {
    c->err = "refine: need 1..2^24 seeds with events";
    return RKN_E_ARG;
  }
  if (ckpt_every != 0 && (ckpt_every < 8 || ckpt_every % 8 != 0 || ckpt_every > 4096)) {
    c->err = "refine: ckpt_every must be 0 (tuned) or a multiple of 8 in [8, 4096]";
    return RKN_E_ARG;
  }
  for (int64_t s = 0; s < n_seeds; ++s) {
    if (seed_event[s] < 0 || seed_event[s] >= c->n_events || (s > 0 && seed_event[s] < seed_event[s - 1])) {
      c->err = "refine: seed events must be valid and non-decreasing";
      return RKN_E_ARG;
    }
    for (int d = 0; d < 5; ++d)
      if (!std::isfinite(seeds5[5 * s + d])) {
        c->err = "refine: non-finite seed";
        return RKN_E_ARG;
      }
  }
  hipError_t e;
  if ((e = hipSetDevice(c->device)) != hipSuccess) return rerr(c, e, "hipSetDevice");
  c->r_params = *p;
  c->r_params.block_steps = 8;
  c->r_n = n_seeds;
  c->r_ckpt = ckpt_every > 0 ? ckpt_every : 64;
  c->r_nckpt = (p->n_steps + c->r_ckpt - 1) / c->r_ckpt;
  for (float& t : c->r_tune_ms) t = 0.0f;
  const int H = c->max_hits_event > 0 ? c->max_hits_event : 1;
  const int T = scan_tile(c, &c->r_params);
  std::vector<int32_t> ev(seed_event, seed_event + n_seeds);
  // trials: the six step lengths of seed s at positions 6 s .. 6 s + 5, so that an
  // event's trials share its tiles
  std::vector<int32_t> ev6(6 * (size_t)n_seeds);
  for (int64_t i = 0; i < 6 * n_seeds; ++i) ev6[i] = ev[i / 6];
  std::vector<Tile> t1 = slot_tiles(ev, T), t6 = slot_tiles(ev6, T);
  c->r_ntiles = (int64_t)t1.size();
  c->r_ntiles6 = (int64_t)t6.size();
  std::vector<int64_t> ident(6 * n_seeds), base6(6 * n_seeds);
  for (int64_t i = 0; i < 6 * n_seeds; ++i) {
    ident[i] = i;
    base6[i] = i / 6;
  }
  const size_t n = (size_t)n_seeds;
  if ((e = c->r_seeds.ensure(sizeof(double) * 5 * n)) != hipSuccess ||
      (e = c->r_seeds0.ensure(sizeof(double) * 5 * n)) != hipSuccess ||
      (e = c->r_trials.ensure(sizeof(double) * 5 * 6 * n)) != hipSuccess ||
      (e = c->r_event.ensure(sizeof(int32_t) * n)) != hipSuccess ||
      (e = c->r_tiles.ensure(sizeof(Tile) * std::max<size_t>(t1.size(), 1))) != hipSuccess ||
      (e = c->r_tiles6.ensure(sizeof(Tile) * std::max<size_t>(t6.size(), 1))) != hipSuccess ||
      (e = c->r_ident.ensure(sizeof(int64_t) * 6 * n)) != hipSuccess ||
      (e = c->r_base6.ensure(sizeof(int64_t) * 6 * n)) != hipSuccess ||
      (e = c->r_mask.ensure(n * H)) != hipSuccess ||
      (e = c->r_resid.ensure(sizeof(float) * n * H)) != hipSuccess ||
      (e = c->r_argmin.ensure(sizeof(int32_t) * n * H)) != hipSuccess ||
      (e = c->r_resid6.ensure(sizeof(float) * 6 * n * H)) != hipSuccess ||
      (e = c->r_argmin6.ensure(sizeof(int32_t) * 6 * n * H)) != hipSuccess ||
      (e = c->r_phi.ensure(sizeof(double) * n)) != hipSuccess ||
      (e = c->r_phi6.ensure(sizeof(double) * 6 * n)) != hipSuccess ||
      (e = c->r_phicur.ensure(sizeof(double) * n)) != hipSuccess ||
      (e = c->r_list.ensure(sizeof(int2) * n * H)) != hipSuccess ||
      (e = c->r_grad.ensure(sizeof(double) * 5 * n)) != hipSuccess ||
      (e = c->r_jtj.ensure(sizeof(double) * 25 * n)) != hipSuccess ||
      (e = c->r_cgrad.ensure(sizeof(float) * n * H)) != hipSuccess)
    return rerr(c, e, "refine alloc");
  e = hipMemcpyAsync(c->r_seeds.p, seeds5, sizeof(double) * 5 * n, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->r_seeds0.p, seeds5, sizeof(double) * 5 * n, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(c->r_event.p, seed_event, sizeof(int32_t) * n, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && !t1.empty())
    e = hipMemcpyAsync(c->r_tiles.p, t1.data(), sizeof(Tile) * t1.size(), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && !t6.empty())
    e = hipMemcpyAsync(c->r_tiles6.p, t6.data(), sizeof(Tile) * t6.size(), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->r_ident.p, ident.data(), sizeof(int64_t) * 6 * n, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->r_base6.p, base6.data(), sizeof(int64_t) * 6 * n, hipMemcpyHostToDevice, c->stream);
  if (e != hipSuccess) return rerr(c, e, "refine setup");
  // checkpoint interval: given, or the fastest adjoint sweep (with J^T J) among
  // 32, 64, 128 and 256 steps on these seeds
  int chosen = c->r_ckpt;
  if (ckpt_every == 0) {
    static const int cand[4] = {32, 64, 128, 256};
    hipEvent_t t0 = nullptr, t1e = nullptr;
    if ((e = hipEventCreate(&t0)) != hipSuccess || (e = hipEventCreate(&t1e)) != hipSuccess)
      return rerr(c, e, "refine tune");
    float best = INFINITY;
    for (int i = 0; i < 4 && e == hipSuccess; ++i) {
      e = refine_ckpt_buffers(c, cand[i]);
      if (e == hipSuccess) e = refine_forward(c, false, 1, true);
      if (e == hipSuccess) e = hipEventRecord(t0, c->stream);
      if (e == hipSuccess) e = refine_backward(c, nullptr, true);
      if (e == hipSuccess) e = hipEventRecord(t1e, c->stream);
      if (e == hipSuccess) e = hipEventSynchronize(t1e);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1e);
      c->r_tune_ms[i] = ms;
      if (e == hipSuccess && ms < best) {
        best = ms;
        chosen = cand[i];
      }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1e);
    if (e != hipSuccess) return rerr(c, e, "refine tune");
  }
  // the inlier sets: classification at the starting seeds
  e = refine_ckpt_buffers(c, chosen);
  if (e == hipSuccess) e = refine_forward(c, false, 1, true);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return rerr(c, e, "refine setup");
  c->r_ready = true;
  return RKN_OK;
}

rkn_status rkn_refine_info(rkn_ctx* c, int64_t* n_seeds, int32_t* ckpt_every, float* tune_ms) {
  if (!c) return RKN_E_ARG;
  if (!c->r_ready) {
    c->err = "refine: nothing set up";
    return RKN_E_STATE;
  }
  if (n_seeds) *n_seeds = c->r_n;
  if (ckpt_every) *ckpt_every = c->r_ckpt;
  if (tune_ms)
    for (int i = 0; i < 4; ++i) tune_ms[i] = c->r_tune_ms[i];
  return RKN_OK;
}

rkn_status rkn_residuals_fwd(rkn_ctx* c, const double* seeds5, float* resid, double* phi) {
  if (!c) return RKN_E_ARG;
  if (!c->r_ready) {
    c->err = "refine: call rkn_refine_setup first";
    return RKN_E_STATE;
  }
  const bool dev = (c->r_params.ptr_flags & RKN_PTR_DEVICE) != 0;
  const size_t n = (size_t)c->r_n, H = (size_t)(c->max_hits_event > 0 ? c->max_hits_event : 1);
  hipError_t e;
  if ((e = hipSetDevice(c->device)) != hipSuccess) return rerr(c, e, "hipSetDevice");
  if (seeds5 &&
      (e = hipMemcpyAsync(c->r_seeds.p, seeds5, sizeof(double) * 5 * n, dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          c->stream)) != hipSuccess)
    return rerr(c, e, "refine copy");
  if ((e = refine_forward(c, false, 0, true)) != hipSuccess) return rerr(c, e, "refine forward");
  const hipMemcpyKind k = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (resid && (e = hipMemcpyAsync(resid, c->r_resid.p, sizeof(float) * n * H, k, c->stream)) != hipSuccess)
    return rerr(c, e, "refine copy");
  if (phi && (e = hipMemcpyAsync(phi, c->r_phi.p, sizeof(double) * n, k, c->stream)) != hipSuccess)
    return rerr(c, e, "refine copy");
  if (!dev && (e = hipStreamSynchronize(c->stream)) != hipSuccess) return rerr(c, e, "refine sync");
  return RKN_OK;
}

rkn_status rkn_adjoint_bwd(rkn_ctx* c, const float* d_resid, double* d_seed, double* JtJ, double* Jtr) {
  if (!c) return RKN_E_ARG;
  if (!c->r_ready) {
    c->err = "refine: call rkn_refine_setup and rkn_residuals_fwd first";
    return RKN_E_STATE;
  }
  const bool dev = (c->r_params.ptr_flags & RKN_PTR_DEVICE) != 0;
  const size_t n = (size_t)c->r_n, H = (size_t)(c->max_hits_event > 0 ? c->max_hits_event : 1);
  hipError_t e;
  if ((e = hipSetDevice(c->device)) != hipSuccess) return rerr(c, e, "hipSetDevice");
  const float* cg = nullptr;
  if (d_resid) {
    if ((e = hipMemcpyAsync(c->r_cgrad.p, d_resid, sizeof(float) * n * H,
                            dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream)) != hipSuccess)
      return rerr(c, e, "refine copy");
    cg = c->r_cgrad.as<float>();
  }
  if ((e = refine_backward(c, cg, JtJ != nullptr)) != hipSuccess) return rerr(c, e, "adjoint");
  const hipMemcpyKind k = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (d_seed && (e = hipMemcpyAsync(d_seed, c->r_grad.p, sizeof(double) * 5 * n, k, c->stream)) != hipSuccess)
    return rerr(c, e, "refine copy");
  if (JtJ && (e = hipMemcpyAsync(JtJ, c->r_jtj.p, sizeof(double) * 25 * n, k, c->stream)) != hipSuccess)
    return rerr(c, e, "refine copy");
  if (!dev || Jtr) {
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return rerr(c, e, "refine sync");
  }
  if (Jtr) {
    // J^T r = grad(Phi) / 2 when the upstream gradient is the default 2 r
    std::vector<double> g(5 * n);
    if ((e = hipMemcpy(g.data(), c->r_grad.p, sizeof(double) * 5 * n, hipMemcpyDeviceToHost)) != hipSuccess)
      return rerr(c, e, "refine copy");
    for (double& v : g) v *= d_resid ? 1.0 : 0.5;
    if ((e = hipMemcpy(Jtr, g.data(), sizeof(double) * 5 * n, dev ? hipMemcpyHostToDevice : hipMemcpyHostToHost)) !=
        hipSuccess)
      return rerr(c, e, "refine copy");
  }
  return RKN_OK;
}

rkn_status rkn_gn_refine(rkn_ctx* c, int32_t iters, const double* scale, double* seeds_out, double* phi) {
  if (!c) return RKN_E_ARG;
  if (!c->r_ready) {
    c->err = "refine: call rkn_refine_setup first";
    return RKN_E_STATE;
  }
  if (iters < 0 || iters > 1000 || !scale) {
    c->err = "refine: iters in [0, 1000] and a scale vector are required";
    return RKN_E_ARG;
  }
  for (int d = 0; d < 5; ++d)
    if (!(scale[d] > 0) || !std::isfinite(scale[d])) {
      c->err = "refine: scale must be finite and > 0";
      return RKN_E_ARG;
    }
  const bool dev = (c->r_params.ptr_flags & RKN_PTR_DEVICE) != 0;
  const int64_t n = c->r_n;
  hipError_t e;
  if ((e = hipSetDevice(c->device)) != hipSuccess) return rerr(c, e, "hipSetDevice");
  DevBuf phi_hist;
  if ((e = phi_hist.ensure(sizeof(double) * n * (iters + 1))) != hipSuccess) return rerr(c, e, "refine alloc");
  const dim3 g1((unsigned)((n + 255) / 256)), b1(256);
  // start from the setup seeds; the inlier sets stay those of the setup pass
  e = hipMemcpyAsync(c->r_seeds.p, c->r_seeds0.p, sizeof(double) * 5 * n, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = refine_forward(c, false, 0, true);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->r_phicur.p, c->r_phi.p, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream);
  const int H = c->max_hits_event > 0 ? c->max_hits_event : 1;
  for (int it = 0; it < iters && e == hipSuccess; ++it) {
    hipLaunchKernelGGL(copy_phi_kernel, g1, b1, 0, c->stream, n, c->r_phicur.as<double>(), phi_hist.as<double>(),
                       iters + 1, it);
    e = refine_backward(c, nullptr, true);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(gn_solve_kernel, g1, b1, 0, c->stream, n, c->r_jtj.as<double>(), c->r_grad.as<double>(),
                         c->r_seeds.as<double>(), scale[0], scale[1], scale[2], scale[3], scale[4],
                         c->r_trials.as<double>());
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = refine_forward(c, true, 0, true);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(gn_accept_kernel, g1, b1, 0, c->stream, n, c->r_nckpt, H, c->r_trials.as<double>(),
                         c->r_phi6.as<double>(), c->r_tape6.as<float>(), c->r_resid6.as<float>(),
                         c->r_argmin6.as<int32_t>(), c->r_seeds.as<double>(), c->r_phicur.as<double>(),
                         c->r_tape.as<float>(), c->r_resid.as<float>(), c->r_argmin.as<int32_t>());
      e = hipGetLastError();
    }
  }
  if (e == hipSuccess)
    hipLaunchKernelGGL(copy_phi_kernel, g1, b1, 0, c->stream, n, c->r_phicur.as<double>(), phi_hist.as<double>(),
                       iters + 1, iters);
  const hipMemcpyKind k = dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (e == hipSuccess && seeds_out)
    e = hipMemcpyAsync(seeds_out, c->r_seeds.p, sizeof(double) * 5 * n, k, c->stream);
  if (e == hipSuccess && phi) e = hipMemcpyAsync(phi, phi_hist.p, sizeof(double) * n * (iters + 1), k, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  phi_hist.release();
  if (e != hipSuccess) return rerr(c, e, "gn refine");
  return RKN_OK;
}

}  // extern "C"
