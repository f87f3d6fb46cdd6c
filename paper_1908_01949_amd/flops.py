"""Algorithmic FP32 work of the seed scan, per seed-step (roofline accounting).

Convention: add/sub/mul = 1, FMA = 2, sqrt/rcp/div = 1, min/max/compare/select = 0.
Counted on the arithmetic of the method (the RKN step and the exact chord/wire
distance of every pair that the exact pruning keeps); the pruning itself (band,
sector and sphere tests), compensation terms of the FP32 sums, index arithmetic and
the FP64 score sum are not credited.

  F_RKN_UNIFORM  one RKN4 step in B = B_z z^ (only T_x, T_y turn):           44
  F_FIELD        one bilinear (r, z) field evaluation with B_x,y = B_r (x,y)/r: 31
  F_RKN_GRID     one general RKN4 step (127) + three field evaluations:       220
  F_DOCA         exact squared chord/wire distance:                           50

Per seed-step:  F_alg = F_RKN + F_DOCA * q, where q (chord/hit distances per
seed-step) is counted by the oracle's block-pruned score on a sample of the same
workload (the sphere rule the kernel applies; exact: its E equals the brute-force E
bit for bit).
"""
F_RKN_UNIFORM = 44
F_FIELD = 31
F_RKN_GRID = 127 + 3 * F_FIELD
F_DOCA = 50

# MI355X vector peaks (dense, per the vendor): FP32 with packed math, FP64.
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6


def per_seed_step(field_kind: str, pairs_per_step: float) -> float:
    f_rkn = F_RKN_UNIFORM if field_kind == "uniform" else F_RKN_GRID
    return f_rkn + F_DOCA * pairs_per_step
