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

Per seed-step:  F_alg = F_RKN + F_DOCA * q, where q is the number of chord/wire
distances per seed-step that the kernel evaluates on the same workload, counted by
the kernel's own counting instance (rkn_scan_work_counts; the timed instances carry
no counter). The cull rule behind q is exact: Eq. 1 over the pairs it keeps equals
the brute-force score bit for bit (checked on the CPU). The radial band rule alone
would keep far more pairs (h-bar, counted by the oracle's band-pruned mode); crediting
those would credit work the kernel never does.
"""
F_RKN_UNIFORM = 44
F_FIELD = 31
F_RKN_GRID = 127 + 3 * F_FIELD
F_DOCA = 50

# MI355X vector peaks (dense, per the vendor): FP32 with packed math, FP64; and the
# FP32 rate without packed math (one FMA per lane per clock), the kernels' ceiling here.
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_UNPACKED_TFLOPS = 78.6


def per_seed_step(field_kind: str, pairs_per_step: float) -> float:
    f_rkn = F_RKN_UNIFORM if field_kind == "uniform" else F_RKN_GRID
    return f_rkn + F_DOCA * pairs_per_step
