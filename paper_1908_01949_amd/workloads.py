"""The scan workloads that are measured and tested at full size: grids, steps and the
Hough window rules (configuration only; the arithmetic lives in the kernels)."""

# One electron under one turn, uniform 1 T, FP64: 6^5 seeds around the truth seed.
SINGLE_TURN = dict(n_steps=2000, precision=64, half_width=(0.3, 100.0, 10.0, 10.0, 10.0), count=6)

# A 2-3 pass electron with 30 % noise, uniform 1 T, FP32: 16^5 seeds around the truth seed.
MULTI_TURN = dict(n_steps=6000, precision=32, half_width=(0.3, 100.0, 10.0, 10.0, 10.0), count=16)

# One event of 150 hits (20 % noise) in the solenoid map: Hough windows of 12^5 seeds.
HOUGH_EVENT = dict(n_steps=6000, precision=32,
                   hough=dict(min_votes=6, max_cand=4, count=(12, 12, 12, 12, 12), grow=(0, 0, 0, 0, 0),
                              count_max=12, max_seeds_window=12 ** 5))

# 512 events in one batch: Hough windows of 1e3-1e5 seeds per event.
BATCH = dict(n_events=512, n_steps=6000, precision=32,
             hough=dict(min_votes=6, max_cand=4, gran=(0.01, 100.0, 2.5, 2.5, 12.0), center_z=0.0,
                        center_pz=0.0, count=(4, 6, 4, 4, 6), grow=(1, 0, 1, 1, 0), count_max=10,
                        max_seeds_window=25000))

# Refinement of the 8 best seeds per event of the batch: 10 Gauss-Newton iterations,
# a checkpoint every 64 steps, scaled variables (rad, mm, MeV/c x3).
REFINE = dict(k=8, iters=10, ckpt_every=64, scale=(1.0, 100.0, 100.0, 100.0, 100.0))

# Turn-partition reconstruction (section 2.3) of multi-turn events in the solenoid map:
# Hough windows of 7 x 13 x 7 x 7 x 13 seeds for the first partition (8 candidates),
# then windows of 5 x 9 x 5 x 5 x 9 seeds around each predicted neighbour (the
# rkn_turn_params defaults of the binding), the scan cutoff lambda = 64 mm^2,
# classification at 4 mm^2.
TURNS = dict(n_events=128, n_steps=6000, precision=32,
             hough=dict(min_votes=6, max_cand=4, gran=(0.01, 50.0, 2.5, 2.5, 4.0), count=(7, 13, 7, 7, 13),
                        count_max=13))
