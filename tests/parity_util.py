"""Shared helpers of the GPU parity tests (comparison rules, not arithmetic of the method)."""
import numpy as np

SCORE_REL = 1e-4          # FP32 propagation, FP64 score (relative score error bound)
SCORE_ABS = 1e-4          # mm^2 floor for nearly-zero scores
NEAR_TIE = 2e-4           # best-seed near-tie rule: twice the score tolerance


def check_scores(gpu, orc, rel=SCORE_REL, abs_=SCORE_ABS):
    gpu = np.asarray(gpu); orc = np.asarray(orc)
    inf = ~np.isfinite(orc)
    assert np.array_equal(inf, ~np.isfinite(gpu)), "infinite scores differ"
    err = np.abs(gpu[~inf] - orc[~inf])
    tol = rel * np.abs(orc[~inf]) + abs_
    bad = np.nonzero(err > tol)[0]
    assert bad.size == 0, f"{bad.size} scores off, worst rel {np.max(err / np.maximum(np.abs(orc[~inf]), 1e-30)):.3e}"
    return float(np.max(err / np.maximum(np.abs(orc[~inf]), 1e-12))) if err.size else 0.0


def check_best(gpu_index, orc_scores, offset=0, rel=NEAR_TIE):
    """GPU best index equals the oracle's, except at a stated near-tie."""
    s = np.asarray(orc_scores)
    i1 = int(np.argmin(s))          # numpy argmin: lowest index among ties
    e1 = s[i1]
    g = int(gpu_index) - offset
    if g == i1:
        return True
    assert 0 <= g < s.size, f"gpu best {g} out of range"
    assert s[g] <= e1 * (1 + rel) + 1e-12, f"gpu best {g} (E={s[g]}) vs oracle {i1} (E={e1})"
    return False


def check_nin(gpu_nin, orc_nin, max_frac=1e-3):
    gpu_nin = np.asarray(gpu_nin); orc_nin = np.asarray(orc_nin)
    diff = np.abs(gpu_nin.astype(np.int64) - orc_nin)
    assert diff.max(initial=0) <= 1
    assert np.count_nonzero(diff) <= max(1, int(max_frac * diff.size))
    return np.nonzero(diff)[0]
