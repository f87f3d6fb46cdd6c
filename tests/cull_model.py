"""CPU model of the scan kernel's block culling, used to check the kernel's work
counters (test infrastructure; not part of the oracle, whose score is the plain
definition of Eq. 1).

The rule modelled (FP64 here, FP32 in the kernel): steps are taken in blocks of B;
a block's chords span the radii [min over its B+1 points - h/2, max over them]
(every chord point lies within h/2 of one of its ends); the layers considered are
those whose radial extent, widened by the event's largest drift + sqrt(lambda) +
1 mm, meets one of the 1 mm radial bins that range covers; a hit of such a layer is
kept for the block when its wire's line passes within B h/2 + sqrt(lambda) +
0.05 mm + d of the block's middle point (every chord point lies within B h/2 of
it); every kept (block, hit) pair is compared with each of the block's chords.
A dropped pair cannot matter: its distance exceeds d + sqrt(lambda), where the
hit's term of Eq. 1 is lambda whatever the distance.
"""
from __future__ import annotations

import math

import numpy as np

N_BINS = 1024
BAND_MARGIN = 1.0
CULL_MARGIN = 0.05


def _layer_tables(geo, d_max, lam):
    """Per 1 mm radial bin the half-open layer range [l0, l1p) whose widened band meets it."""
    D = d_max + math.sqrt(lam) + BAND_MARGIN
    lo = np.arange(N_BINS, dtype=np.float64)
    hi = lo + 1.0
    hi[-1] = np.inf
    rmin = np.asarray(geo.layer_rmin, np.float64)
    rmax = np.asarray(geo.layer_rmax, np.float64)
    # l0: the first layer not entirely below the bin; l1p: one past the last layer not above it
    l0 = np.searchsorted(rmax + D, lo, side="left")
    l1p = np.searchsorted(rmin - D, hi, side="right")
    return l0, l1p


def blocked_work(O, prm, seed, geo, wire_id, drift, B, want_score=False):
    """(seed-steps, chord distances, E or None) of one seed under the block rule.

    E, when asked for, is Eq. 1 over the minima of the kept pairs' chord distances
    (orc_seg_wire_dist2 on the oracle's FP64 trajectory)."""
    n = prm.n_steps
    h = prm.step_mm
    lam = prm.lambda_mm2
    wire_id = np.asarray(wire_id, np.int32)
    drift = np.asarray(drift, np.float32).astype(np.float64)
    pts = O.trace(prm, seed, np.arange(n + 1, dtype=np.int32))[0][:, :3]
    if not np.all(np.isfinite(pts)):
        return 0, 0, (math.inf if want_score else None)
    l0, l1p = _layer_tables(geo, float(drift.max(initial=0.0)), lam)
    lay = np.asarray(geo.layer_of, np.int64)[wire_id]
    m = np.stack([geo.mx[wire_id], geo.my[wire_id], geo.mz[wire_id]], -1)
    u = np.stack([geo.ux[wire_id], geo.uy[wire_id], geo.uz[wire_id]], -1)
    kcull = 0.5 * B * h + math.sqrt(lam) + CULL_MARGIN
    thr2 = (kcull + drift) ** 2
    d2 = np.full(wire_id.size, np.inf)
    chords = 0
    r = np.hypot(pts[:, 0], pts[:, 1])
    for b0 in range(0, n, B):
        nb = min(B, n - b0)
        rr = r[b0:b0 + nb + 1]
        rmin = max(float(rr.min()) - 0.5 * h, 0.0)
        rmax = float(rr.max())
        b_lo = int(min(rmin, N_BINS - 1))
        b_hi = int(min(rmax, N_BINS - 1))
        L0, L1p = int(l0[b_lo]), int(l1p[b_hi])
        cand = (lay >= L0) & (lay < L1p)
        if not cand.any():
            continue
        c = pts[b0 + nb // 2]
        rv = c[None, :] - m
        t = (rv * u).sum(-1)
        dl2 = (rv * rv).sum(-1) - t * t
        keep = cand & (dl2 <= thr2)
        k = int(keep.sum())
        chords += k * nb
        if want_score and k:
            for i in np.nonzero(keep)[0]:
                w = int(wire_id[i])
                mm = np.array([geo.mx[w], geo.my[w], geo.mz[w]])
                uu = np.array([geo.ux[w], geo.uy[w], geo.uz[w]])
                for j in range(nb):
                    v = O.seg_wire_dist2(pts[b0 + j], pts[b0 + j + 1], mm, uu, float(geo.half_len[w]))
                    if v < d2[i]:
                        d2[i] = v
    E = None
    if want_score:
        E = 0.0
        for i in range(wire_id.size):
            rr_ = math.sqrt(d2[i]) - float(drift[i])
            tq = rr_ * rr_
            E += tq if tq < lam else lam
    return n, chords, E
