"""Pins of the oracle's coarse-to-fine rescans (section 2.2: the seeds with the lowest E
are kept, finer seed sets are built around them, and the scan is repeated)."""
import numpy as np
import pytest

from paper_1908_01949_amd import synth


def _one_event(ev):
    return np.array([0, ev.wire_id.size], np.int32), ev.wire_id, ev.drift


def test_one_round_is_the_k_lowest_of_the_windows(geo, ev1, orc_u):
    """One round = the k lowest (E, then position) of an independent window scan over grids
    of `grid` points (one point where a step is 0) centred on the kept seeds, half-width =
    their steps; each kept seed carries the step of its own grid."""
    prm = orc_u.params(n_steps=2000)
    off, wid, dr = _one_event(ev1)
    t = ev1.truth_seeds[0]
    k, G = 3, 3
    start = np.array([[t + [0.004, 2.0, 1.0, -1.0, 0.5], t + [-0.01, 0.0, 0.5, 0.5, -1.0],
                       t + [0.02, -3.0, -1.0, 1.0, 1.0]]])
    step = np.array([[[0.004, 0.0, 1.0, 1.0, 1.0], [0.006, 3.0, 0.0, 1.5, 1.5],
                      [0.004, 3.0, 1.0, 0.0, 2.0]]])
    out5, ostep, osc, rounds, margin = orc_u.rescan_refine(prm, off, wid, dr, start, step, grid=G,
                                                           max_rounds=1)
    rows = [(0, j, start[0, j], step[0, j], [G if s > 0 else 1 for s in step[0, j]]) for j in range(k)]
    w = synth.make_windows(rows)
    score, _, _, _, _ = orc_u.scan_windows(prm, off, wid, dr, w, mode=1)
    order = np.lexsort((np.arange(score.size), score))
    sizes = np.array([int(np.prod(x["count"])) for x in w])
    base = np.concatenate([[0], np.cumsum(sizes)])
    assert rounds[0] == 1
    for j in range(k):
        g = int(order[j])
        kw = int(np.searchsorted(base, g, side="right") - 1)
        assert np.array_equal(out5[0, j], orc_u.window_seed(w[kw], g - base[kw]))
        assert osc[0, j] == score[g]
        want = np.where(w[kw]["count"] > 1, 2.0 * w[kw]["half_width"] / np.maximum(w[kw]["count"] - 1, 1), 0.0)
        assert np.array_equal(ostep[0, j], want)
    s = score[order[:k + 1]]
    gaps = np.abs(np.diff(s)) / np.maximum(np.abs(s[1:]), np.abs(s[:-1]))
    assert margin[0] == pytest.approx(gaps.min(), rel=1e-12)
    assert np.all(np.diff(osc[0]) >= 0)


def test_truth_on_the_grid_is_found_and_kept(geo, ufield, orc_u):
    """Noise-free hits: the truth seed is on the first round's grid (its centre sits half
    a half-width off in every dimension). The loop finds it, keeps it as the centre of
    every later grid (odd point count) and halves the step each round; with a target
    just above the truth's E it stops after that first round."""
    ev = synth.event_single_turn(geo, ufield, 1, sigma=0.0)
    prm = orc_u.params(n_steps=2000)
    off, wid, dr = _one_event(ev)
    t = ev.truth_seeds[0]
    hw = np.array([0.008, 8.0, 4.0, 4.0, 4.0])
    start = np.array([[t + 0.5 * hw, t + np.array([3.0, -2.0, 1.0, 2.0, -3.0]) * hw]])
    step = np.array([[hw, hw]])
    out5, ostep, osc, rounds, _ = orc_u.rescan_refine(prm, off, wid, dr, start, step, grid=5, max_rounds=3)
    E_t, _, _ = orc_u.score(prm, t, wid, dr, mode=0)
    assert rounds[0] == 3
    np.testing.assert_allclose(out5[0, 0], t, rtol=0, atol=1e-12)
    assert np.array_equal(ostep[0, 0], hw / 8)
    assert osc[0, 0] == pytest.approx(E_t, rel=1e-9, abs=1e-12)
    assert np.all(np.diff(osc[0]) >= 0)
    out5, ostep, osc, rounds, margin = orc_u.rescan_refine(prm, off, wid, dr, start, step, grid=5, max_rounds=3,
                                                           target=np.array([2.0 * E_t + 1e-12]))
    assert rounds[0] == 1
    np.testing.assert_allclose(out5[0, 0], t, rtol=0, atol=1e-12)
    assert np.array_equal(ostep[0, 0], hw / 2)
    assert 0.0 < margin[0] <= 1.0


def test_rounds_compose_and_empty_events(geo, ufield, orc_u):
    """R rounds equal R - 1 rounds followed by one more from their outputs (bit for bit,
    even point count: the centre is not on the grid); an event without kept seeds runs
    no round; a missing seed row stays missing only while fewer seeds than k exist."""
    evs = [synth.event_single_turn(geo, ufield, s) for s in (21, 22, 23)]
    off, wid, dr = synth.pack_events(evs)
    prm = orc_u.params(n_steps=1200)
    k = 2
    start = np.full((3, k, 5), np.nan); step = np.full((3, k, 5), np.nan)
    hw = np.array([0.01, 6.0, 2.0, 2.0, 2.0])
    start[0, 0] = evs[0].truth_seeds[0] + 0.3 * hw; step[0, 0] = hw
    start[0, 1] = evs[0].truth_seeds[0] - 0.7 * hw; step[0, 1] = hw
    start[2, 1] = evs[2].truth_seeds[0] + 0.2 * hw; step[2, 1] = hw * np.array([1, 0, 1, 1, 1])
    a = orc_u.rescan_refine(prm, off, wid, dr, start, step, grid=4, max_rounds=3)
    b = orc_u.rescan_refine(prm, off, wid, dr, start, step, grid=4, max_rounds=2)
    c = orc_u.rescan_refine(prm, off, wid, dr, b[0], b[1], grid=4, max_rounds=1)
    for x, y in zip(a[:3], c[:3]):
        assert np.array_equal(x, y, equal_nan=True)
    assert list(a[3]) == [3, 0, 3] and list(c[3]) == [1, 0, 1]
    assert np.all(np.isnan(a[0][1])) and np.all(np.isnan(a[2][1]))
    # one kept seed with 4^4 grid points (z step 0): both rows filled after a round
    assert np.all(np.isfinite(a[0][2])) and np.all(a[1][2][:, 1] == 0.0)
    assert np.all(a[0][2][:, 1] == start[2, 1, 1])   # z never moves with a zero step


def test_odd_grid_best_never_rises(geo, ev1, orc_u):
    """With an odd point count every grid contains its centre, so an event's lowest E
    cannot rise from one round to the next."""
    prm = orc_u.params(n_steps=2000)
    off, wid, dr = _one_event(ev1)
    t = ev1.truth_seeds[0]
    hw = np.array([0.01, 10.0, 3.0, 3.0, 3.0])
    start = np.array([[t + 0.37 * hw, t - 0.61 * hw]]); step = np.array([[hw, hw]])
    best = []
    for r in (1, 2, 3):
        best.append(orc_u.rescan_refine(prm, off, wid, dr, start, step, grid=3, max_rounds=r)[2][0, 0])
    assert best[0] >= best[1] >= best[2]


def test_argument_errors(ev1, orc_u):
    prm = orc_u.params(n_steps=10)
    off, wid, dr = _one_event(ev1)
    s = np.zeros((1, 1, 5))
    with pytest.raises(ValueError):
        orc_u.rescan_refine(prm, off, wid, dr, s, s, grid=1)
