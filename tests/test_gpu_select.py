"""GPU top-k selection of the best seeds per event (the pick step of the coarse-to-fine
refinement of section 2.2, and the input of the derivative-based refinement).
Selection is index work: compared bit-exactly with a host sort of the GPU's own
scores (order: score, then global index); decoded seeds against the oracle's window
decode."""
import numpy as np
import pytest

from paper_1908_01949_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rk():
    from paper_1908_01949_amd import rknscan
    rknscan.load_library()
    return rknscan


def _expected(score, ev_seed, k):
    ne = ev_seed.size - 1
    idx = np.full((ne, k), -1, np.int64)
    sc = np.full((ne, k), np.inf)
    for e in range(ne):
        lo, hi = int(ev_seed[e]), int(ev_seed[e + 1])
        s = score[lo:hi]
        ok = ~np.isnan(s)
        ii = np.arange(lo, hi)[ok]
        order = np.lexsort((ii, s[ok]))[:k]
        idx[e, :order.size] = ii[order]
        sc[e, :order.size] = s[ok][order]
    return idx, sc


def _decode(orc, windows, ev_seed, idx):
    """Seeds at global indices, through the oracle's window decode (windows ordered by event)."""
    sizes = np.array([int(np.prod(w["count"].astype(np.int64))) for w in windows])
    base = np.concatenate([[0], np.cumsum(sizes)])
    out = np.full(idx.shape + (5,), np.nan)
    for e, row in enumerate(idx):
        for j, g in enumerate(row):
            if g < 0:
                continue
            kw = int(np.searchsorted(base, g, side="right") - 1)
            assert windows[kw]["event"] == e
            out[e, j] = orc.window_seed(windows[kw], int(g - base[kw]))
    return out


def test_windows_topk_matches_host_selection(rk, geo, ufield, orc_u):
    evs = [synth.event_single_turn(geo, ufield, s) for s in (0, 1, 2, 3)]
    off, wid, dr = synth.pack_events(evs)
    c = rk.Context(0)
    c.upload_geometry(geo); c.upload_field(ufield); c.upload_hits(off, wid, dr)
    hw = [0.05, 20.0, 3.0, 3.0, 3.0]
    # event 0: two windows; event 1: none; event 2: a one-seed window; event 3: one window
    w = synth.make_windows([(0, 0, evs[0].truth_seeds[0], hw, [3, 4, 5, 4, 3]),
                            (0, 1, evs[0].truth_seeds[0] + 0.01, hw, [2, 3, 3, 3, 2]),
                            (2, 0, evs[2].truth_seeds[0], hw, [1, 1, 1, 1, 1]),
                            (3, 0, evs[3].truth_seeds[0], hw, [4, 4, 4, 4, 4])])
    sp = rk.make_scan_params(n_steps=1500, precision=32)
    sizes = np.array([int(np.prod(x["count"].astype(np.int64))) for x in w])
    total = int(sizes.sum())
    score = np.zeros(total)
    rk.rkn_scan_windows(c.ctx, sp, w, score, None, np.zeros(4, np.int64), np.zeros(4))
    ev_seed = np.array([0, sizes[:2].sum(), sizes[:2].sum(), sizes[:3].sum(), total])
    for k in (1, 8, 16):
        idx, sc, s5 = rk.rkn_scan_windows_topk(c.ctx, sp, w, k, n_events=4)
        ei, es = _expected(score, ev_seed, k)
        assert np.array_equal(idx, ei) and np.array_equal(sc, es), k
        np.testing.assert_allclose(s5, _decode(orc_u, w, ev_seed, idx), rtol=0, atol=1e-12)
        assert np.all(np.isnan(s5[idx < 0]))
    # argument errors
    for k in (0, 17):
        with pytest.raises(rk.RknError) as e:
            rk.rkn_scan_windows_topk(c.ctx, sp, w, k, n_events=4)
        assert e.value.status == rk.RKN_E_ARG
    c.close()


def test_windows_topk_ties_take_lowest_index(rk, geo, ufield):
    """A window whose px dimension has a zero half-width repeats every seed: equal
    scores, and the lower global index must win."""
    ev = synth.event_single_turn(geo, ufield, 5)
    off, wid, dr = synth.pack_events([ev])
    c = rk.Context(0)
    c.upload_geometry(geo); c.upload_field(ufield); c.upload_hits(off, wid, dr)
    w = synth.make_windows([(0, 0, ev.truth_seeds[0], [0.02, 10.0, 0.0, 2.0, 2.0], [3, 3, 4, 3, 3])])
    sp = rk.make_scan_params(n_steps=1000, precision=32)
    n = int(np.prod(w[0]["count"].astype(np.int64)))
    score = np.zeros(n)
    rk.rkn_scan_windows(c.ctx, sp, w, score, None, np.zeros(1, np.int64), np.zeros(1))
    idx, sc, _ = rk.rkn_scan_windows_topk(c.ctx, sp, w, 12, n_events=1)
    ei, es = _expected(score, np.array([0, n]), 12)
    assert np.array_equal(idx, ei) and np.array_equal(sc, es)
    assert np.any(sc[0, 1:] == sc[0, :-1])      # ties were present
    c.close()


def test_batch_topk_matches_host_selection(rk, geo, sfield, orc_s):
    evs = synth.events_batch(geo, sfield, 6, seed=3)
    off, wid, dr = synth.pack_events(evs)
    c = rk.Context(0)
    c.upload_geometry(geo); c.upload_field(sfield); c.upload_hits(off, wid, dr)
    hp = rk.make_hough_params(b_ref=sfield.b_ref, max_cand=3, gran=(0.01, 100.0, 2.5, 2.5, 12.0),
                              count=(3, 2, 3, 3, 2), grow=(1, 0, 1, 1, 0), count_max=4, max_seeds_window=150)
    rk.rkn_batch_plan(c.ctx, hp, rk.make_scan_params(n_steps=1200, precision=32))
    with pytest.raises(rk.RknError) as e:
        rk.rkn_batch_topk(c.ctx, 8, n_events=len(evs))
    assert e.value.status == rk.RKN_E_STATE
    rk.rkn_batch_launch(c.ctx, None, None)
    w, score, _, ev_seed = rk.rkn_batch_results(c.ctx, len(evs))
    idx, sc, s5 = rk.rkn_batch_topk(c.ctx, 8, n_events=len(evs))
    ei, es = _expected(score, ev_seed, 8)
    assert np.array_equal(idx, ei) and np.array_equal(sc, es)
    np.testing.assert_allclose(s5, _decode(orc_s, w, ev_seed, idx), rtol=0, atol=1e-12)
    # the per-event argmin of the launch is the first pick
    bi = np.zeros(len(evs), np.int64); bs = np.zeros(len(evs))
    rk.rkn_batch_launch(c.ctx, bi, bs)
    assert np.array_equal(bi, idx[:, 0]) and np.array_equal(bs, sc[:, 0])
    c.close()
