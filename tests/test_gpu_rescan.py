"""GPU coarse-to-fine rescans (section 2.2: the lowest-E seeds are kept, finer grids are
built around them and the scan is repeated) against the oracle's loop.

Rule: every kept seed the GPU returns must score, by the oracle, what the GPU
reports (within the score tolerance). An event whose oracle loop has a margin
(smallest relative gap between consecutive E of a round's k + 1 lowest, and between
the lowest E and the target) above the near-tie bound makes every choice the same on
both sides, so its kept seeds, their steps and its round count must be equal. The
bound is 1e-8 in FP64; in FP32 it is four times the largest relative score error
measured on the GPU's kept seeds (E is dominated by the lambda terms of the
outliers, so relative gaps of 1e-6 between a round's best seeds are common, far
below the 1e-4 score tolerance)."""
import numpy as np
import pytest

from paper_1908_01949_amd import synth, workloads

from parity_util import SCORE_ABS, SCORE_REL

pytestmark = pytest.mark.gpu

HW = np.array([0.02, 12.0, 3.0, 3.0, 3.0])


@pytest.fixture(scope="module")
def rk():
    from paper_1908_01949_amd import rknscan
    rknscan.load_library()
    return rknscan


@pytest.fixture(scope="module")
def batch16(geo, sfield):
    return synth.events_batch(geo, sfield, n_events=16, seed=3)


def _starts(evs, k, seed=0):
    """k kept seeds per event scattered around its first truth seed (some events with
    fewer than k, one with none, some with a zero step in z or pz)."""
    rng = np.random.default_rng(seed)
    ne = len(evs)
    start = np.full((ne, k, 5), np.nan)
    step = np.full((ne, k, 5), np.nan)
    for e, ev in enumerate(evs):
        if e == 5:
            continue
        for j in range(k):
            if e % 4 == 3 and j == k - 1:
                continue
            start[e, j] = ev.truth_seeds[0] + rng.uniform(-1.0, 1.0, 5) * HW
            st = HW * rng.uniform(0.5, 1.0, 5)
            if e % 3 == 1:
                st[1 + 3 * (j % 2)] = 0.0
            step[e, j] = st
    return start, step


def _ctx(rk, geo, field, evs):
    off, wid, dr = synth.pack_events(evs)
    c = rk.Context(0)
    c.upload_geometry(geo)
    c.upload_field(field)
    c.upload_hits(off, wid, dr)
    return c, off, wid, dr


def _compare(orc, prm, off, wid, dr, gpu, ref, rel, abs_, tie=None):
    g5, gst, gsc, grd = gpu
    o5, ost, osc, ord_, margin = ref
    ne = g5.shape[0]
    # every kept seed of the GPU scores, by the oracle, what the GPU reports
    rows = [(e, j) for e in range(ne) for j in range(g5.shape[1]) if np.all(np.isfinite(g5[e, j]))]
    se = np.array([e for e, _ in rows], np.int32)
    s5 = np.array([g5[e, j] for e, j in rows])
    sc, _, _, _ = orc.scan_seeds(prm, off, wid, dr, se, s5, mode=1)
    gs = np.array([gsc[e, j] for e, j in rows])
    assert np.all(np.abs(gs - sc) <= rel * np.abs(sc) + abs_)
    err = float(np.max(np.abs(gs - sc) / np.maximum(np.abs(sc), 1e-30)))
    if tie is None:
        tie = max(4.0 * err, 1e-7)
    exact = 0
    tied = []
    for e in range(ne):
        if margin[e] > tie:
            assert grd[e] == ord_[e], e
            np.testing.assert_allclose(g5[e], o5[e], rtol=0, atol=1e-9, err_msg=f"event {e}")
            assert np.array_equal(gst[e], ost[e], equal_nan=True), e
            fin = np.isfinite(osc[e])
            assert np.array_equal(fin, np.isfinite(gsc[e])), e
            assert np.all(np.abs(gsc[e][fin] - osc[e][fin]) <= rel * np.abs(osc[e][fin]) + abs_), e
            exact += 1
        else:
            tied.append(e)
    print(f"rescan parity: {exact} events identical, near-ties {tied} (bound {tie:.2e}, max score error {err:.2e})")
    return exact, tied


_ORACLE_RUNS = {}


def _oracle_loop(orc, prm, off, wid, dr, start, step, G, R, target=None):
    """The oracle's loop (cached: both precisions compare against the same runs)."""
    key = (G, R, prm.turn_stop, None if target is None else target.tobytes())
    if key not in _ORACLE_RUNS:
        _ORACLE_RUNS[key] = orc.rescan_refine(prm, off, wid, dr, start, step, grid=G, max_rounds=R, target=target)
    return _ORACLE_RUNS[key]


@pytest.mark.parametrize("prec,turn_stop", [(64, 0), (32, 0), (64, 1)])
def test_rescan_matches_oracle_loop(rk, geo, sfield, orc_s, batch16, prec, turn_stop):
    """16 events in the solenoid map, k = 2 kept seeds, 4^5 grids, 3 rounds; then the
    same with per-event targets that stop events after different rounds. With
    turn_stop every scored track ends with its turn partition, in both loops."""
    c, off, wid, dr = _ctx(rk, geo, sfield, batch16)
    k, G, R, n_steps = 2, 4, 3, 1500
    start, step = _starts(batch16, k)
    sp = rk.make_scan_params(n_steps=n_steps, precision=prec, turn_stop=turn_stop)
    rp = rk.make_rescan_params(k=k, grid=G, max_rounds=R)
    prm = orc_s.params(n_steps=n_steps, turn_stop=turn_stop)
    rel, abs_, tie = (1e-9, 1e-9, 1e-8) if prec == 64 else (SCORE_REL, SCORE_ABS, None)
    gpu = rk.rkn_rescan_refine(c.ctx, sp, rp, len(batch16), start, step)
    ref = _oracle_loop(orc_s, prm, off, wid, dr, start, step, G, R)
    exact, tied = _compare(orc_s, prm, off, wid, dr, gpu, ref, rel, abs_, tie)
    assert gpu[3][5] == 0 and ref[3][5] == 0 and np.all(np.isnan(gpu[2][5]))
    assert exact >= (12 if prec == 64 else 6), (exact, tied)
    # targets between the oracle's first- and third-round bests stop events early
    one = _oracle_loop(orc_s, prm, off, wid, dr, start, step, G, 1)
    target = np.where(np.isfinite(one[2][:, 0]), 0.5 * (one[2][:, 0] + ref[2][:, 0]), np.inf)
    gpu = rk.rkn_rescan_refine(c.ctx, sp, rp, len(batch16), start, step, target=target)
    ref = _oracle_loop(orc_s, prm, off, wid, dr, start, step, G, R, target)
    exact, tied = _compare(orc_s, prm, off, wid, dr, gpu, ref, rel, abs_, tie)
    assert exact >= (10 if prec == 64 else 5), (exact, tied)
    assert len(set(ref[3].tolist())) >= 2      # the targets stop events after different rounds
    c.close()


def test_rescan_from_batch_equals_explicit_start(rk, geo, sfield, batch16):
    """Starting from the last batch launch equals starting from that launch's k best with
    the steps of their windows given explicitly; device outputs equal host outputs;
    zero rounds return the start."""
    import torch
    c, off, wid, dr = _ctx(rk, geo, sfield, batch16)
    ne, k = len(batch16), 3
    hp = rk.make_hough_params(b_ref=sfield.b_ref, **workloads.BATCH["hough"])
    sp = rk.make_scan_params(n_steps=1500, precision=32)
    rk.rkn_batch_plan(c.ctx, hp, sp)
    rk.rkn_batch_launch(c.ctx)
    idx, sc, s5 = rk.rkn_batch_topk(c.ctx, k, n_events=ne)
    windows, _, _, _ = rk.rkn_batch_results(c.ctx, ne, want_scores=False)
    sizes = np.prod(windows["count"].astype(np.int64), axis=1)
    wbase = np.concatenate([[0], np.cumsum(sizes)])
    kw = np.searchsorted(wbase, np.where(idx >= 0, idx, 0), side="right") - 1
    cnt = windows["count"][kw].astype(np.float64)
    step = np.where(cnt > 1, 2.0 * windows["half_width"][kw] / np.maximum(cnt - 1, 1), 0.0)
    step[idx < 0] = np.nan
    rp = rk.make_rescan_params(k=k, grid=4, max_rounds=2)
    a = rk.rkn_rescan_refine(c.ctx, sp, rp, ne)
    b = rk.rkn_rescan_refine(c.ctx, sp, rp, ne, s5, step)
    for x, y in zip(a, b):
        assert np.array_equal(x, y, equal_nan=True)
    assert np.all(a[3][np.any(idx >= 0, axis=1)] == 2)
    # device pointers
    dsp = rk.make_scan_params(n_steps=1500, precision=32, ptr_flags=1)
    dev = torch.device("cuda", 0)
    outs = (torch.zeros((ne, k, 5), dtype=torch.float64, device=dev),
            torch.zeros((ne, k, 5), dtype=torch.float64, device=dev),
            torch.zeros((ne, k), dtype=torch.float64, device=dev), torch.zeros(ne, dtype=torch.int32, device=dev))
    d5, dstep = torch.from_numpy(s5).to(dev), torch.from_numpy(step).to(dev)
    torch.cuda.synchronize()         # the context runs on its own stream
    rk.rkn_rescan_refine(c.ctx, dsp, rp, ne, d5, dstep, None, *outs)
    rk.rkn_synchronize(c.ctx)
    for x, y in zip(outs, b):
        assert np.array_equal(x.cpu().numpy(), y, equal_nan=True)
    # zero rounds: the start rows come back, no score, no round
    z = rk.rkn_rescan_refine(c.ctx, sp, rk.make_rescan_params(k=k, grid=4, max_rounds=0), ne, s5, step)
    assert np.array_equal(z[0], s5, equal_nan=True) and np.array_equal(z[1], step, equal_nan=True)
    assert np.all(np.isnan(z[2])) and np.all(z[3] == 0)
    c.close()


def test_rescan_argument_errors(rk, geo, ufield, ev1):
    c, off, wid, dr = _ctx(rk, geo, ufield, [ev1])
    sp = rk.make_scan_params(n_steps=100)
    s = np.zeros((1, 1, 5))
    for bad in (dict(k=0), dict(k=17), dict(grid=1), dict(grid=17), dict(max_rounds=65)):
        kw = dict(k=1, grid=3, max_rounds=1)
        kw.update(bad)
        with pytest.raises(rk.RknError) as e:
            rk.rkn_rescan_refine(c.ctx, sp, rk.make_rescan_params(**kw), 1, np.zeros((1, kw["k"], 5)),
                                 np.zeros((1, kw["k"], 5)))
        assert e.value.status == rk.RKN_E_ARG
    rp = rk.make_rescan_params(k=1, grid=3, max_rounds=1)
    rp.reserved = 1
    with pytest.raises(rk.RknError) as e:
        rk.rkn_rescan_refine(c.ctx, sp, rp, 1, s, s)
    assert e.value.status == rk.RKN_E_ARG
    rp.reserved = 0
    with pytest.raises(rk.RknError) as e:          # no batch launched to start from
        rk.rkn_rescan_refine(c.ctx, sp, rp, 1)
    assert e.value.status == rk.RKN_E_STATE
    with pytest.raises(rk.RknError) as e:          # start without steps
        rk.load_library()
        st = rk.load_library().rkn_rescan_refine(c.ctx, rk.C.byref(sp), rk.C.byref(rp), rk._ptr(s), None, None,
                                                 None, None, None, None)
        rk._check(c.ctx, st)
    assert e.value.status == rk.RKN_E_ARG
    c.close()
