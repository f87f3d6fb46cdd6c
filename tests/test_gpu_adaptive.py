"""GPU parity of the adaptive-step scan (the error-controlled RKN that section 2.2
cites): per-seed scores and n_in against the oracle's adaptive score, the best seed
per event, the reduction to the fixed-step kernel when h_min = h_max, and argument
checks."""
import numpy as np
import pytest

import oracle
from paper_1908_01949_amd import synth
from tests import parity_util as pu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rk():
    from paper_1908_01949_amd import rknscan
    rknscan.load_library()
    return rknscan


def _note(msg):
    print(msg, flush=True)


def _orc_scores(O, prm, ap, evs, w):
    out = []
    for x in w:
        ev = evs[int(x["event"])]
        n = int(np.prod(x["count"]))
        for k in range(n):
            s = O.window_seed(x, k)
            out.append(O.score_adaptive(prm, ap, s, ev.wire_id, ev.drift)[:2])
    return np.array([o[0] for o in out]), np.array([o[1] for o in out])


@pytest.mark.parametrize("kind,turn_stop", [("uniform", 0), ("solenoid", 0), ("solenoid", 1)])
def test_adaptive_scan_matches_oracle(rk, geo, ufield, sfield, orc_u, orc_s, kind, turn_stop):
    field, O = (ufield, orc_u) if kind == "uniform" else (sfield, orc_s)
    evs = [synth.event_multi_turn(geo, field, 0), synth.event_multi_turn(geo, field, 1)]
    off, wid, dr = synth.pack_events(evs)
    c = rk.Context(0)
    c.upload_geometry(geo); c.upload_field(field); c.upload_hits(off, wid, dr)
    w = synth.make_windows([(0, 0, evs[0].truth_seeds[0], (0.02, 40.0, 2.0, 2.0, 4.0), (3, 3, 3, 2, 3)),
                            (1, 0, evs[1].truth_seeds[0], (0.01, 20.0, 1.0, 1.0, 2.0), (2, 3, 2, 3, 2))])
    n = int(sum(int(np.prod(x["count"])) for x in w))
    p = rk.make_scan_params(n_steps=6000, precision=32, turn_stop=turn_stop)
    ap = rk.make_adaptive_params(tol_mm=1e-5, h_min_mm=0.25, h_max_mm=4.0)
    sc = np.zeros(n); nin = np.zeros(n, np.int32); bi = np.zeros(2, np.int64); bs = np.zeros(2)
    rk.rkn_scan_windows_adaptive(c.ctx, p, ap, w, sc, nin, bi, bs)
    osc, onin = _orc_scores(O, O.params(n_steps=6000, turn_stop=turn_stop), oracle.OrcAdaptive(1e-5, 0.25, 4.0), evs, w)
    rel = pu.check_scores(sc, osc)
    pu.check_nin(nin, onin, max_frac=0.02)
    n0 = int(np.prod(w[0]["count"]))
    pu.check_best(bi[0], osc[:n0])
    pu.check_best(bi[1], osc[n0:], offset=n0)
    _note(f"{kind} turn_stop={turn_stop}: {n} seeds, max rel score error vs the oracle {rel:.2e}")
    c.close()


@pytest.mark.parametrize("kind", ["uniform", "solenoid"])
def test_adaptive_fp64_matches_oracle(rk, geo, ufield, sfield, orc_u, orc_s, kind):
    """FP64 propagation with the adaptive step size: the same step decisions as the FP64
    oracle except at rounding-level ties, so the scores agree to ~1e-9."""
    field, O = (ufield, orc_u) if kind == "uniform" else (sfield, orc_s)
    evs = [synth.event_single_turn(geo, field, 0), synth.event_multi_turn(geo, field, 1)]
    off, wid, dr = synth.pack_events(evs)
    c = rk.Context(0)
    c.upload_geometry(geo); c.upload_field(field); c.upload_hits(off, wid, dr)
    w = synth.make_windows([(0, 0, evs[0].truth_seeds[0], (0.05, 30.0, 3.0, 3.0, 3.0), (3, 3, 3, 3, 3)),
                            (1, 0, evs[1].truth_seeds[0], (0.01, 20.0, 1.0, 1.0, 2.0), (2, 3, 2, 2, 3))])
    n = int(sum(int(np.prod(x["count"])) for x in w))
    p = rk.make_scan_params(n_steps=2000, precision=64)
    ap = rk.make_adaptive_params()
    sc = np.zeros(n); nin = np.zeros(n, np.int32); bi = np.zeros(2, np.int64); bs = np.zeros(2)
    rk.rkn_scan_windows_adaptive(c.ctx, p, ap, w, sc, nin, bi, bs)
    osc, onin = _orc_scores(O, O.params(n_steps=2000), oracle.OrcAdaptive(1e-5, 0.25, 4.0), evs, w)
    rel = pu.check_scores(sc, osc, rel=1e-8, abs_=1e-8)
    pu.check_nin(nin, onin)
    n0 = int(np.prod(w[0]["count"]))
    pu.check_best(bi[0], osc[:n0])
    pu.check_best(bi[1], osc[n0:], offset=n0)
    _note(f"{kind} FP64 adaptive: {n} seeds, max rel score error vs the oracle {rel:.2e}")
    c.close()


def test_adaptive_with_fixed_step_equals_fixed_kernel(rk, geo, sfield):
    """h_min = h_max = 1 mm: the adaptive kernel takes the fixed steps, so its scores
    equal the fixed-step kernel's to FP32 rounding (same chords; the two round
    differently: the adaptive step compensates its sums and evaluates every stage's
    field at every step, the fixed step folds per block and takes the previous last
    stage's field; each is within ~4e-6 of the oracle's scores, so 1e-5 apart)."""
    ev = synth.event_multi_turn(geo, sfield, 2)
    off, wid, dr = synth.pack_events([ev])
    c = rk.Context(0)
    c.upload_geometry(geo); c.upload_field(sfield); c.upload_hits(off, wid, dr)
    w = synth.make_windows([(0, 0, ev.truth_seeds[0], (0.05, 60.0, 3.0, 3.0, 6.0), (4, 4, 4, 4, 4))])
    p = rk.make_scan_params(n_steps=6000, precision=32)
    n = int(np.prod(w[0]["count"]))
    a = np.zeros(n); b = np.zeros(n)
    rk.rkn_scan_windows_adaptive(c.ctx, p, rk.make_adaptive_params(1e-9, 1.0, 1.0), w, a, None,
                                 np.zeros(1, np.int64), np.zeros(1))
    rk.rkn_scan_windows(c.ctx, p, w, b, None, np.zeros(1, np.int64), np.zeros(1))
    np.testing.assert_allclose(a, b, rtol=1e-5, atol=1e-6)
    for bad in (rk.make_adaptive_params(0.0, 0.25, 4.0), rk.make_adaptive_params(1e-5, 4.0, 1.0)):
        with pytest.raises(rk.RknError):
            rk.rkn_scan_windows_adaptive(c.ctx, p, bad, w, a, None, None, None)
    c.close()


def test_batch_adaptive_equals_window_scan(rk, geo, sfield, orc_s):
    """The batched persistent launch with the adaptive step size gives the window scan's
    adaptive scores (same kernel, captured in the graph), and sampled seeds match the
    oracle's adaptive score."""
    from paper_1908_01949_amd import workloads
    evs = synth.events_batch(geo, sfield, 24, seed=3)
    off, wid, dr = synth.pack_events(evs)
    c = rk.Context(0)
    c.upload_geometry(geo); c.upload_field(sfield); c.upload_hits(off, wid, dr)
    hp = rk.make_hough_params(b_ref=sfield.b_ref, **workloads.BATCH["hough"])
    sp = rk.make_scan_params(n_steps=6000, precision=32)
    ap = rk.make_adaptive_params()
    rk.rkn_batch_plan_adaptive(c.ctx, hp, sp, ap)
    bi = np.zeros(24, np.int64); bs = np.zeros(24)
    rk.rkn_batch_launch(c.ctx, bi, bs)
    w, score, nin, ev_seed = rk.rkn_batch_results(c.ctx, 24)
    n = score.size
    s2 = np.zeros(n); b2 = np.zeros(24, np.int64); e2 = np.zeros(24)
    rk.rkn_scan_windows_adaptive(c.ctx, sp, ap, w, s2, None, b2, e2)
    np.testing.assert_allclose(score, s2, rtol=1e-12, atol=0)
    assert np.array_equal(bi, b2)
    g = np.sort(np.random.default_rng(33).choice(n, 48, replace=False))
    sizes = np.prod(w["count"].astype(np.int64), axis=1)
    base = np.concatenate([[0], np.cumsum(sizes)])
    osc = []
    for k in g:
        wi = int(np.searchsorted(base, k, side="right") - 1)
        e = int(w[wi]["event"])
        s = orc_s.window_seed(w[wi], int(k - base[wi]))
        osc.append(orc_s.score_adaptive(orc_s.params(n_steps=6000), oracle.OrcAdaptive(1e-5, 0.25, 4.0), s,
                                        evs[e].wire_id, evs[e].drift)[0])
    rel = pu.check_scores(score[g], np.array(osc))
    _note(f"adaptive batch: {n} seeds in {len(w)} windows, equal to the window scan, sample rel error {rel:.2e}")
    c.close()


def test_adaptive_wide_hough_window_every_seed(rk, geo, sfield, orc_s):
    """A Hough window of the batch workload (seeds far from any track as well as near
    it), every seed of a coarser grid over its full span, against the oracle's adaptive
    score: chords of up to h_max = 4 mm reach wires that the cull must not drop."""
    from paper_1908_01949_amd import workloads
    evs = synth.events_batch(geo, sfield, 2, seed=11)
    off, wid, dr = synth.pack_events(evs)
    ohp = orc_s.hough_params(b_ref=sfield.b_ref, **workloads.BATCH["hough"])
    ow = orc_s.hough_seed_windows(ohp, off, wid)
    w = ow[[0, int(np.nonzero(ow["event"] == 1)[0][0])]].copy()   # one window of each event
    w["count"] = np.array([3, 4, 3, 3, 4])
    c = rk.Context(0)
    c.upload_geometry(geo); c.upload_field(sfield); c.upload_hits(off, wid, dr)
    n = int(sum(int(np.prod(x["count"])) for x in w))
    p = rk.make_scan_params(n_steps=6000, precision=32)
    ap = rk.make_adaptive_params(tol_mm=1e-5, h_min_mm=0.25, h_max_mm=4.0)
    ne = len(evs)
    sc = np.zeros(n); nin = np.zeros(n, np.int32); bi = np.zeros(ne, np.int64); bs = np.zeros(ne)
    rk.rkn_scan_windows_adaptive(c.ctx, p, ap, w, sc, nin, bi, bs)
    osc, onin = _orc_scores(orc_s, orc_s.params(n_steps=6000), oracle.OrcAdaptive(1e-5, 0.25, 4.0), evs, w)
    rel = pu.check_scores(sc, osc)
    pu.check_nin(nin, onin, max_frac=0.02)
    _note(f"wide Hough windows (events {sorted(set(w['event'].tolist()))}): {n} seeds, max rel score error "
          f"{rel:.2e}, E from {osc.min():.4g} to {osc.max():.4g}")
    c.close()
