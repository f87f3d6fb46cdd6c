"""GPU parity of the batched path: Hough windows -> tiles -> one persistent scan launch
-> per-event argmin, replayed from captured HIP graphs."""
import numpy as np
import pytest

from paper_1908_01949_amd import synth
from tests import parity_util as pu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rk():
    from paper_1908_01949_amd import rknscan
    rknscan.load_library()
    return rknscan


def test_batch_matches_oracle_and_replays(rk, geo, sfield, orc_s):
    evs = synth.events_batch(geo, sfield, 12, seed=1)
    off, wid, dr = synth.pack_events(evs)
    c = rk.Context(0)
    c.upload_geometry(geo); c.upload_field(sfield); c.upload_hits(off, wid, dr)
    kw = dict(b_ref=sfield.b_ref, max_cand=3, gran=(0.01, 100.0, 2.5, 2.5, 12.0), count=(3, 2, 3, 3, 2),
              grow=(1, 0, 1, 1, 0), count_max=5, max_seeds_window=200)
    hp = rk.make_hough_params(**kw)
    n_steps = 1500
    sp = rk.make_scan_params(n_steps=n_steps, precision=32)
    rk.rkn_batch_plan(c.ctx, hp, sp)
    ne = len(evs)
    bi = np.zeros(ne, np.int64); bs = np.zeros(ne)
    rk.rkn_batch_launch(c.ctx, bi, bs)
    nw, ns, th, ts = rk.rkn_batch_info(c.ctx)
    print(f"batch: {nw} windows, {ns} seeds, hough {th:.2f} ms, scan {ts:.2f} ms", flush=True)
    w, score, nin, ev_seed = rk.rkn_batch_results(c.ctx, ne)
    assert nw >= ne and ns == int(sum(np.prod(x["count"].astype(np.int64)) for x in w))
    # windows: the batch expansion keeps exactly the Hough stage's windows
    w_direct = rk.rkn_hough_seed_windows(c.ctx, hp)
    assert np.array_equal(w_direct, w)
    ow = orc_s.hough_seed_windows(orc_s.hough_params(**kw), off, wid)
    assert np.array_equal(ow["count"], w["count"]) and np.array_equal(ow["event"], w["event"])
    np.testing.assert_allclose(ow["center"], w["center"], rtol=0, atol=1e-11)
    # scores against the oracle on the same windows
    osc, onin, obi, obs, _ = orc_s.scan_windows(orc_s.params(n_steps=n_steps), off, wid, dr, w)
    rel = pu.check_scores(score, osc)
    print(f"max rel score error {rel:.2e}", flush=True)
    pu.check_nin(nin, onin)
    for e in range(ne):
        lo, hi = ev_seed[e], ev_seed[e + 1]
        if hi > lo:
            pu.check_best(bi[e], osc[lo:hi], offset=lo)
        else:
            assert bi[e] == -1
    # same kernels as the eager scan: bit-identical scores
    s2 = np.zeros(ns); n2 = np.zeros(ns, np.int32); b2 = np.zeros(ne, np.int64); e2 = np.zeros(ne)
    rk.rkn_scan_windows(c.ctx, sp, w, s2, n2, b2, e2)
    assert np.array_equal(s2, score) and np.array_equal(b2, bi)
    # replays after other work give identical results
    for _ in range(3):
        bi3 = np.zeros(ne, np.int64); bs3 = np.zeros(ne)
        rk.rkn_batch_launch(c.ctx, bi3, bs3)
        _, s3, _, _ = rk.rkn_batch_results(c.ctx, ne)
        assert np.array_equal(s3, score) and np.array_equal(bi3, bi) and np.array_equal(bs3, bs)
        rk.rkn_scan_windows(c.ctx, sp, w[:2], None, None, np.zeros(ne, np.int64), np.zeros(ne))
    c.close()


def test_batch_requires_plan_and_reupload_invalidates(rk, geo, ufield):
    c = rk.Context(0)
    c.upload_geometry(geo); c.upload_field(ufield)
    ev = synth.event_single_turn(geo, ufield, 0)
    off, wid, dr = synth.pack_events([ev])
    c.upload_hits(off, wid, dr)
    with pytest.raises(rk.RknError) as e:
        rk.rkn_batch_launch(c.ctx, np.zeros(1, np.int64), np.zeros(1))
    assert e.value.status == rk.RKN_E_STATE
    rk.rkn_batch_plan(c.ctx, rk.make_hough_params(count=(2, 2, 2, 2, 2), count_max=2),
                      rk.make_scan_params(n_steps=300))
    rk.rkn_batch_launch(c.ctx, np.zeros(1, np.int64), np.zeros(1))
    c.upload_hits(off, wid, dr)
    with pytest.raises(rk.RknError) as e:
        rk.rkn_batch_launch(c.ctx, np.zeros(1, np.int64), np.zeros(1))
    assert e.value.status == rk.RKN_E_STATE
    # a field upload after the plan drops it too (the captured graphs hold the field)
    for fld in (synth.solenoid_field(), ufield):
        rk.rkn_batch_plan(c.ctx, rk.make_hough_params(count=(2, 2, 2, 2, 2), count_max=2),
                          rk.make_scan_params(n_steps=300))
        c.upload_field(fld)
        with pytest.raises(rk.RknError) as e:
            rk.rkn_batch_launch(c.ctx, np.zeros(1, np.int64), np.zeros(1))
        assert e.value.status == rk.RKN_E_STATE
    c.close()


def test_batch_block_sizes_agree_and_autotune(rk, geo, sfield):
    """The cull is exact, so every block size (and workgroup shape) gives the same
    scores up to FP32 rounding of the trajectories (their block-relative sums fold
    into the compensated origin at each block's end, every B steps: ~2e-6 relative,
    far inside the oracle tolerance); the autotuner leaves the batch planned with one
    of them."""
    evs = synth.events_batch(geo, sfield, 10, seed=7)
    off, wid, dr = synth.pack_events(evs)
    c = rk.Context(0)
    c.upload_geometry(geo); c.upload_field(sfield); c.upload_hits(off, wid, dr)
    hp = rk.make_hough_params(b_ref=sfield.b_ref, max_cand=3, gran=(0.01, 100.0, 2.5, 2.5, 12.0),
                              count=(3, 3, 3, 3, 3), grow=(1, 0, 1, 1, 0), count_max=5, max_seeds_window=600)
    ne = len(evs)
    ref = None
    for b in (4, 6, 8):
        rk.rkn_batch_plan(c.ctx, hp, rk.make_scan_params(n_steps=1000, precision=32, block_steps=b))
        bi = np.zeros(ne, np.int64); bs = np.zeros(ne)
        rk.rkn_batch_launch(c.ctx, bi, bs)
        _, score, nin, _ = rk.rkn_batch_results(c.ctx, ne)
        if ref is None:
            ref = (score, nin, bi)
        else:
            d = float(np.max(np.abs(score - ref[0]) / np.maximum(np.abs(ref[0]), 1e-12)))
            print(f"block_steps={b}: max rel score difference to block_steps=4: {d:.2e}", flush=True)
            pu.check_scores(score, ref[0], rel=1e-5, abs_=1e-5)
            pu.check_nin(nin, ref[1])
            ev_seed = rk.rkn_batch_results(c.ctx, ne, want_scores=False)[3]
            for e in range(ne):
                if ev_seed[e + 1] > ev_seed[e]:
                    pu.check_best(bi[e], ref[0][ev_seed[e]:ev_seed[e + 1]], offset=ev_seed[e])
    chosen, ms = rk.rkn_batch_autotune(c.ctx, hp, rk.make_scan_params(n_steps=1000, precision=32),
                                       sample_events=4, reps=1)
    print(f"autotune: chose {chosen}, sample ms {ms}", flush=True)
    assert chosen in (4, 6, 8) and np.isfinite(min(ms))
    bi = np.zeros(ne, np.int64); bs = np.zeros(ne)
    rk.rkn_batch_launch(c.ctx, bi, bs)
    _, score, _, _ = rk.rkn_batch_results(c.ctx, ne)
    pu.check_scores(score, ref[0], rel=1e-5, abs_=1e-5)
    c.close()


def test_batch_on_a_40_layer_chamber(rk, sfield):
    """The batched graph on a 40-layer chamber, where the 12-wave shape does not fit the
    LDS: the plan, its tiles and the captured scan use the 8-wave fallback, and the
    Hough windows, scores, n_in and best seeds match the oracle's."""
    import oracle
    g = synth.make_geometry(n_layers=40)
    evs = synth.events_batch(g, sfield, 3, seed=23, hits_range=(8, 480))
    off, wid, dr = synth.pack_events(evs)
    c = rk.Context(0)
    c.upload_geometry(g); c.upload_field(sfield); c.upload_hits(off, wid, dr)
    kw = dict(b_ref=sfield.b_ref, max_cand=2, gran=(0.01, 100.0, 2.5, 2.5, 12.0), count=(3, 2, 3, 3, 2),
              grow=(1, 0, 1, 1, 0), count_max=4, max_seeds_window=150)
    hp = rk.make_hough_params(**kw)
    n_steps = 1500
    sp = rk.make_scan_params(n_steps=n_steps, precision=32)
    assert rk.rkn_scan_shape(c.ctx, sp) == (6, 512)
    rk.rkn_batch_plan(c.ctx, hp, sp)
    ne = len(evs)
    bi = np.zeros(ne, np.int64); bs = np.zeros(ne)
    rk.rkn_batch_launch(c.ctx, bi, bs)
    w, score, nin, ev_seed = rk.rkn_batch_results(c.ctx, ne)
    c.close()
    O = oracle.Oracle(g, sfield)
    ow = O.hough_seed_windows(O.hough_params(**kw), off, wid)
    assert np.array_equal(ow["count"], w["count"]) and np.array_equal(ow["event"], w["event"])
    np.testing.assert_allclose(ow["center"], w["center"], rtol=0, atol=1e-11)
    osc, onin, obi, obs, _ = O.scan_windows(O.params(n_steps=n_steps), off, wid, dr, w)
    rel = pu.check_scores(score, osc)
    pu.check_nin(nin, onin)
    for e in range(ne):
        lo, hi = ev_seed[e], ev_seed[e + 1]
        if hi > lo:
            pu.check_best(bi[e], osc[lo:hi], offset=lo)
        else:
            assert bi[e] == -1
    print(f"40-layer batch: {len(w)} windows, {score.size} seeds, max rel score error {rel:.2e}", flush=True)
