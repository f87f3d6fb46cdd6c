"""GPU parity of the turn-partition parts (sections 2.3 and 4.2): scans, traces and
Gauss-Newton with the track ending at its turn partition, the predicted seeds of
neighbouring partitions, and the reconstruction loop, each step of which is checked
against the oracle (the prediction from the previous partition's fitted seed, the
classification at the fitted seed over the hits still unclassified) and scored by
Eqs. 2-3 on the synthetic truth."""
import numpy as np
import pytest

from paper_1908_01949_amd import quality, synth
from tests import parity_util as pu

pytestmark = pytest.mark.gpu

N_STEPS = 6000


@pytest.fixture(scope="module")
def rk():
    from paper_1908_01949_amd import rknscan
    rknscan.load_library()
    return rknscan


def _note(msg):
    print(msg, flush=True)


def _ctx(rk, geo, field, evs):
    off, wid, dr = synth.pack_events(evs)
    c = rk.Context(0)
    c.upload_geometry(geo); c.upload_field(field); c.upload_hits(off, wid, dr)
    return c, off, wid, dr


@pytest.mark.parametrize("kind", ["uniform", "solenoid"])
def test_turn_stop_scan_parity(rk, geo, ufield, sfield, orc_u, orc_s, kind):
    """Scores and n_in of windows around the truth seeds of two multi-turn events,
    with the stop rule, element by element against the oracle, for every block size."""
    field, O = (ufield, orc_u) if kind == "uniform" else (sfield, orc_s)
    evs = [synth.event_multi_turn(geo, field, s) for s in (0, 1)]
    c, off, wid, dr = _ctx(rk, geo, field, evs)
    w = synth.make_windows([(e, 0, evs[e].truth_seeds[0], (0.02, 60.0, 3.0, 3.0, 6.0), (3, 5, 3, 3, 5))
                            for e in range(2)] + [(1, 1, evs[1].truth_seeds[0], (0.01, 20.0, 1.0, 1.0, 2.0),
                                                   (2, 3, 1, 2, 3))])
    total = int(sum(int(np.prod(x["count"].astype(np.int64))) for x in w))
    osc, onin, obi, _, _ = O.scan_windows(O.params(n_steps=N_STEPS, turn_stop=1), off, wid, dr, w)
    for bsteps in ((0,) if kind == "uniform" else (4, 6, 8)):
        p = rk.make_scan_params(n_steps=N_STEPS, precision=32, turn_stop=1, block_steps=bsteps)
        score = np.zeros(total); nin = np.zeros(total, np.int32); bi = np.zeros(2, np.int64); bs = np.zeros(2)
        rk.rkn_scan_windows(c.ctx, p, w, score, nin, bi, bs)
        rel = pu.check_scores(score, osc)
        pu.check_nin(nin, onin)
        n0 = int(np.prod(w[0]["count"]))
        pu.check_best(bi[0], osc[:n0])
        pu.check_best(bi[1], osc[n0:], offset=n0)
        _note(f"{kind} block {bsteps}: {total} seeds, max rel score error {rel:.2e}")
    # the stop rule changes the scores (the later turns' hits leave the sum)
    p = rk.make_scan_params(n_steps=N_STEPS, precision=32)
    score_all = np.zeros(total)
    rk.rkn_scan_windows(c.ctx, p, w, score_all, None, np.zeros(2, np.int64), np.zeros(2))
    assert np.mean(score_all < osc) > 0.5
    c.close()


@pytest.mark.parametrize("prec,tol", [(64, 1e-9), (32, 0.05)])
def test_turn_stop_trace_parity(rk, geo, sfield, orc_s, prec, tol):
    c, _, _, _ = _ctx(rk, geo, sfield, [synth.event_multi_turn(geo, sfield, 0)])
    rng = np.random.default_rng(21)
    th = rng.uniform(-np.pi, np.pi, 48)
    a = th + rng.uniform(0.3, 1.2, 48)
    pt = rng.uniform(85, 104, 48)
    seeds = np.stack([th, rng.uniform(-300, 300, 48), pt * np.cos(a), pt * np.sin(a), rng.uniform(-20, 20, 48)], 1)
    steps = np.array([0, 1, 500, 900, 1200, 1600, 2500, 6000], np.int32)
    g = rk.rkn_trace(c.ctx, rk.make_scan_params(n_steps=N_STEPS, precision=prec, turn_stop=1), seeds, steps)
    o = orc_s.trace(orc_s.params(n_steps=N_STEPS, turn_stop=1), seeds, steps)
    d = np.linalg.norm(g[..., :3] - o[..., :3], axis=-1)
    _note(f"trace FP{prec} with the stop rule: max position error {d.max():.3e} mm")
    assert d.max() <= tol
    # every track has ended by 6000 steps: the last two states are the same
    assert np.array_equal(g[:, -1], g[:, -2])
    c.close()


@pytest.mark.parametrize("kind", ["uniform", "solenoid"])
def test_neighbour_seeds_parity(rk, geo, ufield, sfield, orc_u, orc_s, kind):
    field, O = (ufield, orc_u) if kind == "uniform" else (sfield, orc_s)
    evs = [synth.event_multi_turn(geo, field, s) for s in (0, 1, 2)]
    c, _, _, _ = _ctx(rk, geo, field, evs)
    rng = np.random.default_rng(22)
    base = np.array([e.truth_seeds[0] for e in evs])
    seeds = np.concatenate([base, base[np.arange(9) % 3] + rng.normal(0, [0.01, 20, 1, 1, 1], (9, 5))])
    p = rk.make_scan_params(n_steps=N_STEPS, precision=64)
    prm = O.params(n_steps=N_STEPS)
    for d in (1, -1):
        out, found = rk.rkn_neighbour_seeds(c.ctx, p, seeds, d)
        for i, s in enumerate(seeds):
            o = O.neighbour_seed(prm, s, d)
            assert (o is not None) == bool(found[i])
            if o is None:
                assert np.all(np.isnan(out[i]))
                continue
            assert abs(np.angle(np.exp(1j * (out[i, 0] - o[0])))) < 1e-9
            np.testing.assert_allclose(out[i, 1:], o[1:], rtol=0, atol=1e-6)
        _note(f"{kind} direction {d:+d}: {int(found.sum())} of {len(seeds)} predictions found, equal to the oracle's")
    out, found = rk.rkn_neighbour_seeds(c.ctx, p, seeds, 1, max_steps=50)
    assert not found.any()
    with pytest.raises(rk.RknError):
        rk.rkn_neighbour_seeds(c.ctx, p, seeds, 0)
    c.close()


def test_turn_stop_gauss_newton(rk, geo, sfield, orc_s):
    """Gauss-Newton with the stop rule from perturbed truth seeds reaches the oracle's
    Phi (same start, same inlier rule)."""
    evs = [synth.event_multi_turn(geo, sfield, s) for s in (0, 1)]
    c, off, wid, dr = _ctx(rk, geo, sfield, evs)
    rng = np.random.default_rng(23)
    ev = np.array([0, 0, 1, 1], np.int32)
    seeds = np.array([evs[e].truth_seeds[0] for e in ev]) + rng.normal(0, [0.003, 5, 0.5, 0.5, 0.5], (4, 5))
    p = rk.make_scan_params(n_steps=N_STEPS, precision=32, turn_stop=1, lambda_mm2=16.0)
    rk.rkn_refine_setup(c.ctx, p, ev, seeds, 64)
    out = np.zeros((4, 5)); phi = np.zeros((4, 11))
    rk.rkn_gn_refine(c.ctx, 10, np.array([1.0, 100, 100, 100, 100]), out, phi)
    prm = orc_s.params(n_steps=N_STEPS, turn_stop=1, lambda_mm2=16.0)
    for i, e in enumerate(ev):
        so, mo, phio = orc_s.gn_refine(prm, seeds[i], evs[e].wire_id, evs[e].drift, iters=10)
        assert phi[i, 0] == pytest.approx(phio[0], rel=1e-3, abs=1e-3)
        _note(f"seed {i}: Phi {phi[i, 0]:.3f} -> {phi[i, -1]:.4f} (oracle {phio[-1]:.4f})")
        assert phi[i, -1] <= phio[-1] * (1 + 1e-3) + 1e-3
    c.close()


@pytest.mark.parametrize("kind,fine", [("uniform", False), ("solenoid", False), ("solenoid", True)])
def test_find_turns(rk, geo, ufield, sfield, orc_u, orc_s, kind, fine):
    field, O = (ufield, orc_u) if kind == "uniform" else (sfield, orc_s)
    evs = [synth.event_multi_turn(geo, field, s) for s in range(6)]
    c, off, wid, dr = _ctx(rk, geo, field, evs)
    hp = rk.make_hough_params(b_ref=field.b_ref, min_votes=6, max_cand=4, gran=(0.01, 50.0, 2.5, 2.5, 4.0),
                              count=(7, 13, 7, 7, 13), count_max=13)
    sp = rk.make_scan_params(n_steps=N_STEPS, precision=32)
    # fine: the optional (z0, pz0) rescan of the first partition's candidates
    tp = rk.make_turn_params(fine_count=(31, 25), n_candidates=4) if fine else rk.make_turn_params()
    r = rk.rkn_find_turns(c.ctx, hp, sp, tp, wid.size, len(evs))
    lam_c = tp.lambda_classify_mm2
    prm_c = O.params(n_steps=N_STEPS, turn_stop=1, lambda_mm2=lam_c)
    prm = O.params(n_steps=N_STEPS)
    eps, pur, flips = [], [], 0
    for e, x in enumerate(evs):
        lo, hi = off[e], off[e + 1]
        lab = r["hit_turn"][lo:hi]
        nt = int(r["n_turns"][e])
        assert nt >= 1 and lab.max() == nt - 1 and lab.min() >= -1
        pos = r["turn_pos"][e, :nt]
        assert pos[0] == 0 and len(set(pos.tolist())) == nt
        for t in range(nt):
            assert int(np.sum(lab == t)) == r["turn_nhits"][e, t] >= tp.min_hits
            # the classification at the fitted seed over the hits left before it
            left = (lab < 0) | (lab >= t)
            om = O.inlier_mask(prm_c, r["turn_seed"][e, t], x.wire_id[left], x.drift[left]).astype(bool)
            got = (lab[left] == t)
            diff = np.nonzero(om != got)[0]
            if diff.size:
                ok, res, _ = O.residual_jacobian(prm_c, r["turn_seed"][e, t], x.wire_id[left], x.drift[left],
                                                 np.ones(int(left.sum()), np.uint8))
                assert np.all(np.abs(np.abs(res[diff]) - np.sqrt(lam_c)) < 2e-3), (e, t, diff, res[diff])
                flips += diff.size
            # a neighbour's window is centred on the prediction from the partition next to it
            if pos[t] != 0:
                d = 1 if pos[t] > 0 else -1
                src = int(np.nonzero(pos[:t] == pos[t] - d)[0][0])
                pred = O.neighbour_seed(prm, r["turn_seed"][e, src], d)
                assert pred is not None
                assert abs(np.angle(np.exp(1j * (r["turn_center"][e, t, 0] - pred[0])))) < 1e-9
                np.testing.assert_allclose(r["turn_center"][e, t, 1:], pred[1:], rtol=0, atol=1e-6)
        q = quality.turn_quality(x.turn_of, lab)
        eps += [v["eps"] for v in q]
        pur += [v["pi"] for v in q if np.isfinite(v["pi"])]
        _note(f"{kind} event {e}: true turns {np.bincount(x.turn_of[x.turn_of >= 0]).tolist()}, found "
              f"{[(int(pos[t]), int(r['turn_nhits'][e, t])) for t in range(nt)]}, "
              f"eps/pi {[(round(v['eps'], 2), round(v['pi'], 2)) for v in q]}")
    _note(f"{kind} (fine rescan {fine}): mean eps {np.mean(eps):.2f}, mean pi {np.mean(pur):.2f}, {flips} boundary flips")
    # every event finds its first partition mostly within one true turn
    assert np.mean(pur) >= 0.5
    # the context's hits are the caller's again: a plain scan still runs on them
    w = synth.make_windows([(0, 0, evs[0].truth_seeds[0], (0.01, 10, 1, 1, 1), (2, 2, 2, 2, 2))])
    sc = np.zeros(32)
    rk.rkn_scan_windows(c.ctx, sp, w, sc, None, np.zeros(len(evs), np.int64), np.zeros(len(evs)))
    osc, _, _, _, _ = O.scan_windows(O.params(n_steps=N_STEPS), off, wid, dr, w)
    pu.check_scores(sc, osc)
    c.close()


def test_find_turns_edges_and_errors(rk, geo, sfield):
    """One partition at most with max_turns = 1; nothing found when min_hits exceeds
    every event's hits; a small event next to a large one; invalid parameters raise
    and leave the context's hits as they were."""
    evs = [synth.event_multi_turn(geo, sfield, 3), synth.event_fixed_total(geo, sfield, 2, n_total=8, noise_frac=0.0)]
    c, off, wid, dr = _ctx(rk, geo, sfield, evs)
    hp = rk.make_hough_params(b_ref=sfield.b_ref, min_votes=6, max_cand=4, gran=(0.01, 50.0, 2.5, 2.5, 4.0),
                              count=(7, 13, 7, 7, 13), count_max=13)
    sp = rk.make_scan_params(n_steps=N_STEPS, precision=32)
    r = rk.rkn_find_turns(c.ctx, hp, sp, rk.make_turn_params(max_turns=1), wid.size, 2)
    assert r["n_turns"][0] == 1 and r["n_turns"][1] == 0
    lab = r["hit_turn"]
    assert set(np.unique(lab[off[0]:off[1]])) <= {-1, 0} and np.all(lab[off[1]:off[2]] == -1)
    r = rk.rkn_find_turns(c.ctx, hp, sp, rk.make_turn_params(min_hits=10000), wid.size, 2)
    assert np.all(r["n_turns"] == 0) and np.all(r["hit_turn"] == -1)
    for bad in (dict(max_turns=0), dict(max_turns=17), dict(min_hits=0), dict(lambda_classify_mm2=0.0),
                dict(n_candidates=0), dict(count=(0, 9, 5, 5, 9)), dict(fine_count=(0, 1))):
        with pytest.raises(rk.RknError):
            rk.rkn_find_turns(c.ctx, hp, sp, rk.make_turn_params(**bad), wid.size, 2)
    with pytest.raises(rk.RknError):
        rk.rkn_find_turns(c.ctx, hp, rk.make_scan_params(n_steps=N_STEPS, precision=64), rk.make_turn_params(),
                          wid.size, 2)
    with pytest.raises(rk.RknError):   # Hough and scan charges differ
        rk.rkn_find_turns(c.ctx, hp, rk.make_scan_params(n_steps=N_STEPS, precision=32, charge=1.0),
                          rk.make_turn_params(), wid.size, 2)
    with pytest.raises(rk.RknError):
        rk.rkn_batch_plan(c.ctx, hp, rk.make_scan_params(n_steps=N_STEPS, precision=32, charge=1.0))
    # the caller's hits are in place: the loop gives the same answer again
    r2 = rk.rkn_find_turns(c.ctx, hp, sp, rk.make_turn_params(max_turns=1), wid.size, 2)
    assert np.array_equal(r2["n_turns"], [1, 0])
    c.close()


def test_turn_stop_fp64_scan_and_batch(rk, geo, ufield, sfield, orc_u):
    """The FP64 scan with the stop rule against the oracle (uniform field), and the
    batched graph with the stop rule equal to the window scan on the batch's windows."""
    from paper_1908_01949_amd import workloads
    ev = synth.event_multi_turn(geo, ufield, 4)
    c, off, wid, dr = _ctx(rk, geo, ufield, [ev])
    w = synth.make_windows([(0, 0, ev.truth_seeds[0], (0.02, 40.0, 2.0, 2.0, 4.0), (3, 4, 3, 3, 4))])
    n = int(np.prod(w[0]["count"]))
    p = rk.make_scan_params(n_steps=N_STEPS, precision=64, turn_stop=1)
    sc = np.zeros(n); nin = np.zeros(n, np.int32); bi = np.zeros(1, np.int64); bs = np.zeros(1)
    rk.rkn_scan_windows(c.ctx, p, w, sc, nin, bi, bs)
    osc, onin, _, _, _ = orc_u.scan_windows(orc_u.params(n_steps=N_STEPS, turn_stop=1), off, wid, dr, w)
    rel = pu.check_scores(sc, osc, rel=1e-9, abs_=1e-9)
    assert np.array_equal(nin, onin)
    pu.check_best(bi[0], osc)
    _note(f"FP64 with the stop rule: {n} seeds, max rel error {rel:.2e}")
    c.close()
    evs = synth.events_batch(geo, sfield, 16, seed=4)
    c, off, wid, dr = _ctx(rk, geo, sfield, evs)
    hp = rk.make_hough_params(b_ref=sfield.b_ref, **workloads.BATCH["hough"])
    sp = rk.make_scan_params(n_steps=N_STEPS, precision=32, turn_stop=1)
    rk.rkn_batch_plan(c.ctx, hp, sp)
    bi = np.zeros(16, np.int64); bs = np.zeros(16)
    rk.rkn_batch_launch(c.ctx, bi, bs)
    wb, score, _, _ = rk.rkn_batch_results(c.ctx, 16)
    s2 = np.zeros(score.size); b2 = np.zeros(16, np.int64)
    rk.rkn_scan_windows(c.ctx, sp, wb, s2, None, b2, np.zeros(16))
    np.testing.assert_allclose(score, s2, rtol=1e-12, atol=0)
    assert np.array_equal(bi, b2)
    _note(f"batch with the stop rule: {score.size} seeds equal to the window scan")
    c.close()
