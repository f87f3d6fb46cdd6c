"""GPU parity of the hit classification and of the two-direction quality count
(section 2.2): classified-hit masks against the oracle's classification of the same
seeds, exit-side windows (the time-reversed track, opposite charge) against the
oracle's Hough stage, and N_c from both directions against the oracle's masks."""
import numpy as np
import pytest

from paper_1908_01949_amd import synth
from tests import parity_util as pu

pytestmark = pytest.mark.gpu

N_STEPS = 6000
SQRT_LAM = 8.0


@pytest.fixture(scope="module")
def rk():
    from paper_1908_01949_amd import rknscan
    rknscan.load_library()
    return rknscan


def _check_mask(O, prm, gmask, seed, x):
    """GPU mask equals the oracle's, except hits whose residual is within rounding of
    the classification boundary |D - d| = sqrt(lambda)."""
    nh = x.wire_id.size
    om = O.inlier_mask(prm, seed, x.wire_id, x.drift).astype(bool)
    g = gmask[:nh].astype(bool)
    assert not np.any(gmask[nh:])
    diff = np.nonzero(g != om)[0]
    if diff.size:
        _, r, _ = O.residual_jacobian(prm, seed, x.wire_id, x.drift, np.ones(nh, np.uint8))
        assert np.all(np.abs(np.abs(r[diff]) - SQRT_LAM) < 1e-3), (diff, r[diff])
    return diff.size


@pytest.mark.parametrize("kind", ["uniform", "solenoid"])
def test_classify_matches_oracle(rk, geo, ufield, sfield, kind):
    field = ufield if kind == "uniform" else sfield
    import oracle
    O = oracle.Oracle(geo, field)
    evs = [synth.event_fixed_total(geo, field, s, n_total=150, noise_frac=0.2) for s in (4, 5, 6)]
    off, wid, dr = synth.pack_events(evs)
    c = rk.Context(0)
    c.upload_geometry(geo); c.upload_field(field); c.upload_hits(off, wid, dr)
    rng = np.random.default_rng(3)
    ev = np.array([2, 0, 1, 0, 2, 1] * 2, np.int32)   # any event order
    amp = np.array([0.003, 3.0, 0.6, 0.6, 1.0])
    s5 = np.array([evs[e].truth_seeds[0] for e in ev]) + amp * rng.uniform(-1, 1, (ev.size, 5))
    H = int(np.diff(off).max())
    for charge in (-1.0, 1.0):
        p = rk.make_scan_params(n_steps=N_STEPS, precision=32, charge=charge)
        mask, n_in = rk.rkn_classify_hits(c.ctx, p, ev, s5, H)
        prm = O.params(n_steps=N_STEPS, charge=charge)
        flips = 0
        for i, e in enumerate(ev):
            flips += _check_mask(O, prm, mask[i], s5[i], evs[e])
            assert n_in[i] == int(mask[i].sum())
        # the classification agrees with the scan's n_in for the same seeds
        sc = np.zeros(ev.size); nin2 = np.zeros(ev.size, np.int32)
        rk.rkn_scan_seeds(c.ctx, p, ev, s5, sc, nin2, np.zeros(3, np.int64), np.zeros(3))
        pu.check_nin(n_in, nin2)
        print(f"{kind} charge {charge:+.0f}: {ev.size} seeds, {flips} boundary flips", flush=True)
    c.close()


def test_exit_side_windows_and_common_hits(rk, geo, sfield, orc_s):
    """Entrance scan (electron) and exit scan (time-reversed: opposite charge) of
    single-track events; their best seeds classify mostly the same hits (N_c), the
    GPU's N_c equals the count of the oracle's masks, and exit-side windows equal the
    oracle's Hough stage with the opposite charge."""
    evs = [synth.event_fixed_total(geo, sfield, s, n_total=120, noise_frac=0.1) for s in (7, 8, 9, 10)]
    off, wid, dr = synth.pack_events(evs)
    c = rk.Context(0)
    c.upload_geometry(geo); c.upload_field(sfield); c.upload_hits(off, wid, dr)
    H = int(np.diff(off).max())
    kw = dict(b_ref=sfield.b_ref, min_votes=6, max_cand=2, gran=(0.01, 100.0, 2.5, 2.5, 12.0), count=(5, 7, 5, 5, 7),
              grow=(1, 0, 1, 1, 0), count_max=9, max_seeds_window=12000)
    best = {}
    for charge in (-1.0, 1.0):
        w = rk.rkn_hough_seed_windows(c.ctx, rk.make_hough_params(charge=charge, **kw))
        ow = orc_s.hough_seed_windows(orc_s.hough_params(charge=charge, **kw), off, wid)
        assert np.array_equal(ow["count"], w["count"]) and np.array_equal(ow["event"], w["event"])
        np.testing.assert_allclose(ow["center"], w["center"], rtol=0, atol=1e-11)
        p = rk.make_scan_params(n_steps=N_STEPS, precision=32, charge=charge)
        idx, sc, s5 = rk.rkn_scan_windows_topk(c.ctx, p, w, 1, n_events=len(evs))
        assert np.all(idx[:, 0] >= 0)
        best[charge] = s5[:, 0]
    ev = np.arange(len(evs), dtype=np.int32)
    p = rk.make_scan_params(n_steps=N_STEPS, precision=32, charge=-1.0)
    m_in, m_out, n_common = rk.rkn_bidirectional_common(c.ctx, p, ev, best[-1.0], best[1.0], H)
    for e, x in enumerate(evs):
        nh = x.wire_id.size
        om_in = orc_s.inlier_mask(orc_s.params(n_steps=N_STEPS, charge=-1.0), best[-1.0][e], x.wire_id, x.drift)
        om_out = orc_s.inlier_mask(orc_s.params(n_steps=N_STEPS, charge=1.0), best[1.0][e], x.wire_id, x.drift)
        oc = int((om_in.astype(bool) & om_out.astype(bool)).sum())
        assert abs(int(n_common[e]) - oc) <= 2, (e, n_common[e], oc)
        assert n_common[e] == int((m_in[e, :nh].astype(bool) & m_out[e, :nh].astype(bool)).sum())
        true_hits = int((~x.is_noise).sum())
        print(f"event {e}: {nh} hits ({true_hits} true), entrance {int(m_in[e].sum())}, exit {int(m_out[e].sum())}, "
              f"common {int(n_common[e])} (oracle {oc})", flush=True)
        # the paper's quality cut keeps these clean single-track events
        assert n_common[e] >= 20
    c.close()


def test_mask_rows_fully_defined(rk, geo, sfield):
    """Columns past an event's hit count are 0 even where the buffers held ones from
    an earlier classification of larger events, so the counts only see real hits."""
    big = [synth.event_fixed_total(geo, sfield, s, n_total=150, noise_frac=0.3) for s in (4, 5)]
    small = [synth.event_fixed_total(geo, sfield, s, n_total=n, noise_frac=0.1) for s, n in ((6, 60), (7, 45))]
    c = rk.Context(0)
    c.upload_geometry(geo); c.upload_field(sfield)
    p = rk.make_scan_params(n_steps=N_STEPS, precision=32, lambda_mm2=1e6)   # every reached hit is in
    for evs in (big, small):
        off, wid, dr = synth.pack_events(evs)
        c.upload_hits(off, wid, dr)
        H = int(np.diff(off).max())
        ev = np.array([0, 1, 0, 1], np.int32)
        s5 = np.array([evs[e].truth_seeds[0] for e in ev])
        mask, n_in = rk.rkn_classify_hits(c.ctx, p, ev, s5, H)
        for i, e in enumerate(ev):
            nh = evs[e].wire_id.size
            assert not mask[i, nh:].any() and n_in[i] == int(mask[i].sum()) > 0
        _, _, n_common = rk.rkn_bidirectional_common(c.ctx, p, ev, s5, s5, H)
        assert np.all(n_common <= np.diff(off)[ev])
    c.close()
