"""GPU parity of the paper's two-kernel form of the scan (section 4.2: record every
step, then one lane per wire finds its distance of closest approach): scores, n_in
and the best seed per event against the oracle element by element, against the fused
kernel to rounding, across trajectory chunks, with the turn-partition stop, and for
an event without windows."""
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


def _note(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("kind,turn_stop", [("uniform", 0), ("solenoid", 0), ("solenoid", 1)])
def test_two_kernel_matches_oracle_and_fused(rk, geo, ufield, sfield, orc_u, orc_s, kind, turn_stop):
    field, O = (ufield, orc_u) if kind == "uniform" else (sfield, orc_s)
    evs = [synth.event_multi_turn(geo, field, 0), synth.event_fixed_total(geo, field, 1, n_total=80),
           synth.event_multi_turn(geo, field, 2)]
    off, wid, dr = synth.pack_events(evs)
    c = rk.Context(0)
    c.upload_geometry(geo); c.upload_field(field); c.upload_hits(off, wid, dr)
    # event 1 has no window; ragged grids
    w = synth.make_windows([(0, 0, evs[0].truth_seeds[0], (0.03, 60.0, 3.0, 3.0, 6.0), (3, 5, 4, 3, 5)),
                            (2, 0, evs[2].truth_seeds[0], (0.02, 40.0, 2.0, 2.0, 4.0), (2, 3, 3, 3, 4)),
                            (2, 1, evs[2].truth_seeds[0], (0.0, 10.0, 0.0, 0.0, 1.0), (1, 7, 1, 1, 1))])
    n = int(sum(int(np.prod(x["count"].astype(np.int64))) for x in w))
    p = rk.make_scan_params(n_steps=6000, precision=32, turn_stop=turn_stop)
    s2 = np.zeros(n); n2 = np.zeros(n, np.int32); b2 = np.zeros(3, np.int64); e2 = np.zeros(3)
    rk.rkn_scan_windows_two_kernel(c.ctx, p, w, s2, n2, b2, e2)
    s1 = np.zeros(n); n1 = np.zeros(n, np.int32); b1 = np.zeros(3, np.int64); e1 = np.zeros(3)
    rk.rkn_scan_windows(c.ctx, p, w, s1, n1, b1, e1)
    osc, onin, obi, _, _ = O.scan_windows(O.params(n_steps=6000, turn_stop=turn_stop), off, wid, dr, w)
    rel = pu.check_scores(s2, osc)
    pu.check_nin(n2, onin)
    # the fused kernel's chords are the same: scores agree to rounding
    np.testing.assert_allclose(s2, s1, rtol=2e-6, atol=1e-6)
    n0 = int(np.prod(w[0]["count"]))
    pu.check_best(b2[0], osc[:n0])
    pu.check_best(b2[2], osc[n0:], offset=n0)
    assert b2[1] == -1 and e2[1] == np.inf
    assert e2[0] == s2[b2[0]] and e2[2] == s2[b2[2]]
    _note(f"{kind} turn_stop={turn_stop}: {n} seeds, max rel error vs oracle {rel:.2e}, "
          f"vs fused {np.max(np.abs(s2 - s1) / np.maximum(s1, 1e-9)):.2e}")
    c.close()


def test_two_kernel_chunks(rk, geo, ufield, orc_u):
    """More seeds than one 4 GiB trajectory chunk holds (about 55 900 at 6000 steps):
    every seed against the fused kernel, a sample against the oracle."""
    ev = synth.event_multi_turn(geo, ufield, 3)
    off, wid, dr = synth.pack_events([ev])
    c = rk.Context(0)
    c.upload_geometry(geo); c.upload_field(ufield); c.upload_hits(off, wid, dr)
    w = synth.make_windows([(0, 0, ev.truth_seeds[0], (0.3, 100.0, 10.0, 10.0, 10.0), (10, 10, 10, 8, 10))])
    n = 80000
    p = rk.make_scan_params(n_steps=6000, precision=32)
    s2 = np.zeros(n); b2 = np.zeros(1, np.int64); e2 = np.zeros(1)
    rk.rkn_scan_windows_two_kernel(c.ctx, p, w, s2, None, b2, e2)
    s1 = np.zeros(n); b1 = np.zeros(1, np.int64); e1 = np.zeros(1)
    rk.rkn_scan_windows(c.ctx, p, w, s1, None, b1, e1)
    np.testing.assert_allclose(s2, s1, rtol=2e-6, atol=1e-6)
    assert b2[0] == int(np.argmin(s2))
    g = np.sort(np.random.default_rng(9).choice(n, 96, replace=False))
    seeds = np.array([orc_u.window_seed(w[0], int(k)) for k in g])
    osc, _, _, _ = orc_u.scan_seeds(orc_u.params(n_steps=6000), off, wid, dr, np.zeros(g.size, np.int32), seeds)
    rel = pu.check_scores(s2[g], osc)
    _note(f"80000 seeds in two chunks: equal to the fused kernel to rounding, sample rel error {rel:.2e}")
    c.close()
