"""Pins of the turn-partition parts of the oracle (sections 2.3 and 4.2) and of the
track-finding quality of Eqs. 2-3: the end of a turn partition and the neighbouring
partition's seed against the closed-form helix of a uniform field, the four score
paths against each other under the stop rule, the time reversal of the prediction in
the solenoid map, and the truth-labelled multi-turn events."""
import numpy as np
import pytest
from scipy.optimize import brentq

import oracle
from paper_1908_01949_amd import quality, synth

KAPPA = 0.299792458
R0 = 500.0


def _outward_seed(rng, pt=(85.0, 104.0), pz=(-20.0, 20.0)):
    th = rng.uniform(-np.pi, np.pi)
    a = th + rng.uniform(0.3, 1.2)      # direction with a positive radial component
    p_t = rng.uniform(*pt)
    return np.array([th, rng.uniform(-300, 300), p_t * np.cos(a), p_t * np.sin(a), rng.uniform(*pz)])


def _helix(seed, s, bz=1.0, q=-1.0):
    """Closed-form helix through the seed (uniform B_z), position at arc lengths s."""
    th, z0, px, py, pz = seed
    pm = np.sqrt(px * px + py * py + pz * pz)
    t = np.array([px, py, pz]) / pm
    w = -KAPPA * q * bz / pm                       # rotation rate of T_perp per unit arc
    c0 = complex(R0 * np.cos(th), R0 * np.sin(th))
    tp = complex(t[0], t[1])
    s = np.asarray(s, np.float64)
    xy = c0 + tp * (np.exp(1j * w * s) - 1) / (1j * w)
    return np.stack([xy.real, xy.imag, z0 + t[2] * s], -1)


def _exit_arc(seed):
    """Arc length of the first return of the closed-form helix to r = R0."""
    s = np.linspace(1e-3, 4000.0, 400001)
    r = np.hypot(*_helix(seed, s)[:, :2].T)
    k = np.nonzero(r < R0)[0][0]
    return brentq(lambda v: np.hypot(*_helix(seed, np.array([v]))[0, :2]) - R0, s[k - 1], s[k], xtol=1e-12)


@pytest.fixture(scope="module")
def orc_uni(geo, ufield):
    return oracle.Oracle(geo, ufield)


def test_turn_end_against_closed_form_helix(orc_uni):
    rng = np.random.default_rng(11)
    for _ in range(12):
        seed = _outward_seed(rng)
        s_exit = _exit_arc(seed)
        n_star = int(np.ceil(s_exit))               # first whole step inside r < R0
        if abs(s_exit - round(s_exit)) < 1e-6:
            continue
        prm = orc_uni.params(n_steps=6000, turn_stop=1)
        st = orc_uni.trace(prm, seed, np.array([n_star - 1, n_star, n_star + 1, 6000]))[0]
        ref = _helix(seed, np.array([n_star - 1.0, n_star]))
        np.testing.assert_allclose(st[:2, :3], ref, rtol=0, atol=1e-6)
        assert np.hypot(*st[0, :2]) >= R0 > np.hypot(*st[1, :2])
        # states beyond the end stay at the last one
        assert np.array_equal(st[2], st[1]) and np.array_equal(st[3], st[1])
        # without the stop rule the track goes on
        free = orc_uni.trace(orc_uni.params(n_steps=6000), seed, np.array([n_star + 1]))[0, 0]
        assert np.linalg.norm(free[:3] - st[1, :3]) > 0.5


@pytest.mark.parametrize("kind", ["uniform", "solenoid"])
def test_turn_stop_scores_agree(geo, ufield, sfield, kind):
    """Brute force, band-pruned and block-culled scores (the kernel's rule, modelled in
    tests/cull_model.py) are identical under the stop rule, and equal the score of the
    same track cut to its own step count."""
    from tests.cull_model import blocked_work
    field = ufield if kind == "uniform" else sfield
    O = oracle.Oracle(geo, field)
    ev = synth.event_multi_turn(geo, field, 1)
    stop = O.params(n_steps=6000, turn_stop=1)
    rng = np.random.default_rng(12)
    seeds = [ev.truth_seeds[0]] + [ev.truth_seeds[0] + rng.normal(0, [0.01, 5, 1, 1, 1]) for _ in range(3)]
    for s in seeds:
        E0, n0, _ = O.score(stop, s, ev.wire_id, ev.drift, mode=0)
        E1, n1, _ = O.score(stop, s, ev.wire_id, ev.drift, mode=1)
        for B in (4, 6, 8):
            _, _, Eb = blocked_work(O, stop, s, geo, ev.wire_id, ev.drift, B, want_score=True)
            assert Eb == E0
        assert E1 == E0 and n1 == n0
        # the step count of the turn: the first state inside r < R0
        tr = O.trace(O.params(n_steps=6000), s, np.arange(6001))[0]
        inside = np.nonzero(np.hypot(tr[1:, 0], tr[1:, 1]) < R0)[0]
        n_star = int(inside[0]) + 1
        Ec, nc, _ = O.score(O.params(n_steps=n_star), s, ev.wire_id, ev.drift, mode=0)
        assert Ec == E0 and nc == n0


def test_neighbour_seed_closed_form_uniform(orc_uni):
    """In a uniform field the track returns to the same (x, y) after each turn: the
    next entrance seed is (theta0, z0 + 2 pi R pz / pT, p) and the previous one has
    z0 - 2 pi R pz / pT."""
    rng = np.random.default_rng(13)
    prm = orc_uni.params(n_steps=6000)
    for _ in range(10):
        seed = _outward_seed(rng, pz=(-25.0, 25.0))
        pt = np.hypot(seed[2], seed[3])
        pitch = 2 * np.pi * (pt / KAPPA) * seed[4] / pt
        for d in (1, -1):
            nb = orc_uni.neighbour_seed(prm, seed, d)
            assert nb is not None
            assert abs(np.angle(np.exp(1j * (nb[0] - seed[0])))) < 1e-9
            assert nb[1] == pytest.approx(seed[1] + d * pitch, abs=1e-5)
            np.testing.assert_allclose(nb[2:], seed[2:], rtol=0, atol=1e-7)


def test_neighbour_seed_time_reversal_solenoid(geo, sfield):
    """Next then previous returns the starting seed in the (r, z) map (the RKN map is
    time-reversible to its truncation error), and a track that never re-enters the
    seed cylinder within the step limit gives no prediction."""
    O = oracle.Oracle(geo, sfield)
    prm = O.params(n_steps=6000)
    rng = np.random.default_rng(14)
    for _ in range(6):
        seed = _outward_seed(rng)
        nx = O.neighbour_seed(prm, seed, 1)
        back = O.neighbour_seed(prm, nx, -1)
        assert abs(np.angle(np.exp(1j * (back[0] - seed[0])))) < 1e-7
        np.testing.assert_allclose(back[1:], seed[1:], rtol=0, atol=1e-5)
    assert O.neighbour_seed(prm, seed, 1, max_steps=50) is None


@pytest.mark.parametrize("kind", ["uniform", "solenoid"])
def test_truth_turns_and_classification(geo, ufield, sfield, kind):
    """Truth labels of multi-turn events: every true hit has a pass index, the passes
    follow the predicted neighbour seeds, and the stop-ruled truth seed of each pass
    classifies all of its hits."""
    field = ufield if kind == "uniform" else sfield
    O = oracle.Oracle(geo, field)
    stop = O.params(n_steps=6000, turn_stop=1, lambda_mm2=4.0)
    for sd in (0, 2):
        ev = synth.event_multi_turn(geo, field, sd)
        t = ev.turn_of
        assert np.all((t >= 0) == ~ev.is_noise) and t.max() >= 1
        s = ev.truth_seeds[0]
        for k in range(t.max() + 1):
            m = O.inlier_mask(stop, s, ev.wire_id, ev.drift).astype(bool)
            assert np.all(m[t == k]), (sd, k)
            s = O.neighbour_seed(O.params(n_steps=6000), s, 1)


def test_quality_eqs_2_3_hand_example():
    true = np.array([0, 0, 0, 0, 1, 1, 1, -1, 2])
    found = np.array([0, 0, 0, 1, 1, 1, -1, 0, -1])
    q = quality.turn_quality(true, found)
    assert q[0] == dict(n_hits=4, eps=0.75, pi=1.0, found=0)          # the noise hit is not in the sum
    assert q[1]["eps"] == pytest.approx(2 / 3) and q[1]["pi"] == pytest.approx(2 / 3) and q[1]["found"] == 1
    assert q[2]["eps"] == 0.0 and np.isnan(q[2]["pi"]) and q[2]["found"] == -1
    # two found partitions owned by one true partition: the larger share counts
    q = quality.turn_quality(np.array([0, 0, 0, 1]), np.array([0, 1, 1, -1]))
    assert q[0]["found"] == 1 and q[0]["eps"] == pytest.approx(2 / 3) and q[1]["eps"] == 0.0


def test_loop_defaults_follow_the_paper():
    """The turn loop's stop rule and the two-direction cut use the paper's numbers, and
    the window around a predicted seed spans at least the paper's resolution of the
    predicted (z0, pz0)."""
    import json
    import os
    from paper_1908_01949_amd import rknscan
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))
    tp = rknscan.make_turn_params()
    assert tp.min_hits == g["stop_unclassified_hits"]["value"]
    assert tp.half_width[1] >= g["turn_seed_resolution_z0_mm"]["value"]
    assert tp.half_width[4] >= g["turn_seed_resolution_pz0_MeV"]["value"]
    import inspect
    import bench
    assert inspect.signature(bench.bidirectional_leg).parameters["n_c_min"].default == g["common_hits_cut"]["value"]


@pytest.mark.parametrize("kind", ["uniform", "solenoid"])
def test_time_reversed_track_retraces_the_curve(geo, ufield, sfield, kind):
    """The reading of the exit-side scan: a state reversed in direction and propagated
    with the opposite charge retraces the same curve back to the seed point (the RKN map
    is time-reversible to its truncation error)."""
    field = ufield if kind == "uniform" else sfield
    O = oracle.Oracle(geo, field)
    rng = np.random.default_rng(15)
    for _ in range(4):
        seed = _outward_seed(rng)
        ok, x0, T0, lam = O.seed_state(O.params(), seed)
        x, T = x0.copy(), T0.copy()
        for _ in range(900):
            x, T = O.rkn_step(lam, 1.0, x, T)
        xr, Tr = x.copy(), -T
        for _ in range(900):
            xr, Tr = O.rkn_step(-lam, 1.0, xr, Tr)
        assert np.linalg.norm(xr - x0) < 1e-6, np.linalg.norm(xr - x0)
        assert np.linalg.norm(-Tr - T0) < 1e-9
