"""Pins of the oracle's adaptive step size (the error-controlled RKN that section 2.2
cites): the error estimate's order, the closed-form helix, the path length and step
bounds, the reduction to the fixed-step method when h_min = h_max, and the score
against the fixed 1 mm step."""
import numpy as np
import pytest

import oracle
from paper_1908_01949_amd import synth

KAPPA = 0.299792458


def _helix_at(seed, s, bz=1.0, q=-1.0, R0=500.0):
    th, z0, px, py, pz = seed
    pm = np.sqrt(px * px + py * py + pz * pz)
    t = np.array([px, py, pz]) / pm
    w = -KAPPA * q * bz / pm
    c0 = complex(R0 * np.cos(th), R0 * np.sin(th))
    xy = c0 + complex(t[0], t[1]) * (np.exp(1j * w * s) - 1) / (1j * w)
    return np.stack([xy.real, xy.imag, z0 + t[2] * s], -1)


def test_error_estimate_is_fourth_order(orc_u):
    x = np.array([500.0, 0.0, 10.0]); T = np.array([0.3, 0.9, 0.1]); T /= np.linalg.norm(T)
    lam = -KAPPA / 100.0
    errs = [orc_u.rkn_trial(lam, h, x, T)[2] for h in (8.0, 4.0, 2.0, 1.0)]
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(np.abs(ratios - 16.0) < 1.0), ratios
    # the trial step is the fixed-step formula
    xn, Tn, _ = orc_u.rkn_trial(lam, 1.0, x, T)
    xf, Tf = orc_u.rkn_step(lam, 1.0, x, T)
    assert np.array_equal(xn, xf) and np.array_equal(Tn, Tf)


def test_adaptive_trace_on_the_helix(orc_u):
    rng = np.random.default_rng(31)
    prm = orc_u.params(n_steps=6000)
    ap = oracle.OrcAdaptive(1e-5, 0.25, 4.0)
    for _ in range(6):
        th = rng.uniform(-np.pi, np.pi); a = th + rng.uniform(0.3, 1.2); pt = rng.uniform(85, 104)
        seed = np.array([th, rng.uniform(-200, 200), pt * np.cos(a), pt * np.sin(a), rng.uniform(-20, 20)])
        pts, arc, rej = orc_u.adaptive_trace(prm, ap, seed)
        steps = np.diff(arc)
        assert arc[-1] == pytest.approx(6000.0, abs=1e-9)
        assert np.all(steps[:-1] <= 4.0 + 1e-12) and np.all(steps[:-1] >= 0.25 - 1e-12)
        dev = np.linalg.norm(pts - _helix_at(seed, arc), axis=1)
        assert dev.max() < 1e-3, dev.max()
        assert steps.size < 2000          # far fewer than 6000 fixed steps


def test_adaptive_reduces_to_fixed_step(orc_u, orc_s, geo):
    """h_min = h_max = step: every trial is taken at the fixed step, so the chords and
    the score are the fixed-step method's, bit for bit."""
    for O, field in ((orc_u, synth.uniform_field()), (orc_s, synth.solenoid_field())):
        ev = synth.event_fixed_total(geo, field, 0, n_total=60, noise_frac=0.2) if O is orc_u else \
            synth.event_multi_turn(geo, field, 0)
        for ts in (0, 1):
            prm = O.params(n_steps=3000, turn_stop=ts)
            ap = oracle.OrcAdaptive(1e-12, 1.0, 1.0)
            E, nin, ns = O.score_adaptive(prm, ap, ev.truth_seeds[0], ev.wire_id, ev.drift)
            E0, nin0, _ = O.score(prm, ev.truth_seeds[0], ev.wire_id, ev.drift, mode=0)
            assert E == E0 and nin == nin0


def test_adaptive_score_close_to_fixed(geo, sfield, orc_s):
    ev = synth.event_multi_turn(geo, sfield, 1)
    prm = orc_s.params(n_steps=6000)
    ap = oracle.OrcAdaptive(1e-5, 0.25, 4.0)
    rng = np.random.default_rng(32)
    for s in [ev.truth_seeds[0]] + [ev.truth_seeds[0] + rng.normal(0, [0.005, 3, 0.5, 0.5, 0.5]) for _ in range(3)]:
        E, nin, ns = orc_s.score_adaptive(prm, ap, s, ev.wire_id, ev.drift)
        E0, nin0, _ = orc_s.score(prm, s, ev.wire_id, ev.drift, mode=1)
        # chords up to 4 mm: sagitta 4^2 / (8 R) < 0.006 mm on each distance
        assert abs(E - E0) <= 2e-3 * E0 and abs(nin - nin0) <= 1 and ns < 2000
