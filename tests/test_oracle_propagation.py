"""Pins of the oracle's field, seed state and RKN propagation (CPU only).

Each test checks the oracle against something other than itself: the closed-form
helix, the theoretical order of the Runge-Kutta-Nystrom formula, invariants of the
exact dynamics (|p| and Busch's canonical angular momentum), and exactness
properties of bilinear interpolation.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_1908_01949_amd import synth

KAPPA = 0.299792458
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def helix_closed_form(seed, s, q=-1.0, B=1.0, R0=500.0):
    """Exact solution of dT/ds = (kappa q/|p|) T x B z^ from the seed point (written out here)."""
    x0 = np.array([R0 * math.cos(seed[0]), R0 * math.sin(seed[0]), seed[1]])
    pm = np.linalg.norm(seed[2:])
    t0 = np.asarray(seed[2:]) / pm
    a = KAPPA * q * B / pm
    sa, ca = math.sin(a * s), math.cos(a * s)
    x = np.array([x0[0] + (t0[0] * sa + t0[1] * (1 - ca)) / a,
                  x0[1] + (t0[1] * sa + t0[0] * (ca - 1)) / a,
                  x0[2] + t0[2] * s])
    t = np.array([t0[0] * ca + t0[1] * sa, t0[1] * ca - t0[0] * sa, t0[2]])
    return x, t


def _seed(p=104.97, pz=15.0, theta=0.0, z=-300.0):
    pt = math.sqrt(p * p - pz * pz)
    return np.array([theta, z, -pt * math.sin(theta + 0.3), pt * math.cos(theta + 0.3), pz])


def test_golden_constants_used_by_generator():
    g = json.load(open(GOLDEN))
    assert synth.R0_SEED == g["seed_radius_mm"]["value"]
    assert synth.P_SIGNAL == g["signal_momentum_MeV"]["value"]
    assert synth.make_geometry().n_layers == g["n_sense_layers"]["value"]


def test_seed_state(orc_u):
    prm = orc_u.params()
    ok, x, T, lam = orc_u.seed_state(prm, [0.7, 12.5, 3.0, 4.0, 12.0])
    assert ok
    np.testing.assert_allclose(x, [500 * math.cos(0.7), 500 * math.sin(0.7), 12.5], rtol=0, atol=1e-12)
    np.testing.assert_allclose(T, np.array([3.0, 4.0, 12.0]) / 13.0, rtol=0, atol=1e-15)
    assert lam == pytest.approx(KAPPA * -1.0 / 13.0, rel=1e-15)
    ok, *_ = orc_u.seed_state(prm, [0.0, 0.0, 1e-4, 0.0, 0.0])
    assert not ok


def test_helix_three_turns(orc_u):
    """|oracle - closed-form helix| <= 1e-7 mm after three turns at h = 1 mm."""
    seed = _seed()
    n = 6600
    prm = orc_u.params(step_mm=1.0, n_steps=n)
    st = orc_u.trace(prm, seed, [0, 1, 100, n])[0]
    for k, s in enumerate([0, 1, 100, n]):
        x, t = helix_closed_form(seed, float(s))
        assert np.linalg.norm(st[k, :3] - x) <= 1e-7
        assert np.linalg.norm(st[k, 3:] - t) <= 1e-10


def test_order_four(orc_u):
    """Halving h divides the global error by 2^4 (observed order 4 +- 0.1)."""
    seed = _seed()
    errs = []
    for h in (4.0, 2.0, 1.0):
        n = int(round(6600 / h))
        prm = orc_u.params(step_mm=h, n_steps=n)
        st = orc_u.trace(prm, seed, [n])[0, 0]
        errs.append(np.linalg.norm(st[:3] - helix_closed_form(seed, n * h)[0]))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(o - 4.0) < 0.1 for o in orders), orders


def test_signal_radius(orc_u):
    """p = 104.97 MeV/c at 1 T gives R = p / (kappa B) = 350.142 mm and a 2200 mm turn."""
    seed = np.array([0.0, 0.0, 0.0, 104.97, 0.0])
    prm = orc_u.params(step_mm=1.0)
    n = np.arange(0, 2200, 50, dtype=np.int32)
    st = orc_u.trace(prm, seed, n)[0]
    xy = st[:, :2]
    # fit a circle through the sampled points (algebraic least squares)
    A = np.c_[2 * xy, np.ones(len(xy))]
    sol = np.linalg.lstsq(A, (xy ** 2).sum(1), rcond=None)[0]
    R = math.sqrt(sol[2] + sol[0] ** 2 + sol[1] ** 2)
    assert R == pytest.approx(104.97 / KAPPA, abs=1e-6)
    assert 2 * math.pi * 104.97 / KAPPA == pytest.approx(2200.0, abs=0.1)


def test_electron_turns_counter_clockwise(orc_u):
    """q = -1 in +z field: T rotates counter-clockwise seen from +z (T x dT/ds along +z)."""
    seed = np.array([0.0, 0.0, 0.0, 100.0, 10.0])
    prm = orc_u.params(step_mm=1.0)
    st = orc_u.trace(prm, seed, [0, 1])[0]
    t0, t1 = st[0, 3:], st[1, 3:]
    assert np.cross(t0, t1)[2] > 0


def test_momentum_magnitude_conserved(orc_s):
    """The magnetic force does no work: |T| stays 1 in the solenoid map to RKN truncation."""
    seed = _seed(pz=12.0, z=-200.0)
    prm = orc_s.params(step_mm=1.0)
    st = orc_s.trace(prm, seed, np.arange(0, 6001, 1000, dtype=np.int32))[0]
    assert np.max(np.abs(np.linalg.norm(st[:, 3:], axis=1) - 1.0)) <= 1e-11


def test_busch_invariant_linear_bottle(geo):
    """Busch: L = |p|(x T_y - y T_x) + kappa q r A_phi is conserved in an axisymmetric field.

    B_z = 1 + b z, B_r = -b r / 2 is divergence- and curl-free with A_phi = r (1 + b z)/2,
    and bilinear interpolation reproduces it exactly, so the oracle's grid path must
    conserve L to the RKN truncation error (relative <= 1e-10 over 6000 steps).
    """
    import oracle
    b = 2.0 ** -14                      # dyadic so that grid nodes are exact in float32
    f = synth.linear_bottle_field(b)
    O = oracle.Oracle(geo, f)
    seed = _seed(pz=8.0, z=-100.0)
    pm = np.linalg.norm(seed[2:])
    prm = O.params(step_mm=1.0)
    st = O.trace(prm, seed, np.arange(0, 6001, 500, dtype=np.int32))[0]
    assert np.all(np.abs(st[:, 2]) < 1000) and np.all(np.hypot(st[:, 0], st[:, 1]) < 900)
    x, y, z = st[:, 0], st[:, 1], st[:, 2]
    r2 = x * x + y * y
    L = pm * (x * st[:, 4] - y * st[:, 3]) + KAPPA * -1.0 * r2 * (1 + b * z) / 2
    assert np.max(np.abs(L - L[0])) <= 1e-10 * abs(L[0]), (L - L[0])
    # and the field really varies along the track (the test is not vacuous)
    Bz = np.array([O.field_eval(s[:3])[2] for s in st])
    assert np.ptp(Bz) > 0.01


def test_field_grid_nodes_and_linear_exactness(geo, sfield):
    import oracle
    O = oracle.Oracle(geo, sfield)
    rn = np.linspace(0, 900, 65); zn = np.linspace(-1000, 1000, 129)
    for (i, j) in [(0, 64), (10, 20), (64, 128), (33, 77)]:
        B = O.field_eval([rn[i], 0.0, zn[j]])
        assert B[2] == float(sfield.bz_grid[j, i])
        assert B[0] == float(sfield.br_grid[j, i])
    # linear field reproduced exactly at arbitrary points inside the grid
    b = 2.0 ** -12
    Ol = oracle.Oracle(geo, synth.linear_bottle_field(b))
    rng = np.random.default_rng(1)
    for _ in range(50):
        r = rng.uniform(1, 899); ph = rng.uniform(0, 2 * np.pi); z = rng.uniform(-999, 999)
        B = Ol.field_eval([r * math.cos(ph), r * math.sin(ph), z])
        assert B[2] == pytest.approx(1 + b * z, abs=1e-13)
        assert math.hypot(B[0], B[1]) == pytest.approx(b * r / 2, abs=1e-13)
        # B_r points inward (B_r < 0) for b > 0
        assert B[0] * math.cos(ph) + B[1] * math.sin(ph) < 0
    # clamped to the edge outside the grid
    assert Ol.field_eval([0.0, 0.0, 5000.0])[2] == pytest.approx(1 + b * 1000, abs=1e-12)
    assert Ol.field_eval([0.0, 0.0, 0.0])[0] == 0.0


def test_constant_grid_equals_uniform(geo, orc_u):
    """A grid holding B_z = 1 everywhere reproduces the uniform path to rounding."""
    import oracle
    O = oracle.Oracle(geo, synth.constant_grid_field(1.0))
    seed = _seed()
    prm = O.params(step_mm=1.0)
    a = O.trace(prm, seed, [2000])[0, 0]
    b = orc_u.trace(prm, seed, [2000])[0, 0]
    assert np.max(np.abs(a - b)) <= 1e-9


def test_field_rotation_invariant(orc_s):
    rng = np.random.default_rng(3)
    for _ in range(20):
        r = rng.uniform(0, 880); z = rng.uniform(-950, 950)
        ph1, ph2 = rng.uniform(0, 2 * np.pi, 2)
        B1 = orc_s.field_eval([r * math.cos(ph1), r * math.sin(ph1), z])
        B2 = orc_s.field_eval([r * math.cos(ph2), r * math.sin(ph2), z])
        assert np.linalg.norm(B1) == pytest.approx(np.linalg.norm(B2), rel=1e-12)


@pytest.mark.parametrize("fieldname", ["solenoid", "bottle"])
def test_last_stage_point_meets_next_start(geo, sfield, fieldname):
    """The last stage of a step evaluates the field at p_n + h t_n + h^2/2 k3; over three
    turns that point stays within 1e-5 mm of the next step's start p_{n+1} (the formula
    predicts h^3 |lam B|^2 / 6 ~ 1e-6 mm), below the FP32 spacing of positions there
    (3e-5 mm at 500 mm), and the map's field differs between the two points by less than
    1e-8 relative, below FP32 rounding: the reason an FP32 propagation may take the one
    field for the other."""
    import oracle
    field = sfield if fieldname == "solenoid" else synth.linear_bottle_field(2.0 ** -11)
    O = oracle.Oracle(geo, field)
    prm = O.params(n_steps=6000)
    ok, x, T, lam = O.seed_state(prm, _seed(pz=8.0))
    assert ok
    h = 1.0
    worst_d = worst_b = 0.0
    for n in range(6000):
        k1 = lam * np.cross(T, O.field_eval(x))
        xm = x + 0.5 * h * T + 0.125 * h * h * k1
        Bm = O.field_eval(xm)
        k2 = lam * np.cross(T + 0.5 * h * k1, Bm)
        k3 = lam * np.cross(T + 0.5 * h * k2, Bm)
        x4 = x + h * T + 0.5 * h * h * k3
        B4 = O.field_eval(x4)
        x, T = O.rkn_step(lam, h, x, T)
        worst_d = max(worst_d, float(np.linalg.norm(x4 - x)))
        worst_b = max(worst_b, float(np.linalg.norm(B4 - O.field_eval(x)) / np.linalg.norm(B4)))
    assert 1e-8 < worst_d < 1e-5
    assert worst_b < 1e-8
