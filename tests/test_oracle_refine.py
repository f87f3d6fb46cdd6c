"""Pins of the oracle's refinement pieces: FP64 forward sensitivities of the inlier
residuals (against central finite differences), their consistency with the score of
Eq. 1, and Gauss-Newton convergence on noise-free events."""
import numpy as np
import pytest

from paper_1908_01949_amd import synth

SCALE = np.array([1.0, 100.0, 100.0, 100.0, 100.0])


def _case(geo, which):
    import oracle
    if which == "uniform":
        f = synth.uniform_field(1.0)
        ev = synth.event_multi_turn(geo, f, 1, sigma=0.0, noise_frac=0.0)
    else:
        f = synth.solenoid_field()
        ev = synth.event_fixed_total(geo, f, 0, n_total=120, noise_frac=0.0, sigma=0.0)
    return oracle.Oracle(geo, f), ev


@pytest.mark.parametrize("which,tol", [("uniform", 1e-6), ("solenoid", 1e-3)])
def test_jacobian_vs_finite_differences(geo, which, tol):
    """Central differences with h_k = 1e-6 max(|s_k|, scale_k) (the bilinear map's
    derivative jumps at cell edges, so the map case gets a looser bound)."""
    O, ev = _case(geo, which)
    prm = O.params(n_steps=6000)
    s0 = ev.truth_seeds[0] + np.array([0.002, 1.5, 0.4, -0.3, 0.5])
    m = O.inlier_mask(prm, s0, ev.wire_id, ev.drift)
    assert m.sum() > 50
    ok, r, J = O.residual_jacobian(prm, s0, ev.wire_id, ev.drift, m)
    assert ok
    for k in range(5):
        hk = 1e-6 * max(abs(s0[k]), SCALE[k])
        sp = s0.copy(); sp[k] += hk
        sm = s0.copy(); sm[k] -= hk
        _, rp, _ = O.residual_jacobian(prm, sp, ev.wire_id, ev.drift, m)
        _, rm, _ = O.residual_jacobian(prm, sm, ev.wire_id, ev.drift, m)
        fd = (rp - rm) / (2 * hk)
        sel = m.astype(bool)
        err = np.abs(J[sel, k] - fd[sel]).max()
        assert err <= tol * np.abs(fd[sel]).max(), (k, err)
    # non-inliers carry nothing
    assert np.all(J[~m.astype(bool)] == 0)


def test_residuals_consistent_with_score(geo):
    """On the inlier set Phi = E - (N - n_in) lambda (Eq. 1 split into in and out terms)."""
    O, ev = _case(geo, "uniform")
    prm = O.params(n_steps=6000)
    s0 = ev.truth_seeds[0] + np.array([0.01, 5.0, 1.0, -1.0, 1.0])
    m = O.inlier_mask(prm, s0, ev.wire_id, ev.drift)
    _, r, _ = O.residual_jacobian(prm, s0, ev.wire_id, ev.drift, m)
    E, n_in, _ = O.score(prm, s0, ev.wire_id, ev.drift)
    assert n_in == int(m.sum())
    phi = float((r[m.astype(bool)] ** 2).sum())
    assert phi == pytest.approx(E - (ev.wire_id.size - n_in) * prm.lambda_mm2, rel=1e-10)


@pytest.mark.parametrize("which,ztol", [("uniform", 1e-3), ("solenoid", 5e-3)])
def test_gauss_newton_converges_to_truth(geo, which, ztol):
    """Noise-free hits, a start in the basin: Phi falls fast and the seed reaches the truth."""
    O, ev = _case(geo, which)
    prm = O.params(n_steps=6000)
    s0 = ev.truth_seeds[0] + np.array([0.002, 1.5, 0.4, -0.3, 0.5])
    s, m, phi = O.gn_refine(prm, s0, ev.wire_id, ev.drift, scale=SCALE, iters=10)
    assert np.all(np.diff(phi) <= 0)
    assert phi[-1] < 1e-4 and phi[3] < 1e-2 * phi[0]
    err = s - ev.truth_seeds[0]
    assert abs(err[0]) * 500.0 < 1e-3 and abs(err[1]) < ztol
    assert np.all(np.abs(err[2:]) < 2e-3)
