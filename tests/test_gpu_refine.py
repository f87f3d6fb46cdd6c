"""GPU parity of the differentiated refinement: checkpointed FP32 forward pass, adjoint
backward sweep (gradient, J^T J, J^T r) and Gauss-Newton, each against the oracle's
FP64 forward sensitivities on the same seeded events.

Tolerances, from the arithmetic: the GPU propagates in FP32 with compensated sums,
so positions carry ~1e-4 mm of rounding over 6000 steps and a chord-wire distance
another eps32 * |p - m| ~ 6e-5 mm; residuals are compared at 1e-3 mm (1/200 of the
0.2 mm drift resolution). The tangent maps are FP32 per step and accumulated in FP64;
N = 6000 steps of relative rounding 6e-8 bound the relative error of a derivative by
N * u * (a few) ~ 1e-3, the bound used for J^T c and J^T J (Frobenius, in the scaled
variables D = diag(1, 100, 100, 100, 100) that make the columns comparable).

Where that bound is reached: the rows of J carry the tangent maps' FP32 rounding
accumulated along the path, which grows linearly with the steps a hit lies behind
(the phase of a helix is linear in its path length): N u = 6000 x 6e-8 = 3.6e-4 for
the rows of the last hits of a 6000-step multi-turn track, and 2 N u = 7.2e-4 for
J^T J. Measured: J^T c over hits passing >= 0.5 mm from their wire 3.4e-4, J^T J
8.3e-4 on the uniform multi-turn events without the turn stop; with the turn stop
(about a third of the steps) and on the single-turn solenoid events, 1e-5 to 4e-4.
The 1e-3 bound is 2.8 N u."""
import numpy as np
import pytest

from paper_1908_01949_amd import synth

pytestmark = pytest.mark.gpu

SCALE = np.array([1.0, 100.0, 100.0, 100.0, 100.0])
R_ABS = 1e-3        # mm, residual agreement
DER_REL = 1e-3      # relative derivative agreement (see module docstring)
N_STEPS = 6000


@pytest.fixture(scope="module")
def rk():
    from paper_1908_01949_amd import rknscan
    rknscan.load_library()
    return rknscan


def _events(geo, field, kind):
    if kind == "uniform":
        return [synth.event_multi_turn(geo, field, s, sigma=0.2, noise_frac=0.3) for s in (3, 4, 5)]
    return [synth.event_fixed_total(geo, field, s, n_total=150, noise_frac=0.2, sigma=0.2) for s in (1, 2, 3)]


def _seeds(evs, per_event, rng):
    """Seeds grouped by event: truth plus a scaled perturbation inside the basin."""
    amp = np.array([0.002, 1.5, 0.4, 0.4, 0.5])
    ev, s5 = [], []
    for e, x in enumerate(evs):
        for _ in range(per_event):
            ev.append(e)
            s5.append(x.truth_seeds[0] + amp * rng.uniform(-1.0, 1.0, 5))
    return np.array(ev, np.int32), np.array(s5)


def _setup(rk, geo, field, kind, per_event=4, seed=0, turn_stop=0):
    evs = _events(geo, field, kind)
    off, wid, dr = synth.pack_events(evs)
    c = rk.Context(0)
    c.upload_geometry(geo); c.upload_field(field); c.upload_hits(off, wid, dr)
    ev, s5 = _seeds(evs, per_event, np.random.default_rng(seed))
    sp = rk.make_scan_params(n_steps=N_STEPS, precision=32, turn_stop=turn_stop)
    rk.rkn_refine_setup(c.ctx, sp, ev, s5, ckpt_every=64)
    H = int(np.diff(off).max())
    return c, evs, off, ev, s5, H


def _orc(geo, field):
    import oracle
    return oracle.Oracle(geo, field)


def _forward(rk, c, n, H, seeds=None):
    resid = np.zeros((n, H), np.float32)
    phi = np.zeros(n)
    rk.rkn_residuals_fwd(c.ctx, seeds, resid, phi)
    return resid, phi


@pytest.mark.parametrize("kind", ["uniform", "solenoid"])
def test_residuals_match_oracle(rk, geo, ufield, sfield, kind):
    field = ufield if kind == "uniform" else sfield
    O = _orc(geo, field)
    prm = O.params(n_steps=N_STEPS)
    c, evs, off, ev, s5, H = _setup(rk, geo, field, kind)
    n = ev.size
    resid, phi = _forward(rk, c, n, H)
    worst, flips = 0.0, 0
    for p in range(n):
        x = evs[ev[p]]
        nh = x.wire_id.size
        assert np.all(np.isnan(resid[p, nh:]))
        gmask = ~np.isnan(resid[p, :nh])
        om = O.inlier_mask(prm, s5[p], x.wire_id, x.drift).astype(bool)
        _, r_all, _ = O.residual_jacobian(prm, s5[p], x.wire_id, x.drift, np.ones(nh, np.uint8))
        # the classification may differ only where |r| is within rounding of sqrt(lambda)
        diff = gmask != om
        flips += int(diff.sum())
        assert np.all(np.abs(np.abs(r_all[diff]) - np.sqrt(prm.lambda_mm2)) < R_ABS), p
        both = gmask & om
        err = np.abs(resid[p, :nh][both] - r_all[both])
        worst = max(worst, float(err.max(initial=0.0)))
        assert err.max(initial=0.0) < R_ABS, (p, err.max())
        # Phi is the FP64 sum of the squared inlier residuals
        phi_o = float((r_all[gmask] ** 2).sum())
        assert abs(phi[p] - phi_o) <= R_ABS * (2.0 * np.abs(r_all[gmask]).sum() + gmask.sum() * R_ABS), p
        assert phi[p] == pytest.approx(float((resid[p, :nh][gmask].astype(np.float64) ** 2).sum()), rel=1e-6)
    print(f"{kind}: {n} seeds, max |dr| {worst:.2e} mm, classification flips {flips}", flush=True)
    c.close()


@pytest.mark.parametrize("kind,turn_stop", [("uniform", 0), ("solenoid", 0), ("uniform", 1), ("solenoid", 1)])
def test_adjoint_matches_oracle_sensitivities(rk, geo, ufield, sfield, kind, turn_stop):
    """With turn_stop the forward pass freezes each track at the end of its turn
    partition and the backward sweep recomputes the same frozen steps (identity step
    Jacobians); the oracle stops its sensitivities there too."""
    field = ufield if kind == "uniform" else sfield
    O = _orc(geo, field)
    prm = O.params(n_steps=N_STEPS, turn_stop=turn_stop)
    c, evs, off, ev, s5, H = _setup(rk, geo, field, kind, seed=1, turn_stop=turn_stop)
    n = ev.size
    resid, phi = _forward(rk, c, n, H)
    g = np.zeros((n, 5)); A = np.zeros((n, 5, 5)); jtr = np.zeros((n, 5))
    rk.rkn_adjoint_bwd(c.ctx, None, g, A, jtr)
    np.testing.assert_allclose(jtr, 0.5 * g, rtol=1e-15, atol=0)
    # an arbitrary upstream gradient: the adjoint gives J^T cvec
    rng = np.random.default_rng(7)
    cvec = rng.standard_normal((n, H)).astype(np.float32)
    gc = np.zeros((n, 5))
    rk.rkn_adjoint_bwd(c.ctx, cvec, gc, None, None)
    # the same with the upstream gradient kept only on hits passing >= 0.5 mm from
    # their wire: J^T c over rows whose closest-approach direction is well conditioned
    dfar = np.zeros((n, H), bool)
    for p in range(n):
        x = evs[ev[p]]
        nh = x.wire_id.size
        dfar[p, :nh] = ~np.isnan(resid[p, :nh]) & (resid[p, :nh] + x.drift >= 0.5)
    cfar = np.where(dfar, cvec, 0.0).astype(np.float32)
    gfar = np.zeros((n, 5))
    rk.rkn_adjoint_bwd(c.ctx, cfar, gfar, None, None)
    werr_a = werr_c = werr_g = werr_f = 0.0
    for p in range(n):
        x = evs[ev[p]]
        nh = x.wire_id.size
        gm = (~np.isnan(resid[p, :nh])).astype(np.uint8)
        dmin = float(np.min(resid[p, :nh][gm.astype(bool)] + x.drift[gm.astype(bool)], initial=np.inf))
        ok, r, J = O.residual_jacobian(prm, s5[p], x.wire_id, x.drift, gm)
        assert ok
        JD = J * SCALE
        Ao = JD.T @ JD
        Ag = A[p] * np.outer(SCALE, SCALE)
        ea = np.linalg.norm(Ag - Ao) / np.linalg.norm(Ao)
        co = JD.T @ np.where(gm.astype(bool), cvec[p, :nh], 0.0)
        ec = np.linalg.norm(gc[p] * SCALE - co) / (np.linalg.norm(JD) * np.linalg.norm(cvec[p, :nh][gm.astype(bool)]))
        fm = dfar[p, :nh]
        if fm.any():
            cf = np.where(fm, cvec[p, :nh], 0.0)
            ef = np.linalg.norm(gfar[p] * SCALE - JD.T @ cf) / (np.linalg.norm(JD[fm]) * np.linalg.norm(cf[fm]))
            werr_f = max(werr_f, ef)
        # gradient of Phi: residual differences (<= R_ABS) enter through J^T
        go = 2.0 * JD.T @ np.where(gm.astype(bool), r, 0.0)
        tol_g = DER_REL * np.linalg.norm(go) + 2.0 * np.linalg.norm(JD) * R_ABS * np.sqrt(gm.sum())
        eg = np.linalg.norm(g[p] * SCALE - go)
        werr_a, werr_c, werr_g = max(werr_a, ea), max(werr_c, ec), max(werr_g, eg / tol_g)
        assert ea < DER_REL, (p, ea, dmin)
        assert ec < DER_REL, (p, ec)
        assert eg < tol_g, (p, eg, tol_g)
    # rounding along the path, not ill-conditioned small-distance rows, sets the error
    assert werr_f < DER_REL
    print(f"{kind} turn_stop={turn_stop}: J^T J rel {werr_a:.2e}, J^T c rel {werr_c:.2e}, J^T c over hits with "
          f"D >= 0.5 mm rel {werr_f:.2e}, grad err/tol {werr_g:.2e}", flush=True)
    c.close()


@pytest.mark.parametrize("kind", ["uniform", "solenoid"])
def test_adjoint_gradient_matches_gpu_finite_differences(rk, geo, ufield, sfield, kind):
    """Self-consistency of the GPU pair: grad . v against a central difference of the
    GPU's own Phi along v. Single-turn events, so that every hit has one closest
    pass and Phi is smooth along v; the step moves the seed by ~0.05 mm (Phi's FP32
    noise enters through 2 sum|r| times the ~1e-4 mm FP32 residual noise)."""
    field = ufield if kind == "uniform" else sfield
    evs = [synth.event_single_turn(geo, field, s) for s in (1, 2, 3)]
    off, wid, dr = synth.pack_events(evs)
    c = rk.Context(0)
    c.upload_geometry(geo); c.upload_field(field); c.upload_hits(off, wid, dr)
    # D = |closest-approach vector| is not differentiable at D = 0: the seeds are chosen
    # beforehand, by the oracle's distances, among candidates around the truth, so that
    # every inlier of each stays >= 0.15 mm from its wire (the stencil below moves the
    # trajectory by at most ~0.05 mm)
    O = _orc(geo, field)
    prm = O.params(n_steps=2000)
    cev, cs5 = _seeds(evs, 16, np.random.default_rng(2))
    keep = []
    for q in range(cev.size):
        if sum(1 for k in keep if cev[k] == cev[q]) == 6:
            continue                      # at most 6 seeds per event
        x = evs[cev[q]]
        D = np.sqrt(O.doca2(prm, cs5[q], x.wire_id))
        inl = (D - x.drift) ** 2 < prm.lambda_mm2
        if inl.any() and D[inl].min() >= 0.15:
            keep.append(q)
    keep = np.array(keep, int)
    assert keep.size >= 12, keep.size
    ev, s5 = cev[keep], cs5[keep]
    rk.rkn_refine_setup(c.ctx, rk.make_scan_params(n_steps=2000), ev, s5)
    n, H = ev.size, int(np.diff(off).max())
    resid, _ = _forward(rk, c, n, H)
    g = np.zeros((n, 5))
    rk.rkn_adjoint_bwd(c.ctx, None, g, None, None)
    rng = np.random.default_rng(3)
    v = rng.standard_normal((n, 5)) / SCALE
    v *= 0.05 / np.abs(v * np.array([500.0, 1.0, 500.0, 500.0, 500.0])).max(axis=1, keepdims=True)
    _, pp = _forward(rk, c, n, H, s5 + v)
    _, pm = _forward(rk, c, n, H, s5 - v)
    fd = (pp - pm) / 2.0
    an = (g * v).sum(axis=1)
    noise = 2.0 * np.nansum(np.abs(resid), axis=1) * 1e-4
    tol = 2e-2 * np.abs(an) + noise
    err = np.abs(fd - an)
    print(f"{kind}: {n} seeds chosen from {cev.size}; FD vs adjoint worst err/tol {np.max(err / tol):.2e}, "
          f"worst rel {np.max(err / np.abs(an)):.2e}", flush=True)
    assert np.all(err < tol), (err, tol)
    c.close()


@pytest.mark.parametrize("kind", ["uniform", "solenoid"])
def test_gauss_newton_matches_oracle(rk, geo, ufield, sfield, kind):
    field = ufield if kind == "uniform" else sfield
    O = _orc(geo, field)
    prm = O.params(n_steps=N_STEPS)
    c, evs, off, ev, s5, H = _setup(rk, geo, field, kind, per_event=3, seed=4)
    n, iters = ev.size, 8
    out = np.zeros((n, 5)); phi = np.zeros((n, iters + 1))
    rk.rkn_gn_refine(c.ctx, iters, SCALE, out, phi)
    assert np.all(np.diff(phi, axis=1) <= 0)
    for p in range(n):
        x = evs[ev[p]]
        so, mo, phio = O.gn_refine(prm, s5[p], x.wire_id, x.drift, scale=SCALE, iters=iters)
        assert phi[p, 0] == pytest.approx(phio[0], rel=1e-3, abs=1e-3)
        # the GPU's minimum is as good as the oracle's: the oracle's Phi at the GPU seed
        ok, r, _ = O.residual_jacobian(prm, out[p], x.wire_id, x.drift, mo)
        assert ok
        phi_at_gpu = float((r[mo.astype(bool)] ** 2).sum())
        assert phi_at_gpu <= phio[-1] * (1 + 1e-3) + 1e-3, (p, phi_at_gpu, phio[-1])
        assert phi[p, -1] <= phio[-1] * (1 + 1e-3) + 1e-2, (p, phi[p, -1], phio[-1])
        # and it converged: at least a factor 10 below the start when the start was off
        if phio[0] > 10.0 * phio[-1]:
            assert phi[p, -1] < 0.2 * phi[p, 0]
    print(f"{kind}: GN Phi start {phi[:, 0].mean():.3g} -> {phi[:, -1].mean():.3g}", flush=True)
    # a second call starts again from the setup seeds: identical results
    out2 = np.zeros((n, 5)); phi2 = np.zeros((n, iters + 1))
    rk.rkn_gn_refine(c.ctx, iters, SCALE, out2, phi2)
    assert np.array_equal(out, out2) and np.array_equal(phi, phi2)
    c.close()


def test_refine_argument_and_state_errors(rk, geo, ufield):
    c = rk.Context(0)
    c.upload_geometry(geo); c.upload_field(ufield)
    evs = _events(geo, ufield, "uniform")[:2]
    off, wid, dr = synth.pack_events(evs)
    c.upload_hits(off, wid, dr)
    s5 = np.array([e.truth_seeds[0] for e in evs])
    with pytest.raises(rk.RknError) as e:
        rk.rkn_residuals_fwd(c.ctx, None, None, None)
    assert e.value.status == rk.RKN_E_STATE
    with pytest.raises(rk.RknError) as e:
        rk.rkn_refine_setup(c.ctx, rk.make_scan_params(n_steps=100, precision=64), np.array([0, 1], np.int32), s5)
    assert e.value.status == rk.RKN_E_ARG
    with pytest.raises(rk.RknError) as e:
        rk.rkn_refine_setup(c.ctx, rk.make_scan_params(n_steps=100), np.array([1, 0], np.int32), s5)
    assert e.value.status == rk.RKN_E_ARG
    with pytest.raises(rk.RknError) as e:
        rk.rkn_refine_setup(c.ctx, rk.make_scan_params(n_steps=100), np.array([0, 1], np.int32), s5, ckpt_every=12)
    assert e.value.status == rk.RKN_E_ARG
    rk.rkn_refine_setup(c.ctx, rk.make_scan_params(n_steps=100), np.array([0, 1], np.int32), s5)
    rk.rkn_residuals_fwd(c.ctx, None, None, np.zeros(2))
    c.upload_hits(off, wid, dr)      # new hits invalidate the refinement state
    with pytest.raises(rk.RknError) as e:
        rk.rkn_adjoint_bwd(c.ctx, None, np.zeros((2, 5)), None, None)
    assert e.value.status == rk.RKN_E_STATE
    c.close()


def test_batch_survives_refine_and_larger_eager_scans(rk, geo, sfield):
    """The captured batch graphs keep private scan scratch: refinement and eager scans
    that need more scratch do not disturb a planned batch."""
    evs = synth.events_batch(geo, sfield, 4, seed=5)
    off, wid, dr = synth.pack_events(evs)
    c = rk.Context(0)
    c.upload_geometry(geo); c.upload_field(sfield); c.upload_hits(off, wid, dr)
    hp = rk.make_hough_params(b_ref=sfield.b_ref, max_cand=2, count=(2, 2, 2, 2, 2), count_max=2, max_seeds_window=32)
    rk.rkn_batch_plan(c.ctx, hp, rk.make_scan_params(n_steps=800, precision=32))
    ne = len(evs)
    b1 = np.zeros(ne, np.int64); e1 = np.zeros(ne)
    rk.rkn_batch_launch(c.ctx, b1, e1)
    # refinement, then an FP64 eager scan over a large window set (more scratch)
    ev = np.arange(ne, dtype=np.int32)
    rk.rkn_refine_setup(c.ctx, rk.make_scan_params(n_steps=800), ev, np.array([x.truth_seeds[0] for x in evs]))
    rk.rkn_gn_refine(c.ctx, 2, SCALE, np.zeros((ne, 5)), np.zeros((ne, 3)))
    w = synth.make_windows([(e, 0, evs[e].truth_seeds[0], [0.01, 5.0, 1.0, 1.0, 1.0], [4, 4, 4, 4, 4])
                            for e in range(ne)])
    rk.rkn_scan_windows(c.ctx, rk.make_scan_params(n_steps=800, precision=64), w, None, None,
                        np.zeros(ne, np.int64), np.zeros(ne))
    b2 = np.zeros(ne, np.int64); e2 = np.zeros(ne)
    rk.rkn_batch_launch(c.ctx, b2, e2)
    assert np.array_equal(b1, b2) and np.array_equal(e1, e2)
    c.close()


def test_autograd_function_matches_adjoint_entry_point(rk, geo, ufield):
    """torch.autograd over the residuals: seeds.grad of sum(r^2) equals the library's
    default-gradient adjoint (upstream 2 r is exact in FP32); a backward that does not
    follow the last forward is refused."""
    import torch
    from paper_1908_01949_amd.refine import Refinement
    evs = _events(geo, ufield, "uniform")
    off, wid, dr = synth.pack_events(evs)
    ev, s5 = _seeds(evs, 2, np.random.default_rng(11))
    n = ev.size
    st = torch.cuda.Stream()
    ca = rk.Context(0, st.cuda_stream)
    ca.upload_geometry(geo); ca.upload_field(ufield); ca.upload_hits(off, wid, dr)
    ref = Refinement(ca, rk.make_scan_params(n_steps=N_STEPS), ev, s5)
    seeds = torch.tensor(s5, device="cuda", requires_grad=True)
    r = ref.residuals(seeds)
    loss = torch.nansum(r.double() ** 2)
    loss.backward()
    # host-pointer twin on its own context
    c, _, _, _, _, H = _setup(rk, geo, ufield, "uniform", per_event=2, seed=11)
    resid, phi = _forward(rk, c, n, H)
    g = np.zeros((n, 5))
    rk.rkn_adjoint_bwd(c.ctx, None, g, None, None)
    np.testing.assert_array_equal(r.detach().cpu().numpy(), resid)
    np.testing.assert_allclose(seeds.grad.cpu().numpy(), g, rtol=1e-12, atol=0)
    assert float(loss.detach()) == pytest.approx(phi.sum(), rel=1e-6)
    # stale backward
    r1 = ref.residuals(seeds)
    ref.residuals(seeds)
    with pytest.raises(RuntimeError):
        torch.nansum(r1.double() ** 2).backward()
    c.close(); ca.close()


def test_checkpoint_tuner(rk, geo, sfield):
    """ckpt_every = 0 times the adjoint sweep for 32, 64, 128 and 256 steps and keeps
    the fastest; the gradient and J^T J equal those of an explicit setup with the
    chosen interval (the segment chaining only reassociates FP64 sums)."""
    c, evs, off, ev, s5, H = _setup(rk, geo, sfield, "solenoid", per_event=4, seed=9)
    sp = rk.make_scan_params(n_steps=N_STEPS, precision=32)
    rk.rkn_refine_setup(c.ctx, sp, ev, s5, 0)
    n, k, ms = rk.rkn_refine_info(c.ctx)
    print(f"checkpoint tuner: chose {k}, sweeps {ms} ms", flush=True)
    assert n == ev.size and k in (32, 64, 128, 256) and all(m > 0 for m in ms)
    _forward(rk, c, n, H)
    g1 = np.zeros((n, 5)); A1 = np.zeros((n, 5, 5))
    rk.rkn_adjoint_bwd(c.ctx, None, g1, A1, None)
    for kk in (k, 64 if k != 64 else 32):
        rk.rkn_refine_setup(c.ctx, sp, ev, s5, kk)
        assert rk.rkn_refine_info(c.ctx)[1] == kk
        _forward(rk, c, n, H)
        g2 = np.zeros((n, 5)); A2 = np.zeros((n, 5, 5))
        rk.rkn_adjoint_bwd(c.ctx, None, g2, A2, None)
        np.testing.assert_allclose(g2, g1, rtol=1e-9, atol=1e-9 * np.abs(g1).max())
        np.testing.assert_allclose(A2, A1, rtol=1e-9, atol=1e-9 * np.abs(A1).max())
    with pytest.raises(rk.RknError) as e:
        rk.rkn_refine_setup(c.ctx, sp, ev, s5, 20)
    assert e.value.status == rk.RKN_E_ARG
    c.close()
