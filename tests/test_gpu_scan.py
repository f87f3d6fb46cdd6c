"""GPU parity of the propagation and the scan against the FP64 oracle (through the C ABI).

Tolerances (stated, not tuned): FP64 trajectories <= 1e-9 mm, FP32 trajectories
<= 0.05 mm after three turns, scores <= 1e-4 relative, best-seed index identical
except at a near-tie (runner-up within 2e-4 relative), n_in identical except for a
hit on the lambda boundary.
"""
import math

import numpy as np
import pytest

from paper_1908_01949_amd import synth
from tests import parity_util as pu

pytestmark = pytest.mark.gpu


def _note(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def rk():
    from paper_1908_01949_amd import rknscan
    rknscan.load_library()
    return rknscan


@pytest.fixture(scope="module")
def ctx_u(rk, geo, ufield):
    c = rk.Context(0)
    c.upload_geometry(geo)
    c.upload_field(ufield)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx_s(rk, geo, sfield):
    c = rk.Context(0)
    c.upload_geometry(geo)
    c.upload_field(sfield)
    yield c
    c.close()


def _seeds(rng, n, pz_max=20.0):
    th = rng.uniform(-np.pi, np.pi, n)
    p = rng.uniform(70, 106, n)
    pz = rng.uniform(-pz_max, pz_max, n)
    pt = np.sqrt(p * p - pz * pz)
    ph = th + np.pi / 2 + rng.uniform(-0.6, 0.6, n)
    return np.stack([th, rng.uniform(-300, 300, n), pt * np.cos(ph), pt * np.sin(ph), pz], -1)


# ---------------------------------------------------------------------------------------
# trajectories (rkn_trace)
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("fieldname,prec,tol", [("u", 64, 1e-9), ("u", 32, 0.05),
                                                ("s", 64, 1e-9), ("s", 32, 0.05)])
def test_trace_parity(rk, ctx_u, ctx_s, orc_u, orc_s, fieldname, prec, tol):
    ctx, O = (ctx_u, orc_u) if fieldname == "u" else (ctx_s, orc_s)
    _note(f"trace parity field={fieldname} precision={prec}")
    rng = np.random.default_rng(100 + prec)
    seeds = _seeds(rng, 64)
    steps = np.array([0, 1, 7, 500, 2200, 4400, 6600], np.int32)   # 3 turns = 6600 mm
    p = rk.make_scan_params(n_steps=6600, precision=prec)
    g = rk.rkn_trace(ctx.ctx, p, seeds, steps)
    o = O.trace(O.params(n_steps=6600), seeds, steps)
    dpos = np.linalg.norm(g[..., :3] - o[..., :3], axis=-1)
    _note(f"  max position error {dpos.max():.3e} mm (tol {tol})")
    assert dpos.max() <= tol
    assert np.abs(g[..., 3:] - o[..., 3:]).max() <= (1e-12 if prec == 64 else 1e-5)


# ---------------------------------------------------------------------------------------
# scans
# ---------------------------------------------------------------------------------------
def _scan_both(rk, ctx, O, ev_list, windows, n_steps, prec, lam=64.0, block_steps=0, mode=1, turn_stop=0):
    off, wid, dr = synth.pack_events(ev_list)
    ctx.upload_hits(off, wid, dr)
    total = int(sum(int(np.prod(w["count"].astype(np.int64))) for w in windows))
    p = rk.make_scan_params(n_steps=n_steps, precision=prec, lambda_mm2=lam, block_steps=block_steps,
                            turn_stop=turn_stop)
    score = np.zeros(total); nin = np.zeros(total, np.int32)
    bi = np.zeros(len(ev_list), np.int64); bs = np.zeros(len(ev_list))
    rk.rkn_scan_windows(ctx.ctx, p, windows, score, nin, bi, bs)
    osc, onin, obi, obs, _ = O.scan_windows(O.params(n_steps=n_steps, lambda_mm2=lam, turn_stop=turn_stop),
                                            off, wid, dr, windows, mode=mode)
    return score, nin, bi, bs, osc, onin, obi, obs


def test_scan_single_turn_fp64(rk, ctx_u, orc_u, ev1):
    """One event, uniform 1 T, FP64, 6^5 = 7776 seeds over theta+-0.3, z+-100, p+-10, 2000 steps."""
    _note("scan single-turn FP64 6^5")
    w = synth.make_windows([(0, 0, ev1.truth_seeds[0], [0.3, 100, 10, 10, 10], [6] * 5)])
    score, nin, bi, bs, osc, onin, obi, obs = _scan_both(rk, ctx_u, orc_u, [ev1], w, 2000, 64)
    rel = pu.check_scores(score, osc, rel=1e-9, abs_=1e-9)
    _note(f"  max rel score error {rel:.2e}")
    assert np.array_equal(nin, onin)
    pu.check_best(bi[0], osc)
    assert bs[0] == pytest.approx(osc.min(), rel=1e-9)


@pytest.mark.parametrize("turn_stop", [0, 1])
def test_scan_solenoid_fp64(rk, ctx_s, orc_s, geo, sfield, turn_stop):
    """FP64 scan in the (r, z) field map: one event, 6^5 = 7776 seeds over theta+-0.3,
    z+-100, p+-10, 2000 steps, with and without the end of the turn partition."""
    _note(f"scan solenoid FP64 6^5 turn_stop={turn_stop}")
    ev = synth.event_single_turn(geo, sfield, 2)
    w = synth.make_windows([(0, 0, ev.truth_seeds[0], [0.3, 100, 10, 10, 10], [6] * 5)])
    score, nin, bi, bs, osc, onin, obi, obs = _scan_both(rk, ctx_s, orc_s, [ev], w, 2000, 64, turn_stop=turn_stop)
    rel = pu.check_scores(score, osc, rel=1e-9, abs_=1e-9)
    _note(f"  max rel score error {rel:.2e}")
    assert np.array_equal(nin, onin)
    pu.check_best(bi[0], osc)
    assert bs[0] == pytest.approx(osc.min(), rel=1e-9)


def test_scan_multi_turn_fp32(rk, ctx_u, orc_u, geo, ufield):
    """2-3 turn event with 30 % noise, FP32 propagation, 6000 steps, 4^5 grid + ragged tail."""
    _note("scan multi-turn FP32 4^5+ragged")
    ev = synth.event_multi_turn(geo, ufield, 0)
    t = ev.truth_seeds[0]
    w = synth.make_windows([(0, 0, t, [0.04, 15, 2, 2, 2], [4, 4, 4, 4, 4]),
                            (0, 1, t + np.array([0.01, 5, 0.5, -0.5, 0.3]), [0.01, 3, 0.5, 0.5, 0.5], [3, 1, 5, 1, 7])])
    score, nin, bi, bs, osc, onin, obi, obs = _scan_both(rk, ctx_u, orc_u, [ev], w, 6000, 32)
    rel = pu.check_scores(score, osc)
    _note(f"  max rel score error {rel:.2e}")
    pu.check_nin(nin, onin)
    pu.check_best(bi[0], osc)


def test_scan_solenoid_fp32(rk, ctx_s, orc_s, geo, sfield):
    """Field map (65x129 bilinear) event with 150 hits, 20 % noise, FP32."""
    _note("scan solenoid FP32 3^5")
    ev = synth.event_fixed_total(geo, sfield, 0, n_total=150, noise_frac=0.2)
    w = synth.make_windows([(0, 0, ev.truth_seeds[0], [0.03, 20, 3, 3, 3], [3] * 5)])
    score, nin, bi, bs, osc, onin, obi, obs = _scan_both(rk, ctx_s, orc_s, [ev], w, 6000, 32)
    rel = pu.check_scores(score, osc)
    _note(f"  max rel score error {rel:.2e}")
    pu.check_nin(nin, onin)
    pu.check_best(bi[0], osc)


@pytest.mark.parametrize("block_steps", [4, 6, 8])
def test_scan_block_steps_and_ragged_steps(rk, ctx_u, orc_u, ev1, block_steps):
    """n_steps not a multiple of the block; every block size gives the oracle's scores."""
    _note(f"scan block_steps={block_steps} n_steps=1999")
    w = synth.make_windows([(0, 0, ev1.truth_seeds[0], [0.1, 30, 4, 4, 4], [3, 3, 3, 3, 3])])
    score, nin, bi, bs, osc, onin, obi, obs = _scan_both(rk, ctx_u, orc_u, [ev1], w, 1999, 32,
                                                         block_steps=block_steps)
    pu.check_scores(score, osc)
    pu.check_best(bi[0], osc)


@pytest.mark.parametrize("block_steps", [4, 6, 8])
def test_scan_solenoid_workgroup_shapes(rk, ctx_s, orc_s, geo, sfield, block_steps):
    """Field map, every workgroup shape (16, 12 and 8 waves): several tiles, a ragged
    tile tail and a step count that no block size divides."""
    _note(f"scan solenoid block_steps={block_steps} 1280+105 seeds, 1999 steps")
    ev = synth.event_fixed_total(geo, sfield, 2, n_total=150, noise_frac=0.2)
    t = ev.truth_seeds[0]
    w = synth.make_windows([(0, 0, t, [0.03, 20, 3, 3, 3], [4, 4, 4, 4, 5]),
                            (0, 1, t + np.array([0.01, 5, 0.5, -0.5, 0.3]), [0.01, 3, 0.5, 0.5, 0.5], [3, 1, 5, 1, 7])])
    score, nin, bi, bs, osc, onin, obi, obs = _scan_both(rk, ctx_s, orc_s, [ev], w, 1999, 32,
                                                         block_steps=block_steps)
    rel = pu.check_scores(score, osc)
    _note(f"  max rel score error {rel:.2e}")
    pu.check_nin(nin, onin)
    pu.check_best(bi[0], osc)


def test_scan_max_hits_event(rk, ctx_s, orc_s, geo, sfield):
    """An event at the hit limit (512 hits, mostly noise): the wide workgroup shapes no
    longer fit in LDS, the scan falls back to 8 waves and still matches the oracle."""
    _note("scan 512-hit event, solenoid FP32")
    ev = synth.event_fixed_total(geo, sfield, 3, n_total=512, noise_frac=0.7)
    assert ev.wire_id.size == 512
    w = synth.make_windows([(0, 0, ev.truth_seeds[0], [0.03, 20, 3, 3, 3], [3, 3, 3, 3, 4])])
    off, wid, dr = synth.pack_events([ev])
    ctx_s.upload_hits(off, wid, dr)
    bsteps, tile = rk.rkn_scan_shape(ctx_s.ctx, rk.make_scan_params(n_steps=1500, precision=32))
    _note(f"  shape {bsteps}-step blocks, {tile} seeds per tile")
    score, nin, bi, bs, osc, onin, obi, obs = _scan_both(rk, ctx_s, orc_s, [ev], w, 1500, 32)
    rel = pu.check_scores(score, osc)
    _note(f"  max rel score error {rel:.2e}")
    pu.check_nin(nin, onin)
    pu.check_best(bi[0], osc)


def test_scan_multi_event_edge_cases(rk, ctx_u, orc_u, geo, ufield, ev1):
    """Several events: one with no hits, one with no window, a seed with |p| ~ 0, lambda = 16."""
    _note("scan multi-event edge cases")
    ev2 = synth.event_single_turn(geo, ufield, 5)
    empty = synth.Event(np.zeros(0, np.int32), np.zeros(0, np.float32), np.zeros(0, bool),
                        np.zeros(0, np.int32), np.zeros(0), np.zeros((0, 5)), np.zeros(0))
    evs = [ev1, empty, ev2, ev1]
    w = synth.make_windows([
        (0, 0, ev1.truth_seeds[0], [0.05, 10, 2, 2, 2], [2, 2, 3, 2, 2]),
        (1, 0, ev1.truth_seeds[0], [0.05, 10, 2, 2, 2], [2, 1, 1, 1, 3]),
        (2, 0, ev2.truth_seeds[0], [0.05, 10, 2, 2, 2], [3, 3, 3, 3, 3]),
        (2, 1, [0.0, 0.0, 0.0, 0.0, 0.0], [0, 0, 0, 0, 0], [1, 1, 1, 1, 1]),     # |p| = 0
    ])
    score, nin, bi, bs, osc, onin, obi, obs = _scan_both(rk, ctx_u, orc_u, evs, w, 2000, 32, lam=16.0)
    pu.check_scores(score, osc)
    assert np.all(score[48:51] == 0.0)                 # no hits: E = 0
    assert np.isinf(score[-1]) and nin[-1] == 0
    assert bi[3] == -1 and np.isinf(bs[3])             # event with no window
    assert bi[1] == 48                                  # all-zero plateau: lowest index
    for e in (0, 2):
        assert bi[e] == obi[e] or pu.check_best(bi[e], osc)


def test_scan_seeds_matches_oracle(rk, ctx_u, orc_u, geo, ufield, ev1):
    """Explicit seed list in scrambled event order across two events."""
    _note("scan explicit seeds")
    ev2 = synth.event_single_turn(geo, ufield, 6)
    off, wid, dr = synth.pack_events([ev1, ev2])
    ctx_u.upload_hits(off, wid, dr)
    rng = np.random.default_rng(4)
    s1 = synth.random_seeds(rng, ev1.truth_seeds[0], [0.05, 20, 3, 3, 3], 300)
    s2 = synth.random_seeds(rng, ev2.truth_seeds[0], [0.05, 20, 3, 3, 3], 200)
    seeds = np.concatenate([s1, s2]); sev = np.r_[np.zeros(300), np.ones(200)].astype(np.int32)
    perm = rng.permutation(500)
    seeds, sev = seeds[perm], sev[perm]
    p = rk.make_scan_params(n_steps=2000, precision=32)
    score = np.zeros(500); nin = np.zeros(500, np.int32); bi = np.zeros(2, np.int64); bs = np.zeros(2)
    rk.rkn_scan_seeds(ctx_u.ctx, p, sev, seeds, score, nin, bi, bs)
    osc, onin, obi, obs = orc_u.scan_seeds(orc_u.params(n_steps=2000), off, wid, dr, sev, seeds)
    pu.check_scores(score, osc)
    pu.check_nin(nin, onin)
    for e in range(2):
        idx = np.nonzero(sev == e)[0]
        g = int(bi[e]); assert sev[g] == e
        best = idx[np.argmin(osc[idx])]
        assert g == best or osc[g] <= osc[best] * (1 + pu.NEAR_TIE)


def test_scan_device_outputs_torch(rk, geo, ufield, orc_u, ev1):
    """Device-pointer outputs on torch's current stream (stream-ordered)."""
    import torch
    _note("scan device outputs")
    stream = torch.cuda.current_stream().cuda_stream
    c = rk.Context(0, stream)
    c.upload_geometry(geo); c.upload_field(ufield)
    off, wid, dr = synth.pack_events([ev1])
    c.upload_hits(off, wid, dr)
    w = synth.make_windows([(0, 0, ev1.truth_seeds[0], [0.1, 30, 4, 4, 4], [3] * 5)])
    p = rk.make_scan_params(n_steps=2000, precision=32, ptr_flags=rk.RKN_PTR_DEVICE)
    score = torch.zeros(243, dtype=torch.float64, device="cuda")
    nin = torch.zeros(243, dtype=torch.int32, device="cuda")
    bi = torch.zeros(1, dtype=torch.int64, device="cuda"); bs = torch.zeros(1, dtype=torch.float64, device="cuda")
    rk.rkn_scan_windows(c.ctx, p, w, score, nin, bi, bs)
    torch.cuda.synchronize()
    osc, onin, obi, obs, _ = orc_u.scan_windows(orc_u.params(n_steps=2000), off, wid, dr, w)
    pu.check_scores(score.cpu().numpy(), osc)
    pu.check_best(int(bi.cpu()[0]), osc)
    c.close()


def test_scan_repeatable(rk, ctx_u, ev1):
    """Two identical scans give bit-identical scores (no order-dependent reductions)."""
    off, wid, dr = synth.pack_events([ev1])
    ctx_u.upload_hits(off, wid, dr)
    w = synth.make_windows([(0, 0, ev1.truth_seeds[0], [0.3, 100, 10, 10, 10], [4] * 5)])
    p = rk.make_scan_params(n_steps=2000, precision=32)
    outs = []
    for _ in range(2):
        s = np.zeros(1024); n = np.zeros(1024, np.int32); bi = np.zeros(1, np.int64); bs = np.zeros(1)
        rk.rkn_scan_windows(ctx_u.ctx, p, w, s, n, bi, bs)
        outs.append((s, n, bi))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2][0] == outs[1][2][0]


def test_argument_errors(rk, geo, ufield, ev1):
    """Invalid arguments and call order give error codes, never a crash."""
    c = rk.Context(0)
    w = synth.make_windows([(0, 0, ev1.truth_seeds[0], [0.1, 30, 4, 4, 4], [2] * 5)])
    p = rk.make_scan_params()
    out = (np.zeros(32), np.zeros(32, np.int32), np.zeros(1, np.int64), np.zeros(1))
    with pytest.raises(rk.RknError) as e:
        rk.rkn_scan_windows(c.ctx, p, w, *out)
    assert e.value.status == rk.RKN_E_STATE
    c.upload_geometry(geo)
    with pytest.raises(rk.RknError) as e:
        rk.rkn_upload_hits(c.ctx, [0, 2], [0, 99999], [1.0, 1.0])
    assert e.value.status == rk.RKN_E_ARG
    with pytest.raises(rk.RknError) as e:
        rk.rkn_upload_hits(c.ctx, [0, 1], [3], [float("nan")])
    assert e.value.status == rk.RKN_E_ARG
    with pytest.raises(rk.RknError) as e:
        rk.rkn_upload_hits(c.ctx, [0, 600], np.arange(600), np.ones(600))
    assert e.value.status == rk.RKN_E_CAPACITY
    c.upload_field(ufield)
    off, wid, dr = synth.pack_events([ev1])
    c.upload_hits(off, wid, dr)
    for bad in (dict(n_steps=0), dict(step_mm=-1.0), dict(precision=16), dict(lambda_mm2=float("nan")),
                dict(block_steps=5)):
        with pytest.raises(rk.RknError) as e:
            rk.rkn_scan_windows(c.ctx, rk.make_scan_params(**bad), w, *out)
        assert e.value.status == rk.RKN_E_ARG
    wbad = w.copy(); wbad[0]["count"][2] = 0
    with pytest.raises(rk.RknError) as e:
        rk.rkn_scan_windows(c.ctx, p, wbad, *out)
    assert e.value.status == rk.RKN_E_ARG
    wbad = w.copy(); wbad[0]["event"] = 3
    with pytest.raises(rk.RknError):
        rk.rkn_scan_windows(c.ctx, p, wbad, *out)
    # the context still works after errors
    rk.rkn_scan_windows(c.ctx, p, w, *out)
    assert np.isfinite(out[0]).all()
    c.close()


@pytest.mark.parametrize("kind", ["uniform", "solenoid"])
def test_scan_rotation_invariance(rk, geo, ufield, sfield, kind):
    """Both fields are symmetric about the z axis: rotating every wire and every seed by
    the same angle about it leaves each seed's score unchanged (up to rounding), for
    angles that move the event's hits across the azimuth sectors and the -pi/pi seam."""
    import dataclasses
    field = ufield if kind == "uniform" else sfield
    ev = synth.event_fixed_total(geo, field, 3, n_total=120, noise_frac=0.2)
    off, wid, dr = synth.pack_events([ev])
    w = synth.make_windows([(0, 0, ev.truth_seeds[0], (0.03, 40.0, 3.0, 3.0, 4.0), (3, 3, 3, 3, 3))])
    n = 243
    p = rk.make_scan_params(n_steps=6000, precision=32)
    ref = None
    for ang in (0.0, 0.7, np.pi - 0.01, 2.9, -1.3):
        ca, sa = np.cos(ang), np.sin(ang)
        g2 = dataclasses.replace(geo, mx=ca * geo.mx - sa * geo.my, my=sa * geo.mx + ca * geo.my,
                                 ux=ca * geo.ux - sa * geo.uy, uy=sa * geo.ux + ca * geo.uy)
        # explicit seeds: a window's (px, py) grid would not rotate with the seeds
        seeds = np.array([synth_window_seed(w[0], k) for k in range(n)])
        rs = seeds.copy()
        rs[:, 0] = seeds[:, 0] + ang
        rs[:, 2] = ca * seeds[:, 2] - sa * seeds[:, 3]
        rs[:, 3] = sa * seeds[:, 2] + ca * seeds[:, 3]
        c = rk.Context(0)
        c.upload_geometry(g2); c.upload_field(field); c.upload_hits(off, wid, dr)
        sc = np.zeros(n); nin = np.zeros(n, np.int32)
        rk.rkn_scan_seeds(c.ctx, p, np.zeros(n, np.int32), rs, sc, nin, np.zeros(1, np.int64), np.zeros(1))
        c.close()
        if ref is None:
            ref = (sc.copy(), nin.copy())
            continue
        np.testing.assert_allclose(sc, ref[0], rtol=2e-5, atol=1e-4)
        assert np.abs(nin - ref[1]).max() <= 1
        _note(f"{kind} rotated by {ang:+.2f} rad: max rel score change {np.max(np.abs(sc - ref[0]) / np.maximum(ref[0], 1e-9)):.1e}")


def synth_window_seed(win, k):
    """Seed k of a window's grid (theta slowest, pz fastest), for building explicit seeds."""
    cnt = [int(x) for x in win["count"]]
    idx = []
    for d in range(4, -1, -1):
        idx.append(k % cnt[d]); k //= cnt[d]
    idx = idx[::-1]
    return np.array([win["center"][d] if cnt[d] <= 1 else
                     win["center"][d] - win["half_width"][d] + 2 * win["half_width"][d] * idx[d] / (cnt[d] - 1)
                     for d in range(5)])


@pytest.mark.parametrize("kind", ["uniform", "solenoid"])
def test_scan_z_mirror_invariance(rk, geo, ufield, sfield, kind):
    """Both fields are mirror-symmetric in z (B_r odd, B_z even): mirroring the wires
    (u_z -> -u_z, which swaps the stereo signs) and the seeds (z0 -> -z0, pz -> -pz)
    leaves each seed's score unchanged up to rounding."""
    import dataclasses
    field = ufield if kind == "uniform" else sfield
    ev = synth.event_fixed_total(geo, field, 3, n_total=120, noise_frac=0.2)
    off, wid, dr = synth.pack_events([ev])
    w = synth.make_windows([(0, 0, ev.truth_seeds[0], (0.03, 40.0, 3.0, 3.0, 4.0), (3, 3, 3, 3, 3))])
    seeds = np.array([synth_window_seed(w[0], k) for k in range(243)])
    p = rk.make_scan_params(n_steps=6000, precision=32)
    out = []
    for mirror in (False, True):
        g2 = dataclasses.replace(geo, mz=-geo.mz, uz=-geo.uz) if mirror else geo
        s2 = seeds.copy()
        if mirror:
            s2[:, 1] = -s2[:, 1]
            s2[:, 4] = -s2[:, 4]
        c = rk.Context(0)
        c.upload_geometry(g2); c.upload_field(field); c.upload_hits(off, wid, dr)
        sc = np.zeros(243); nin = np.zeros(243, np.int32)
        rk.rkn_scan_seeds(c.ctx, p, np.zeros(243, np.int32), s2, sc, nin, np.zeros(1, np.int64), np.zeros(1))
        c.close()
        out.append((sc, nin))
    np.testing.assert_allclose(out[1][0], out[0][0], rtol=2e-5, atol=1e-4)
    assert np.abs(out[1][1] - out[0][1]).max() <= 1
    _note(f"{kind} z-mirror: max rel score change {np.max(np.abs(out[1][0] - out[0][0]) / np.maximum(out[0][0], 1e-9)):.1e}")


def test_hit_order_invariance(rk, geo, sfield):
    """The upload sorts each event's hits (layer, twisted azimuth): uploading them in
    another order gives the same scores (to FP64 summation order) and classification
    masks that follow the caller's order."""
    ev = synth.event_fixed_total(geo, sfield, 5, n_total=130, noise_frac=0.2)
    w = synth.make_windows([(0, 0, ev.truth_seeds[0], (0.03, 40.0, 3.0, 3.0, 4.0), (3, 3, 3, 3, 3))])
    perm = np.random.default_rng(16).permutation(ev.wire_id.size)
    p = rk.make_scan_params(n_steps=6000, precision=32)
    res = []
    for order in (np.arange(ev.wire_id.size), perm):
        c = rk.Context(0)
        c.upload_geometry(geo); c.upload_field(sfield)
        c.upload_hits(np.array([0, order.size], np.int32), ev.wire_id[order], ev.drift[order])
        sc = np.zeros(243); nin = np.zeros(243, np.int32)
        rk.rkn_scan_windows(c.ctx, p, w, sc, nin, np.zeros(1, np.int64), np.zeros(1))
        mask, _ = rk.rkn_classify_hits(c.ctx, p, np.zeros(4, np.int32),
                                       np.array([synth_window_seed(w[0], k) for k in (0, 60, 121, 242)]), order.size)
        c.close()
        res.append((sc, nin, mask))
    np.testing.assert_allclose(res[1][0], res[0][0], rtol=1e-12, atol=1e-12)
    assert np.array_equal(res[1][1], res[0][1])
    assert np.array_equal(res[1][2][:, :perm.size], res[0][2][:, perm])
    _note("hit order: scores, n_in and masks follow the permutation")


# ---------------------------------------------------------------------------------------
# work counters of the kernel against the CPU model of its culling rule
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("fieldname", ["u", "s"])
def test_work_counts_match_cull_model(rk, geo, ufield, sfield, ctx_u, ctx_s, fieldname):
    """The counting instance of the scan kernel takes every step and evaluates the chord
    distances of exactly the (block, hit) pairs the cull rule keeps (tests/cull_model.py,
    FP64): the counts agree up to pairs whose sphere or band test sits within FP32
    rounding of its bound."""
    import oracle
    from tests.cull_model import blocked_work
    field = ufield if fieldname == "u" else sfield
    ctx = ctx_u if fieldname == "u" else ctx_s
    ev = synth.event_multi_turn(geo, field, 7, sigma=0.2, noise_frac=0.3)
    off, wid, dr = synth.pack_events([ev])
    ctx.upload_hits(off, wid, dr)
    n_steps = 3000
    w = synth.make_windows([(0, 0, ev.truth_seeds[0], [0.02, 20.0, 3.0, 3.0, 3.0], [2, 2, 2, 2, 2])])
    p = rk.make_scan_params(n_steps=n_steps, precision=32)
    B, _ = rk.rkn_scan_shape(ctx.ctx, p)
    steps, tests, chords = rk.rkn_scan_work_counts(ctx.ctx, p, w)
    O = oracle.Oracle(geo, field)
    prm = O.params(n_steps=n_steps)
    m_steps = m_chords = 0
    for k in range(32):
        s, c, _ = blocked_work(O, prm, O.window_seed(w[0], k), geo, ev.wire_id, ev.drift, B)
        m_steps += s
        m_chords += c
    _note(f"{fieldname}: B={B} steps {steps} tests {tests} chords {chords} (model {m_chords}), "
          f"chords/seed-step {chords / steps:.4f}")
    assert steps == m_steps == 32 * n_steps
    assert abs(chords - m_chords) <= 0.005 * m_chords + 2 * B
    assert tests >= chords // B > 0


@pytest.mark.parametrize("n_layers,tile", [(6, 768), (40, 512)])
def test_scan_other_layer_counts(rk, sfield, n_layers, tile):
    """Chambers of 6 and 40 layers in the field map: the per-event layer and sector
    tables are sized by the geometry (with 40 layers the 12-wave shape no longer fits
    the LDS and the scan falls back to 8-wave workgroups); scores, n_in and the best
    seed match the oracle's."""
    import oracle
    g = synth.make_geometry(n_layers=n_layers)
    evs = synth.events_batch(g, sfield, 1, seed=21, hits_range=(8, 480))
    off, wid, dr = synth.pack_events(evs)
    c = rk.Context(0)
    c.upload_geometry(g); c.upload_field(sfield); c.upload_hits(off, wid, dr)
    w = synth.make_windows([(0, 0, evs[0].truth_seeds[0], [0.03, 20, 3, 3, 3], [3, 4, 3, 3, 4])])
    p = rk.make_scan_params(n_steps=3000, precision=32)
    assert rk.rkn_scan_shape(c.ctx, p) == (6, tile)
    n = int(np.prod(w[0]["count"]))
    score = np.zeros(n); nin = np.zeros(n, np.int32); bi = np.zeros(1, np.int64); bs = np.zeros(1)
    rk.rkn_scan_windows(c.ctx, p, w, score, nin, bi, bs)
    c.close()
    O = oracle.Oracle(g, sfield)
    osc, onin, obi, obs, _ = O.scan_windows(O.params(n_steps=3000), off, wid, dr, w)
    rel = pu.check_scores(score, osc)
    pu.check_nin(nin, onin)
    pu.check_best(bi[0], osc)
    _note(f"{n_layers} layers, {wid.size} hits, tile {tile}: {n} seeds, max rel score error {rel:.2e}")
