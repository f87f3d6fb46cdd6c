#!/usr/bin/env python3
"""Benchmark of the batched RKN seed scan on one MI355X.

One step = one pass of the hot path over a batch of 512 synthetic events: circle
Hough stage and seed windows for every event, one persistent scan launch over all
seeds (6000 RKN steps of 1 mm, FP32 propagation, FP64 scores) and the per-event
argmin, replayed from captured HIP graphs with inputs already in HBM.

Prints one JSON line (stdout). Progress goes to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from paper_1908_01949_amd import rknscan as rk  # noqa: E402  (loads the HIP runtime first)
from paper_1908_01949_amd import flops, quality, synth, workloads  # noqa: E402

METRIC = "RKN seed-steps/s & events/s, %FP32 vector peak; plain scan vs adjoint-refined"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def batch_hough_params(field):
    """Window rule of the batched workload: 1e3-1e5 seeds per event."""
    return rk.make_hough_params(b_ref=field.b_ref, **workloads.BATCH["hough"])


def cpu_baseline_leg(geo, field, events, windows, ev_seed_off, gpu_scores, n_steps, lam, seconds):
    """The FP64 oracle timed on this host's cores (OpenMP threads) on a bounded random
    sample of the same batch, and on one thread (the paper's serial CPU) on a smaller
    sample. The oracle runs in its band-pruned mode, whose E is the brute-force E; the
    (chord, hit) pairs it evaluates per seed-step are the band-rule work count."""
    import ctypes
    import oracle
    gomp = ctypes.CDLL("libgomp.so.1")
    O = oracle.Oracle(geo, field)
    prm = O.params(n_steps=n_steps, lambda_mm2=lam)
    off, wid, dr = synth.pack_events(events)
    sizes = np.array([int(np.prod(w["count"].astype(np.int64))) for w in windows])
    wbase = np.concatenate([[0], np.cumsum(sizes)])
    total = int(wbase[-1])
    rng = np.random.default_rng(2024)

    def draw(n):
        g = np.sort(rng.choice(total, size=n, replace=False))
        k = np.searchsorted(wbase, g, side="right") - 1
        seeds = np.array([O.window_seed(windows[kk], gg - wbase[kk]) for kk, gg in zip(k, g)])
        return g, windows["event"][k].astype(np.int32), seeds

    cores = int(gomp.omp_get_max_threads())
    g, se, seeds = draw(min(64, total))
    t = time.perf_counter()
    pairs = []
    sc, _, _, _ = O.scan_seeds(prm, off, wid, dr, se, seeds, mode=1, pairs=pairs)
    dt = time.perf_counter() - t
    n = int(min(total, max(64, 64 * seconds / max(dt, 1e-3))))
    if n > 64:
        g, se, seeds = draw(n)
        pairs = []
        t = time.perf_counter()
        sc, _, _, _ = O.scan_seeds(prm, off, wid, dr, se, seeds, mode=1, pairs=pairs)
        dt = time.perf_counter() - t
    rel = float(np.max(np.abs(gpu_scores[g] - sc) / np.maximum(np.abs(sc), 1e-12)))
    # one thread, on the first seeds of the sample (about a quarter of the time budget)
    m1 = max(4, min(len(g), int(len(g) * 0.25 / max(cores, 1))))
    gomp.omp_set_num_threads(1)
    t = time.perf_counter()
    O.scan_seeds(prm, off, wid, dr, se[:m1], seeds[:m1], mode=1)
    dt1 = time.perf_counter() - t
    gomp.omp_set_num_threads(cores)
    return dict(value=len(g) * n_steps / dt, unit="seed-steps/s", cores=cores, kind="oracle",
                sample=f"{len(g)} seeds drawn uniformly from the {total} of the batch, {n_steps} steps each, "
                       f"FP64 band-pruned oracle, OpenMP over seeds, {dt:.1f} s",
                value_1_thread=m1 * n_steps / dt1,
                sample_1_thread=f"the first {m1} seeds of that sample on one thread, {dt1:.1f} s"), \
        dict(hbar_c11=pairs[0] / (len(g) * n_steps), sample_max_rel_score_err=rel)


def measured_traffic():
    """HBM bytes per scan launch from the committed counter record (FETCH_SIZE and
    WRITE_SIZE runs scaled by a plain copy's counts), or None when the kernel sources
    differ from the ones the counters were taken on."""
    path = os.path.join(ROOT, "profiles", "scan_kernel_512ev_solenoid_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    return int(rec["traffic_bytes"]) if rec.get("kernel_source_sha256") == kernel_source_hash() else None


def kernel_source_hash():
    """SHA-256 of the scan kernel's sources with comments and blank space removed."""
    import hashlib
    h = hashlib.sha256()
    for fn in ("scan.hip", "device_math.hpp", "internal.hpp"):
        with open(os.path.join(ROOT, "paper_1908_01949_amd", "csrc", fn)) as f:
            for line in f:
                code = line.split("//", 1)[0].strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()


def _sync_time(fn):
    import torch
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return r, time.perf_counter() - t


def refine_leg(ctx, sp, n_events, t_coarse, k=8, gn_iters=10, max_rounds=10, rtol=1e-3,
               scale=(1.0, 100.0, 100.0, 100.0, 100.0), grid=6):
    """Refinement of the k best seeds per event of the batch just scanned, two ways:
    (a) Gauss-Newton with the adjoint sweep (gn_iters iterations), and (b) the paper's
    coarse-to-fine rescans (section 2.2) through rkn_rescan_refine: grid^5 grids around
    the k kept seeds, half-width = the previous grid step, max_rounds rounds. (b) runs
    twice: all rounds, as the paper does, and stopping each event once its lowest E is
    within rtol * Phi_GN of the E of its best Gauss-Newton seed (the same residual
    accuracy in mm^2). Times include the shared coarse scan; the targets and the
    accuracy checks are not timed."""
    ne = n_events
    (idx, sc, s5), t_topk = _sync_time(lambda: rk.rkn_batch_topk(ctx.ctx, k, n_events=ne))
    ok = idx >= 0
    ev_of = np.repeat(np.arange(ne, dtype=np.int32), k).reshape(ne, k)
    seed_event = ev_of[ok]
    seeds = s5[ok]
    # (a) Gauss-Newton
    p = rk.make_scan_params(n_steps=sp.n_steps, precision=32, lambda_mm2=sp.lambda_mm2)
    nsd = seed_event.size
    # the checkpoint interval is tuned once (untimed), then used by the timed leg
    rk.rkn_refine_setup(ctx.ctx, p, seed_event, seeds, 0)
    _, ckpt, tune_ms = rk.rkn_refine_info(ctx.ctx)
    log(f"checkpoint tuner: {ckpt} steps (adjoint sweeps for 32/64/128/256: {tune_ms})")

    def gn():
        rk.rkn_refine_setup(ctx.ctx, p, seed_event, seeds, ckpt)
        out = np.zeros((nsd, 5)); phi = np.zeros((nsd, gn_iters + 1))
        rk.rkn_gn_refine(ctx.ctx, gn_iters, np.asarray(scale), out, phi)
        return out, phi
    (gn_seeds, gn_phi), t_gn = _sync_time(gn)
    phi_fin = gn_phi[:, -1]
    best_slot = np.full(ne, -1)
    for e in range(ne):
        sl = np.nonzero(seed_event == e)[0]
        if sl.size:
            best_slot[e] = sl[np.argmin(phi_fin[sl])]
    has = best_slot >= 0
    phi_gn = np.where(has, phi_fin[np.maximum(best_slot, 0)], np.nan)
    log(f"refine: {nsd} seeds, top-{k} {t_topk * 1e3:.1f} ms, GN {gn_iters} it {t_gn * 1e3:.1f} ms, "
        f"Phi {np.nanmean(gn_phi[:, 0]):.3g} -> {np.nanmean(phi_fin):.3g}")
    # E of each event's best GN seed (untimed): the rescans' target in their own score
    e_gn = np.full(ne, np.inf)
    if has.any():
        ev_h = np.nonzero(has)[0].astype(np.int32)
        sc_gn, _, _, _ = rk.rkn_scan_seeds(ctx.ctx, sp, ev_h, gn_seeds[best_slot[has]], np.zeros(ev_h.size),
                                           np.zeros(ev_h.size, np.int32), np.zeros(ne, np.int64), np.zeros(ne))
        e_gn[has] = sc_gn
    target = np.where(has, e_gn + rtol * phi_gn, -np.inf)

    def phi_on_gn_set(cand):
        """Phi of cand[e] on the inlier set of event e's best GN seed (not timed)."""
        trial = gn_seeds.copy()
        sel = has & np.all(np.isfinite(cand), axis=1)
        trial[best_slot[sel]] = cand[sel]
        ph = np.zeros(nsd)
        rk.rkn_residuals_fwd(ctx.ctx, trial, None, ph)
        out = np.full(ne, np.inf)
        out[sel] = ph[best_slot[sel]]
        return out

    # (b) the paper's rescans from the batch's k best, all rounds, then with the stop rule
    rp = rk.make_rescan_params(k=k, grid=grid, max_rounds=max_rounds)
    (r5, rstep, rsc, rrounds), t_full = _sync_time(lambda: rk.rkn_rescan_refine(ctx.ctx, sp, rp, ne))
    (q5, qstep, qsc, qrounds), t_stop = _sync_time(
        lambda: rk.rkn_rescan_refine(ctx.ctx, sp, rp, ne, target=target))
    full_reach_e = int(np.sum(has & (rsc[:, 0] <= target)))
    stop_reach_e = int(np.sum(has & (qsc[:, 0] <= target)))
    ph_full = phi_on_gn_set(r5[:, 0, :])
    ph_stop = phi_on_gn_set(q5[:, 0, :])
    full_reach_phi = int(np.sum(has & (ph_full <= (1.0 + rtol) * phi_gn)))
    stop_reach_phi = int(np.sum(has & (ph_stop <= (1.0 + rtol) * phi_gn)))
    valid0 = ok.sum(axis=1)
    per_grid = grid ** 5

    def seeds_scanned(rounds):
        r = rounds.astype(np.int64)
        return int(np.sum(np.where(r > 0, valid0 + (r - 1) * k, 0)) * per_grid)
    log(f"rescans: all {max_rounds} rounds {t_full * 1e3:.1f} ms (E within target: {full_reach_e} events, "
        f"Phi: {full_reach_phi}); with the stop rule {t_stop * 1e3:.1f} ms, mean rounds "
        f"{qrounds[has].mean():.2f} (E: {stop_reach_e}, Phi: {stop_reach_phi})")
    t_a = t_coarse + t_topk + t_gn
    t_b = t_coarse + t_full
    t_c = t_coarse + t_stop
    return dict(
        seeds=int(nsd), k=k, gn_iters=gn_iters, ckpt_every=ckpt, ckpt_tune_ms=[round(x, 3) for x in tune_ms],
        ms_coarse=round(t_coarse * 1e3, 2), ms_topk=round(t_topk * 1e3, 2), ms_gn=round(t_gn * 1e3, 2),
        rescan_grid=f"{grid}^5", ms_rescans_all_rounds=round(t_full * 1e3, 2),
        ms_rescans_stopped=round(t_stop * 1e3, 2), rescan_seeds_all_rounds=seeds_scanned(rrounds),
        rescan_seeds_stopped=seeds_scanned(qrounds),
        events_per_s_gn=ne / t_a, events_per_s_rescan_all_rounds=ne / t_b, events_per_s_rescan_stopped=ne / t_c,
        speedup_vs_paper_rescans=t_b / t_a, speedup_vs_stopped_rescans=t_c / t_a,
        # the coarse scan is shared: the refinement stages alone, and the end-to-end
        # ratio a zero-cost refinement would reach against the paper's ten rounds
        refinement_stage_speedup=t_full / (t_topk + t_gn),
        speedup_bound_shared_coarse=t_b / t_coarse,
        rescan_rounds_mean_stopped=float(qrounds[has].mean()) if has.any() else 0.0,
        events_with_seeds=int(has.sum()),
        events_reaching_gn_e_all_rounds=full_reach_e, events_reaching_gn_e_stopped=stop_reach_e,
        events_reaching_gn_phi_all_rounds=full_reach_phi, events_reaching_gn_phi_stopped=stop_reach_phi,
        phi_gn_mean=float(np.nanmean(phi_gn)), phi_start_mean=float(np.nanmean(gn_phi[:, 0])),
        rule=f"stopped rescans end an event once its lowest E <= E(best GN seed) + {rtol:g} Phi_GN; "
             f"reach counts: E by that rule, Phi as Phi(best rescan seed) <= (1+{rtol:g}) Phi_GN on the GN "
             f"inlier set; <= {max_rounds} rounds")


def bidirectional_leg(ctx, field, sp, n_events, t_entrance, n_hits_max, n_c_min=20):
    """Section 2.2's two-direction scan: the batch is scanned again from seed sets at the
    chamber exit (the time-reversed track: the circle Hough stage and the scan with the
    opposite charge), and each event's best entrance and exit seeds classify its hits;
    the event is kept when at least n_c_min hits are classified from both sides."""
    ne = n_events
    ent_idx, _, ent_s5 = rk.rkn_batch_topk(ctx.ctx, 1, n_events=ne)
    hp_exit = rk.make_hough_params(b_ref=field.b_ref, charge=-sp.charge, **workloads.BATCH["hough"])
    sp_exit = rk.make_scan_params(n_steps=sp.n_steps, precision=sp.precision, lambda_mm2=sp.lambda_mm2,
                                  charge=-sp.charge, block_steps=sp.block_steps)
    rk.rkn_batch_plan(ctx.ctx, hp_exit, sp_exit)
    rk.rkn_batch_launch(ctx.ctx, None, None)
    _, t_exit = _sync_time(lambda: rk.rkn_batch_launch(ctx.ctx, None, None))
    ext_idx, _, ext_s5 = rk.rkn_batch_topk(ctx.ctx, 1, n_events=ne)
    both = (ent_idx[:, 0] >= 0) & (ext_idx[:, 0] >= 0)
    ev = np.nonzero(both)[0].astype(np.int32)
    (_, _, n_common), t_cls = _sync_time(lambda: rk.rkn_bidirectional_common(
        ctx.ctx, sp, ev, ent_s5[ev, 0], ext_s5[ev, 0], n_hits_max))
    kept = int((n_common >= n_c_min).sum())
    t_all = t_entrance + t_exit + t_cls
    log(f"bidirectional: exit scan {t_exit * 1e3:.1f} ms, classification {t_cls * 1e3:.1f} ms, "
        f"{kept} of {ev.size} events with N_c >= {n_c_min}")
    return dict(ms_entrance=round(t_entrance * 1e3, 2), ms_exit=round(t_exit * 1e3, 2),
                ms_classify=round(t_cls * 1e3, 2), events_per_s=ne / t_all, events_with_both=int(ev.size),
                events_kept=kept, n_c_min=n_c_min, n_c_mean=float(n_common.mean()) if ev.size else 0.0)


def turns_leg(geo, field, n_events):
    """Section 2.3's reconstruction loop over multi-turn events (2-3 passes, 30 % noise)
    in the same field: time per call (inputs resident, host outputs) and the track
    finding quality of Eqs. 2-3 against the synthetic truth, averaged over the true
    turn partitions."""
    wl = workloads.TURNS
    t0 = time.time()
    evs = synth.events_multi_turn(geo, field, n_events, seed=1, n_steps=wl["n_steps"])
    off, wid, dr = synth.pack_events(evs)
    log(f"turn partitions: {n_events} multi-turn events, {wid.size} hits in {time.time() - t0:.1f} s")
    c = rk.Context(0)
    c.upload_geometry(geo); c.upload_field(field); c.upload_hits(off, wid, dr)
    hp = rk.make_hough_params(b_ref=field.b_ref, **wl["hough"])
    sp = rk.make_scan_params(n_steps=wl["n_steps"], precision=wl["precision"])
    tp = rk.make_turn_params()
    rk.rkn_find_turns(c.ctx, hp, sp, tp, wid.size, n_events)       # warm-up (code objects, buffers)
    r, dt = _sync_time(lambda: rk.rkn_find_turns(c.ctx, hp, sp, tp, wid.size, n_events))
    c.close()
    eps, pur, last_eps, last_pur = [], [], [], []
    for e, x in enumerate(evs):
        q = quality.turn_quality(x.turn_of, r["hit_turn"][off[e]:off[e + 1]])
        eps += [v["eps"] for v in q]
        pur += [v["pi"] for v in q if np.isfinite(v["pi"])]
        last_eps.append(q[-1]["eps"])
        if np.isfinite(q[-1]["pi"]):
            last_pur.append(q[-1]["pi"])
    out = dict(events=n_events, ms=round(dt * 1e3, 1), events_per_s=n_events / dt,
               partitions_per_event=float(r["n_turns"].mean()),
               true_partitions_per_event=float(np.mean([x.turn_of.max() + 1 for x in evs])),
               mean_eps=float(np.mean(eps)), mean_pi=float(np.mean(pur)),
               last_turn_eps=float(np.mean(last_eps)), last_turn_pi=float(np.mean(last_pur)),
               unclassified_frac=float(np.mean(r["hit_turn"] < 0)))
    log(f"turn partitions: {out}")
    return out


def adaptive_batch_leg(ctx, hp, sp, n_events, t_fixed, reps=2):
    """The same batch with the adaptive step size (error-controlled RKN, tol 1e-5 mm,
    steps 0.25-4 mm over the same 6000 mm path), planned and replayed like the
    fixed-step batch; not the headline (its steps are not 1 mm RKN steps)."""
    import torch
    ap = rk.make_adaptive_params()
    rk.rkn_batch_plan_adaptive(ctx.ctx, hp, sp, ap)
    rk.rkn_batch_launch(ctx.ctx, None, None)
    torch.cuda.synchronize()
    t = time.perf_counter()
    ms_scan = []
    for _ in range(reps):
        rk.rkn_batch_launch(ctx.ctx, None, None)
        ms_scan.append(rk.rkn_batch_info(ctx.ctx)[3])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / reps
    out = dict(ms_step=round(dt * 1e3, 1), ms_scan=round(float(np.mean(ms_scan)), 1), events_per_s=n_events / dt,
               speedup_over_fixed_step=round(t_fixed / dt, 2), tol_mm=ap.tol_mm, h_min_mm=ap.h_min_mm,
               h_max_mm=ap.h_max_mm)
    log(f"adaptive batch: {out}")
    return out


def other_workloads(geo, reps=3):
    """The single-event workloads, timed on the GPU (device outputs, inputs resident):
    a 6^5 FP64 scan of a single-turn event, a 16^5 FP32 scan of a multi-turn event
    (both uniform 1 T) and the Hough windows (12^5 per candidate) of a 150-hit event
    in the solenoid map."""
    import torch
    out = {}
    uf, sf = synth.uniform_field(1.0), synth.solenoid_field()
    cases = []
    ev1 = synth.event_single_turn(geo, uf, 0)
    wl = workloads.SINGLE_TURN
    cases.append(("single_turn_6^5_fp64", uf, ev1, wl, synth.make_windows(
        [(0, 0, ev1.truth_seeds[0], wl["half_width"], [wl["count"]] * 5)])))
    ev2 = synth.event_multi_turn(geo, uf, 0)
    wl = workloads.MULTI_TURN
    cases.append(("multi_turn_16^5_fp32", uf, ev2, wl, synth.make_windows(
        [(0, 0, ev2.truth_seeds[0], wl["half_width"], [wl["count"]] * 5)])))
    ev3 = synth.event_fixed_total(geo, sf, 0, n_total=150, noise_frac=0.2)
    cases.append(("hough_event_12^5_fp32", sf, ev3, workloads.HOUGH_EVENT, None))
    for name, field, ev, wl, w in cases:
        off, wid, dr = synth.pack_events([ev])
        c = rk.Context(0)
        c.upload_geometry(geo); c.upload_field(field); c.upload_hits(off, wid, dr)
        t_hough = 0.0
        if w is None:
            hp = rk.make_hough_params(b_ref=field.b_ref, **wl["hough"])
            w = rk.rkn_hough_seed_windows(c.ctx, hp)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                rk.rkn_hough_seed_windows(c.ctx, hp)
            t_hough = (time.perf_counter() - t) / reps
        n = int(np.prod(w["count"].astype(np.int64), axis=1).sum())
        p = rk.make_scan_params(n_steps=wl["n_steps"], precision=wl["precision"], ptr_flags=rk.RKN_PTR_DEVICE)
        score = torch.empty(n, dtype=torch.float64, device="cuda")
        bi = torch.empty(1, dtype=torch.int64, device="cuda"); bs = torch.empty(1, dtype=torch.float64, device="cuda")
        rk.rkn_scan_windows(c.ctx, p, w, score, None, bi, bs)
        rk.rkn_synchronize(c.ctx)
        t = time.perf_counter()
        for _ in range(reps):
            rk.rkn_scan_windows(c.ctx, p, w, score, None, bi, bs)
        rk.rkn_synchronize(c.ctx)
        dt = (time.perf_counter() - t) / reps
        out[name] = dict(seeds=n, steps=wl["n_steps"], ms_scan=round(dt * 1e3, 3),
                         seed_steps_per_s=n * wl["n_steps"] / dt, hough_ms=round(t_hough * 1e3, 3) or None)
        # roofline of this scan: the kernel's own count of chord distances (untimed
        # counting instance) in the same flop model, against the peak of its precision
        k_steps, _, k_chords = rk.rkn_scan_work_counts(c.ctx, p, w)
        q = k_chords / k_steps
        f_alg = flops.per_seed_step(field.kind, q)
        peak = flops.PEAK_FP64_TFLOPS if wl["precision"] == 64 else flops.PEAK_FP32_TFLOPS
        ach = f_alg * n * wl["n_steps"] / dt / 1e12
        out[name]["roofline"] = dict(bound="alu", achieved=round(ach, 3), peak=peak, unit="TFLOP/s",
                                     frac=round(ach / peak, 4), flops_per_seed_step=round(f_alg, 2),
                                     q_kernel=round(q, 5))
        if wl["precision"] == 32:
            # the paper's record-then-DCA form of the same scan (section 4.2), for comparison
            rk.rkn_scan_windows_two_kernel(c.ctx, p, w, score, None, bi, bs)
            rk.rkn_synchronize(c.ctx)
            t = time.perf_counter()
            rk.rkn_scan_windows_two_kernel(c.ctx, p, w, score, None, bi, bs)
            rk.rkn_synchronize(c.ctx)
            t2 = time.perf_counter() - t
            out[name]["ms_two_kernel"] = round(t2 * 1e3, 3)
            out[name]["fused_speedup_over_two_kernel"] = round(t2 / dt, 2)
        # the adaptive step size over the same path length (tol 1e-5 mm, steps 0.25-4 mm)
        ap = rk.make_adaptive_params()
        rk.rkn_scan_windows_adaptive(c.ctx, p, ap, w, score, None, bi, bs)
        rk.rkn_synchronize(c.ctx)
        t = time.perf_counter()
        rk.rkn_scan_windows_adaptive(c.ctx, p, ap, w, score, None, bi, bs)
        rk.rkn_synchronize(c.ctx)
        t3 = time.perf_counter() - t
        out[name]["ms_adaptive"] = round(t3 * 1e3, 3)
        out[name]["adaptive_speedup"] = round(dt / t3, 2)
        log(f"{name}: {out[name]}")
        c.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--events", type=int, default=512)
    ap.add_argument("--rkn-steps", type=int, default=6000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-refine", action="store_true", help="skip the refinement comparison")
    ap.add_argument("--no-other", action="store_true", help="skip the single-event workloads")
    ap.add_argument("--no-bidir", action="store_true", help="skip the two-direction scan")
    ap.add_argument("--no-adaptive", action="store_true", help="skip the adaptive-step batch")
    ap.add_argument("--turn-events", type=int, default=workloads.TURNS["n_events"],
                    help="multi-turn events of the turn-partition loop (0 = skip)")
    ap.add_argument("--block-steps", type=int, default=0, help="RKN steps per cull block (0 = default)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.empty(args.copy_calibration << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied {args.copy_calibration} MiB three times")
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the scan is measured on one GPU only (events shard across GPUs without any "
              "exchange between them); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    log(f"generating {args.events} events ...")
    t0 = time.time()
    geo = synth.make_geometry()
    field = synth.solenoid_field()
    events = synth.events_batch(geo, field, args.events, seed=0, n_steps=args.rkn_steps)
    off, wid, dr = synth.pack_events(events)
    log(f"  {wid.size} hits in {time.time() - t0:.1f} s")

    stream = torch.cuda.current_stream().cuda_stream
    ctx = rk.Context(0, stream)
    ctx.upload_geometry(geo)
    ctx.upload_field(field)
    ctx.upload_hits(off, wid, dr)
    lam = 64.0
    sp = rk.make_scan_params(n_steps=args.rkn_steps, precision=32, lambda_mm2=lam, block_steps=args.block_steps)
    hp = batch_hough_params(field)
    tune_ms = None
    if args.block_steps == 0:
        # untimed: the autotuner times each block size on the first events and leaves
        # the batch planned with the fastest
        chosen, tune_ms = rk.rkn_batch_autotune(ctx.ctx, hp, sp)
        sp.block_steps = chosen
        log(f"autotune: block sizes 4/6/8 -> {[round(v, 1) for v in tune_ms]} ms on the sample, chose {chosen}")
    else:
        rk.rkn_batch_plan(ctx.ctx, hp, sp)
    bsteps, tile = rk.rkn_scan_shape(ctx.ctx, sp)
    log(f"scan shape: {bsteps}-step blocks, {tile} seeds per tile ({tile // 64} waves)")
    ne = args.events
    bi = np.zeros(ne, np.int64); bs = np.zeros(ne)
    for i in range(args.warmup):
        rk.rkn_batch_launch(ctx.ctx, bi, bs)
        log(f"warmup {i}: {rk.rkn_batch_info(ctx.ctx)}")
    torch.cuda.synchronize()
    ms_h, ms_s = [], []
    t = time.perf_counter()
    for i in range(args.steps):
        rk.rkn_batch_launch(ctx.ctx, bi, bs)
        nw, ns, th, ts = rk.rkn_batch_info(ctx.ctx)
        ms_h.append(th); ms_s.append(ts)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    seed_steps = ns * args.rkn_steps
    value = seed_steps * args.steps / dt
    log(f"timed {args.steps} steps: {dt * 1e3 / args.steps:.1f} ms/step, {nw} windows, {ns} seeds, "
        f"hough {np.mean(ms_h):.2f} ms, scan {np.mean(ms_s):.2f} ms")

    windows, scores, _, ev_seed_off = rk.rkn_batch_results(ctx.ctx, ne)
    # untimed: the kernel's counting instance over the same windows gives the chord
    # distances it evaluates per seed-step (the work the roofline credits)
    k_steps, k_tests, k_chords = rk.rkn_scan_work_counts(ctx.ctx, sp, windows)
    q_kernel = k_chords / k_steps
    log(f"kernel work counts: {k_steps} seed-steps, {k_tests} sphere tests, {k_chords} chord distances "
        f"(q = {q_kernel:.4f} per seed-step)")
    cpu = None
    work = None
    if not args.no_cpu_baseline:
        cpu, work = cpu_baseline_leg(geo, field, events, windows, ev_seed_off, scores, args.rkn_steps,
                                     lam, args.cpu_seconds)
        log(f"cpu baseline: {cpu}")
        log(f"band-rule work and sample parity: {work}")
    bwaves = tile // 64
    f_alg = flops.per_seed_step("rz", q_kernel)
    achieved = f_alg * seed_steps / (np.mean(ms_s) * 1e-3) / 1e12
    roof = dict(bound="alu", achieved=round(achieved, 3), peak=flops.PEAK_FP32_TFLOPS, unit="TFLOP/s",
                frac=round(achieved / flops.PEAK_FP32_TFLOPS, 4), traffic=measured_traffic(),
                frac_unpacked_fp32=round(achieved / flops.PEAK_FP32_UNPACKED_TFLOPS, 4),
                flops_per_seed_step=round(f_alg, 2), q_kernel=round(q_kernel, 5),
                sphere_tests_per_seed_step=round(k_tests / k_steps, 5),
                kernel=f"scan_kernel<float, rz field, {bsteps}-step blocks, {bwaves} waves>")
    if work is not None:
        # the band rule's (chord, hit) pairs per seed-step, as the oracle counts them
        roof["hbar_c11"] = round(work["hbar_c11"], 4)
        roof["flops_per_seed_step_c11"] = round(flops.per_seed_step("rz", work["hbar_c11"]), 2)
    out = {
        "metric": METRIC, "value": value, "unit": "seed-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{ne} events, 1-3 e- with p~U[60,105] MeV/c, 40-300 hits with 10-40% noise, "
                               f"65x129 (r,z) solenoid map, circle-Hough windows (1e3-1e5 seeds/event), "
                               f"{args.rkn_steps} RKN steps of 1 mm, FP64 scores and argmin",
                   "n_events": ne, "n_seeds": int(ns), "n_windows": int(nw), "rkn_steps": args.rkn_steps,
                   "lambda_mm2": lam, "block_steps": bsteps, "seeds_per_tile": tile,
                   "block_steps_autotuned_ms": None if tune_ms is None else [round(v, 2) for v in tune_ms]},
        "events_per_s": ne * args.steps / dt,
        "ms_hough": float(np.mean(ms_h)), "ms_scan": float(np.mean(ms_s)),
        "roofline": roof, "cpu_baseline": cpu,
    }
    if work is not None:
        out["sample_max_rel_score_err"] = work["sample_max_rel_score_err"]
    if not args.no_refine:
        out["refine"] = refine_leg(ctx, sp, ne, dt / args.steps)
        log(f"refine: {out['refine']}")
    if not args.no_bidir:
        out["bidirectional"] = bidirectional_leg(ctx, field, sp, ne, dt / args.steps, int(np.diff(off).max()))
    if not args.no_adaptive:
        out["adaptive_batch"] = adaptive_batch_leg(ctx, hp, sp, ne, dt / args.steps)
    ctx.close()
    if args.turn_events > 0:
        out["turn_partitions"] = turns_leg(geo, field, args.turn_events)
    if not args.no_other:
        out["other_workloads"] = other_workloads(geo)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
