"""Python binding of librknscan (ctypes): argument marshalling only.

Every function here has the name of the C entry point it calls (include/rknscan.h)
and does no arithmetic of the scan; all work runs in the HIP kernels of
``lib/librknscan.so``. Arrays are numpy (host) or torch tensors (device: their
``data_ptr()`` is passed with ``RKN_PTR_DEVICE``). Importing this module on a
machine without the built library raises immediately: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "librknscan.so")

RKN_OK = 0
RKN_E_ARG = -1
RKN_E_STATE = -2
RKN_E_NOMEM = -3
RKN_E_DEVICE = -4
RKN_E_CAPACITY = -5
RKN_E_UNSUPPORTED = -6
RKN_PTR_DEVICE = 1
RKN_MAX_HITS_PER_EVENT = 512
RKN_MAX_LAYERS = 64
RKN_TOPK_MAX = 16

STATUS_NAMES = {0: "RKN_OK", -1: "RKN_E_ARG", -2: "RKN_E_STATE", -3: "RKN_E_NOMEM",
                -4: "RKN_E_DEVICE", -5: "RKN_E_CAPACITY", -6: "RKN_E_UNSUPPORTED"}


class RknError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class rkn_window(C.Structure):
    _fields_ = [("event", C.c_int32), ("candidate", C.c_int32), ("center", C.c_double * 5),
                ("half_width", C.c_double * 5), ("count", C.c_int32 * 5), ("pad", C.c_int32)]


class rkn_hough_params(C.Structure):
    _fields_ = [("n_xy", C.c_int32), ("n_r", C.c_int32), ("xy_half", C.c_double),
                ("r_min", C.c_double), ("r_max", C.c_double), ("min_votes", C.c_int32),
                ("max_cand", C.c_int32), ("R0", C.c_double), ("charge", C.c_double),
                ("b_ref", C.c_double), ("gran", C.c_double * 5), ("center_z", C.c_double),
                ("center_pz", C.c_double), ("count", C.c_int32 * 5), ("grow", C.c_int32 * 5),
                ("count_max", C.c_int32), ("pad", C.c_int32), ("max_seeds_window", C.c_int64)]


class rkn_scan_params(C.Structure):
    _fields_ = [("R0", C.c_double), ("charge", C.c_double), ("step_mm", C.c_double),
                ("lambda_mm2", C.c_double), ("n_steps", C.c_int32), ("precision", C.c_int32),
                ("ptr_flags", C.c_int32), ("block_steps", C.c_int32), ("turn_stop", C.c_int32),
                ("reserved", C.c_int32)]


class rkn_turn_params(C.Structure):
    _fields_ = [("half_width", C.c_double * 5), ("count", C.c_int32 * 5), ("gn_iters", C.c_int32),
                ("gn_scale", C.c_double * 5), ("lambda_classify_mm2", C.c_double),
                ("fine_half_width", C.c_double * 2), ("fine_count", C.c_int32 * 2), ("n_candidates", C.c_int32),
                ("min_hits", C.c_int32), ("max_turns", C.c_int32), ("max_extrap_steps", C.c_int32)]


RKN_TURNS_MAX = 16


class rkn_rescan_params(C.Structure):
    _fields_ = [("k", C.c_int32), ("grid", C.c_int32), ("max_rounds", C.c_int32), ("reserved", C.c_int32)]


def make_rescan_params(k=8, grid=6, max_rounds=10) -> rkn_rescan_params:
    return rkn_rescan_params(int(k), int(grid), int(max_rounds), 0)


class rkn_adaptive_params(C.Structure):
    _fields_ = [("tol_mm", C.c_double), ("h_min_mm", C.c_double), ("h_max_mm", C.c_double)]


def make_adaptive_params(tol_mm=1e-5, h_min_mm=0.25, h_max_mm=4.0) -> rkn_adaptive_params:
    return rkn_adaptive_params(tol_mm, h_min_mm, h_max_mm)


# Exported symbols and their ctypes signatures (the C header declares the same set).
_P = C.c_void_p
_SIGS = {
    "rkn_version": (C.c_char_p, []),
    "rkn_create": (C.c_int32, [C.c_int32, _P, C.POINTER(_P)]),
    "rkn_destroy": (None, [_P]),
    "rkn_last_error": (C.c_char_p, [_P]),
    "rkn_synchronize": (C.c_int32, [_P]),
    "rkn_upload_geometry": (C.c_int32, [_P, C.c_int32, _P, _P, _P, _P, _P, _P, _P, _P, C.c_int32, _P, _P]),
    "rkn_upload_field_uniform": (C.c_int32, [_P, C.c_double]),
    "rkn_upload_field_rz": (C.c_int32, [_P, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_double,
                                        C.c_double, _P, _P]),
    "rkn_upload_hits": (C.c_int32, [_P, C.c_int32, _P, _P, _P]),
    "rkn_hough_seed_windows": (C.c_int32, [_P, _P, C.c_int32, _P, _P]),
    "rkn_hough_accumulator": (C.c_int32, [_P, _P, C.c_int32, C.c_int32, _P]),
    "rkn_scan_windows": (C.c_int32, [_P, _P, C.c_int32, _P, _P, _P, _P, _P]),
    "rkn_scan_seeds": (C.c_int32, [_P, _P, C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "rkn_trace": (C.c_int32, [_P, _P, C.c_int64, _P, C.c_int32, _P, _P]),
    "rkn_batch_plan": (C.c_int32, [_P, _P, _P]),
    "rkn_batch_launch": (C.c_int32, [_P, _P, _P]),
    "rkn_batch_info": (C.c_int32, [_P, _P, _P, _P, _P]),
    "rkn_batch_results": (C.c_int32, [_P, C.c_int32, _P, _P, C.c_int64, _P, _P, _P]),
    "rkn_batch_topk": (C.c_int32, [_P, C.c_int32, _P, _P, _P]),
    "rkn_batch_autotune": (C.c_int32, [_P, _P, _P, C.c_int32, C.c_int32, _P, _P]),
    "rkn_scan_windows_topk": (C.c_int32, [_P, _P, C.c_int32, _P, C.c_int32, _P, _P, _P]),
    "rkn_scan_shape": (C.c_int32, [_P, _P, _P, _P]),
    "rkn_scan_work_counts": (C.c_int32, [_P, _P, C.c_int32, _P, _P]),
    "rkn_classify_hits": (C.c_int32, [_P, _P, C.c_int64, _P, _P, _P, _P]),
    "rkn_bidirectional_common": (C.c_int32, [_P, _P, C.c_int64, _P, _P, _P, _P, _P, _P]),
    "rkn_refine_setup": (C.c_int32, [_P, _P, C.c_int64, _P, _P, C.c_int32]),
    "rkn_refine_info": (C.c_int32, [_P, _P, _P, _P]),
    "rkn_residuals_fwd": (C.c_int32, [_P, _P, _P, _P]),
    "rkn_adjoint_bwd": (C.c_int32, [_P, _P, _P, _P, _P]),
    "rkn_gn_refine": (C.c_int32, [_P, C.c_int32, _P, _P, _P]),
    "rkn_neighbour_seeds": (C.c_int32, [_P, _P, C.c_int64, _P, C.c_int32, C.c_int32, _P, _P]),
    "rkn_find_turns": (C.c_int32, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "rkn_scan_windows_two_kernel": (C.c_int32, [_P, _P, C.c_int32, _P, _P, _P, _P, _P]),
    "rkn_scan_windows_adaptive": (C.c_int32, [_P, _P, _P, C.c_int32, _P, _P, _P, _P, _P]),
    "rkn_batch_plan_adaptive": (C.c_int32, [_P, _P, _P, _P]),
    "rkn_rescan_refine": (C.c_int32, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "rkn_scan_windows_noalloc": (C.c_int32, [_P, _P, C.c_int32, _P, _P, _P, _P, _P]),
}

_lib = None


def preload_hip_runtime() -> None:
    """Load the system HIP runtime by its bare name, process-wide, before torch.

    torch's HIP library asks for ``libamdhip64.so`` while this library asks for
    ``libamdhip64.so.7``; loading the runtime first under the bare name makes both
    bind to one copy. If torch is already imported, this library binds to torch's
    runtime through the shared soname instead. Either way one runtime serves both.
    """
    if "torch" not in sys.modules:
        C.CDLL("libamdhip64.so", mode=C.RTLD_GLOBAL)


def load_library(path: str = LIB_PATH):
    """Load librknscan.so; raise if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        preload_hip_runtime()
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with paper_1908_01949_amd/build.py "
                              "(the seed scan has no CPU fallback)")
        lib = C.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def exported_symbols() -> list[str]:
    return list(_SIGS)


def _ptr(a):
    """Pointer of a numpy array or torch tensor (None passes NULL)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


def _host(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _check(ctx, status):
    if status != RKN_OK:
        msg = load_library().rkn_last_error(ctx)
        raise RknError(status, msg.decode() if msg else "")


def rkn_version() -> str:
    return load_library().rkn_version().decode()


def rkn_create(device: int = 0, stream: int | None = None):
    out = _P()
    st = load_library().rkn_create(device, stream, C.byref(out))
    if st != RKN_OK:
        raise RknError(st, "rkn_create failed")
    return out


def rkn_destroy(ctx) -> None:
    load_library().rkn_destroy(ctx)


def rkn_last_error(ctx) -> str:
    return load_library().rkn_last_error(ctx).decode()


def rkn_synchronize(ctx) -> None:
    _check(ctx, load_library().rkn_synchronize(ctx))


def rkn_upload_geometry(ctx, mx, my, mz, ux, uy, uz, half_len, layer_of, layer_rmin, layer_rmax) -> None:
    a = [_host(v, np.float64) for v in (mx, my, mz, ux, uy, uz, half_len)]
    lo = _host(layer_of, np.int32)
    r0 = _host(layer_rmin, np.float64); r1 = _host(layer_rmax, np.float64)
    _check(ctx, load_library().rkn_upload_geometry(ctx, a[0].size, *[_ptr(v) for v in a], _ptr(lo),
                                                   r0.size, _ptr(r0), _ptr(r1)))


def rkn_upload_field_uniform(ctx, bz: float) -> None:
    _check(ctx, load_library().rkn_upload_field_uniform(ctx, float(bz)))


def rkn_upload_field_rz(ctx, r0, r1, z0, z1, br, bz) -> None:
    br = _host(br, np.float32); bz = _host(bz, np.float32)
    nz, nr = br.shape
    _check(ctx, load_library().rkn_upload_field_rz(ctx, nr, nz, float(r0), float(r1), float(z0), float(z1),
                                                   _ptr(br), _ptr(bz)))


def rkn_upload_hits(ctx, ev_off, wire_id, drift) -> None:
    off = _host(ev_off, np.int32); w = _host(wire_id, np.int32); d = _host(drift, np.float32)
    _check(ctx, load_library().rkn_upload_hits(ctx, off.size - 1, _ptr(off), _ptr(w), _ptr(d)))


def make_scan_params(R0=500.0, charge=-1.0, step_mm=1.0, lambda_mm2=64.0, n_steps=2000, precision=32,
                     ptr_flags=0, block_steps=0, turn_stop=0) -> rkn_scan_params:
    return rkn_scan_params(R0, charge, step_mm, lambda_mm2, n_steps, precision, ptr_flags, block_steps,
                           int(turn_stop), 0)


def make_hough_params(**kw) -> rkn_hough_params:
    d = dict(n_xy=256, n_r=64, xy_half=512.0, r_min=160.0, r_max=416.0, min_votes=6, max_cand=4,
             R0=500.0, charge=-1.0, b_ref=1.0, gran=(0.01, 50.0, 2.5, 2.5, 5.0), center_z=0.0,
             center_pz=0.0, count=(12, 12, 12, 12, 12), grow=(0, 0, 0, 0, 0), count_max=12,
             max_seeds_window=100000)
    d.update(kw)
    hp = rkn_hough_params()
    for k, v in d.items():
        if k in ("gran", "count", "grow"):
            arr = getattr(hp, k)
            for i in range(5):
                arr[i] = v[i]
        else:
            setattr(hp, k, v)
    return hp


def windows_to_c(windows) -> C.Array:
    """numpy structured windows (synth.WINDOW_DTYPE) -> rkn_window array."""
    arr = (rkn_window * max(len(windows), 1))()
    C.memmove(arr, np.ascontiguousarray(windows).ctypes.data, len(windows) * C.sizeof(rkn_window))
    return arr


def windows_from_c(arr, n):
    from paper_1908_01949_amd.synth import WINDOW_DTYPE
    out = np.zeros(n, WINDOW_DTYPE)
    C.memmove(out.ctypes.data, arr, n * C.sizeof(rkn_window))
    return out


def rkn_hough_seed_windows(ctx, hp: rkn_hough_params, max_windows: int = 4096):
    arr = (rkn_window * max(max_windows, 1))()
    n = C.c_int32()
    _check(ctx, load_library().rkn_hough_seed_windows(ctx, C.byref(hp), max_windows, arr, C.byref(n)))
    return windows_from_c(arr, n.value)


def rkn_hough_accumulator(ctx, hp: rkn_hough_params, event: int, out=None):
    if out is None:
        out = np.zeros(hp.n_xy * hp.n_xy * hp.n_r, np.uint32)
    flags = RKN_PTR_DEVICE if hasattr(out, "data_ptr") else 0
    _check(ctx, load_library().rkn_hough_accumulator(ctx, C.byref(hp), event, flags, _ptr(out)))
    return out


def rkn_scan_windows(ctx, p: rkn_scan_params, windows, score=None, n_in=None, best_index=None,
                     best_score=None):
    """Outputs: numpy arrays (host) or torch tensors (set p.ptr_flags = RKN_PTR_DEVICE)."""
    w = windows_to_c(windows)
    _check(ctx, load_library().rkn_scan_windows(ctx, C.byref(p), len(windows), w, _ptr(score), _ptr(n_in),
                                                _ptr(best_index), _ptr(best_score)))
    return score, n_in, best_index, best_score


def rkn_scan_windows_noalloc(ctx, p: rkn_scan_params, windows, score, n_in, best_index, best_score):
    """rkn_scan_windows with no allocation; outputs are device pointers (torch tensors)."""
    w = windows_to_c(windows)
    _check(ctx, load_library().rkn_scan_windows_noalloc(ctx, C.byref(p), len(windows), w, _ptr(score), _ptr(n_in),
                                                        _ptr(best_index), _ptr(best_score)))
    return score, n_in, best_index, best_score


def rkn_scan_work_counts(ctx, p: rkn_scan_params, windows):
    """(seed-steps, sphere tests, chord distances) of the scan of these windows, from
    the kernel's counting instance."""
    w = windows_to_c(windows)
    counts = np.zeros(3, np.int64)
    _check(ctx, load_library().rkn_scan_work_counts(ctx, C.byref(p), len(windows), w, _ptr(counts)))
    return tuple(int(v) for v in counts)


def rkn_scan_windows_two_kernel(ctx, p: rkn_scan_params, windows, score=None, n_in=None, best_index=None,
                                best_score=None):
    """rkn_scan_windows computed by the record-then-DCA kernels (same outputs)."""
    w = windows_to_c(windows)
    _check(ctx, load_library().rkn_scan_windows_two_kernel(ctx, C.byref(p), len(windows), w, _ptr(score), _ptr(n_in),
                                                           _ptr(best_index), _ptr(best_score)))
    return score, n_in, best_index, best_score


def rkn_scan_windows_adaptive(ctx, p: rkn_scan_params, ap: rkn_adaptive_params, windows, score=None, n_in=None,
                              best_index=None, best_score=None):
    """rkn_scan_windows with the adaptive step size (same outputs)."""
    w = windows_to_c(windows)
    _check(ctx, load_library().rkn_scan_windows_adaptive(ctx, C.byref(p), C.byref(ap), len(windows), w, _ptr(score),
                                                         _ptr(n_in), _ptr(best_index), _ptr(best_score)))
    return score, n_in, best_index, best_score


def rkn_scan_shape(ctx, p: rkn_scan_params):
    """(block_steps, seeds_per_tile) the scan uses for these parameters on the current hits."""
    b = C.c_int32(); t = C.c_int32()
    _check(ctx, load_library().rkn_scan_shape(ctx, C.byref(p), C.byref(b), C.byref(t)))
    return b.value, t.value


def rkn_scan_windows_topk(ctx, p: rkn_scan_params, windows, k, index=None, score=None, seeds5=None,
                          n_events=None):
    """k best seeds per event of a window scan; host outputs are allocated when None
    (n_events required then)."""
    if index is None:
        index = np.zeros((n_events, k), np.int64)
        score = np.zeros((n_events, k))
        seeds5 = np.zeros((n_events, k, 5))
    w = windows_to_c(windows)
    _check(ctx, load_library().rkn_scan_windows_topk(ctx, C.byref(p), len(windows), w, int(k), _ptr(index),
                                                     _ptr(score), _ptr(seeds5)))
    return index, score, seeds5


def rkn_scan_seeds(ctx, p: rkn_scan_params, seed_event, seeds5, score=None, n_in=None, best_index=None,
                   best_score=None):
    se = _host(seed_event, np.int32)
    s5 = np.asarray(seeds5, np.float64).reshape(-1, 5)
    cols = [np.ascontiguousarray(s5[:, d]) for d in range(5)]
    _check(ctx, load_library().rkn_scan_seeds(ctx, C.byref(p), se.size, _ptr(se), *[_ptr(c) for c in cols],
                                              _ptr(score), _ptr(n_in), _ptr(best_index), _ptr(best_score)))
    return score, n_in, best_index, best_score


def rkn_trace(ctx, p: rkn_scan_params, seeds5, step_idx, states=None):
    s5 = np.ascontiguousarray(np.asarray(seeds5, np.float64).reshape(-1, 5))
    st = _host(step_idx, np.int32)
    if states is None:
        states = np.zeros((s5.shape[0], st.size, 6))
    _check(ctx, load_library().rkn_trace(ctx, C.byref(p), s5.shape[0], _ptr(s5), st.size, _ptr(st),
                                         _ptr(states)))
    return states


def rkn_batch_plan(ctx, hp: rkn_hough_params, sp: rkn_scan_params) -> None:
    _check(ctx, load_library().rkn_batch_plan(ctx, C.byref(hp), C.byref(sp)))


def rkn_batch_autotune(ctx, hp: rkn_hough_params, sp: rkn_scan_params, sample_events: int = 64, reps: int = 2):
    """Plan the batch with the fastest block size; returns (block_steps, ms[3] for 4, 6, 8)."""
    chosen = C.c_int32()
    ms = (C.c_float * 3)()
    _check(ctx, load_library().rkn_batch_autotune(ctx, C.byref(hp), C.byref(sp), int(sample_events), int(reps),
                                                  C.byref(chosen), ms))
    return chosen.value, list(ms)


def rkn_batch_plan_adaptive(ctx, hp: rkn_hough_params, sp: rkn_scan_params, ap) -> None:
    _check(ctx, load_library().rkn_batch_plan_adaptive(ctx, C.byref(hp), C.byref(sp), C.byref(ap)))


def rkn_batch_launch(ctx, best_index=None, best_score=None):
    _check(ctx, load_library().rkn_batch_launch(ctx, _ptr(best_index), _ptr(best_score)))
    return best_index, best_score


def rkn_batch_topk(ctx, k, index=None, score=None, seeds5=None, n_events=None):
    if index is None:
        index = np.zeros((n_events, k), np.int64)
        score = np.zeros((n_events, k))
        seeds5 = np.zeros((n_events, k, 5))
    _check(ctx, load_library().rkn_batch_topk(ctx, int(k), _ptr(index), _ptr(score), _ptr(seeds5)))
    return index, score, seeds5


def rkn_rescan_refine(ctx, p: rkn_scan_params, rp: rkn_rescan_params, n_events: int, start5=None, step5=None,
                      target=None, out5=None, out_step5=None, out_score=None, rounds=None):
    """The coarse-to-fine rescans (start5/step5 None: from the last batch launch's k
    best). With host pointers, outputs are allocated when None and returned as
    (seeds5, steps5, scores, rounds)."""
    k = rp.k
    dev = bool(p.ptr_flags & 1)
    if not dev:
        if start5 is not None:
            start5 = np.ascontiguousarray(start5, np.float64).reshape(n_events, k, 5)
            step5 = np.ascontiguousarray(step5, np.float64).reshape(n_events, k, 5)
        if target is not None:
            target = np.ascontiguousarray(target, np.float64).reshape(n_events)
        out5 = np.zeros((n_events, k, 5)) if out5 is None else out5
        out_step5 = np.zeros((n_events, k, 5)) if out_step5 is None else out_step5
        out_score = np.zeros((n_events, k)) if out_score is None else out_score
        rounds = np.zeros(n_events, np.int32) if rounds is None else rounds
    _check(ctx, load_library().rkn_rescan_refine(ctx, C.byref(p), C.byref(rp), _ptr(start5), _ptr(step5),
                                                 _ptr(target), _ptr(out5), _ptr(out_step5), _ptr(out_score),
                                                 _ptr(rounds)))
    return out5, out_step5, out_score, rounds


def rkn_batch_info(ctx):
    """(n_windows, n_seeds, ms_hough, ms_scan) of the last batch launch."""
    nw = C.c_int32(); ns = C.c_int64(); th = C.c_float(); ts = C.c_float()
    _check(ctx, load_library().rkn_batch_info(ctx, C.byref(nw), C.byref(ns), C.byref(th), C.byref(ts)))
    return nw.value, ns.value, th.value, ts.value


def rkn_batch_results(ctx, n_events: int, want_scores: bool = True):
    """(windows, scores, n_in, ev_seed_off) of the last batch launch (host arrays)."""
    nw, ns, _, _ = rkn_batch_info(ctx)
    arr = (rkn_window * max(nw, 1))()
    score = np.zeros(max(ns, 1)) if want_scores else None
    nin = np.zeros(max(ns, 1), np.int32) if want_scores else None
    off = np.zeros(n_events + 1, np.int64)
    n = C.c_int32()
    _check(ctx, load_library().rkn_batch_results(ctx, nw, arr, C.byref(n), ns, _ptr(score), _ptr(nin),
                                                 _ptr(off)))
    return windows_from_c(arr, n.value), (score[:ns] if want_scores else None), \
        (nin[:ns] if want_scores else None), off


def rkn_classify_hits(ctx, p: rkn_scan_params, seed_event, seeds5, n_hits_max, mask=None, n_in=None):
    """Inlier masks [n][H] (uint8) and counts [n] of explicit seeds (host arrays if None)."""
    se = _host(seed_event, np.int32)
    s5 = np.ascontiguousarray(np.asarray(seeds5, np.float64).reshape(-1, 5))
    if mask is None and n_in is None:
        mask = np.zeros((se.size, n_hits_max), np.uint8)
        n_in = np.zeros(se.size, np.int32)
    _check(ctx, load_library().rkn_classify_hits(ctx, C.byref(p), se.size, _ptr(se), _ptr(s5), _ptr(mask),
                                                 _ptr(n_in)))
    return mask, n_in


def make_turn_params(half_width=(0.02, 40.0, 3.0, 3.0, 4.0), count=(5, 9, 5, 5, 9), gn_iters=5,
                     gn_scale=(1.0, 100.0, 100.0, 100.0, 100.0), lambda_classify_mm2=4.0,
                     fine_half_width=(300.0, 24.0), fine_count=(1, 1), n_candidates=8, min_hits=10,
                     max_turns=8, max_extrap_steps=6000) -> rkn_turn_params:
    """Defaults chosen on a separate sample of 128 multi-turn events (seed 2): no fine
    (z0, pz0) rescan (fine_count (1, 1)), 8 first-partition candidates, neighbour
    windows of +-(0.02 rad, 40 mm, 3, 3, 4 MeV/c), 5 Gauss-Newton iterations per fit
    (as good as 10 there, in 0.7 of the time)."""
    tp = rkn_turn_params()
    for i in range(5):
        tp.half_width[i] = half_width[i]
        tp.count[i] = count[i]
        tp.gn_scale[i] = gn_scale[i]
    for i in range(2):
        tp.fine_half_width[i] = fine_half_width[i]
        tp.fine_count[i] = fine_count[i]
    tp.n_candidates = n_candidates
    tp.gn_iters = gn_iters
    tp.lambda_classify_mm2 = lambda_classify_mm2
    tp.min_hits = min_hits
    tp.max_turns = max_turns
    tp.max_extrap_steps = max_extrap_steps
    return tp


def rkn_neighbour_seeds(ctx, p: rkn_scan_params, seeds5, direction, max_steps=6000, out5=None, found=None):
    """Seeds of the neighbouring turn partitions ([n][5]) and the found flags."""
    s5 = np.ascontiguousarray(np.asarray(seeds5, np.float64).reshape(-1, 5))
    n = s5.shape[0]
    if out5 is None:
        out5 = np.zeros((n, 5)); found = np.zeros(n, np.int32)
    _check(ctx, load_library().rkn_neighbour_seeds(ctx, C.byref(p), n, _ptr(s5), int(direction), int(max_steps),
                                                   _ptr(out5), _ptr(found)))
    return out5, found


def rkn_find_turns(ctx, hp: rkn_hough_params, sp: rkn_scan_params, tp: rkn_turn_params, n_hits_total, n_events):
    """The turn-partition loop; returns a dict of its outputs (host arrays)."""
    T = int(tp.max_turns)
    out = dict(hit_turn=np.zeros(n_hits_total, np.int32), n_turns=np.zeros(n_events, np.int32),
               turn_seed=np.zeros((n_events, T, 5)), turn_center=np.zeros((n_events, T, 5)),
               turn_pos=np.zeros((n_events, T), np.int32), turn_nhits=np.zeros((n_events, T), np.int32))
    _check(ctx, load_library().rkn_find_turns(ctx, C.byref(hp), C.byref(sp), C.byref(tp), _ptr(out["hit_turn"]),
                                              _ptr(out["n_turns"]), _ptr(out["turn_seed"]), _ptr(out["turn_center"]),
                                              _ptr(out["turn_pos"]), _ptr(out["turn_nhits"])))
    return out


def rkn_bidirectional_common(ctx, p: rkn_scan_params, pair_event, seeds_entry5, seeds_exit5, n_hits_max,
                             mask_entry=None, mask_exit=None, n_common=None):
    """Per pair: the entrance and exit masks and the number of hits in both."""
    se = _host(pair_event, np.int32)
    a = np.ascontiguousarray(np.asarray(seeds_entry5, np.float64).reshape(-1, 5))
    b = np.ascontiguousarray(np.asarray(seeds_exit5, np.float64).reshape(-1, 5))
    if n_common is None:
        mask_entry = np.zeros((se.size, n_hits_max), np.uint8)
        mask_exit = np.zeros((se.size, n_hits_max), np.uint8)
        n_common = np.zeros(se.size, np.int32)
    _check(ctx, load_library().rkn_bidirectional_common(ctx, C.byref(p), se.size, _ptr(se), _ptr(a), _ptr(b),
                                                        _ptr(mask_entry), _ptr(mask_exit), _ptr(n_common)))
    return mask_entry, mask_exit, n_common


def rkn_refine_setup(ctx, p: rkn_scan_params, seed_event, seeds5, ckpt_every: int = 64) -> None:
    se = _host(seed_event, np.int32)
    s5 = np.ascontiguousarray(np.asarray(seeds5, np.float64).reshape(-1, 5))
    _check(ctx, load_library().rkn_refine_setup(ctx, C.byref(p), se.size, _ptr(se), _ptr(s5), int(ckpt_every)))


def rkn_refine_info(ctx):
    """(n_seeds, ckpt_every, tune_ms[4]) of the current refinement setup."""
    n = C.c_int64(); k = C.c_int32(); ms = (C.c_float * 4)()
    _check(ctx, load_library().rkn_refine_info(ctx, C.byref(n), C.byref(k), ms))
    return n.value, k.value, list(ms)


def rkn_residuals_fwd(ctx, seeds5=None, resid=None, phi=None):
    s5 = None if seeds5 is None else (seeds5 if hasattr(seeds5, "data_ptr") else
                                      np.ascontiguousarray(np.asarray(seeds5, np.float64).reshape(-1, 5)))
    _check(ctx, load_library().rkn_residuals_fwd(ctx, _ptr(s5), _ptr(resid), _ptr(phi)))
    return resid, phi


def rkn_adjoint_bwd(ctx, d_resid=None, d_seed=None, JtJ=None, Jtr=None):
    dr = None if d_resid is None else (d_resid if hasattr(d_resid, "data_ptr") else _host(d_resid, np.float32))
    _check(ctx, load_library().rkn_adjoint_bwd(ctx, _ptr(dr), _ptr(d_seed), _ptr(JtJ), _ptr(Jtr)))
    return d_seed, JtJ, Jtr


def rkn_gn_refine(ctx, iters, scale, seeds_out=None, phi=None):
    sc = _host(scale, np.float64)
    _check(ctx, load_library().rkn_gn_refine(ctx, int(iters), _ptr(sc), _ptr(seeds_out), _ptr(phi)))
    return seeds_out, phi


class Context:
    """Convenience owner of an rkn_ctx (destroyed with the object)."""

    def __init__(self, device: int = 0, stream: int | None = None):
        self.ctx = rkn_create(device, stream)
        self.stream = stream

    def close(self):
        if getattr(self, "ctx", None) is not None:
            rkn_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def upload_geometry(self, geo):
        rkn_upload_geometry(self.ctx, geo.mx, geo.my, geo.mz, geo.ux, geo.uy, geo.uz, geo.half_len,
                            geo.layer_of, geo.layer_rmin, geo.layer_rmax)

    def upload_field(self, field):
        if field.kind == "uniform":
            rkn_upload_field_uniform(self.ctx, field.bz)
        else:
            rkn_upload_field_rz(self.ctx, field.r0, field.r1, field.z0, field.z1, field.br_grid, field.bz_grid)

    def upload_hits(self, ev_off, wire_id, drift):
        rkn_upload_hits(self.ctx, ev_off, wire_id, drift)
        off = np.asarray(ev_off)
        self.n_events = off.size - 1
        self.max_hits = int(np.diff(off).max(initial=0))
