"""The allocation-free window scan (rkn_scan_windows_noalloc) through the C ABI: the
same scores, n_in and per-event best as rkn_scan_windows on two calls in a row, the
second smaller, with no device allocation during the calls."""
import numpy as np
import pytest

from paper_1908_01949_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rk():
    from paper_1908_01949_amd import rknscan
    rknscan.load_library()
    return rknscan


def _run_both(rk, c, windows, n_events, precision):
    import torch
    dev = torch.device("cuda", 0)
    total = int(sum(int(np.prod(w["count"].astype(np.int64))) for w in windows))
    p = rk.make_scan_params(n_steps=2000, precision=precision)
    ref = (np.zeros(total), np.zeros(total, np.int32), np.zeros(n_events, np.int64), np.zeros(n_events))
    rk.rkn_scan_windows(c.ctx, p, windows, *ref)
    pd = rk.make_scan_params(n_steps=2000, precision=precision, ptr_flags=rk.RKN_PTR_DEVICE)
    out = (torch.full((total,), -1.0, dtype=torch.float64, device=dev),
           torch.full((total,), -1, dtype=torch.int32, device=dev),
           torch.full((n_events,), -7, dtype=torch.int64, device=dev),
           torch.full((n_events,), -1.0, dtype=torch.float64, device=dev))
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info(0)[0]
    rk.rkn_scan_windows_noalloc(c.ctx, pd, windows, *out)
    rk.rkn_synchronize(c.ctx)
    free1 = torch.cuda.mem_get_info(0)[0]
    got = tuple(x.cpu().numpy() for x in out)
    return ref, got, free0 - free1


@pytest.mark.parametrize("precision", [32, 64])
def test_noalloc_equals_scan_windows_twice(rk, geo, sfield, precision):
    evs = synth.events_batch(geo, sfield, 6, seed=5)
    off, wid, dr = synth.pack_events(evs)
    c = rk.Context(0)
    c.upload_geometry(geo); c.upload_field(sfield); c.upload_hits(off, wid, dr)
    hw = [0.03, 30.0, 4.0, 4.0, 4.0]
    big = synth.make_windows([(e, j, evs[e].truth_seeds[0] + 0.01 * j, hw, [5, 4, 4, 4, 5])
                              for e in range(6) for j in range(2)])
    small = synth.make_windows([(1, 0, evs[1].truth_seeds[0], hw, [3, 3, 3, 3, 3]),
                                (4, 0, evs[4].truth_seeds[0], hw, [2, 3, 2, 3, 2])])
    for windows in (big, small):
        ref, got, used = _run_both(rk, c, windows, 6, precision)
        for a, b in zip(ref, got):
            assert np.array_equal(a, b)
        assert used == 0
    # events without windows in the small call: no best seed
    assert got[2][0] == -1 and np.isinf(got[3][0])
    # host outputs are refused; so is a request whose tiles do not fit the work array
    with pytest.raises(rk.RknError) as e:
        rk.rkn_scan_windows_noalloc(c.ctx, rk.make_scan_params(n_steps=10), small, None, None,
                                    np.zeros(6, np.int64), np.zeros(6))
    assert e.value.status == rk.RKN_E_ARG
    import torch
    huge = synth.make_windows([(0, 0, evs[0].truth_seeds[0], hw, [64, 64, 64, 64, 64])] * 4)
    bi = torch.zeros(6, dtype=torch.int64, device="cuda"); bs = torch.zeros(6, dtype=torch.float64, device="cuda")
    with pytest.raises(rk.RknError) as e:
        rk.rkn_scan_windows_noalloc(c.ctx, rk.make_scan_params(n_steps=10, ptr_flags=rk.RKN_PTR_DEVICE), huge,
                                    None, None, bi, bs)
    assert e.value.status == rk.RKN_E_CAPACITY
    c.close()
