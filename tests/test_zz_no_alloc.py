"""The allocation-free render entry point (rxgs_render_noalloc) through the C
ABI: its outputs equal rxgs_render's bit for bit (same kernels, same
workspace layout carved from the static scratch array) on two calls in a row,
the second with fewer receivers and views; no device buffer comes from the
context's allocator during the calls; a render too large for the array is
refused with E_OOM and a message naming the scratch region."""
import ctypes
import math

import numpy as np
import pytest

from paper_2605_24290_amd import scenes as S

from .parity import gpu, needs_gpu

pytestmark = [gpu, needs_gpu]


def _call_noalloc(r, rx, tx, mode, rx_off=None):
    import torch
    from paper_2605_24290_amd import rxgs
    L = rxgs.lib()
    rx_t = torch.as_tensor(np.asarray(rx, np.float32)).cuda().contiguous()
    N = rx_t.shape[0]
    H, W = r.grid.H, r.grid.W
    C = torch.full((N, 2, H, W), float("nan"), device="cuda")
    P = torch.full((N,), float("nan"), device="cuda")
    Sm = torch.full((N, 2), float("nan"), device="cuda")
    A = torch.full((N, H, W), float("nan"), device="cuda")
    m = rxgs.MODE_TX if mode == "tx" else rxgs.MODE_RX
    tx_t, Q, off = None, 0, None
    if m == rxgs.MODE_TX:
        tx_t = torch.as_tensor(np.asarray(tx, np.float32)).cuda().reshape(-1, 3).contiguous()
        Q = tx_t.shape[0]
        rx_off = [0, N] if rx_off is None else rx_off
        off = (ctypes.c_int32 * (Q + 1))(*rx_off)
    st = L.rxgs_render_noalloc(r._ctx, m, Q, None if tx_t is None else ctypes.c_void_p(tx_t.data_ptr()), off, N,
                               ctypes.c_void_p(rx_t.data_ptr()), ctypes.c_void_p(C.data_ptr()),
                               ctypes.c_void_p(P.data_ptr()), ctypes.c_void_p(Sm.data_ptr()),
                               ctypes.c_void_p(A.data_ptr()), r._stream())
    torch.cuda.synchronize()
    return st, C, P, Sm, A


def _reference(r, rx, tx, mode, rx_off=None):
    import torch
    C, P, Sm, A = r.render(rx, tx=tx, rx_off=rx_off, mode=mode, want_csum=True, want_amp=True)
    torch.cuda.synchronize()
    return C, P, Sm, A


@pytest.mark.parametrize("use_mlp", [False, True])
def test_noalloc_equals_render_twice(use_mlp):
    import torch
    from paper_2605_24290_amd import rxgs
    grid = S.Grid(45, 90, -math.pi / 2, math.pi / 45)
    wl = S.make_workload("c0", K=3000, N=6, Q=2, grid=grid, use_mlp=use_mlp)
    alloc = rxgs.TorchAllocator()
    r = rxgs.Renderer(grid, allocator=alloc)
    sc = wl.scene
    r.upload_scene(sc.means, sc.log_scales, sc.quats, sc.logits, radiance=sc.radiance, features=sc.features)
    if use_mlp:
        r.upload_mlp(S.flat_mlp(wl.mlp))
    calls = [("tx", wl.rx, wl.tx, [0, 4, 6]), ("rx", wl.rx[:3], None, None)]   # the second smaller
    refs = [_reference(r, rx, tx, mode, off) for mode, rx, tx, off in calls]
    n0, b0 = alloc.n_alloc, alloc.bytes_alloc
    for (mode, rx, tx, off), ref in zip(calls, refs):
        st, C, P, Sm, A = _call_noalloc(r, rx, tx, mode, off)
        assert st == 0, rxgs.lib().rxgs_last_error(r._ctx)
        for got, exp in zip((C, P, Sm, A), ref):
            assert torch.equal(got, exp), (mode, (got - exp).abs().max().item())
    assert (alloc.n_alloc, alloc.bytes_alloc) == (n0, b0), "the allocation-free calls allocated"
    r.close()


def test_noalloc_rejects_a_render_beyond_the_scratch():
    from paper_2605_24290_amd import rxgs
    wl = S.make_workload("c1", K=50_000, N=64)
    r = rxgs.Renderer(wl.grid)
    sc = wl.scene
    r.upload_scene(sc.means, sc.log_scales, sc.quats, sc.logits, features=sc.features)
    r.upload_mlp(S.flat_mlp(wl.mlp))
    st, C, P, _, _ = _call_noalloc(r, wl.rx, wl.tx, "rx")
    assert st == 2   # E_OOM
    assert b"scratch region exhausted" in rxgs.lib().rxgs_last_error(r._ctx)
    # a small render still works afterwards
    st, C, _, _, _ = _call_noalloc(r, wl.rx[:1], None, "rx")
    assert st == 0
    r.close()
