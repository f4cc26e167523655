"""Coverage-map render streamed in receiver chunks (rxgs_render_chunked)
against one rxgs_render over all receivers: the same spectra and power per
receiver (1e-6 of the receiver's largest |C|: a chunk may change the
receiver's slot in its blend workgroup), several chunks, transmitters split
across chunks, and a budget below one receiver's workspace rejected."""
import math

import numpy as np
import pytest

from paper_2605_24290_amd import scenes as S

from .parity import gpu, needs_gpu, renderer_for

pytestmark = [gpu, needs_gpu]


@pytest.mark.parametrize("case", ["tx", "tx_three", "rx"])
def test_chunked_equals_single_render(case):
    import torch
    from paper_2605_24290_amd import rxgs
    Q = 3 if case == "tx_three" else 1
    N = 100 if case != "rx" else 40
    wl = S.make_workload("c1", K=5000, N=N, Q=Q)
    mode = "rx" if case == "rx" else "tx"
    rx_off = [0, 45, 45, 100] if case == "tx_three" else None
    r = renderer_for(wl)
    C0, P0, _ = r.render(wl.rx, tx=wl.tx, rx_off=rx_off, mode=mode)
    views = (Q if mode == "tx" else N)
    budget = rxgs.workspace_estimate(mode, min(views, 2), max(N // 4, 1), wl.scene.K, wl.grid.H, wl.grid.W)
    C1, P1, nch = r.render_chunked(wl.rx, tx=wl.tx, rx_off=rx_off, mode=mode, budget_bytes=budget)
    torch.cuda.synchronize()
    print(f"[chunked] {case}: {nch} chunks")
    assert nch >= 3
    a, b = C0.cpu().numpy(), C1.cpu().numpy()
    scale = np.abs(a).reshape(N, -1).max(axis=1)
    err = np.abs(a - b).reshape(N, -1).max(axis=1) / np.maximum(scale, 1e-30)
    assert err.max() <= 1e-6, err.max()
    p0, p1 = P0.cpu().numpy(), P1.cpu().numpy()
    assert np.abs(p0 - p1).max() <= 1e-6 * np.abs(p0).max()
    with pytest.raises(rxgs.RxgsError):
        r.render_chunked(wl.rx, tx=wl.tx, rx_off=rx_off, mode=mode, budget_bytes=1024)
    r.close()
