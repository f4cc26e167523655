"""The scale workload: 1,000,000 Gaussians in a 40 x 40 x 4 m box (log-scales
N(-1.0, 0.5^2)), 90 x 360 grid, MLP radiance.

* Training step over 512 receivers as RX-mode views (forward with saved
  state, L2 loss, hand-written backward): the loss gradient is kept on one
  sampled receiver, so the oracle's reverse mode over that receiver alone is
  the exact reference for every gradient (1e-4 of each tensor's largest
  entry), and its spectrum is checked against the oracle's.
* Coverage map of 4,096 receivers of one transmitter streamed in receiver
  chunks (default budget: half the free device memory), a sampled receiver
  against the oracle, and the same map in at least four chunks against it.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_24290_amd import scenes as S

from .parity import compare_spectra, gpu, needs_gpu, renderer_for

pytestmark = [gpu, needs_gpu]

FIELDS_MLP = ["means", "log_scales", "quats", "logits", "features", "mlp"]


def _threads():
    return len(os.sched_getaffinity(0))


def test_scale_training_step_rx_sampled():
    import torch
    from paper_2605_24290_amd import rxgs
    wl = S.make_workload("c4")
    N = wl.rx.shape[0]
    j = 7
    print(f"[scale] {wl.scene.K} Gaussians, {N} RX views, loss on receiver {j}", flush=True)
    r = renderer_for(wl)
    dev = torch.device("cuda", 0)
    rx = torch.as_tensor(wl.rx, device=dev)
    saved = rxgs.Saved(r)
    C, P, _ = r.render(rx, mode="rx", saved=saved)
    Y = torch.as_tensor(wl.targets[j], device=dev)
    dC = torch.zeros_like(C)
    dC[j] = 2.0 * (C[j] - Y)
    g = r.backward(saved, C, dC, None)
    torch.cuda.synchronize()
    gg = {k: v.cpu().numpy().astype(np.float64) for k, v in g.items()}
    Cj = C[j:j + 1].cpu().numpy()
    info = saved.info()
    print(f"[scale] pairs {info['D']}, visible {info['n_visible']}", flush=True)
    saved.close()
    r.close()
    rxs = wl.rx[[j]]
    cen, rv = O.views_for("rx", wl.tx, rxs)
    ora = O.render(wl.scene, wl.grid, cen, rxs, rv, mlp=wl.mlp, nthreads=_threads())
    compare_spectra(Cj, ora, max_flagged=1e-2)
    dCo = 2.0 * (ora["C"] - wl.targets[[j]])
    go = O.backward(wl.scene, wl.grid, cen, rxs, rv, dCo, None, mlp=wl.mlp, nthreads=_threads())
    worst = {}
    for f in FIELDS_MLP:
        a, b = gg[f].ravel(), go[f].ravel()
        worst[f] = float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
    print("[scale grad parity]", {k: f"{v:.2e}" for k, v in worst.items()})
    for f, e in worst.items():
        assert e <= 1e-4, f"{f}: {e:.3e}"


def test_scale_coverage_map_chunked():
    import torch
    wl = S.make_workload("c4", N=4096, targets=False)
    N = wl.rx.shape[0]
    print(f"[scale] coverage: {wl.scene.K} Gaussians, {N} receivers of one transmitter", flush=True)
    r = renderer_for(wl)
    dev = torch.device("cuda", 0)
    rx = torch.as_tensor(wl.rx, device=dev)
    tx = torch.as_tensor(wl.tx, device=dev)
    C, P, n1 = r.render_chunked(rx, tx=tx, mode="tx")
    from paper_2605_24290_amd import rxgs
    budget = rxgs.workspace_estimate("tx", 1, N // 4, wl.scene.K, wl.grid.H, wl.grid.W)
    C4, P4, n4 = r.render_chunked(rx, tx=tx, mode="tx", budget_bytes=budget)
    scale = C.abs().reshape(N, -1).amax(dim=1).clamp_min(1e-30)
    err = (C - C4).abs().reshape(N, -1).amax(dim=1) / scale
    worst = float(err.max().cpu())
    print(f"[scale] coverage chunks {n1} and {n4}; worst difference {worst:.2e}", flush=True)
    assert n4 >= 4 and worst <= 1e-6
    assert float((P - P4).abs().max().cpu()) <= 1e-6 * float(P.abs().max().cpu())
    j = 1000
    Cj = C[j:j + 1].cpu().numpy()
    Pj = P[j:j + 1].cpu().numpy()
    r.close()
    rxs = wl.rx[[j]]
    cen, rv = O.views_for("tx", wl.tx, rxs)
    ora = O.render(wl.scene, wl.grid, cen, rxs, rv, mlp=wl.mlp, nthreads=_threads())
    compare_spectra(Cj, ora, max_flagged=1e-2)
    assert np.abs(Pj - ora["power"]).max() <= 1e-4 * np.abs(ora["power"]).max()
