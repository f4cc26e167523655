"""The deterministic backward (rxgs_set_deterministic) through the C ABI: two
backwards of one saved state, and a backward of a second saved render of the
same inputs, give the same bits in every gradient; the gradients match the
FP64 oracle's reverse mode within 1e-4 (per tensor, max error over max) and
the float-atomic backward within 1e-5; the accumulating form adds.  Cases:
direct radiance in both view modes, the training step's MLP subset, a TX view
of 20 receivers (blocks of 4 receivers, two receiver groups per work item),
several transmitters, and a grid of more than 255 tiles (pairs sorted by
tile in two passes instead of placed directly)."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_24290_amd import scenes as S

from .parity import gpu, needs_gpu, renderer_for
from .test_gpu_backward import FIELDS_DIRECT, FIELDS_MLP, _compare

pytestmark = [gpu, needs_gpu]


def _run(wl, mode, dC, dP=None, rx_off=None, det=True, repeats=2):
    import torch
    from paper_2605_24290_amd import rxgs
    r = renderer_for(wl)
    r.deterministic(det)
    out = []
    for _ in range(repeats):
        saved = rxgs.Saved(r)
        C, P, _ = r.render(wl.rx, tx=wl.tx, rx_off=rx_off, mode=mode, saved=saved)
        dC_t = torch.as_tensor(dC, dtype=torch.float32, device=C.device)
        dP_t = None if dP is None else torch.as_tensor(dP, dtype=torch.float32, device=C.device)
        g1 = r.backward(saved, C, dC_t, dP_t)
        g1 = {k: v.clone() for k, v in g1.items()}
        if det:   # (the float-atomic backward may differ in the last bits)
            g2 = r.backward(saved, C, dC_t, dP_t)
            torch.cuda.synchronize()
            for k in g1:
                assert torch.equal(g1[k], g2[k]), f"{k}: a second backward of one state differs"
        out.append(g1)
        saved.close()
    if repeats > 1:
        for k in out[0]:
            assert torch.equal(out[0][k], out[1][k]), f"{k}: a second saved render's backward differs"
    r.close()
    return {k: v.cpu().numpy().astype(np.float64) for k, v in out[0].items()}


def _check(wl, mode, dC, dP=None, rx_off=None, fields=FIELDS_MLP, rv=None):
    gd = _run(wl, mode, dC, dP, rx_off)
    ga = _run(wl, mode, dC, dP, rx_off, det=False, repeats=1)
    if rv is None:
        cen, rv = O.views_for(mode, wl.tx, wl.rx)
    else:
        cen = wl.tx.astype(np.float64)
    go = O.backward(wl.scene, wl.grid, cen, wl.rx, rv, dC, dP, mlp=wl.mlp)
    _compare(gd, go, fields)
    worst = {}
    for f in fields:
        scale = max(np.abs(ga[f]).max(), 1e-30)
        worst[f] = np.abs(gd[f] - ga[f]).max() / scale
        assert worst[f] <= 1e-5, (f, worst[f])
    print("[det vs atomic]", {k: f"{v:.1e}" for k, v in worst.items()})


@pytest.mark.parametrize("mode", ["tx", "rx"])
def test_deterministic_direct_radiance(mode):
    wl = S.make_workload("c0", K=600, N=4)
    rng = np.random.default_rng(21)
    dC = rng.normal(size=(4, 2, wl.grid.H, wl.grid.W)).astype(np.float32)
    dP = rng.normal(size=(4,)).astype(np.float32)
    _check(wl, mode, dC, dP, fields=FIELDS_DIRECT)


@pytest.mark.parametrize("mode", ["tx", "rx"])
def test_deterministic_mlp_training_subset(mode):
    full = S.make_workload("c2", K=100_000, N=32)
    sc = full.scene
    sub = S.Scene(sc.means[:256], sc.log_scales[:256], sc.quats[:256], sc.logits[:256], features=sc.features[:256])
    wl = S.Workload(sub, full.tx, full.rx[:8], full.grid, full.mlp, full.targets[:8], name="c2-subset")
    rng = np.random.default_rng(22)
    dC = rng.normal(size=(8, 2, wl.grid.H, wl.grid.W)).astype(np.float32)
    _check(wl, mode, dC)


def test_deterministic_many_receivers_and_transmitters():
    grid = S.Grid(45, 90, -math.pi / 2, math.pi / 45)
    wl = S.make_workload("c1", K=1500, N=23, Q=2, grid=grid)
    rng = np.random.default_rng(23)
    dC = rng.normal(size=(23, 2, grid.H, grid.W)).astype(np.float32)
    dP = rng.normal(size=(23,)).astype(np.float32)
    rv = np.array([0] * 20 + [1] * 3, dtype=np.int32)
    _check(wl, "tx", dC, dP, rx_off=[0, 20, 23], rv=rv)


def test_deterministic_two_pass_pair_sort():
    """A 4 deg x 1 deg grid of 23 x 45 = 1035 tiles: the pairs are emitted
    and sorted by tile in two passes (grids over 255 tiles), and the
    deterministic backward's partials sit at the pairs' emission slots, which
    it derives from each entry's first slot and the tile's rank in its
    rectangle, whatever order the sort left."""
    grid = S.Grid(90, 720, 0.0, math.pi / 180)
    wl = S.make_workload("c1", K=800, N=2, grid=grid)
    rng = np.random.default_rng(24)
    dC = rng.normal(size=(2, 2, grid.H, grid.W)).astype(np.float32)
    _check(wl, "rx", dC)


def test_deterministic_accumulate_adds():
    import torch
    from paper_2605_24290_amd import rxgs
    wl = S.make_workload("c0", K=500, N=3)
    r = renderer_for(wl)
    r.deterministic(True)
    saved = rxgs.Saved(r)
    C, _, _ = r.render(wl.rx, tx=wl.tx, mode="rx", saved=saved)
    dC = torch.ones_like(C)
    g = r.backward(saved, C, dC)
    g1 = {k: v.clone() for k, v in g.items()}
    g2 = r.backward(saved, C, dC, grads=g, accumulate=True)
    torch.cuda.synchronize()
    for k in g1:
        a, b = g2[k].cpu().numpy(), 2.0 * g1[k].cpu().numpy()
        assert np.abs(a - b).max() <= 1e-6 * max(np.abs(b).max(), 1e-30), k
    saved.close()
    r.close()
