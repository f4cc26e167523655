"""GPU checks of the boundary's optional outputs and modes, through the C ABI.

* Amplitude output (App. E.2: |R| = sqrt(Re^2 + Im^2 + 1e-8)) against the
  oracle's spectrum, and its gradient (dL/damp) against the oracle's reverse
  mode fed the same loss through the chain rule.
* Accumulating backward: two backwards added into one set of buffers equal
  the sum of two overwriting ones.
* The radix sort's look-back fallback (the path a bounded wait takes when it
  expires), forced from the host, gives the same order bit for bit.
* The torch.autograd.Function: torch.autograd.backward through one render and
  through two renders of one scene summed into one loss (c2 subset: 256
  Gaussians, 8 receivers), against Renderer.backward and the oracle.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_24290_amd import scenes as S

from .parity import FLAG_MARGIN, compare_spectra, gpu, needs_gpu, oracle_render, renderer_for

pytestmark = [gpu, needs_gpu]

FIELDS_MLP = ["means", "log_scales", "quats", "logits", "features", "mlp"]


def _rel(a, b):
    return float(np.abs(np.asarray(a, np.float64) - b).max() / max(np.abs(b).max(), 1e-30))


def _subset_c2(n_rx=8, K=256):
    full = S.make_workload("c2", K=100_000, N=32)
    sc = full.scene
    sub = S.Scene(sc.means[:K], sc.log_scales[:K], sc.quats[:K], sc.logits[:K], features=sc.features[:K])
    return S.Workload(sub, full.tx, full.rx[:n_rx], full.grid, full.mlp, full.targets[:n_rx], name="c2-subset")


@pytest.mark.parametrize("mode", ["tx", "rx"])
def test_amplitude_output_and_gradient(mode):
    import torch
    from paper_2605_24290_amd import rxgs
    wl = S.make_workload("c1", K=3000, N=6)
    r = renderer_for(wl)
    saved = rxgs.Saved(r)
    C, P, _, A = r.render(wl.rx, tx=wl.tx, mode=mode, saved=saved, want_amp=True)
    torch.cuda.synchronize()
    ora = oracle_render(wl, mode)
    Co = ora["C"]
    amp_o = np.sqrt(Co[:, 0] ** 2 + Co[:, 1] ** 2 + 1e-8)
    ok = ora["margin"] >= FLAG_MARGIN
    An = A.cpu().numpy()
    for j in range(An.shape[0]):
        err = np.abs(An[j] - amp_o[j]) / amp_o[j].max()
        assert err[ok[j]].max() <= 1e-4, (j, err[ok[j]].max())
    # the amplitude equals the formula on the GPU's own spectrum
    Cn = C.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(An, np.sqrt(Cn[:, 0] ** 2 + Cn[:, 1] ** 2 + 1e-8), rtol=2e-7, atol=1e-12)
    # loss = sum(dA * amp): the GPU gets dA, the oracle gets the same loss as
    # dL/dC = dA C / amp (chain rule through its own spectrum)
    rng = np.random.default_rng(11)
    dA = rng.normal(size=An.shape).astype(np.float32)
    g = r.backward(saved, C, None, None, dA=torch.as_tensor(dA, device=C.device))
    torch.cuda.synchronize()
    dC_o = dA.astype(np.float64)[:, None] * Co / amp_o[:, None]
    cen, rv = O.views_for(mode, wl.tx, wl.rx)
    go = O.backward(wl.scene, wl.grid, cen, wl.rx, rv, dC_o, None, mlp=wl.mlp)
    for f in FIELDS_MLP:
        e = _rel(g[f].cpu().numpy(), go[f])
        assert e <= 1e-4, (f, e)
    saved.close()
    r.close()


def test_backward_accumulate_adds():
    import torch
    from paper_2605_24290_amd import rxgs
    wl = S.make_workload("c1", K=3000, N=4)
    r = renderer_for(wl)
    saved = rxgs.Saved(r)
    C, P, _ = r.render(wl.rx, tx=wl.tx, mode="rx", saved=saved)
    rng = np.random.default_rng(3)
    d1 = torch.as_tensor(rng.normal(size=tuple(C.shape)).astype(np.float32), device=C.device)
    d2 = torch.as_tensor(rng.normal(size=tuple(C.shape)).astype(np.float32), device=C.device)
    g1 = {k: v.clone() for k, v in r.backward(saved, C, d1).items()}
    g2 = {k: v.clone() for k, v in r.backward(saved, C, d2).items()}
    acc = {k: v.clone() for k, v in g1.items()}
    r.backward(saved, C, d2, grads=acc, accumulate=True)
    torch.cuda.synchronize()
    for k in g1:
        want = (g1[k].double() + g2[k].double()).cpu().numpy()
        got = acc[k].double().cpu().numpy()
        # float atomics in a different order: last bits only
        assert _rel(got, want) <= 1e-5, (k, _rel(got, want))
    saved.close()
    r.close()


def test_sort_lookback_fallback_is_exact(monkeypatch):
    """Every radix-sort tile after a segment's first counts its predecessors'
    digits directly (the expired-wait path); both sorts must give the same
    order, hence bit-identical outputs and exports."""
    import torch
    from paper_2605_24290_amd import rxgs
    wl = S.make_workload("c1", K=20_000, N=3)
    r = renderer_for(wl)

    def run():
        s = rxgs.Saved(r)
        C, P, _ = r.render(wl.rx, tx=wl.tx, mode="rx", saved=s)
        torch.cuda.synchronize()
        info = s.info()
        V, Kp, D, T = info["V"], info["K_pad"], info["D"], info["tiles"]
        ex = (s.export(rxgs.EXPORT_ORDER, np.int32, (V, Kp)), s.export(rxgs.EXPORT_NVIS, np.int32, (V,)),
              s.export(rxgs.EXPORT_PAIRS, np.int32, (D,)), s.export(rxgs.EXPORT_RANGES, np.uint32, (V * T, 2)))
        out = (C.cpu().numpy(), P.cpu().numpy(), info, ex)
        s.close()
        return out

    C0, P0, i0, e0 = run()
    monkeypatch.setenv("RXGS_SORT_SPIN_LIMIT", "-1")
    C1, P1, i1, e1 = run()
    monkeypatch.delenv("RXGS_SORT_SPIN_LIMIT")
    print("[sort fallback] tiles:", i0["n_sort_fallbacks"], "->", i1["n_sort_fallbacks"])
    assert i0["n_sort_fallbacks"] == 0
    assert i1["n_sort_fallbacks"] > 0
    nv = e0[1]
    assert np.array_equal(nv, e1[1])
    for v in range(len(nv)):
        assert np.array_equal(e0[0][v, :nv[v]], e1[0][v, :nv[v]])
    assert np.array_equal(e0[2], e1[2]) and np.array_equal(e0[3], e1[3])
    assert np.array_equal(C0, C1) and np.array_equal(P0, P1)
    r.close()


@pytest.mark.parametrize("mode", ["tx", "rx"])
def test_autograd_function_matches_backward_and_oracle(mode):
    import torch
    from paper_2605_24290_amd import rxgs
    from paper_2605_24290_amd.autograd import rx_render
    wl = _subset_c2()
    sc = wl.scene
    dev = torch.device("cuda", 0)
    leaves = {k: torch.tensor(np.asarray(v, np.float32), device=dev, requires_grad=True)
              for k, v in dict(means=sc.means, log_scales=sc.log_scales, quats=sc.quats, logits=sc.logits,
                               features=sc.features, mlp=S.flat_mlp(wl.mlp)).items()}
    rx = torch.tensor(wl.rx, device=dev)
    tx = torch.tensor(wl.tx, device=dev)
    Y = torch.tensor(wl.targets, device=dev)
    r = rxgs.Renderer(wl.grid)
    C, P = rx_render(r, leaves["means"], leaves["log_scales"], leaves["quats"], leaves["logits"],
                     leaves["features"], leaves["mlp"], rx, tx=tx, mode=mode)
    loss = ((C - Y) ** 2).sum()
    torch.autograd.backward(loss)
    got = {k: v.grad.detach().cpu().numpy().astype(np.float64) for k, v in leaves.items()}
    # the same through Renderer.backward
    r2 = renderer_for(wl)
    s2 = rxgs.Saved(r2)
    C2, _, _ = r2.render(wl.rx, tx=wl.tx, mode=mode, saved=s2)
    g2 = r2.backward(s2, C2, 2.0 * (C2 - Y))
    torch.cuda.synchronize()
    # the oracle's reverse mode of the same loss
    ora = oracle_render(wl, mode)
    cen, rv = O.views_for(mode, wl.tx, wl.rx)
    go = O.backward(sc, wl.grid, cen, wl.rx, rv, 2.0 * (ora["C"] - wl.targets), None, mlp=wl.mlp)
    for k in FIELDS_MLP:
        assert _rel(got[k], g2[k].double().cpu().numpy()) <= 1e-5, k
        assert _rel(got[k], go[k]) <= 1e-4, (k, _rel(got[k], go[k]))
    s2.close()
    r2.close()
    r.close()


def test_autograd_two_renders_one_loss():
    """Two transmitters' renders of one scene summed into one loss: the
    gradient is the sum of the two renders' oracle gradients."""
    import torch
    from paper_2605_24290_amd import rxgs
    from paper_2605_24290_amd.autograd import rx_render
    wl = _subset_c2(n_rx=6)
    sc = wl.scene
    dev = torch.device("cuda", 0)
    leaves = {k: torch.tensor(np.asarray(v, np.float32), device=dev, requires_grad=True)
              for k, v in dict(means=sc.means, log_scales=sc.log_scales, quats=sc.quats, logits=sc.logits,
                               features=sc.features, mlp=S.flat_mlp(wl.mlp)).items()}
    tx2 = np.stack([wl.tx[0], wl.rx[5]]).astype(np.float32)   # a second transmitter
    r = rxgs.Renderer(wl.grid)
    rx = torch.tensor(wl.rx[:5], device=dev)
    Y = torch.tensor(wl.targets[:5], device=dev)
    loss = 0.0
    for q in range(2):
        C, P = rx_render(r, leaves["means"], leaves["log_scales"], leaves["quats"], leaves["logits"],
                         leaves["features"], leaves["mlp"], rx, tx=torch.tensor(tx2[q:q + 1], device=dev), mode="tx")
        loss = loss + ((C - Y) ** 2).sum() + 0.5 * P.sum()
    torch.autograd.backward(loss)
    got = {k: v.grad.detach().cpu().numpy().astype(np.float64) for k, v in leaves.items()}
    want = {k: 0.0 for k in FIELDS_MLP}
    for q in range(2):
        cen, rv = O.views_for("tx", tx2[q:q + 1], wl.rx[:5])
        ora = O.render(sc, wl.grid, cen, wl.rx[:5], rv, mlp=wl.mlp)
        go = O.backward(sc, wl.grid, cen, wl.rx[:5], rv, 2.0 * (ora["C"] - wl.targets[:5]),
                        np.full(5, 0.5), mlp=wl.mlp)
        for k in FIELDS_MLP:
            want[k] = want[k] + go[k]
    for k in FIELDS_MLP:
        assert _rel(got[k], want[k]) <= 1e-4, (k, _rel(got[k], want[k]))
    r.close()


def test_caller_allocator_receives_every_device_byte():
    """A context made with allocator callbacks (PyTorch's caching allocator)
    takes all its device memory through them: scene, MLP, workspace, saved
    state and backward scratch.  The device's free memory shrinks by no more
    than what PyTorch reserved, and everything is handed back at the end."""
    import torch
    from paper_2605_24290_amd import rxgs
    wl = S.make_workload("c1", K=50_000, N=32)
    sc = wl.scene
    # load the library's kernels with an ordinary context first (code objects)
    r0 = renderer_for(S.make_workload("c1", K=2000, N=2))
    r0.render(S.make_workload("c1", K=2000, N=2).rx, mode="rx")
    r0.close()
    torch.cuda.synchronize()
    tensors = [torch.tensor(np.asarray(a, np.float32), device="cuda")
               for a in (sc.means, sc.log_scales, sc.quats, sc.logits, sc.features, S.flat_mlp(wl.mlp), wl.rx)]
    C = torch.empty((32, 2, wl.grid.H, wl.grid.W), device="cuda")
    P = torch.empty((32,), device="cuda")
    dC = torch.randn_like(C)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    res0 = torch.cuda.memory_reserved()
    al = rxgs.TorchAllocator()
    r = rxgs.Renderer(wl.grid, allocator=al)
    r.upload_scene(*tensors[:4], features=tensors[4])
    r.upload_mlp(tensors[5])
    saved = rxgs.Saved(r)
    r.render(tensors[6], mode="rx", saved=saved, out=(C, P))
    g = r.backward(saved, C, dC)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    res1 = torch.cuda.memory_reserved()
    used = free0 - free1
    grown = res1 - res0
    print(f"[allocator] {al.n_alloc} blocks, {al.live_bytes / 2**20:.1f} MiB live; device used "
          f"{used / 2**20:.1f} MiB, torch reserved +{grown / 2**20:.1f} MiB")
    assert al.n_alloc > 0 and al.live_bytes > (100 << 20)
    # the gradient tensors g come from torch too; the slack covers events and streams
    assert used <= grown + (16 << 20), (used, grown)
    saved.close()
    r.close()
    assert al.live_bytes == 0 and al.n_free == al.n_alloc
    del g
