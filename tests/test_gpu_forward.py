"""GPU parity of the forward path against the FP64 oracle.

Bit-exact: FP32 depth keys, tile binning, the (view, tile, depth, index) pair
order and the tile ranges (re-derived by the oracle's integer binning from the
GPU's exported FP32 records).  Within 1e-4 (per-receiver max error over max
|C|): spectra, power, radiance.  Cases cover both view modes, ragged tiles, the
azimuth seam, the poles of a full-sphere grid, several transmitters with
uneven receiver counts (one with none), no Gaussians, zero-opacity Gaussians
and repeat determinism.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_24290_amd import scenes as S

from .parity import FLAG_MARGIN, compare_spectra, gpu, needs_gpu, oracle_render, renderer_for

pytestmark = [gpu, needs_gpu]

GRID_SMALL = S.Grid(45, 90, -math.pi / 2, math.pi / 45)     # 4 deg, full sphere, ragged tiles


def _wl(preset="c0", **kw):
    return S.make_workload(preset, **kw)


def _render(r, wl, mode, saved=None, rx=None, tx=None, rx_off=None):
    import torch
    rx = wl.rx if rx is None else rx
    tx = wl.tx if tx is None else tx
    C, P, Sm = r.render(rx, tx=tx, rx_off=rx_off, mode=mode, saved=saved, want_csum=True)
    torch.cuda.synchronize()
    return C.cpu().numpy(), P.cpu().numpy(), Sm.cpu().numpy()


def _check_binning(r, saved, wl, mode):
    from paper_2605_24290_amd import rxgs
    info = saved.info()
    V, Kp, K, D, T = info["V"], info["K_pad"], info["K"], info["D"], info["tiles"]
    ext = saved.export(rxgs.EXPORT_BIN, np.float32, (V, Kp, 4))[:, :K]
    keys = saved.export(rxgs.EXPORT_KEYS, np.uint32, (V, Kp))[:, :K]
    op = saved.export(rxgs.EXPORT_OPACITY, np.float32, (V, Kp))[:, :K]
    order = saved.export(rxgs.EXPORT_ORDER, np.int32, (V, Kp))
    nvis = saved.export(rxgs.EXPORT_NVIS, np.int32, (V,))
    pairs = saved.export(rxgs.EXPORT_PAIRS, np.int32, (D,))
    ranges = saved.export(rxgs.EXPORT_RANGES, np.uint32, (V * T, 2))
    # keys bit-exact against the oracle's FP32 key
    cen, _ = O.views_for(mode, wl.tx, wl.rx)
    kb, near, pr = O.project(wl.scene, wl.grid, cen)
    diff = np.argwhere(keys != kb)
    assert diff.size == 0, (diff[:5], keys[tuple(diff[:5].T)], kb[tuple(diff[:5].T)])
    # binning boxes within tolerance of the FP64 projection (visible ones):
    # centre, and the padded half-extents of the ellipse q <= 2 ln(255 o)
    # (R6: x 1.0001 + 0.01 px) from the oracle's projected covariance
    vis = ~near & (op >= np.float32(1 / 255))
    assert np.abs(ext[..., 0][vis] - pr[..., 0][vis]).max() < 1e-4 * wl.grid.W
    assert np.abs(ext[..., 1][vis] - pr[..., 1][vis]).max() < 1e-3
    assert np.abs(op[~near] - pr[..., 5][~near]).max() < 1e-6
    qmax = 2.0 * np.log(op.astype(np.float64) * 255.0)
    for ax, cov in ((2, 6), (3, 8)):
        want = np.sqrt(np.maximum(qmax * pr[..., cov], 0.0)) * 1.0001 + 0.01
        err = np.abs(ext[..., ax].astype(np.float64) - want)[vis]
        assert (err <= 2e-6 * want[vis] + 1e-5).all(), (ax, err.max())
    # the blend records at each sorted position: pixel position to 1e-5 px,
    # conic to 1e-5 of its largest coefficient, log2 opacity
    rec = saved.export(rxgs.EXPORT_RECORDS, np.float32, (V, Kp, 8)).astype(np.float64)
    l2e = 1.4426950408889634
    for v in range(V):
        n = int(nvis[v])
        k = order[v, :n]
        assert np.abs(rec[v, :n, 0] + rec[v, :n, 1] - pr[v, k, 0]).max(initial=0) <= 1e-5
        assert np.abs(rec[v, :n, 2] + rec[v, :n, 3] - pr[v, k, 1]).max(initial=0) <= 1e-5
        conic = np.stack([rec[v, :n, 4] / (-0.5 * l2e), rec[v, :n, 5] / -l2e, rec[v, :n, 6] / (-0.5 * l2e)], axis=1)
        ref = pr[v, k, 2:5]
        scale = np.maximum(np.abs(ref[:, 0]), np.abs(ref[:, 2]))[:, None]
        assert (np.abs(conic - ref) <= 1e-5 * scale).all(), np.abs((conic - ref) / scale).max()
        assert np.abs(rec[v, :n, 7] - np.log2(pr[v, k, 5])).max(initial=0) <= 1e-6
    # pairs and order bit-exact against the oracle's integer binning
    seg, kk = O.bin_records(ext[..., 0], ext[..., 1], ext[..., 2], ext[..., 3], op, keys, wl.grid)
    assert seg.size == D
    v_of = pairs // Kp
    s_of = pairs % Kp
    assert (s_of < nvis[v_of]).all()
    g_k = order[v_of, s_of]
    assert np.array_equal(g_k, kk)
    assert np.array_equal(v_of, seg // T)
    # ranges: each segment's [start, end) covers exactly its pairs
    exp_rng = np.zeros((V * T, 2), dtype=np.int64)
    if D:
        u, first = np.unique(seg, return_index=True)
        last = np.r_[first[1:], D]
        exp_rng[u, 0] = first
        exp_rng[u, 1] = last
    assert np.array_equal(ranges.astype(np.int64), exp_rng)
    return info


@pytest.mark.parametrize("mode", ["tx", "rx"])
def test_c0_forward_parity(mode):
    """1,024 Gaussians, 4 receivers, 90 x 180 at 2 degrees, direct radiance."""
    from paper_2605_24290_amd import rxgs
    wl = _wl("c0")
    r = renderer_for(wl)
    saved = rxgs.Saved(r)
    C, P, Sm = _render(r, wl, mode, saved=saved)
    info = _check_binning(r, saved, wl, mode)
    assert info["D"] > 0
    ora = oracle_render(wl, mode)
    worst, frac = compare_spectra(C, ora)
    scale = np.abs(ora["power"]).max()
    assert np.abs(P - ora["power"]).max() <= 1e-4 * scale
    # the coherent sum: per receiver within 1e-4 of the sum of |C| over its pixels
    # (the bound of summing errors of at most 1e-4 max|C| per pixel without cancellation)
    abs_sum = np.abs(ora["C"]).sum(axis=(2, 3))   # (N, 2): per receiver and channel
    assert (np.abs(Sm - ora["csum"]) <= 1e-4 * abs_sum).all()
    # transmittance and stop index agree with the oracle where not flagged
    Tg = saved.export(rxgs.EXPORT_TFINAL, np.float32, (info["V"] if mode == "tx" else info["N"], 90, 180))
    if mode == "rx":
        ok = ora["margin"] >= FLAG_MARGIN
        assert np.abs(Tg - ora["T_final"])[ok].max() < 1e-4
    r.close()


@pytest.mark.parametrize("mode", ["tx", "rx"])
def test_mlp_forward_parity_small(mode):
    """MLP radiance: 3,000 Gaussians, 8 receivers, 90 x 360 at 1 degree."""
    from paper_2605_24290_amd import rxgs
    wl = _wl("c1", K=3000, N=8)
    r = renderer_for(wl)
    saved = rxgs.Saved(r)
    C, P, _ = _render(r, wl, mode, saved=saved)
    info = _check_binning(r, saved, wl, mode)
    # radiance at each sorted position against the oracle MLP
    rad = saved.export(rxgs.EXPORT_RADIANCE, np.float32, (info["N"], info["K_pad"], 2))
    order = saved.export(rxgs.EXPORT_ORDER, np.int32, (info["V"], info["K_pad"]))
    nvis = saved.export(rxgs.EXPORT_NVIS, np.int32, (info["V"],))
    ref = O.radiance(wl.scene, wl.rx, mlp=wl.mlp)
    for j in range(info["N"]):
        v = 0 if mode == "tx" else j
        ks = order[v, :nvis[v]]
        got = rad[j, :nvis[v]]
        exp = ref[j, ks]
        assert np.abs(got - exp).max() <= 1e-5 * max(1.0, np.abs(exp).max())
    ora = oracle_render(wl, mode)
    compare_spectra(C, ora)
    assert np.abs(P - ora["power"]).max() <= 1e-4 * np.abs(ora["power"]).max()
    r.close()


@pytest.mark.parametrize("case", ["large_activations", "large_features", "tiny_w2", "tx_ragged_receivers"])
def test_mlp_radiance_ranges_and_items(case):
    """Split-FP16 MLP against the FP64 oracle MLP outside the usual ranges:
    layer-1 activations beyond the FP16 range (scaled path), features beyond it
    (stored layer-1 term instead of the in-kernel one), a W2 near the FP32
    subnormal range (FP32 fallback), and 37 receivers of one view (three
    receiver blocks per work item, the last one ragged)."""
    from paper_2605_24290_amd import rxgs
    N = 37 if case == "tx_ragged_receivers" else 6
    wl = _wl("c1", K=2500, N=N)
    if case == "large_activations":
        wl.mlp[0] = wl.mlp[0] * np.float32(2.0 ** 16)
    elif case == "large_features":   # beyond the FP16 range: the stored layer-1 term is used
        wl.scene.features = wl.scene.features * np.float32(2.0 ** 16)
    elif case == "tiny_w2":
        wl.mlp[2] = wl.mlp[2] * np.float32(2.0 ** -100)
        wl.mlp[3] = wl.mlp[3] + np.float32(2.0 ** -101)
    mode = "tx" if case == "tx_ragged_receivers" else "rx"
    r = renderer_for(wl)
    saved = rxgs.Saved(r)
    _render(r, wl, mode, saved=saved)
    info = saved.info()
    rad = saved.export(rxgs.EXPORT_RADIANCE, np.float32, (info["N"], info["K_pad"], 2))
    order = saved.export(rxgs.EXPORT_ORDER, np.int32, (info["V"], info["K_pad"]))
    nvis = saved.export(rxgs.EXPORT_NVIS, np.int32, (info["V"],))
    ref = O.radiance(wl.scene, wl.rx, mlp=wl.mlp)
    worst = 0.0
    for j in range(info["N"]):
        v = 0 if mode == "tx" else j
        ks = order[v, :nvis[v]]
        got = rad[j, :nvis[v]].astype(np.float64)
        exp = ref[j, ks]
        scale = max(np.abs(exp).max(), 1e-300)
        worst = max(worst, float(np.abs(got - exp).max() / scale))
    print(f"[mlp] {case}: worst radiance error {worst:.3e} of the largest value")
    assert worst <= 1e-5
    saved.close()
    r.close()


@pytest.mark.parametrize("case", ["one_tx", "several_tx", "tiny_w2", "large_activations"])
def test_lazy_tx_radiance_bit_identical(case):
    """TX mode without saved state evaluates the pair MLP only on the blocks of
    32 sorted positions that some pixel composites (marked by a weights-only
    pass over the view); spectra and power must equal, bit for bit, those of
    the saved render, which evaluates every visible position, and match the
    oracle."""
    from paper_2605_24290_amd import rxgs
    rx_off = None
    if case == "several_tx":   # 6 receivers (weights pass), none, 2 and 1 (all blocks live)
        wl = _wl("c1", K=3000, N=9, Q=4)
        rx_off = [0, 6, 6, 8, 9]
    else:
        wl = _wl("c1", K=3000, N=12)
    if case == "tiny_w2":
        wl.mlp[2] = wl.mlp[2] * np.float32(2.0 ** -100)
        wl.mlp[3] = wl.mlp[3] + np.float32(2.0 ** -101)
    elif case == "large_activations":
        wl.mlp[0] = wl.mlp[0] * np.float32(2.0 ** 16)
    r = renderer_for(wl)
    C0, P0, S0 = _render(r, wl, "tx", rx_off=rx_off)
    saved = rxgs.Saved(r)
    C1, P1, S1 = _render(r, wl, "tx", saved=saved, rx_off=rx_off)
    assert np.array_equal(C0, C1) and np.array_equal(P0, P1) and np.array_equal(S0, S1)
    if case == "several_tx":
        cen = wl.tx.astype(np.float64)
        rv = np.array([0] * 6 + [2] * 2 + [3], dtype=np.int32)
        ora = O.render(wl.scene, wl.grid, cen, wl.rx, rv, mlp=wl.mlp)
    else:
        ora = oracle_render(wl, "tx")
    compare_spectra(C0, ora)
    saved.close()
    r.close()


def test_several_transmitters_uneven_receivers():
    """Three transmitters with 3, 0 and 5 receivers in one launch (TX mode)."""
    wl = _wl("c1", K=2000, N=8, Q=3, grid=GRID_SMALL)
    r = renderer_for(wl)
    rx_off = [0, 3, 3, 8]
    C, P, _ = _render(r, wl, "tx", rx_off=rx_off)
    cen = wl.tx.astype(np.float64)
    rv = np.array([0, 0, 0, 2, 2, 2, 2, 2], dtype=np.int32)
    ora = O.render(wl.scene, wl.grid, cen, wl.rx, rv, mlp=wl.mlp)
    compare_spectra(C, ora)
    r.close()


def test_full_sphere_small_grid_rx_mode():
    """Full-sphere grid with ragged tiles (45 x 90), receivers as views."""
    wl = _wl("c0", K=3000, N=5, grid=GRID_SMALL)
    r = renderer_for(wl)
    C, P, _ = _render(r, wl, "rx")
    compare_spectra(C, oracle_render(wl, "rx"))
    r.close()


@pytest.mark.parametrize("mode", ["tx", "rx"])
def test_large_grid_two_pass_pair_sort(mode):
    """200 x 400 full-sphere grid: 13 x 25 = 325 tiles per view, so the pair
    sort takes two 8-bit passes and tile ranges come from the sorted keys."""
    from paper_2605_24290_amd import rxgs
    grid = S.Grid(200, 400, -math.pi / 2.0, math.pi / 200.0)
    wl = _wl("c0", K=700, N=3, grid=grid)
    r = renderer_for(wl)
    saved = rxgs.Saved(r)
    C, P, _ = _render(r, wl, mode, saved=saved)
    info = _check_binning(r, saved, wl, mode)
    assert info["tiles"] > 255
    compare_spectra(C, oracle_render(wl, mode))
    saved.close()
    r.close()


@pytest.mark.parametrize("mode", ["rx", "tx"])
def test_direct_binning_equals_pair_sort(mode, monkeypatch):
    """Grids of at most 255 tiles place each pair in its tile list directly
    (per-chunk tile counts from the first emission, a per-view scan, ranked
    placement); RXGS_PAIR_SORT=1 takes the emission plus stable pair sort
    instead.  At full c1 size (50k Gaussians, 64 receivers, 90 x 360) both
    give the same pairs, ranges and outputs, bit for bit."""
    from paper_2605_24290_amd import rxgs
    wl = _wl("c1")
    out = []
    for env in ("0", "1"):
        monkeypatch.setenv("RXGS_PAIR_SORT", env)
        r = renderer_for(wl)
        saved = rxgs.Saved(r)
        C, P, Sm = _render(r, wl, mode, saved=saved)
        info = saved.info()
        pairs = saved.export(rxgs.EXPORT_PAIRS, np.int32, (info["D"],))
        ranges = saved.export(rxgs.EXPORT_RANGES, np.uint32, (info["V"] * info["tiles"], 2))
        out.append((C, P, Sm, pairs, ranges))
        saved.close()
        r.close()
    (C0, P0, S0, p0, g0), (C1, P1, S1, p1, g1) = out
    assert p0.size > 200_000 and np.array_equal(p0, p1)
    assert np.array_equal(g0, g1)
    assert np.array_equal(C0, C1) and np.array_equal(P0, P1) and np.array_equal(S0, S1)


def test_no_gaussians_and_zero_opacity():
    import torch
    from paper_2605_24290_amd import rxgs
    wl = _wl("c0", K=600, N=3)
    r = renderer_for(wl)
    C0, P0, _ = _render(r, wl, "rx")
    # zero-opacity Gaussians change nothing, bit for bit
    sc = wl.scene
    rng = np.random.default_rng(3)
    extra = 300
    r.upload_scene(np.concatenate([sc.means, rng.uniform(0, 10, (extra, 3)).astype(np.float32)]),
                   np.concatenate([sc.log_scales, np.full((extra, 3), -1.0, np.float32)]),
                   np.concatenate([sc.quats, np.tile([[1, 0, 0, 0]], (extra, 1)).astype(np.float32)]),
                   np.concatenate([sc.logits, np.full(extra, -30.0, np.float32)]),
                   radiance=np.concatenate([sc.radiance, np.ones((extra, 2), np.float32)]))
    C1, P1, _ = _render(r, wl, "rx")
    assert np.array_equal(C0, C1) and np.array_equal(P0, P1)
    # no Gaussians at all: zero spectra, unit transmittance
    r.upload_scene(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32), np.zeros((0, 4), np.float32),
                   np.zeros((0,), np.float32), radiance=np.zeros((0, 2), np.float32))
    saved = rxgs.Saved(r)
    C2, P2, _ = _render(r, wl, "tx", saved=saved)
    assert not C2.any() and not P2.any()
    T = saved.export(rxgs.EXPORT_TFINAL, np.float32, (1, wl.grid.H, wl.grid.W))
    assert (T == 1).all()
    # no receivers: a no-op
    C3, P3, _ = r.render(np.zeros((0, 3), np.float32), tx=wl.tx, mode="tx")
    torch.cuda.synchronize()
    assert C3.shape[0] == 0
    r.close()


def test_repeat_is_bit_identical_and_receivers_permute():
    wl = _wl("c1", K=4000, N=6)
    r = renderer_for(wl)
    for mode in ("tx", "rx"):
        a = _render(r, wl, mode)
        b = _render(r, wl, mode)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        perm = np.array([4, 2, 0, 5, 1, 3])
        c = _render(r, wl, mode, rx=wl.rx[perm])
        assert np.array_equal(a[0][perm], c[0])
    r.close()


def test_invalid_arguments_raise():
    from paper_2605_24290_amd import rxgs
    wl = _wl("c0", K=50, N=2)
    r = renderer_for(wl)
    with pytest.raises(rxgs.RxgsError):
        r.render(wl.rx, tx=wl.tx, rx_off=[0, 3], mode="tx")
    bad = wl.scene.means.copy()
    bad[3, 1] = np.nan
    with pytest.raises(rxgs.RxgsError):
        r.upload_scene(bad, wl.scene.log_scales, wl.scene.quats, wl.scene.logits, radiance=wl.scene.radiance)
    r.close()


def test_saved_binning_exports_on_demand():
    """A saved state's binning boxes, raw keys and opacities are computed on
    their first export (from the saved view centres): equal on repeated
    exports and equal to those of a second saved render of the same batch;
    refused once the scene has changed before that first export."""
    from paper_2605_24290_amd import rxgs
    wl = _wl("c0", K=300, N=3)
    r = renderer_for(wl)
    s1, s2 = rxgs.Saved(r), rxgs.Saved(r)
    r.render(wl.rx, tx=wl.tx, mode="rx", saved=s1)
    r.render(wl.rx, tx=wl.tx, mode="rx", saved=s2)
    info = s1.info()
    V, Kp = info["V"], info["K_pad"]
    k1 = s1.export(rxgs.EXPORT_KEYS, np.uint32, (V, Kp))
    b1 = s1.export(rxgs.EXPORT_BIN, np.float32, (V, Kp, 4))
    assert np.array_equal(k1, s1.export(rxgs.EXPORT_KEYS, np.uint32, (V, Kp)))
    assert np.array_equal(k1, s2.export(rxgs.EXPORT_KEYS, np.uint32, (V, Kp)))
    assert np.array_equal(b1, s2.export(rxgs.EXPORT_BIN, np.float32, (V, Kp, 4)))
    assert np.array_equal(s1.export(rxgs.EXPORT_OPACITY, np.float32, (V, Kp)),
                          s2.export(rxgs.EXPORT_OPACITY, np.float32, (V, Kp)))
    # keys of real Gaussians are their FP32 squared distances (bit patterns)
    K = wl.scene.K
    assert np.isfinite(k1[:, :K].view(np.float32)).all()
    s3 = rxgs.Saved(r)
    r.render(wl.rx, tx=wl.tx, mode="rx", saved=s3)
    sc = wl.scene
    r.upload_scene(sc.means, sc.log_scales, sc.quats, sc.logits, radiance=sc.radiance)
    with pytest.raises(rxgs.RxgsError):
        s3.export(rxgs.EXPORT_BIN, np.float32, (V, Kp, 4))
    for s in (s1, s2, s3):
        s.close()
    r.close()
