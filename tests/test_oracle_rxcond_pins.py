"""Pins of the oracle's receiver-conditioned radiance (the paper's FiLM global
branch, occupancy-grid local branch and FLE / SH basis; Sec. 4.3.2, App. E.2,
App. E.5, Alg. 1 stage 2) against facts fixed by mathematics and by library
routines:

* the basis is orthonormal on the sphere (Gauss-Legendre x uniform-azimuth
  quadrature, exact for these band-limited products);
* the complex FLE basis is scipy's spherical harmonic up to the Condon-Shortley
  sign (-1)^m for m >= 0, and the real SH basis is built from it by the
  textbook real combinations;
* with both branches' final layers zero (the paper's initialisation) the
  radiance is the plain basis expansion of the base coefficients;
* a global final layer with zero weights and bias (alpha, beta) applies the
  affine map (1 + alpha) phi + beta to every component (eq. film_apply); a
  local one applies its per-Gaussian (alpha', beta') after it, the same for
  every component (eq. combined_local; App. E.5 "per-Gaussian scale and
  shift"), so beta' adds beta' sum_l B_l to the radiance;
* special weights that pass the inputs through the global MLP expose the
  receiver encoding (eq. rx_enc), the (degree, order) features and the
  embeddings, and through the local MLP its six inputs (eq. local);
* the occupancy grid of one or two Gaussians is 1 - prod (1 - o G) at the
  voxel centres within 2 sigma, 0 elsewhere (App. E.5), and each probe reads
  the voxel whose centre is nearest (found here by brute force over all
  centres), giving T = prod (1 - V) and the mean density of eq. (transmittance).
"""
import math

import numpy as np
import pytest
import scipy.special as sp

from oracle import oracle as O
from paper_2605_24290_amd import scenes as S

SQ2 = math.sqrt(2.0)


def _idx(l, m):
    return l * l + l + m


def _dirs(n_theta=24, n_phi=48):
    """Gauss-Legendre nodes in cos(theta) and uniform azimuths, with weights."""
    x, w = sp.roots_legendre(n_theta)
    ph = (np.arange(n_phi) + 0.5) * 2 * np.pi / n_phi
    th = np.arccos(x)
    T, PH = np.meshgrid(th, ph, indexing="ij")
    W = np.outer(w, np.full(n_phi, 2 * np.pi / n_phi))
    d = np.stack([np.sin(T) * np.cos(PH), np.sin(T) * np.sin(PH), np.cos(T)], axis=-1)
    return d.reshape(-1, 3), W.ravel(), T.ravel(), PH.ravel()


@pytest.mark.parametrize("kind,lmax", [(O.BASIS_FLE, 9), (O.BASIS_SH, 4), (O.BASIS_SH, 9)])
def test_basis_is_orthonormal(oracle_lib, kind, lmax):
    d, w, _, _ = _dirs()
    L = (lmax + 1) ** 2
    B = np.stack([O.basis(kind, lmax, di) for di in d])          # (n, L, 2)
    Z = B[..., 0] + 1j * B[..., 1]
    gram = (Z * w[:, None]).T @ Z.conj()
    assert np.abs(gram - np.eye(L)).max() < 1e-12


def test_fle_basis_is_scipy_spherical_harmonic(oracle_lib):
    """B_{l,m} = (-1)^m Y_l^m for m >= 0 and Y_l^m for m < 0 (scipy's Y_l^m
    carries the Condon-Shortley phase); low orders by hand: B_00 = 1/sqrt(4 pi),
    B_10 = sqrt(3/(4 pi)) cos(theta), B_11 = sqrt(3/(8 pi)) sin(theta) e^{i phi}."""
    d, _, th, ph = _dirs(7, 11)
    for di, t, p in zip(d, th, ph):
        B = O.basis(O.BASIS_FLE, 9, di)
        Z = B[:, 0] + 1j * B[:, 1]
        for l in range(10):
            for m in range(-l, l + 1):
                y = complex(sp.sph_harm_y(l, m, t, p))
                exp = (-1) ** m * y if m >= 0 else y
                assert abs(Z[_idx(l, m)] - exp) < 1e-12, (l, m)
        assert abs(Z[0] - 1 / math.sqrt(4 * math.pi)) < 1e-14
        assert abs(Z[_idx(1, 0)] - math.sqrt(3 / (4 * math.pi)) * math.cos(t)) < 1e-14
        assert abs(Z[_idx(1, 1)] - math.sqrt(3 / (8 * math.pi)) * math.sin(t) * np.exp(1j * p)) < 1e-14
        # the real SH basis: m = 0 as is, m > 0 sqrt2 Re, m < 0 sqrt2 Im of B_{l,|m|}
        R = O.basis(O.BASIS_SH, 9, di)
        assert np.abs(R[:, 1]).max() == 0.0
        for l in range(10):
            for m in range(-l, l + 1):
                zb = Z[_idx(l, abs(m))]
                exp = zb.real if m == 0 else (SQ2 * zb.real if m > 0 else SQ2 * zb.imag)
                assert abs(R[_idx(l, m), 0] - exp) < 1e-12


def _small_scene(K=6, seed=3):
    wl = S.make_workload(S.Preset("t", K, 2, (3.0, 3.0, 2.0), -1.2, 0.3, S.GRID_90x180, False), seed=seed)
    return wl


def _expand(model, coeffs, B):
    """sum_l phi_{l,c} B_l as a complex number per channel (phi, B complex)."""
    return (coeffs[..., 0] + 1j * coeffs[..., 1]).T @ (B[:, 0] + 1j * B[:, 1])


@pytest.mark.parametrize("kind", [O.BASIS_FLE, O.BASIS_SH])
def test_zero_final_layers_give_the_plain_basis_expansion(oracle_lib, kind):
    wl = _small_scene()
    m = S.make_rxcond_model(wl.scene.K, kind=kind, lmax=4, C=2, F=6, H=32, zero_final=True)
    cen = wl.tx.astype(np.float64)
    rad = O.rxcond_radiance(m, wl.scene, cen, wl.rx, [0, 0], occ=O.occupancy(wl.scene, 16))
    for j in range(2):
        for k in range(wl.scene.K):
            B = O.basis(kind, 4, wl.scene.means[k].astype(np.float64) - cen[0])
            exp = _expand(m, m.coeffs[k].astype(np.float64), B)
            got = rad[j, :, k, 0] + 1j * rad[j, :, k, 1]
            assert np.abs(got - exp).max() < 1e-12


def test_affine_modulations_closed_form(oracle_lib):
    """Global final layer W3 = 0 with bias (alpha, beta) per channel, then a
    local final layer W3 = 0 with bias (alpha', beta') per channel, shared by
    the components: phi -> (1 + alpha') ((1 + alpha) phi + beta) + beta'."""
    wl = _small_scene(K=5, seed=4)
    lmax, C = 3, 2
    m = S.make_rxcond_model(wl.scene.K, kind=O.BASIS_FLE, lmax=lmax, C=C, F=4, H=16, zero_final=True)
    P = S.split_rxcond_params(m)
    rng = np.random.default_rng(9)
    gb = rng.normal(size=4 * C).astype(np.float32)
    lb = rng.normal(size=4 * C).astype(np.float32)
    P[7][:] = gb
    P[13][:] = lb
    cen = wl.tx.astype(np.float64)
    rad = O.rxcond_radiance(m, wl.scene, cen, wl.rx, [0, 0], occ=O.occupancy(wl.scene, 16))
    g = gb.astype(np.float64).reshape(C, 4)
    q = lb.astype(np.float64).reshape(C, 4)
    for k in range(wl.scene.K):
        B = O.basis(O.BASIS_FLE, lmax, wl.scene.means[k].astype(np.float64) - cen[0])
        Bz = B[:, 0] + 1j * B[:, 1]
        phi = m.coeffs[k, ..., 0].astype(np.float64) + 1j * m.coeffs[k, ..., 1]       # (L, C)
        t = (1 + g[:, 0] + 1j * g[:, 1]) * phi + (g[:, 2] + 1j * g[:, 3])
        u = (1 + q[..., 0] + 1j * q[..., 1]) * t + (q[..., 2] + 1j * q[..., 3])
        exp = (u * Bz[:, None]).sum(axis=0)
        for j in range(2):
            assert np.abs(rad[j, :, k, 0] + 1j * rad[j, :, k, 1] - exp).max() < 1e-12


def test_global_branch_inputs_by_pass_through_weights(oracle_lib):
    """With identity first and second layers (hidden width = input width) and
    a final layer reading input i into alpha_re, the radiance of a Gaussian
    with phi = (1, 0) in component 0 only, seen along +z (B_00 = 1/sqrt(4 pi),
    every other component times phi = 0), is (1 + relu(x_i)) / sqrt(4 pi):
    x = [sin(W r), cos(W r) interleaved per frequency; deg/lmax, ord/lmax;
    e_l].  Here l = 0, so deg = ord = 0 and e_0 is the first embedding row."""
    F, lmax = 3, 2
    gin = 6 * F + 2 + 16
    sc = S.Scene(np.array([[0.0, 0.0, 1.0]]), np.full((1, 3), -2.0), np.array([[1.0, 0, 0, 0]]), np.array([0.0]),
                 radiance=np.zeros((1, 2)))
    m = S.make_rxcond_model(1, kind=O.BASIS_FLE, lmax=lmax, C=1, F=F, H=gin, zero_final=True)
    m.coeffs[:] = 0
    m.coeffs[0, 0, 0, 0] = 1.0
    P = S.split_rxcond_params(m)
    rng = np.random.default_rng(2)
    P[0][:] = rng.normal(size=P[0].shape)            # general frequency vectors
    P[1][:] = np.abs(rng.normal(size=P[1].shape))    # embeddings > 0 (survive the ReLU)
    P[2][:] = np.eye(gin)
    P[4][:] = np.eye(gin)
    r = np.array([[0.7, -1.3, 0.4]])
    W = P[0].astype(np.float64)
    x = np.zeros(gin)
    x[0:6 * F:2] = np.sin(W @ r[0])
    x[1:6 * F:2] = np.cos(W @ r[0])
    x[6 * F + 2:] = P[1][0]
    for i in range(gin):
        P[6][:] = 0
        P[6][0, i] = 1.0
        rad = O.rxcond_radiance(m, sc, np.zeros((1, 3)), r, [0], occ=O.occupancy(sc, 8))
        exp = (1 + max(x[i], 0.0)) / math.sqrt(4 * math.pi)
        assert abs(rad[0, 0, 0, 0] - exp) < 1e-12, i
        assert abs(rad[0, 0, 0, 1]) < 1e-12
    # component (deg 2, ord 1): its features are deg / lmax = 1, ord / lmax = 1/2
    # and its own embedding row; seen along (1, 1, 1) where B_21 is non-zero
    m.coeffs[:] = 0
    m.coeffs[0, _idx(2, 1), 0, 0] = 1.0
    sc2 = S.Scene(np.array([[1.0, 1.0, 1.0]]), sc.log_scales, sc.quats, sc.logits, radiance=sc.radiance)
    B21 = O.basis(O.BASIS_FLE, lmax, [1.0, 1.0, 1.0])[_idx(2, 1)]
    x2 = x.copy()
    x2[6 * F], x2[6 * F + 1] = 1.0, 0.5
    x2[6 * F + 2:] = P[1][_idx(2, 1)]
    for i in range(6 * F, gin):
        P[6][:] = 0
        P[6][0, i] = 1.0
        rad = O.rxcond_radiance(m, sc2, np.zeros((1, 3)), r, [0], occ=O.occupancy(sc2, 8))
        exp = (1 + max(x2[i], 0.0)) * (B21[0] + 1j * B21[1])
        assert abs(rad[0, 0, 0, 0] + 1j * rad[0, 0, 0, 1] - exp) < 1e-12, i


def test_local_branch_inputs_by_pass_through_weights(oracle_lib):
    """Local MLP with identity layers (width 6) and a final layer reading input
    i into alpha'_re of channel 0: the radiance of phi = (1, 0) in component
    0 seen along +z is (1 + relu(f_i)) / sqrt(4 pi), f = [(r - p)/|r - p|;
    |r - p|; T; rho] with the local features reported by the oracle."""
    sc = S.Scene(np.array([[0.0, 0.0, 1.0], [0.4, 0.1, 1.2]]), np.full((2, 3), -1.0),
                 np.array([[1.0, 0, 0, 0]] * 2), np.array([2.0, 1.0]), radiance=np.zeros((2, 2)))
    m = S.make_rxcond_model(2, kind=O.BASIS_FLE, lmax=1, C=1, F=2, H=6, zero_final=True)
    m.coeffs[:] = 0
    m.coeffs[:, 0, 0, 0] = 1.0
    P = S.split_rxcond_params(m)
    P[8][:] = np.eye(6)
    P[10][:] = np.eye(6)
    r = np.array([[0.1, -0.2, 1.05]])
    occ = O.occupancy(sc, 12)
    _, f = O.rxcond_radiance(m, sc, np.zeros((1, 3)), r, [0], occ=occ, want_feats=True)
    v = r[0] - sc.means[0]
    assert np.abs(f[0, 0, :3] - v / np.linalg.norm(v)).max() < 1e-15
    assert abs(f[0, 0, 3] - np.linalg.norm(v)) < 1e-15
    for i in range(6):
        P[12][:] = 0
        P[12][0, i] = 1.0
        rad = O.rxcond_radiance(m, sc, np.zeros((1, 3)), r, [0], occ=occ)
        exp = (1 + max(f[0, 0, i], 0.0)) / math.sqrt(4 * math.pi)
        assert abs(rad[0, 0, 0, 0] - exp) < 1e-12, i


def test_occupancy_one_and_two_gaussians(oracle_lib):
    """V at every voxel centre: 1 - prod over the Gaussians within 2 sigma (the
    largest scale) of (1 - o exp(-d^2 / (2 sigma^2))), with the grid spanning
    the box of the means."""
    means = np.array([[0.2, 0.5, 0.1], [1.4, 1.1, 0.9], [0.9, 0.4, 0.6]])
    ls = np.array([[-1.3, -1.6, -1.5], [-1.1, -1.4, -1.2], [-1.8, -1.2, -1.7]])
    logits = np.array([0.3, 1.2, -0.4])
    sc = S.Scene(means, ls, np.tile([1.0, 0, 0, 0], (3, 1)), logits, radiance=np.zeros((3, 2)))
    G = 20
    grid, lo, hi = O.occupancy(sc, G)
    assert np.array_equal(lo, means.min(axis=0)) and np.array_equal(hi, means.max(axis=0))
    vs = (hi - lo) / G
    idx = np.arange(G)
    X = lo[None, None, None, :] + (np.stack(np.meshgrid(idx, idx, idx, indexing="ij"), -1)[..., ::-1] + 0.5) * vs
    prod = np.ones((G, G, G))
    for k in range(3):
        sig = math.exp(ls[k].max())
        o = 1 / (1 + math.exp(-logits[k]))
        d2 = ((X - means[k]) ** 2).sum(-1)
        prod *= np.where(d2 <= 4 * sig * sig, 1 - o * np.exp(-0.5 * d2 / sig ** 2), 1.0)
    assert np.abs(grid - (1 - prod)).max() < 1e-13
    assert (grid > 0).sum() > 50 and (grid == 0).sum() > 50


def test_probes_read_the_nearest_voxel(oracle_lib):
    """T and rho of eq. (transmittance) from 16 probes at t = 0.05 .. 0.95 on
    the segment from the Gaussian to the receiver, each reading the voxel
    whose centre is nearest (brute force over all G^3 centres here), 0
    outside the box."""
    wl = _small_scene(K=30, seed=8)
    sc = S.Scene(*[None if a is None else np.asarray(a, np.float64) for a in
                   (wl.scene.means, wl.scene.log_scales, wl.scene.quats, wl.scene.logits, wl.scene.radiance)])
    G = 10
    occ = O.occupancy(sc, G)
    grid, lo, hi = occ
    m = S.make_rxcond_model(sc.K, lmax=1, C=1, F=2, H=8)
    rx = np.array([[1.5, 1.5, 1.0], [3.5, -0.5, 0.2]])   # the second outside the box
    _, f = O.rxcond_radiance(m, sc, np.zeros((1, 3)), rx, [0, 0], occ=occ, want_feats=True)
    vs = (hi - lo) / G
    idx = np.arange(G)
    cz, cy, cx = np.meshgrid(idx, idx, idx, indexing="ij")
    centres = lo + (np.stack([cx, cy, cz], -1) + 0.5) * vs
    checked = 0
    for j in range(2):
        for k in range(sc.K):
            T, tot = 1.0, 0.0
            for s in range(16):
                t = 0.05 + 0.9 * s / 15
                q = sc.means[k] + t * (rx[j] - sc.means[k])
                if (q < lo).any() or (q >= hi).any():
                    v = 0.0
                else:
                    dist = ((centres - q) ** 2).sum(-1)
                    v = grid.ravel()[np.argmin(dist)]
                    checked += 1
                T *= 1 - v
                tot += v
            assert abs(f[j, k, 4] - T) < 1e-12 and abs(f[j, k, 5] - tot / 16) < 1e-12
    assert checked > 100


def test_render_with_conditioned_radiance_channels(oracle_lib):
    """Each (receiver, channel) row of render_rxcond equals a plain render of
    that row's radiance (direct radiance given per Gaussian), so multi-channel
    rendering composites every channel with the same weights."""
    wl = _small_scene(K=40, seed=5)
    grid = S.Grid(12, 24, -math.pi / 2, math.pi / 12)
    m = S.make_rxcond_model(wl.scene.K, kind=O.BASIS_SH, lmax=2, C=3, F=3, H=16)
    cen = wl.tx.astype(np.float64)
    occ = O.occupancy(wl.scene, 16)
    out = O.render_rxcond(wl.scene, m, grid, cen, wl.rx, [0, 0], occ=occ)
    rad = O.rxcond_radiance(m, wl.scene, cen, wl.rx, [0, 0], occ=occ)
    for j in range(2):
        for c in range(3):
            sc = S.Scene(wl.scene.means, wl.scene.log_scales, wl.scene.quats, wl.scene.logits, radiance=rad[j, c])
            ref = O.render(sc, grid, cen, wl.rx[j:j + 1], [0])
            assert np.array_equal(out["C"][3 * j + c], ref["C"][0])
