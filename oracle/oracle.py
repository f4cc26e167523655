"""ctypes front end of the FP64 CPU oracle (``rxgs_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg call this module; the product path never does.  It imports
nothing from the GPU package and the GPU package imports nothing from it.

Every function takes plain numpy arrays (FP32 inputs are widened to FP64 here)
and returns FP64 results.  View conventions: in mode ``"tx"`` the views are the
transmitters and receiver j uses view ``q`` for ``rx_off[q] <= j < rx_off[q+1]``
(Alg. 1: one transmitter-centred sphere shared by its receivers); in mode
``"rx"`` receiver j is its own view, centred at its position.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rxgs_oracle.c")
SRCS = [SRC, os.path.join(HERE, "rxcond_oracle.c")]
LIB = os.path.join(HERE, "liboracle.so")

TILE_W = 16
TILE_H = 16
NMLP = 64 * 68 + 64 + 64 * 64 + 64 + 2 * 64 + 2

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-o", LIB + ".tmp", *SRCS, "-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(f) for f in SRCS):
            build()
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        up = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        fp = ctypes.POINTER(ctypes.c_float)
        i64p = ctypes.POINTER(ctypes.c_int64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        ci, cd = ctypes.c_int, ctypes.c_double
        L.orc_render.argtypes = [ci, dp, dp, dp, dp, dp, dp, dp, ci, dp, ci, dp, ip, ci, ci, cd, cd, ci,
                                 dp, dp, ip, dp, dp, dp, u64p, ip]
        L.orc_render.restype = ci
        L.orc_project.argtypes = [ci, dp, dp, dp, dp, ci, dp, ci, ci, cd, cd, up, ip, dp]
        L.orc_project.restype = ci
        L.orc_project_jacobian.argtypes = [dp, dp, dp, cd, dp, ci, ci, cd, cd, dp]
        L.orc_project_jacobian.restype = ci
        L.orc_radiance.argtypes = [ci, dp, dp, dp, ci, dp, ci, dp]
        L.orc_radiance.restype = ci
        L.orc_backward.argtypes = [ci, dp, dp, dp, dp, dp, dp, dp, ci, dp, ci, dp, ip, ci, ci, cd, cd, ci,
                                   dp, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_backward.restype = ci
        L.orc_bin.argtypes = [ci, ci, fp, fp, fp, fp, fp, up, ci, ci, ci, ci, i64p, i32p, ctypes.c_int64]
        L.orc_bin.restype = ctypes.c_int64
        L.orc_render_rad.argtypes = [ci, dp, dp, dp, dp, dp, ci, dp, ci, ip, ci, ci, cd, cd, ci,
                                     dp, dp, ip, dp, dp, dp, u64p, ip]
        L.orc_render_rad.restype = ci
        L.orc_basis.argtypes = [ci, ci, cd, cd, cd, dp]
        L.orc_basis.restype = ci
        L.orc_occupancy.argtypes = [ci, dp, dp, dp, ci, ci, dp, dp, dp]
        L.orc_occupancy.restype = ci
        L.orc_rxcond_param_count.argtypes = [ci, ci, ci, ci]
        L.orc_rxcond_param_count.restype = ctypes.c_long
        L.orc_rxcond_radiance.argtypes = [ci, ci, ci, ci, ci, ci, ci, dp, dp, dp, ci, dp, ci, dp, ip, ci, dp, dp,
                                          dp, ci, dp, dp]
        L.orc_rxcond_radiance.restype = ci
        _lib = L
    return _lib


def _d(a):
    if a is None:
        return None, None
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ptr(a, ct):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ct))


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


def views_for(mode: str, tx, rx, rx_off=None):
    """(centres V x 3, rx_view N) for a render mode."""
    rx = np.asarray(rx, dtype=np.float64).reshape(-1, 3)
    N = rx.shape[0]
    if mode == "rx":
        return rx.copy(), np.arange(N, dtype=np.int32)
    if mode != "tx":
        raise ValueError("mode must be 'tx' or 'rx'")
    tx = np.asarray(tx, dtype=np.float64).reshape(-1, 3)
    if rx_off is None:
        if tx.shape[0] != 1:
            raise ValueError("rx_off is needed with several transmitters")
        rx_off = [0, N]
    rx_off = np.asarray(rx_off, dtype=np.int64)
    rv = np.zeros(N, dtype=np.int32)
    for q in range(tx.shape[0]):
        rv[rx_off[q]:rx_off[q + 1]] = q
    return tx.copy(), rv


def _scene_args(scene, mlp):
    means, pm = _d(scene.means)
    ls, pl = _d(scene.log_scales)
    qu, pq = _d(scene.quats)
    lg, pg = _d(scene.logits)
    rad = feat = ml = None
    prad = pfeat = pml = None
    if scene.features is not None and mlp is not None:
        feat, pfeat = _d(scene.features)
        flat = np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in mlp])
        assert flat.size == NMLP
        ml, pml = _d(flat)
    else:
        rad, prad = _d(scene.radiance)
    keep = (means, ls, qu, lg, rad, feat, ml)
    return keep, (pm, pl, pq, pg, prad, pfeat, pml)


def render(scene, grid, centres, rx, rx_view, mlp=None, nthreads=None, want_hash=False):
    """Forward render.  Returns a dict with C (N,2,H,W), T_final, ncomp and
    nclamp (clamped composited entries) (N,H,W), margin (N,H,W), power (N),
    csum (N,2) and optionally rowhash (N,H)."""
    L = lib()
    keep, ptrs = _scene_args(scene, mlp)
    cen, pc = _d(np.asarray(centres).reshape(-1, 3))
    rxa, prx = _d(np.asarray(rx).reshape(-1, 3))
    rv = np.ascontiguousarray(np.asarray(rx_view, dtype=np.int32))
    N, V, K = rxa.shape[0], cen.shape[0], scene.K
    H, W = grid.H, grid.W
    C = np.zeros((N, 2, H, W))
    T = np.zeros((N, H, W))
    nc = np.zeros((N, H, W), dtype=np.int32)
    ncl = np.zeros((N, H, W), dtype=np.int32)
    mg = np.zeros((N, H, W))
    pw = np.zeros(N)
    cs = np.zeros((N, 2))
    rh = np.zeros((N, H), dtype=np.uint64) if want_hash else None
    nt = nthreads or default_threads()
    rc = L.orc_render(K, *ptrs, V, pc, N, prx, _ptr(rv, ctypes.c_int), H, W, grid.el0, grid.del_el, nt,
                      _ptr(C, ctypes.c_double), _ptr(T, ctypes.c_double), _ptr(nc, ctypes.c_int),
                      _ptr(mg, ctypes.c_double), _ptr(pw, ctypes.c_double), _ptr(cs, ctypes.c_double),
                      _ptr(rh, ctypes.c_uint64), _ptr(ncl, ctypes.c_int))
    if rc != 0:
        raise RuntimeError(f"orc_render failed ({rc})")
    del keep
    out = dict(C=C, T_final=T, ncomp=nc, nclamp=ncl, margin=mg, power=pw, csum=cs)
    if want_hash:
        out["rowhash"] = rh
    return out


def project(scene, grid, centres):
    """Per (view, Gaussian): keybits (V,K) u32, nearcull (V,K) bool and
    proj (V,K,9) = u, v, conic a, b, c, opacity, covariance A, B, Cc."""
    L = lib()
    keep, ptrs = _scene_args(scene, None)
    cen, pc = _d(np.asarray(centres).reshape(-1, 3))
    V, K = cen.shape[0], scene.K
    kb = np.zeros((V, K), dtype=np.uint32)
    nc = np.zeros((V, K), dtype=np.int32)
    pr = np.zeros((V, K, 9))
    L.orc_project(K, ptrs[0], ptrs[1], ptrs[2], ptrs[3], V, pc, grid.H, grid.W, grid.el0, grid.del_el,
                  _ptr(kb, ctypes.c_uint32), _ptr(nc, ctypes.c_int), _ptr(pr, ctypes.c_double))
    del keep
    return kb, nc.astype(bool), pr


def project_jacobian(p, ls, q, logit, centre, grid):
    """6 x 11 Jacobian of (u, v, a, b, c, o) w.r.t. (mean, log-scale, quat, logit)."""
    L = lib()
    pa, pp = _d(p)
    la, pl = _d(ls)
    qa, pq = _d(q)
    ca, pc = _d(centre)
    jac = np.zeros((6, 11))
    L.orc_project_jacobian(pp, pl, pq, float(logit), pc, grid.H, grid.W, grid.el0, grid.del_el,
                           _ptr(jac, ctypes.c_double))
    del pa, la, qa, ca
    return jac


def radiance(scene, rx, mlp=None, nthreads=None):
    """Radiance of every (receiver, Gaussian) pair, (N, K, 2)."""
    L = lib()
    keep, ptrs = _scene_args(scene, mlp)
    rxa, prx = _d(np.asarray(rx).reshape(-1, 3))
    N, K = rxa.shape[0], scene.K
    out = np.zeros((N, K, 2))
    L.orc_radiance(K, ptrs[4], ptrs[5], ptrs[6], N, prx, nthreads or default_threads(),
                   _ptr(out, ctypes.c_double))
    del keep
    return out


def backward(scene, grid, centres, rx, rx_view, dC, dP=None, mlp=None, nthreads=None):
    """Gradients of L given dL/dC (N,2,H,W) and dL/dP (N).  Returns a dict with
    means, log_scales, quats, logits and radiance, or features and mlp (flat)."""
    L = lib()
    keep, ptrs = _scene_args(scene, mlp)
    cen, pc = _d(np.asarray(centres).reshape(-1, 3))
    rxa, prx = _d(np.asarray(rx).reshape(-1, 3))
    rv = np.ascontiguousarray(np.asarray(rx_view, dtype=np.int32))
    dCa, pdC = _d(dC)
    dPa, pdP = _d(dP)
    N, V, K = rxa.shape[0], cen.shape[0], scene.K
    g = dict(means=np.zeros((K, 3)), log_scales=np.zeros((K, 3)), quats=np.zeros((K, 4)),
             logits=np.zeros(K))
    use_mlp = ptrs[6] is not None
    if use_mlp:
        g["features"] = np.zeros((K, 32))
        g["mlp"] = np.zeros(NMLP)
    else:
        g["radiance"] = np.zeros((K, 2))
    dp = ctypes.c_double
    rc = L.orc_backward(K, *ptrs, V, pc, N, prx, _ptr(rv, ctypes.c_int), grid.H, grid.W, grid.el0,
                        grid.del_el, nthreads or default_threads(), pdC, pdP,
                        _ptr(g["means"], dp), _ptr(g["log_scales"], dp), _ptr(g["quats"], dp),
                        _ptr(g["logits"], dp), _ptr(g.get("radiance"), dp),
                        _ptr(g.get("features"), dp), _ptr(g.get("mlp"), dp))
    if rc != 0:
        raise RuntimeError(f"orc_backward failed ({rc})")
    del keep, dCa, dPa
    return g


def bin_records(u, v, rup, rvp, o, keybits, grid, tile_w=TILE_W, tile_h=TILE_H):
    """Expected sorted (segment, Gaussian index) pairs from FP32 records of shape (V, K)."""
    L = lib()
    arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float32)) for a in (u, v, rup, rvp, o)]
    kb = np.ascontiguousarray(np.asarray(keybits, dtype=np.uint32))
    V, K = kb.shape
    fp = ctypes.c_float
    args = [_ptr(a, fp) for a in arrs]
    n = L.orc_bin(V, K, *args, _ptr(kb, ctypes.c_uint32), grid.H, grid.W, tile_w, tile_h, None, None, 0)
    seg = np.zeros(max(n, 1), dtype=np.int64)
    kk = np.zeros(max(n, 1), dtype=np.int32)
    n2 = L.orc_bin(V, K, *args, _ptr(kb, ctypes.c_uint32), grid.H, grid.W, tile_w, tile_h,
                   _ptr(seg, ctypes.c_int64), _ptr(kk, ctypes.c_int32), n)
    assert n2 == n
    return seg[:n], kk[:n]


# ---------------------------------------------------------------------------
# the paper's conditioned radiance (rxcond_oracle.c)

BASIS_FLE = 0
BASIS_SH = 1


def basis(kind: int, lmax: int, d) -> np.ndarray:
    """Basis values at direction d (3,): (L, 2) Re / Im, component index deg^2 + deg + ord."""
    L = (lmax + 1) ** 2
    out = np.zeros((L, 2))
    d = np.asarray(d, dtype=np.float64)
    rc = lib().orc_basis(kind, lmax, float(d[0]), float(d[1]), float(d[2]), _ptr(out, ctypes.c_double))
    if rc != 0:
        raise ValueError("bad basis arguments")
    return out


def occupancy(scene, G: int = 128, nthreads=None):
    """(grid (G, G, G) indexed [z, y, x], lo (3,), hi (3,)) of the scene's Gaussians."""
    means, pm = _d(scene.means)
    ls, pl = _d(scene.log_scales)
    lg, pg = _d(scene.logits)
    lo = np.zeros(3)
    hi = np.zeros(3)
    grid = np.zeros((G, G, G))
    rc = lib().orc_occupancy(scene.K, pm, pl, pg, G, nthreads or default_threads(), _ptr(lo, ctypes.c_double),
                             _ptr(hi, ctypes.c_double), _ptr(grid, ctypes.c_double))
    if rc != 0:
        raise RuntimeError(f"orc_occupancy failed ({rc})")
    del means, ls, lg
    return grid, lo, hi


def rxcond_param_count(lmax: int, C: int, F: int, H: int) -> int:
    return int(lib().orc_rxcond_param_count(lmax, C, F, H))


def rxcond_radiance(model, scene, centres, rx, rx_view, occ=None, nthreads=None, want_feats=False):
    """Conditioned radiance of every (receiver, channel, Gaussian): (N, C, K, 2),
    and the local-branch inputs (N, K, 6) when want_feats.  model has kind,
    lmax, C, F, H, S, G, coeffs (K, L, C, 2) and params (flat)."""
    L = lib()
    means, pm = _d(scene.means)
    co, pco = _d(model.coeffs)
    pa, ppa = _d(model.params)
    assert pa.size == rxcond_param_count(model.lmax, model.C, model.F, model.H)
    cen, pc = _d(np.asarray(centres).reshape(-1, 3))
    rxa, prx = _d(np.asarray(rx).reshape(-1, 3))
    rv = np.ascontiguousarray(np.asarray(rx_view, dtype=np.int32))
    if occ is None:
        occ = occupancy(scene, model.G, nthreads)
    grid, lo, hi = occ
    G = grid.shape[0]
    assert grid.shape == (G, G, G)
    gr, pgr = _d(grid)
    lo_, plo = _d(lo)
    hi_, phi = _d(hi)
    N, K = rxa.shape[0], scene.K
    out = np.zeros((N, model.C, K, 2))
    feats = np.zeros((N, K, 6)) if want_feats else None
    rc = L.orc_rxcond_radiance(model.kind, model.lmax, model.C, model.F, model.H, model.S, K, pm, pco, ppa,
                               cen.shape[0], pc, N, prx, _ptr(rv, ctypes.c_int), G, plo, phi, pgr,
                               nthreads or default_threads(), _ptr(out, ctypes.c_double),
                               _ptr(feats, ctypes.c_double))
    if rc != 0:
        raise RuntimeError(f"orc_rxcond_radiance failed ({rc})")
    del means, co, pa, cen, rxa, gr, lo_, hi_
    return (out, feats) if want_feats else out


def render_rad(scene, grid, centres, rad_rx, rx_view, nthreads=None, want_hash=False):
    """Forward render with per-receiver radiance rad_rx (N, K, 2) given
    (receiver j uses view rx_view[j]); outputs as render()."""
    L = lib()
    means, pm = _d(scene.means)
    ls, pl = _d(scene.log_scales)
    qu, pq = _d(scene.quats)
    lg, pg = _d(scene.logits)
    rr, prr = _d(rad_rx)
    cen, pc = _d(np.asarray(centres).reshape(-1, 3))
    rv = np.ascontiguousarray(np.asarray(rx_view, dtype=np.int32))
    N, V, K = rr.shape[0], cen.shape[0], scene.K
    assert rr.shape == (N, K, 2)
    H, W = grid.H, grid.W
    C = np.zeros((N, 2, H, W))
    T = np.zeros((N, H, W))
    nc = np.zeros((N, H, W), dtype=np.int32)
    ncl = np.zeros((N, H, W), dtype=np.int32)
    mg = np.zeros((N, H, W))
    pw = np.zeros(N)
    cs = np.zeros((N, 2))
    rh = np.zeros((N, H), dtype=np.uint64) if want_hash else None
    rc = L.orc_render_rad(K, pm, pl, pq, pg, prr, V, pc, N, _ptr(rv, ctypes.c_int), H, W, grid.el0, grid.del_el,
                          nthreads or default_threads(), _ptr(C, ctypes.c_double), _ptr(T, ctypes.c_double),
                          _ptr(nc, ctypes.c_int), _ptr(mg, ctypes.c_double), _ptr(pw, ctypes.c_double),
                          _ptr(cs, ctypes.c_double), _ptr(rh, ctypes.c_uint64), _ptr(ncl, ctypes.c_int))
    if rc != 0:
        raise RuntimeError(f"orc_render_rad failed ({rc})")
    del means, ls, qu, lg, rr, cen
    out = dict(C=C, T_final=T, ncomp=nc, nclamp=ncl, margin=mg, power=pw, csum=cs)
    if want_hash:
        out["rowhash"] = rh
    return out


def render_rxcond(scene, model, grid, centres, rx, rx_view, nthreads=None, occ=None):
    """Render with the conditioned radiance: every (receiver, channel) is one
    output row (receiver-major), composited over its receiver's view.  C
    (N * C, 2, H, W) and the other outputs of render()."""
    rad = rxcond_radiance(model, scene, centres, rx, rx_view, occ=occ, nthreads=nthreads)   # (N, C, K, 2)
    N, Ch = rad.shape[0], rad.shape[1]
    rv = np.repeat(np.asarray(rx_view, dtype=np.int32), Ch)
    return render_rad(scene, grid, centres, rad.reshape(N * Ch, scene.K, 2), rv, nthreads=nthreads)
