"""Dense NumPy twin of the oracle for tiny scenes (TEST INFRASTRUCTURE ONLY).

A second formulation of the same definition, written differently on purpose,
so that the two check each other:

* the projection Jacobian is taken numerically (central differences of the
  azimuth / elevation map) instead of from the analytic formula;
* the rotation matrix comes from ``scipy.spatial.transform.Rotation``;
* compositing is dense: a pixels x Gaussians weight matrix in depth-key order,
  a mask for the 1/255 skip, an exclusive cumulative product for the
  transmittance and a ``T_before >= 1e-4`` test for the early stop
  (Alg. 1, stage 3), instead of a per-pixel loop with a break;
* the MLP first layer is split into its receiver part and its Gaussian part,
  relu(W1a gamma(r) + W1b f + b1), the form the spec calls the global
  and local branches (Sec. 4.3.2), instead of one 68-wide product.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.spatial.transform import Rotation
from scipy.special import expit

ALPHA_MIN = 1.0 / 255.0
W_MAX = 0.99
T_EPS = 1e-4
DILATE = 0.3


def _angles(d):
    """Azimuth in [0, 2pi) and elevation of direction vectors d (..., 3)."""
    h = np.maximum(np.hypot(d[..., 0], d[..., 1]), 1e-6)
    az = np.mod(np.arctan2(d[..., 1], d[..., 0]), 2 * math.pi)
    el = np.arctan2(d[..., 2], h)
    return az, el


def _key32(means, c):
    m = np.asarray(means, dtype=np.float32)
    cc = np.asarray(c, dtype=np.float32)
    d = m - cc
    s = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]
    s = s + d[:, 2] * d[:, 2]
    return s.astype(np.float32)


def project(scene, grid, c):
    """u, v, conic (K,3), opacity, key (f32) and near flag for one view."""
    p = np.asarray(scene.means, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    d = p - c
    az, el = _angles(d)
    u = az / grid.del_az - 0.5
    v = (el - grid.el0) / grid.del_el - 0.5
    K = p.shape[0]
    J = np.zeros((K, 2, 3))
    for a in range(3):
        hstep = 1e-5 * np.maximum(np.linalg.norm(d, axis=1), 1.0)
        e = np.zeros(3)
        e[a] = 1.0
        azp, elp = _angles(d + hstep[:, None] * e)
        azm, elm = _angles(d - hstep[:, None] * e)
        daz = np.mod(azp - azm + math.pi, 2 * math.pi) - math.pi
        J[:, 0, a] = daz / (2 * hstep) / grid.del_az
        J[:, 1, a] = (elp - elm) / (2 * hstep) / grid.del_el
    q = np.asarray(scene.quats, dtype=np.float64)
    R = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()
    s2 = np.exp(2.0 * np.asarray(scene.log_scales, dtype=np.float64))
    Sig = np.einsum("kij,kj,klj->kil", R, s2, R)
    Spx = np.einsum("kai,kij,kbj->kab", J, Sig, J) + DILATE * np.eye(2)
    con = np.linalg.inv(Spx)
    conic = np.stack([con[:, 0, 0], con[:, 0, 1], con[:, 1, 1]], axis=1)
    o = expit(np.asarray(scene.logits, dtype=np.float64))
    key = _key32(scene.means, c)
    near = key < np.float32(0.04)
    return u, v, conic, o, key, near, Spx


def encode(r):
    r = np.asarray(r, dtype=np.float64)
    out = np.zeros(36)
    for d in range(3):
        for f in range(6):
            out[12 * d + 2 * f] = math.sin(r[d] * 2.0 ** f)
            out[12 * d + 2 * f + 1] = math.cos(r[d] * 2.0 ** f)
    return out


def radiance(scene, rx, mlp=None):
    rx = np.asarray(rx, dtype=np.float64).reshape(-1, 3)
    K = scene.K
    if mlp is None or scene.features is None:
        rad = np.asarray(scene.radiance, dtype=np.float64)
        return np.broadcast_to(rad, (rx.shape[0], K, 2)).copy()
    W1, b1, W2, b2, W3, b3 = [np.asarray(a, dtype=np.float64) for a in mlp]
    local = np.asarray(scene.features, dtype=np.float64) @ W1[:, 36:].T + b1      # (K, 64)
    out = np.zeros((rx.shape[0], K, 2))
    for j in range(rx.shape[0]):
        glob = W1[:, :36] @ encode(rx[j])                                          # (64,)
        h1 = np.maximum(local + glob[None, :], 0.0)
        h2 = np.maximum(h1 @ W2.T + b2, 0.0)
        out[j] = h2 @ W3.T + b3
    return out


def render(scene, grid, centres, rx, rx_view, mlp=None):
    centres = np.asarray(centres, dtype=np.float64).reshape(-1, 3)
    rx = np.asarray(rx, dtype=np.float64).reshape(-1, 3)
    H, W = grid.H, grid.W
    rad = radiance(scene, rx, mlp)
    rows, cols = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    rows = rows.ravel()
    cols = cols.ravel()
    N = rx.shape[0]
    C = np.zeros((N, 2, H * W))
    Tf = np.ones((N, H * W))
    views = {}
    for j in range(N):
        vi = int(rx_view[j])
        if vi not in views:
            u, v, conic, o, key, near, _ = project(scene, grid, centres[vi])
            idx = np.nonzero(~near)[0]
            order = idx[np.lexsort((idx, key[idx].view(np.uint32)))]
            du = cols[:, None] - u[None, order]
            du = np.mod(du + W / 2.0, W) - W / 2.0
            dv = rows[:, None] - v[None, order]
            a, b, c = conic[order, 0], conic[order, 1], conic[order, 2]
            qf = a * du * du + 2 * b * du * dv + c * dv * dv
            w = np.minimum(W_MAX, o[order] * np.exp(-0.5 * qf))
            mask = w >= ALPHA_MIN
            fac = 1.0 - np.where(mask, w, 0.0)
            Tb = np.concatenate([np.ones((H * W, 1)), np.cumprod(fac, axis=1)[:, :-1]], axis=1)
            inc = mask & (Tb >= T_EPS)
            wt = np.where(inc, Tb * w, 0.0)
            Tend = np.prod(np.where(inc, 1.0 - w, 1.0), axis=1)
            views[vi] = (order, wt, Tend)
        order, wt, Tend = views[vi]
        s = rad[j][order]
        C[j, 0] = wt @ s[:, 0]
        C[j, 1] = wt @ s[:, 1]
        Tf[j] = Tend
    C = C.reshape(N, 2, H, W)
    power = (C ** 2).sum(axis=(1, 2, 3))
    return dict(C=C, T_final=Tf.reshape(N, H, W), power=power)
