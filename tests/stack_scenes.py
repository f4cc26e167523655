"""Hand-built scenes whose compositing has a closed form: Gaussians stacked on
the line of sight of one pixel centre.

The angular grid puts the centre of row i at elevation el0 + (i + 1/2) del_el
and column c at azimuth (c + 1/2) 2 pi / W (the grid convention of the
renderer and of the oracle).  A Gaussian whose mean lies on that ray projects
to (u, v) = (c, i) exactly, so its Mahalanobis distance at that pixel is 0 and
its weight there is min(0.99, o) with o = sigmoid(logit) (Alg. 1 stage 3).
"""
import math

import numpy as np

from paper_2605_24290_amd import scenes as S


def pixel_ray(grid, row, col):
    """Unit direction of the centre of pixel (row, col)."""
    az = (col + 0.5) * grid.del_az
    el = grid.el0 + (row + 0.5) * grid.del_el
    return np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])


def sigmoid(x):
    return 1.0 / (1.0 + math.exp(-x))


def stack(grid, row, col, centre, dists, logits, sigma, radiance, dtype=np.float64):
    """Isotropic Gaussians at centre + d * ray(row, col), one per distance."""
    d = pixel_ray(grid, row, col)
    m = len(dists)
    means = np.asarray(centre, dtype=np.float64)[None, :] + np.asarray(dists, dtype=np.float64)[:, None] * d[None, :]
    return S.Scene(means.astype(dtype), np.full((m, 3), math.log(sigma)).astype(dtype),
                   np.tile([[1.0, 0.0, 0.0, 0.0]], (m, 1)).astype(dtype),
                   np.asarray(logits, dtype=np.float64).reshape(m).astype(dtype),
                   radiance=np.asarray(radiance, dtype=np.float64).reshape(m, 2).astype(dtype))


def stop_index(o, eps=1e-4, m_max=1000):
    """First count n of equal weights o (with T = (1 - o)^n) that takes T below eps."""
    T = 1.0
    for n in range(1, m_max + 1):
        T *= 1.0 - o
        if T < eps:
            return n
    return None


def closed_form(o, radiance, n):
    """C = sum_{i < n} o (1 - o)^i s_i and T = (1 - o)^n for n equal weights o."""
    s = np.asarray(radiance, dtype=np.float64)
    w = o * (1.0 - o) ** np.arange(n)
    return (w[:, None] * s[:n]).sum(axis=0), (1.0 - o) ** n
