"""Seeded synthetic inputs for the multi-receiver Gaussian rasterizer.

This module only draws random numbers in a fixed order and packs them into
arrays.  It holds none of the rendering arithmetic, so both the GPU path and
the CPU oracle can take their inputs from it without sharing any of the
method's code.

Workload shapes follow the paper's spatial-spectrum setting (90 x 360 angular
grid at 1 degree, one transmitter, tens of receivers, tens of thousands of
Gaussians; Sec. 5 and App. F.2), with synthetic scenes in place of its
dataset, which is not available.  The base seed 8371 is the split seed the
paper uses for its datasets (App. F).

Draw order inside one ``numpy.random.Generator(PCG64(seed))``:
  1 means U(box) (K x 3)
  2 log-scales N(mu, sd^2) (K x 3)
  3 quaternions N(0,1)^4, normalised, (w, x, y, z) (K x 4)
  4 opacity logits N(0, 1) (K)
  5 direct radiance: amplitude exp(N(0, 0.5^2)), phase U[0, 2 pi) -> (Re, Im)
    or features N(0, 1) (K x 32)
  6 transmitters U(box) (Q x 3)
  7 receivers U(box) (N x 3)
  8 MLP weights, Xavier-uniform, zero biases
  9 target spectra 0.5 N(0, 1) (N x 2 x H x W), when asked for
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BASE_SEED = 8371
FEAT_DIM = 32
ENC_DIM = 36          # 3 axes x 6 frequencies x (sin, cos)
HIDDEN = 64
MLP_IN = ENC_DIM + FEAT_DIM
# W1 (64x68), b1 (64), W2 (64x64), b2 (64), W3 (2x64), b3 (2)
MLP_SHAPES = ((HIDDEN, MLP_IN), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,), (2, HIDDEN), (2,))
MLP_NPARAM = sum(int(np.prod(s)) for s in MLP_SHAPES)


@dataclasses.dataclass(frozen=True)
class Grid:
    """Angular grid: rows are elevation, columns azimuth over the full circle.

    Row i is centred at el0 + (i + 1/2) * del_el, column c at (c + 1/2) * 2 pi / W.
    """
    H: int
    W: int
    el0: float      # radians
    del_el: float   # radians

    @property
    def del_az(self) -> float:
        return 2.0 * math.pi / self.W


GRID_90x360 = Grid(90, 360, 0.0, math.pi / 180.0)          # 1 deg, el in [0, 90) deg
GRID_90x180 = Grid(90, 180, -math.pi / 2.0, math.pi / 90.0)  # 2 deg, full sphere


@dataclasses.dataclass
class Scene:
    means: np.ndarray        # (K, 3) f32
    log_scales: np.ndarray   # (K, 3) f32
    quats: np.ndarray        # (K, 4) f32, (w, x, y, z)
    logits: np.ndarray       # (K,) f32
    radiance: np.ndarray | None = None   # (K, 2) f32, direct (Re, Im)
    features: np.ndarray | None = None   # (K, 32) f32

    @property
    def K(self) -> int:
        return int(self.means.shape[0])


@dataclasses.dataclass
class Workload:
    scene: Scene
    tx: np.ndarray            # (Q, 3) f32
    rx: np.ndarray            # (N, 3) f32
    grid: Grid
    mlp: list | None = None   # [W1, b1, W2, b2, W3, b3] f32
    targets: np.ndarray | None = None  # (N, 2, H, W) f32
    name: str = ""


@dataclasses.dataclass(frozen=True)
class Preset:
    name: str
    K: int
    N: int
    box: tuple
    ls_mu: float
    ls_sd: float
    grid: Grid
    use_mlp: bool
    Q: int = 1
    targets: bool = False


PRESETS = {
    # 1,024 Gaussians, 4 receivers, 90x180 @ 2 deg, direct radiance
    "c0": Preset("c0", 1024, 4, (10.0, 10.0, 3.0), -1.5, 0.3, GRID_90x180, False),
    # 50k Gaussians, 64 receivers, 90x360, conditioning MLP
    "c1": Preset("c1", 50_000, 64, (10.0, 10.0, 3.0), -1.5, 0.3, GRID_90x360, True),
    # 100k Gaussians, 32 receivers, MLP, L2 targets
    "c2": Preset("c2", 100_000, 32, (10.0, 10.0, 3.0), -1.5, 0.3, GRID_90x360, True, targets=True),
    # serving scene: 200k Gaussians resident
    "c3": Preset("c3", 200_000, 0, (10.0, 10.0, 3.0), -1.5, 0.3, GRID_90x360, True),
    # scale: 1M Gaussians in a 40x40x4 box, 512 receivers
    "c4": Preset("c4", 1_000_000, 512, (40.0, 40.0, 4.0), -1.0, 0.5, GRID_90x360, True, targets=True),
    # the paper's own measurement shape (8x6x3 m room, ~32k Gaussians, 21 receivers)
    "paper": Preset("paper", 32_000, 21, (8.0, 6.0, 3.0), -1.5, 0.3, GRID_90x360, True),
}
_PRESET_INDEX = {"c0": 0, "c1": 1, "c2": 2, "c3": 3, "c4": 4, "paper": 5}


def _uniform_box(rng: np.random.Generator, n: int, box) -> np.ndarray:
    return rng.uniform(0.0, 1.0, size=(n, 3)) * np.asarray(box, dtype=np.float64)


def xavier_mlp(rng: np.random.Generator) -> list:
    """Xavier-uniform weights (bound sqrt(6 / (fan_in + fan_out))), zero biases."""
    out = []
    for shape in MLP_SHAPES:
        if len(shape) == 2:
            fo, fi = shape
            bound = math.sqrt(6.0 / (fi + fo))
            out.append(rng.uniform(-bound, bound, size=shape).astype(np.float32))
        else:
            out.append(np.zeros(shape, dtype=np.float32))
    return out


def make_workload(preset: str | Preset = "c0", *, K: int | None = None, N: int | None = None,
                  Q: int | None = None, seed: int | None = None, box=None,
                  grid: Grid | None = None, use_mlp: bool | None = None,
                  targets: bool | None = None) -> Workload:
    """Draw one seeded workload.  Overrides change sizes but not the draw order."""
    p = PRESETS[preset] if isinstance(preset, str) else preset
    K = p.K if K is None else K
    N = p.N if N is None else N
    Q = p.Q if Q is None else Q
    box = p.box if box is None else box
    grid = p.grid if grid is None else grid
    use_mlp = p.use_mlp if use_mlp is None else use_mlp
    targets = p.targets if targets is None else targets
    if seed is None:
        seed = BASE_SEED + 1000 * _PRESET_INDEX.get(p.name, 9)
    rng = np.random.Generator(np.random.PCG64(seed))

    means = _uniform_box(rng, K, box)
    log_scales = rng.normal(p.ls_mu, p.ls_sd, size=(K, 3))
    q = rng.normal(0.0, 1.0, size=(K, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    logits = rng.normal(0.0, 1.0, size=(K,))
    radiance = features = None
    if use_mlp:
        features = rng.normal(0.0, 1.0, size=(K, FEAT_DIM)).astype(np.float32)
    else:
        amp = np.exp(rng.normal(0.0, 0.5, size=(K,)))
        ph = rng.uniform(0.0, 2.0 * math.pi, size=(K,))
        radiance = np.stack([amp * np.cos(ph), amp * np.sin(ph)], axis=1).astype(np.float32)
    tx = _uniform_box(rng, Q, box).astype(np.float32)
    rx = _uniform_box(rng, N, box).astype(np.float32)
    mlp = xavier_mlp(rng) if use_mlp else None
    tgt = None
    if targets:
        tgt = (0.5 * rng.normal(0.0, 1.0, size=(N, 2, grid.H, grid.W))).astype(np.float32)
    scene = Scene(means.astype(np.float32), log_scales.astype(np.float32),
                  q.astype(np.float32), logits.astype(np.float32), radiance, features)
    return Workload(scene, tx, rx, grid, mlp, tgt, name=p.name)


def flat_mlp(mlp: list) -> np.ndarray:
    """Concatenate [W1, b1, W2, b2, W3, b3] (row-major, out x in) into one f32 vector."""
    return np.concatenate([np.asarray(a, dtype=np.float32).ravel() for a in mlp])


def unflat_mlp(v: np.ndarray) -> list:
    out, off = [], 0
    for shape in MLP_SHAPES:
        n = int(np.prod(shape))
        out.append(np.asarray(v[off:off + n]).reshape(shape))
        off += n
    return out


def poisson_queries(rng: np.random.Generator, rate: float, count: int, box,
                    max_rx: int = 256) -> list:
    """Serving queries: Exp(rate) gaps; receiver count floor(exp(U(0, ln(max_rx+1)))),
    clipped to [1, max_rx]; transmitter and receivers uniform in the box."""
    t = 0.0
    out = []
    for _ in range(count):
        t += rng.exponential(1.0 / rate)
        n = int(math.floor(math.exp(rng.uniform(0.0, math.log(max_rx + 1)))))
        n = min(max(n, 1), max_rx)
        txq = _uniform_box(rng, 1, box).astype(np.float32)[0]
        rxq = _uniform_box(rng, n, box).astype(np.float32)
        out.append((t, txq, rxq))
    return out


def serving_queries(seed: int, count: int, box, max_rx: int = 256):
    """Seeded serving queries at unit rate: Exp(1) inter-arrival gaps (scale by
    1 / rate), receiver counts floor(exp(U(0, ln(max_rx + 1)))) clipped to
    [1, max_rx], transmitter and receivers uniform in the box."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0, size=count)
    out = []
    for i in range(count):
        n = int(math.floor(math.exp(rng.uniform(0.0, math.log(max_rx + 1)))))
        n = min(max(n, 1), max_rx)
        txq = _uniform_box(rng, 1, box).astype(np.float32)[0]
        rxq = _uniform_box(rng, n, box).astype(np.float32)
        out.append((float(gaps[i]), txq, rxq))
    return out


# ---------------------------------------------------------------------------
# The paper's receiver-conditioned radiance model (Sec. 4.3.2; App. E.2, E.5)

EMB_DIM = 16          # component embedding width d_c (App. E Table 4)
BASIS_FLE = 0         # complex Fourier-Legendre basis (App. E.2)
BASIS_SH = 1          # real spherical harmonics (the RF-3DGS backbone, Sec. 5)


def rxcond_shapes(lmax: int, C: int, F: int, H: int) -> list:
    """Shapes of the conditioning parameters, in the order of the flat vector:
    Fourier frequency vectors (3F x 3), component embeddings (L x 16), the
    global MLP (W1, b1, W2, b2, W3, b3; input 6F + 2 + 16, output 4C) and the
    local MLP (input 6, output 4C: one complex scale and shift per channel,
    shared by the components); matrices are (out, in)."""
    L = (lmax + 1) ** 2
    gin = 6 * F + 2 + EMB_DIM
    return [(3 * F, 3), (L, EMB_DIM),
            (H, gin), (H,), (H, H), (H,), (4 * C, H), (4 * C,),
            (H, 6), (H,), (H, H), (H,), (4 * C, H), (4 * C,)]


@dataclasses.dataclass
class RxCondModel:
    kind: int            # BASIS_FLE or BASIS_SH
    lmax: int
    C: int               # complex signal channels
    F: int               # Fourier bands per axis
    H: int               # hidden width of both MLPs
    coeffs: np.ndarray   # (K, L, C, 2) f32 base coefficients (Re, Im)
    params: np.ndarray   # flat f32, rxcond_shapes order
    S: int = 16          # occupancy probes per (receiver, Gaussian)
    G: int = 128         # occupancy grid resolution

    @property
    def L(self) -> int:
        return (self.lmax + 1) ** 2


def make_rxcond_model(K: int, *, kind: int = BASIS_FLE, lmax: int = 9, C: int = 1, F: int = 6, H: int = 64,
                      seed: int = BASE_SEED + 7000, coeff_sd: float = 0.3, zero_final: bool = False) -> RxCondModel:
    """Seeded synthetic stand-in for a trained conditioning model: frequency
    vectors at 2^f along each axis (their initialisation, App. E.5),
    embeddings N(0, 1), Xavier-uniform weights with zero biases (final layers
    too unless zero_final, the paper's initialisation), base coefficients
    N(0, coeff_sd^2).  Draw order: coefficients, embeddings, weight matrices
    in rxcond_shapes order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    L = (lmax + 1) ** 2
    coeffs = rng.normal(0.0, coeff_sd, size=(K, L, C, 2)).astype(np.float32)
    shapes = rxcond_shapes(lmax, C, F, H)
    parts = []
    freq = np.zeros((3 * F, 3), dtype=np.float32)
    for d in range(3):
        for f in range(F):
            freq[d * F + f, d] = 2.0 ** f
    parts.append(freq)
    parts.append(rng.normal(0.0, 1.0, size=shapes[1]).astype(np.float32))
    final = {6, 7, 12, 13}
    for i, shape in enumerate(shapes[2:], start=2):
        if len(shape) == 2 and not (zero_final and i in final):
            fo, fi = shape
            bound = math.sqrt(6.0 / (fi + fo))
            parts.append(rng.uniform(-bound, bound, size=shape).astype(np.float32))
        else:
            parts.append(np.zeros(shape, dtype=np.float32))
    params = np.concatenate([p.ravel() for p in parts])
    return RxCondModel(kind, lmax, C, F, H, coeffs, params)


def split_rxcond_params(model: RxCondModel) -> list:
    """The flat parameter vector cut into its rxcond_shapes arrays (views)."""
    out, off = [], 0
    for shape in rxcond_shapes(model.lmax, model.C, model.F, model.H):
        n = int(np.prod(shape))
        out.append(model.params[off:off + n].reshape(shape))
        off += n
    assert off == model.params.size
    return out
