"""Shared helpers of the GPU parity tests (comparison rules and runners).

Comparison rule for spectra: per receiver, max over pixels and channels of
|C_gpu - C_oracle| divided by max |C_oracle| must stay below the tolerance,
except at pixels whose oracle decision margin (relative distance of w to 1/255
or 0.99, of T to 1e-4, of the azimuth offset to W/2) is below FLAG_MARGIN =
1e-5: there an FP32 rounding (the blend exponent carries ~1e-5 absolute, a
relative 7e-6 in the weight) may legitimately flip a skip / clamp / stop
decision.  Flagged pixels are counted, their share is bounded, and their
error is bounded too: a flipped decision moves C by at most about one
entry's T w |s| (w near 1/255 for a skip, a 1e-5 change of w for the clamp,
T below 1e-4 for the stop), so FLAGGED_TOL = 1e-2 of max |C|.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2605_24290_amd import scenes as S

TOL = 1e-4
FLAG_MARGIN = 1e-5
MAX_FLAGGED = 2e-3
FLAGGED_TOL = 1e-2


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def renderer_for(wl):
    from paper_2605_24290_amd import rxgs
    r = rxgs.Renderer(wl.grid)
    sc = wl.scene
    r.upload_scene(sc.means, sc.log_scales, sc.quats, sc.logits, radiance=sc.radiance, features=sc.features)
    if sc.features is not None:
        r.upload_mlp(S.flat_mlp(wl.mlp))
    return r


def compare_spectra(C_gpu, ora, tol=TOL, flag=FLAG_MARGIN, max_flagged=MAX_FLAGGED, rx_index=None):
    C_ora = ora["C"]
    if rx_index is not None:
        C_gpu = C_gpu[rx_index]
    N = C_ora.shape[0]
    flagged = ora["margin"] < flag
    worst = 0.0
    for j in range(N):
        scale = max(np.abs(C_ora[j]).max(), 1e-30)
        err = np.abs(C_gpu[j].astype(np.float64) - C_ora[j]).max(axis=0) / scale
        bad = (err > tol) & ~flagged[j]
        assert not bad.any(), (f"receiver {j}: {int(bad.sum())} pixels over {tol}, worst "
                               f"{err[~flagged[j]].max():.3e} at {np.unravel_index(np.argmax(np.where(flagged[j], 0, err)), err.shape)}")
        worst = max(worst, float(err[~flagged[j]].max()) if (~flagged[j]).any() else 0.0)
    frac = float(flagged.mean())
    wf = 0.0
    for j in range(N):
        if flagged[j].any():
            scale = max(np.abs(C_ora[j]).max(), 1e-30)
            wf = max(wf, float((np.abs(C_gpu[j].astype(np.float64) - C_ora[j]).max(axis=0) / scale)[flagged[j]].max()))
    print(f"[parity] worst rel err {worst:.3e}, flagged pixels {frac:.2e} (worst there {wf:.2e})")
    assert frac <= max_flagged, f"flagged fraction {frac:.2e}"
    assert wf <= FLAGGED_TOL, f"error at a flagged pixel {wf:.2e}"
    return worst, frac


def oracle_render(wl, mode, rx=None, nthreads=None):
    rx = wl.rx if rx is None else rx
    cen, rv = O.views_for(mode, wl.tx, rx)
    return O.render(wl.scene, wl.grid, cen, rx, rv, mlp=wl.mlp, nthreads=nthreads)


gpu = pytest.mark.gpu
needs_gpu = pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
