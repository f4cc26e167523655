"""Nearest-first emission (an option, off by default) against the full lists.

With it on, rxgs_render emits per view only its 4096 nearest depth-sorted
entries when the scene has more, and redoes any view with a pixel still open
at the end of that prefix (compositing stops at a pixel once its transmittance is below 1e-4,
Alg. 1).  Spectra and power must be bit-identical to the render over the full
lists, without and with saved state, in both view modes: on a dense scene
(every view complete after the prefix) and on a sparse one (views redone).
Gradients from the two saved states must agree to 1e-6 (float atomics).
"""
import numpy as np
import pytest

from paper_2605_24290_amd import scenes as S

from .parity import compare_spectra, gpu, needs_gpu, oracle_render, renderer_for

pytestmark = [gpu, needs_gpu]


def _pair(r, wl, mode, saved_cls=None):
    import torch
    outs = []
    for cut in (True, False):
        r.near_cut(cut)
        saved = saved_cls(r) if saved_cls else None
        C, P, Sm = r.render(wl.rx, tx=wl.tx, mode=mode, saved=saved, want_csum=True)
        grads = None
        if saved is not None:
            rng = np.random.default_rng(11)
            dC = torch.as_tensor(rng.normal(size=tuple(C.shape)).astype(np.float32), device=C.device)
            g = r.backward(saved, C, dC, None)
            grads = {k: v.cpu().numpy().astype(np.float64) for k, v in g.items()}
        torch.cuda.synchronize()
        outs.append((C.cpu().numpy(), P.cpu().numpy(), Sm.cpu().numpy(), grads))
        if saved is not None:
            saved.close()
    r.near_cut(False)   # the default
    return outs


@pytest.mark.parametrize("scene", ["dense", "sparse"])
@pytest.mark.parametrize("mode", ["tx", "rx"])
def test_near_cut_equals_full_lists(scene, mode):
    from paper_2605_24290_amd import rxgs
    if scene == "dense":
        wl = S.make_workload("c1", K=20000, N=12)
    else:   # about 4.7 Gaussians per cubic metre: many rays stay open past the prefix
        wl = S.make_workload("c1", K=30000, N=6, box=(40.0, 40.0, 4.0))
    r = renderer_for(wl)
    before = r.views_redone()
    (Ca, Pa, Sa, _), (Cb, Pb, Sb, _) = _pair(r, wl, mode)
    redone = r.views_redone() - before
    print(f"[near] {scene} {mode}: views redone {redone}")
    assert np.array_equal(Ca, Cb) and np.array_equal(Pa, Pb) and np.array_equal(Sa, Sb)
    if scene == "sparse":
        assert redone > 0
    (Ca, Pa, Sa, ga), (Cb, Pb, Sb, gb) = _pair(r, wl, mode, rxgs.Saved)
    assert np.array_equal(Ca, Cb) and np.array_equal(Pa, Pb)
    for f in ga:
        scale = max(np.abs(gb[f]).max(), 1e-30)
        assert np.abs(ga[f] - gb[f]).max() <= 1e-6 * scale, f
    if scene == "sparse":
        compare_spectra(Ca, oracle_render(wl, mode))
    r.close()
