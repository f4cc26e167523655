"""Continuous-batching server on the GPU: a query's result is the same alone
and in a mix of concurrently batched queries, equals a direct render, respects
the memory budget, supports cancellation, and reports latency percentiles."""
import math

import numpy as np
import pytest

from paper_2605_24290_amd import scenes as S

from .parity import gpu, needs_gpu, renderer_for

pytestmark = [gpu, needs_gpu]


def _renderer(K=20_000):
    wl = S.make_workload("c3", K=K, N=1)
    return wl, renderer_for(wl)


@pytest.mark.parametrize("mode", ["tx", "rx"])
def test_alone_equals_mix_and_direct_render(mode):
    import torch
    from paper_2605_24290_amd import rxgs
    wl, r = _renderer()
    qs = S.serving_queries(123, 24, wl.scene.means.max(axis=0), max_rx=40)
    srv = rxgs.Server(r, mode=mode, slots=2, max_queries_per_batch=16, want_spectra=True)
    probe = qs[5]
    t = srv.submit(probe[1], probe[2])
    p_alone, C_alone, info_alone = srv.poll(t, 30_000)
    assert info_alone["batch_queries"] == 1
    tickets = [srv.submit(q[1], q[2]) for q in qs]
    res = [srv.poll(tk, 60_000) for tk in tickets]
    p_mix, C_mix, info_mix = res[5]
    assert max(i["batch_queries"] for _, _, i in res) > 1, "no query was batched with another"
    scale = np.abs(C_alone).max()
    assert np.abs(C_mix - C_alone).max() <= 1e-4 * scale
    assert np.abs(p_mix - p_alone).max() <= 1e-4 * np.abs(p_alone).max()
    print(f"[serving] alone vs mix bit-identical: {np.array_equal(C_mix, C_alone)} "
          f"(batch of {info_mix['batch_queries']} queries)")
    # direct render of the same query
    C, P, _ = r.render(probe[2], tx=probe[1][None], mode=mode)
    torch.cuda.synchronize()
    assert np.abs(C.cpu().numpy() - C_alone).max() <= 1e-4 * scale
    st = srv.stats()
    assert st["completed"] == 25 and st["failed"] == 0
    srv.stop()
    r.close()


def test_memory_budget_caps_batches_and_cancel():
    from paper_2605_24290_amd import rxgs
    wl, r = _renderer()
    K, H, W = wl.scene.K, wl.grid.H, wl.grid.W
    budget = rxgs.workspace_estimate("tx", 2, 80, K, H, W)
    qs = S.serving_queries(7, 30, wl.scene.means.max(axis=0), max_rx=40)
    srv = rxgs.Server(r, mode="tx", slots=1, max_queries_per_batch=64, mem_budget_bytes=budget)
    tickets = [srv.submit(q[1], q[2]) for q in qs]
    srv.cancel(tickets[-1])
    for tk in tickets[:-1]:
        _, _, info = srv.poll(tk, 60_000)
        assert rxgs.workspace_estimate("tx", info["batch_queries"], info["batch_receivers"], K, H, W) <= budget
    with pytest.raises(rxgs.RxgsError):
        srv.poll(tickets[-1], 1000)
    big = np.zeros((41, 3), np.float32) + 1.0
    with pytest.raises(rxgs.RxgsError):
        srv.submit(qs[0][1], np.concatenate([big] * 100))
    srv.stop()
    r.close()


def test_open_loop_reports_percentiles():
    from paper_2605_24290_amd import rxgs, serving
    wl, r = _renderer()
    qs = S.serving_queries(9, 60, wl.scene.means.max(axis=0), max_rx=64)
    srv = rxgs.Server(r, mode="tx", slots=2)
    sat = serving.run_burst(srv, qs)
    res = serving.run_open_loop(srv, qs, rate=0.5 * sat["achieved_qps"])
    for k in ("p50_ms", "p99_ms", "achieved_qps"):
        assert math.isfinite(res[k]) and res[k] > 0
    assert res["p99_ms"] >= res["p50_ms"]
    print("[serving]", sat, res)
    srv.stop()
    r.close()
