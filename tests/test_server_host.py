"""The serving scheduler against the library's host-only executor (no GPU):
continuous batching routes every result to its ticket, the admission budget
caps each batch, a batch that fails at launch (the allocator returned NULL:
E_OOM) or on the device is replayed once and only its own tickets can fail,
the worker keeps serving afterwards, and cancel / stop / invalid queries
behave as the ABI states.  The host executor's batch "renders" power_j =
tx.x + r.x + 2 r.y + 3 r.z per receiver."""
import numpy as np
import pytest

from paper_2605_24290_amd import rxgs

E_INVALID, E_OOM, E_DEVICE, E_CANCELLED = 1, 2, 3, 7
K, H, W = 200_000, 90, 360


def _queries(n, seed=1, max_rx=20):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        m = int(rng.integers(1, max_rx + 1))
        out.append((rng.uniform(0, 10, 3).astype(np.float32), rng.uniform(0, 10, (m, 3)).astype(np.float32)))
    return out


def _expected(tx, rx):
    return (tx[0] + rx[:, 0] + 2 * rx[:, 1] + 3 * rx[:, 2]).astype(np.float32)


def _server(slots=2, delay_us=2000, fail_launch=0, fail_device=0, budget=1 << 40, max_q=16, max_rx=2048):
    return rxgs.Server(None, mode="tx", slots=slots, max_queries_per_batch=max_q, max_rx_per_batch=max_rx,
                       mem_budget_bytes=budget,
                       host_executor=dict(K=K, H=H, W=W, delay_us=delay_us, fail_launch_mask=fail_launch,
                                          fail_device_mask=fail_device))


def _collect(srv, tickets):
    out = []
    for t in tickets:
        try:
            p, _, info = srv.poll(t, 20_000)
            out.append((0, p, info))
        except rxgs.RxgsError as e:
            out.append((e.status, None, getattr(e, "info", None)))
    return out


def test_results_reach_their_tickets_in_continuous_batches():
    qs = _queries(60)
    srv = _server()
    tickets = [srv.submit(tx, rx) for tx, rx in qs]
    res = _collect(srv, tickets)
    for (tx, rx), (st, p, info) in zip(qs, res):
        assert st == 0
        assert np.array_equal(p, _expected(tx, rx))
        assert info["attempts"] == 1
    assert max(i["batch_queries"] for _, _, i in res) > 1, "nothing was batched"
    s = srv.stats()
    assert s["completed"] == 60 and s["failed"] == 0 and s["failed_batches"] == 0
    assert s["batches"] < 60
    srv.stop()


def test_admission_budget_caps_every_batch():
    budget = rxgs.workspace_estimate("tx", 2, 30, K, H, W)
    qs = _queries(40, seed=3, max_rx=12)
    srv = _server(slots=1, budget=budget, max_q=64)
    res = _collect(srv, [srv.submit(tx, rx) for tx, rx in qs])
    for st, _, info in res:
        assert st == 0
        assert rxgs.workspace_estimate("tx", info["batch_queries"], info["batch_receivers"], K, H, W) <= budget
    with pytest.raises(rxgs.RxgsError) as e:   # one query alone over the per-slot budget
        srv.submit(qs[0][0], np.ones((500, 3), np.float32))
    assert e.value.status == E_INVALID
    assert srv.stats()["rejected"] == 1
    srv.stop()


def test_failed_launch_is_replayed_once_and_fails_only_its_tickets():
    qs = _queries(30, seed=5)
    # launch 0 fails (the allocator returned NULL): its tickets ride a later
    # batch and complete
    srv = _server(slots=1, delay_us=3000, fail_launch=0b1, max_q=4)
    res = _collect(srv, [srv.submit(tx, rx) for tx, rx in qs])
    assert all(st == 0 for st, _, _ in res)
    for (tx, rx), (_, p, _) in zip(qs, res):
        assert np.array_equal(p, _expected(tx, rx))
    assert any(i["attempts"] == 2 for _, _, i in res)
    s = srv.stats()
    assert s["failed_batches"] == 1 and s["failed"] == 0 and s["completed"] == 30 and s["replayed"] >= 1
    srv.stop()
    # launches 0 and 1 fail: tickets that rode both fail with E_OOM, every
    # other ticket completes, and the worker keeps serving
    srv = _server(slots=1, delay_us=3000, fail_launch=0b11, max_q=4)
    tickets = [srv.submit(tx, rx) for tx, rx in qs]
    res = _collect(srv, tickets)
    failed = [i for i, (st, _, _) in enumerate(res) if st != 0]
    assert failed, "the scripted failures did not fail any ticket"
    for i in failed:
        st, _, info = res[i]
        assert st == E_OOM and info["attempts"] == 2
    done = [i for i in range(len(qs)) if i not in failed]
    assert len(failed) <= 4 and len(done) == len(qs) - len(failed)
    for i in done:
        assert np.array_equal(res[i][1], _expected(*qs[i]))
    s = srv.stats()
    assert s["failed_batches"] == 2 and s["failed"] == len(failed) and s["completed"] == len(done)
    st, p, _ = _collect(srv, [srv.submit(*qs[0])])[0]
    assert st == 0 and np.array_equal(p, _expected(*qs[0]))
    srv.stop()


def test_device_failure_is_replayed():
    qs = _queries(20, seed=7)
    srv = _server(slots=2, fail_device=0b1)
    res = _collect(srv, [srv.submit(tx, rx) for tx, rx in qs])
    assert all(st == 0 for st, _, _ in res)
    assert any(i["attempts"] == 2 for _, _, i in res)
    for (tx, rx), (_, p, _) in zip(qs, res):
        assert np.array_equal(p, _expected(tx, rx))
    s = srv.stats()
    assert s["failed_batches"] == 1 and s["failed"] == 0 and s["completed"] == 20
    srv.stop()
    # failing twice: E_DEVICE for the tickets that rode both batches
    srv = _server(slots=1, fail_device=0b11, max_q=3)
    res = _collect(srv, [srv.submit(tx, rx) for tx, rx in qs[:6]])
    codes = [st for st, _, _ in res]
    assert E_DEVICE in codes and 0 in codes
    srv.stop()


def test_cancel_stop_and_invalid_queries():
    qs = _queries(30, seed=9)
    srv = _server(slots=1, delay_us=20_000, max_q=1)
    tickets = [srv.submit(tx, rx) for tx, rx in qs]
    assert srv.cancel(tickets[-1]) == 0
    with pytest.raises(rxgs.RxgsError) as e:
        srv.poll(tickets[-1], 1000)
    assert e.value.status == E_CANCELLED
    bad = qs[0][1].copy()
    bad[0, 0] = np.nan
    with pytest.raises(rxgs.RxgsError):
        srv.submit(qs[0][0], bad)
    with pytest.raises(rxgs.RxgsError):
        srv.submit(qs[0][0], np.ones((3000, 3), np.float32))   # over max_rx_per_batch
    st, p, _ = _collect(srv, tickets[:1])[0]
    assert st == 0
    srv.stop()   # cancels what is still queued
    s = srv.stats() if srv._h is not None else None
    assert s is None


def test_host_executor_rejects_bad_options():
    with pytest.raises(rxgs.RxgsError):
        rxgs.Server(None, slots=0, mem_budget_bytes=1 << 30, host_executor=dict())
    with pytest.raises(rxgs.RxgsError):
        rxgs.Server(None, mem_budget_bytes=1 << 30, want_spectra=True, host_executor=dict())
