"""Host-side batch planning of the serving loop (no GPU): arrival-order
prefix, receiver and query caps, and the workspace budget."""
from paper_2605_24290_amd import rxgs

K, H, W = 200_000, 90, 360


def test_prefix_caps():
    take, b = rxgs.plan_batch([10, 20, 30, 40], "tx", K, H, W, 1 << 40, 55, 64)
    assert take == 2   # 10 + 20 <= 55, + 30 > 55
    take, _ = rxgs.plan_batch([10, 20, 30, 40], "tx", K, H, W, 1 << 40, 1000, 3)
    assert take == 3
    take, _ = rxgs.plan_batch([], "tx", K, H, W, 1 << 40, 1000, 3)
    assert take == 0


def test_budget_limits_prefix():
    one = rxgs.workspace_estimate("tx", 1, 100, K, H, W)
    two = rxgs.workspace_estimate("tx", 2, 200, K, H, W)
    assert 0 < one < two
    take, b = rxgs.plan_batch([100, 100, 100], "tx", K, H, W, two, 10_000, 64)
    assert take == 2 and b == two
    take, _ = rxgs.plan_batch([100], "tx", K, H, W, one - 1, 10_000, 64)
    assert take == 0


def test_rx_mode_costs_more_per_receiver():
    assert rxgs.workspace_estimate("rx", 1, 64, K, H, W) > rxgs.workspace_estimate("tx", 1, 64, K, H, W)
    assert rxgs.workspace_estimate("tx", 1, 0, K, H, W) == 0
