"""Scheduler policy of the serving loop on a simulated clock (no GPU):
budget never exceeded, FIFO order within a network, no starvation, request
splitting, bucket choice, batches from different networks in flight together."""
import numpy as np
import pytest

from paper_1701_03891_amd.serve import FakeExecutor, Request, Server

BUCKETS = (1, 2, 4, 8, 16, 32)


def _bytes(net, bucket):
    return (net + 1) * 1000 * bucket


def _cost(net, bucket):
    return 1e-3 * (1 + 0.1 * bucket) * (net + 1)


def _requests(n, n_nets, qps, max_imgs, seed):
    g = np.random.default_rng(seed)
    t = np.cumsum(g.exponential(1.0 / qps, size=n))
    return [Request(i, int(g.integers(0, n_nets)), int(g.integers(1, max_imgs + 1)), float(t[i])) for i in range(n)]


def test_all_requests_complete_within_budget_and_in_order():
    ex = FakeExecutor(3, _bytes, _cost)
    budget = 3 * 32 * 1000 + 5000
    srv = Server(ex, 3, BUCKETS, budget=budget)
    reqs = _requests(400, 3, 800.0, 12, seed=1)
    stats = srv.run(reqs)
    assert all(r.finish is not None and r.done_images == r.n for r in reqs)
    assert srv.adm.peak <= budget and srv.adm.in_flight == 0
    assert stats["max_concurrent_batches"] >= 2          # batches overlap across slots
    # FIFO within a network: images are launched in arrival order
    for k in range(3):
        order = [(p.req.arrival, p.start) for b in srv.batches if b.net == k for p in b.pieces]
        assert order == sorted(order)
    # every image is in exactly one batch, each batch fits its bucket
    assert sum(b.images for b in srv.batches) == sum(r.n for r in reqs)
    assert all(b.images <= b.bucket and b.bucket in BUCKETS for b in srv.batches)
    assert stats["p99_ms"] >= stats["p50_ms"] > 0


def test_large_request_is_split_and_budget_limits_bucket():
    ex = FakeExecutor(2, _bytes, _cost)
    srv = Server(ex, 1, BUCKETS, budget=8 * 1000)   # at most 8 images of net 0 in flight
    reqs = [Request(0, 0, 20, 0.0)]
    srv.run(reqs)
    assert reqs[0].done_images == 20
    assert max(b.bucket for b in srv.batches) <= 8
    assert srv.adm.peak <= 8000


def test_no_starvation_under_a_flood_of_one_net():
    ex = FakeExecutor(1, _bytes, _cost)
    srv = Server(ex, 2, BUCKETS, budget=1 << 30)
    reqs = [Request(i, 0, 32, 1e-4 * i) for i in range(50)]
    reqs.append(Request(50, 1, 1, 2e-4))
    srv.run(reqs)
    late = reqs[-1]
    # the lone request of net 1 is served right after the batch in flight when it arrived
    assert late.finish is not None and late.latency < 4 * _cost(0, 32) + _cost(1, 1)


def test_image_over_budget_is_rejected():
    ex = FakeExecutor(1, _bytes, _cost)
    with pytest.raises(ValueError):
        Server(ex, 2, BUCKETS, budget=1500)   # net 1 needs 2000 bytes for one image


def test_continuous_batching_merges_waiting_requests():
    ex = FakeExecutor(1, _bytes, _cost)
    srv = Server(ex, 1, BUCKETS, budget=1 << 30)
    reqs = [Request(i, 0, 3, 0.0) for i in range(5)]   # 15 images waiting at once
    srv.run(reqs)
    assert srv.batches[0].images == 15 and srv.batches[0].bucket == 16
