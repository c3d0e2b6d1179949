"""Serving loop on the GPU: graph-replayed batches of mixed networks overlap on
two or four streams, and every request's result is bit-identical to recovering
that request alone (per-image results do not depend on the batch they run in).
The mix holds all nine networks of the serving workload: 32x32, 64x64 and
128x128 images at M/N = 0.10, 0.25 and 0.50."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("slots", [2, 4])
def test_served_results_equal_results_alone(slots):
    import torch

    import paper_1701_03891_amd as P
    from paper_1701_03891_amd import serve
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    nets, phis = serve.make_workload(sizes=(32, 64, 128), ratios=(0.10, 0.25, 0.50))
    assert len(nets) == 9
    buckets = (1, 2, 4, 8, 16, 32, 64)
    ex = serve.GraphExecutor(nets, n_slots=slots, buckets=buckets, budget=8 << 30)
    reqs = serve.make_requests(nets, phis, 400, qps=20000.0, max_images=24)
    assert {r.net for r in reqs} == set(range(9))
    srv = serve.Server(ex, len(nets), buckets, budget=8 << 30)
    stats = srv.run(reqs)
    torch.cuda.synchronize()
    print("serving:", stats)
    assert all(r.finish is not None for r in reqs)
    assert stats["max_concurrent_batches"] >= 2
    assert stats["mean_batch"] > 1.5        # requests were merged
    ctx = P.Context(0)
    alone = [ctx.prepare(*shape, params, prec=prec) for shape, params, prec in nets]
    mism = 0
    for r in reqs:
        ref = alone[r.net].recover(r.y)
        if not torch.equal(ref, r.out):
            mism += 1
    for a in alone:
        a.free()
    ctx.close()
    ex.close()
    assert mism == 0, f"{mism} requests differ from their results alone"
    assert stats["p99_ms"] >= stats["p50_ms"] > 0


def test_small_budget_caps_buckets_and_bounds_device_memory():
    """A 1 GiB budget on 4 slots: the executor allocates exactly the budget for batches
    (one 256 MiB arena per slot, workspace plus staging), the 128 x 128 networks are
    capped below the largest bucket, every batch fits its arena, and every request's
    result is still bit-identical to recovering it alone."""
    import torch

    import paper_1701_03891_amd as P
    from paper_1701_03891_amd import serve
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    nets, phis = serve.make_workload(sizes=(32, 64, 128), ratios=(0.10, 0.25, 0.50))
    buckets = (1, 2, 4, 8, 16, 32, 64, 128, 256)
    budget = 1 << 30
    import gc
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    alloc0, free0 = torch.cuda.memory_allocated(), torch.cuda.mem_get_info()[0]
    ex = serve.GraphExecutor(nets, n_slots=4, buckets=buckets, budget=budget)
    torch.cuda.synchronize()
    # the bytes the executor takes through torch are its arenas, exactly the budget's share,
    # plus the few hundred bytes torch's graph capture keeps for itself
    arenas = torch.cuda.memory_allocated() - alloc0
    used = free0 - torch.cuda.mem_get_info()[0]
    print(f"executor: arenas {arenas / 2**20:.0f} MiB (budget {budget / 2**20:.0f} MiB); device-wide "
          f"{used / 2**20:.0f} MiB including the prepared networks' weights")
    assert 4 * ex.arena_bytes <= arenas <= 4 * ex.arena_bytes + (64 << 10)
    assert ex.arena_bytes * 4 <= budget
    caps = [max(b for b in buckets if ex.admissible(k, b)) for k in range(9)]
    print("largest admissible bucket per net:", caps)
    assert max(caps[6:]) < 256 and min(caps[:3]) == 256
    reqs = serve.make_requests(nets, phis, 300, qps=50000.0, max_images=32)
    srv = serve.Server(ex, len(nets), buckets, budget=budget)
    stats = srv.run(reqs)
    torch.cuda.synchronize()
    assert all(r.finish is not None for r in reqs)
    assert all(ex.batch_bytes(b.net, b.bucket) <= ex.arena_bytes for b in srv.batches)
    assert all(b.bucket <= caps[b.net] for b in srv.batches)
    assert srv.adm.peak <= budget
    ctx = P.Context(0)
    alone = [ctx.prepare(*shape, params, prec=prec) for shape, params, prec in nets]
    mism = sum(0 if torch.equal(alone[r.net].recover(r.y), r.out) else 1 for r in reqs)
    for a in alone:
        a.free()
    ctx.close()
    ex.close()
    print("serving at 1 GiB:", stats)
    assert mism == 0
