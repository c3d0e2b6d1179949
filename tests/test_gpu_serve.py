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
    ex = serve.GraphExecutor(nets, n_slots=slots, buckets=buckets)
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
