"""Continuous-batching recovery server on one GPU.

Requests (each a few images of one size and measurement ratio, i.e. one
prepared network) arrive over time.  The scheduler keeps one FIFO queue per
network, and whenever an execution slot (a HIP stream with its own libdsi
context and workspace) is free it forms the next batch:

  * fairness: the network whose oldest waiting image arrived first is served
    first, so no network starves;
  * continuous batching: the batch takes every waiting image of that network,
    splitting requests across batches when needed, up to the largest batch
    size ("bucket") the HBM budget admits;
  * admission: the HBM budget is the device memory for batches, allocated once
    as one arena per execution slot (the slot's workspace and staging); a batch
    is formed only in a bucket whose workspace and staging fit an arena, and
    launched only while the bytes of all batches in flight plus its own stay
    within the budget;
  * execution: every admissible (network, bucket, slot) has a HIP graph
    captured once around dsi_recover on the slot's staging buffers; a launch copies the batch's
    measurement vectors into the staging input, replays the graph on the
    slot's stream and records an event; completion is found by polling the
    events, so batches from different networks overlap on the device.

A request's latency is the time from its arrival to the host seeing its last
image done.  The scheduler is written against an Executor interface so its
policy is testable without a GPU (FakeExecutor).
"""
from __future__ import annotations

import collections
import heapq
import time
from dataclasses import dataclass, field

import numpy as np

DEFAULT_BUCKETS = (1, 2, 4, 8, 16, 32, 64, 128, 256)


@dataclass
class Request:
    rid: int
    net: int            # index of the prepared network
    n: int              # images
    arrival: float      # seconds on the server clock
    y: object = None    # [n][M] device tensor (GPU executor)
    done_images: int = 0
    finish: float | None = None
    out: object = None  # [n][n1][n2] device tensor, filled as batches complete

    @property
    def latency(self):
        return None if self.finish is None else self.finish - self.arrival


@dataclass
class Piece:
    req: Request
    start: int   # first image of the request in this batch
    count: int


@dataclass
class Batch:
    net: int
    bucket: int
    pieces: list
    slot: int
    nbytes: int
    launched: float
    handle: object = None

    @property
    def images(self):
        return sum(p.count for p in self.pieces)


class Admission:
    """HBM budget: bytes of the batches in flight never exceed `budget`."""

    def __init__(self, budget: int):
        self.budget = int(budget)
        self.in_flight = 0
        self.peak = 0

    def fits(self, nbytes: int) -> bool:
        return self.in_flight + nbytes <= self.budget

    def take(self, nbytes: int):
        if not self.fits(nbytes):
            raise RuntimeError("admission over budget")
        self.in_flight += nbytes
        self.peak = max(self.peak, self.in_flight)

    def give(self, nbytes: int):
        self.in_flight -= nbytes
        assert self.in_flight >= 0


class Batcher:
    """Per-network FIFO queues of (request, next image)."""

    def __init__(self, n_nets: int):
        self.q = [collections.deque() for _ in range(n_nets)]

    def push(self, req: Request):
        self.q[req.net].append([req, 0])

    def waiting(self) -> int:
        return sum(sum(r.n - s for r, s in q) for q in self.q)

    def oldest_net(self):
        best, t = None, None
        for k, q in enumerate(self.q):
            if q and (t is None or q[0][0].arrival < t):
                best, t = k, q[0][0].arrival
        return best

    def queued_images(self, net: int) -> int:
        return sum(r.n - s for r, s in self.q[net])

    def take(self, net: int, max_images: int) -> list:
        pieces, left = [], max_images
        q = self.q[net]
        while q and left > 0:
            entry = q[0]
            req, start = entry
            cnt = min(req.n - start, left)
            pieces.append(Piece(req, start, cnt))
            left -= cnt
            if start + cnt == req.n:
                q.popleft()
            else:
                entry[1] = start + cnt
        return pieces


class Executor:
    """What the scheduler needs from the device side."""

    n_slots: int = 1

    def batch_bytes(self, net: int, bucket: int) -> int:
        raise NotImplementedError

    def admissible(self, net: int, bucket: int) -> bool:
        """Whether a batch of this bucket can run at all (fits one slot's memory)."""
        return True

    def launch(self, batch: Batch):
        raise NotImplementedError

    def done(self, batch: Batch) -> bool:
        raise NotImplementedError

    def finish(self, batch: Batch):
        """Hand each piece its results (after done())."""

    def now(self) -> float:
        return time.perf_counter()

    def idle(self, until: float | None):
        """Wait a little (nothing to launch and nothing finished)."""
        time.sleep(0.0 if until is None else max(0.0, min(until - self.now(), 2e-4)))


class Server:
    def __init__(self, executor: Executor, n_nets: int, buckets=DEFAULT_BUCKETS, budget: int = 1 << 40):
        self.ex = executor
        self.buckets = tuple(sorted(buckets))
        self.adm = Admission(budget)
        self.batcher = Batcher(n_nets)
        self.free_slots = list(range(executor.n_slots))
        self.in_flight: list[Batch] = []
        self.batches: list[Batch] = []
        self.max_concurrent = 0
        self.n_finished = 0
        smallest = [executor.batch_bytes(k, self.buckets[0]) for k in range(n_nets)]
        for k, b in enumerate(smallest):
            if b > self.adm.budget or not executor.admissible(k, self.buckets[0]):
                raise ValueError(f"net {k}: one image needs {b} bytes, over the budget {self.adm.budget}")

    def _bucket_for(self, net: int, images: int):
        """Smallest bucket holding `images`, shrunk until it fits the free budget."""
        fit = [b for b in self.buckets
               if self.ex.admissible(net, b) and self.adm.fits(self.ex.batch_bytes(net, b))]
        if not fit:
            return None, 0
        cover = [b for b in fit if b >= images]
        bucket = cover[0] if cover else fit[-1]
        return bucket, min(bucket, images)

    def _try_launch(self) -> bool:
        if not self.free_slots:
            return False
        net = self.batcher.oldest_net()
        if net is None:
            return False
        bucket, take = self._bucket_for(net, self.batcher.queued_images(net))
        if bucket is None:
            return False   # wait for memory to free up
        pieces = self.batcher.take(net, take)
        nbytes = self.ex.batch_bytes(net, bucket)
        self.adm.take(nbytes)
        b = Batch(net, bucket, pieces, self.free_slots.pop(0), nbytes, self.ex.now())
        self.ex.launch(b)
        self.in_flight.append(b)
        self.batches.append(b)
        self.max_concurrent = max(self.max_concurrent, len(self.in_flight))
        return True

    def _poll(self) -> bool:
        progressed = False
        for b in list(self.in_flight):
            if self.ex.done(b):
                t = self.ex.now()
                self.ex.finish(b)
                for p in b.pieces:
                    p.req.done_images += p.count
                    if p.req.done_images == p.req.n:
                        p.req.finish = t
                        self.n_finished += 1
                self.in_flight.remove(b)
                self.free_slots.append(b.slot)
                self.adm.give(b.nbytes)
                progressed = True
        return progressed

    def run(self, requests: list, t0: float | None = None) -> dict:
        """Serve requests whose .arrival is relative to the start; returns statistics."""
        arrivals = [(r.arrival, r.rid, r) for r in requests]
        heapq.heapify(arrivals)
        start = self.ex.now() if t0 is None else t0
        for r in requests:
            r.arrival += start
        total = len(requests)
        self.n_finished = 0
        finished = 0
        while finished < total:
            now = self.ex.now()
            while arrivals and arrivals[0][0] + start <= now:
                self.batcher.push(heapq.heappop(arrivals)[2])
            progressed = self._poll()
            while self._try_launch():
                progressed = True
            finished = self.n_finished
            if not progressed and finished < total:
                nxt = arrivals[0][0] + start if arrivals else None
                self.ex.idle(nxt)
        end = self.ex.now()
        lat = np.array([r.latency for r in requests])
        imgs = sum(r.n for r in requests)
        return {"requests": total, "images": imgs, "seconds": end - start,
                "images_per_s": imgs / (end - start), "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
                "batches": len(self.batches), "mean_batch": imgs / max(1, len(self.batches)),
                "max_concurrent_batches": self.max_concurrent, "peak_bytes": self.adm.peak}


# --------------------------------------------------------------- executors
class FakeExecutor(Executor):
    """Cost-model executor on a simulated clock (no GPU): a batch of bucket b on
    net k takes cost(k, b) seconds; slots run in parallel."""

    def __init__(self, n_slots, bytes_fn, cost_fn):
        self.n_slots = n_slots
        self.bytes_fn, self.cost_fn = bytes_fn, cost_fn
        self.t = 0.0
        self.ends = []
        self.log = []

    def batch_bytes(self, net, bucket):
        return self.bytes_fn(net, bucket)

    def now(self):
        return self.t

    def launch(self, batch):
        batch.handle = self.t + self.cost_fn(batch.net, batch.bucket)
        self.ends.append(batch.handle)
        self.log.append(("launch", self.t, batch.net, batch.bucket, batch.images, batch.slot))

    def done(self, batch):
        return self.t >= batch.handle

    def idle(self, until):
        """Jump the simulated clock to the next completion or arrival."""
        pending = [e for e in self.ends if e > self.t]
        nxt = min(pending) if pending else None
        if until is not None and (nxt is None or until < nxt):
            nxt = until
        self.t = nxt if nxt is not None and nxt > self.t else self.t + 1e-6


class GraphExecutor(Executor):
    """libdsi on one GPU, with every byte a batch uses inside the HBM budget.

    The budget is split into one arena per slot (a HIP stream with its own libdsi
    context).  An arena is its context's workspace (dsi_set_workspace) and, in its
    tail, holds the staging buffers of the batch running on the slot, so device
    memory for batches is allocated once, at exactly the budget.  A (net, bucket)
    is admissible when its workspace plus staging fits one arena: a smaller budget
    caps the bucket sizes, and the scheduler never forms a batch that does not fit.
    Per admissible (net, bucket, slot) one HIP graph is captured around dsi_recover.
    The prepared networks (the resident weights) are shared by the slots."""

    def __init__(self, nets, n_slots=4, buckets=DEFAULT_BUCKETS, device=0, budget=16 << 30):
        import torch

        import paper_1701_03891_amd as P
        self.torch, self.P = torch, P
        self.nets = nets            # list of (desc tuple (n1, n2, M), NetParams, prec)
        self.n_slots = n_slots
        self.buckets = tuple(sorted(buckets))
        self.device = device
        dev = f"cuda:{device}"
        self.arena_bytes = (int(budget) // n_slots) // 256 * 256
        self.streams = [torch.cuda.Stream(device) for _ in range(n_slots)]
        self.ctxs = [P.Context(device) for _ in range(n_slots)]
        self.arenas = [torch.empty(self.arena_bytes, dtype=torch.uint8, device=dev) for _ in range(n_slots)]
        for c, a in zip(self.ctxs, self.arenas):
            c.set_workspace(a)
        self.handles = [self.ctxs[0].prepare(*shape, params, prec=prec) for shape, params, prec in nets]
        self.weight_bytes = sum(params.w_fc.numel() * 2 for _, params, _ in nets)   # BF16 W_fc dominates
        self.graphs = {}    # (net, bucket, slot) -> (graph, y_static, x_static)
        self._need = {}     # (net, bucket) -> (workspace bytes, staging bytes)
        rnd = lambda v: (v + 255) // 256 * 256  # noqa: E731
        for k, (shape, params, prec) in enumerate(nets):
            n1, n2, M = shape
            for b in self.buckets:
                self._need[(k, b)] = (self.handles[k].workspace_size(b), rnd(b * M * 4) + rnd(b * n1 * n2 * 4))
            if not self.admissible(k, self.buckets[0]):
                raise ValueError(f"net {k}: a batch of {self.buckets[0]} needs {sum(self._need[(k, self.buckets[0])])} "
                                 f"bytes, over one slot's arena of {self.arena_bytes}")
        torch.cuda.synchronize(device)
        # staging views in the arena's tail, then capture
        for k, (shape, params, prec) in enumerate(nets):
            n1, n2, M = shape
            net = self.handles[k]
            for s in range(n_slots):
                for b in self.buckets:
                    if not self.admissible(k, b):
                        continue
                    _, stage = self._need[(k, b)]
                    tail = self.arenas[s][self.arena_bytes - stage:]
                    ys = tail[:b * M * 4].view(torch.float32).view(b, M)
                    xo = rnd(b * M * 4)
                    xs = tail[xo:xo + b * n1 * n2 * 4].view(torch.float32).view(b, n1, n2)
                    with torch.cuda.stream(self.streams[s]):
                        ys.zero_()
                        self._recover(net, s, ys, xs)      # warm-up outside capture
                    self.streams[s].synchronize()
                    g = torch.cuda.CUDAGraph()
                    with torch.cuda.graph(g, stream=self.streams[s]):
                        self._recover(net, s, ys, xs)
                    self.graphs[(k, b, s)] = (g, ys, xs)
        torch.cuda.synchronize(device)

    def _recover(self, net, slot, ys, xs):
        """dsi_recover of a shared network with this slot's context (workspace)."""
        P = self.P
        P._lib.dsi_recover(self.ctxs[slot].h, net.h, P._ptr(ys), P._ptr(xs), ys.shape[0],
                           P._stream(self.device))

    def admissible(self, net, bucket) -> bool:
        return sum(self._need[(net, bucket)]) <= self.arena_bytes

    def batch_bytes(self, net, bucket):
        return sum(self._need[(net, bucket)])

    def launch(self, batch):
        """Stage inputs, replay the graph, hand the outputs back, all on the slot's stream
        (request y and out tensors are allocated before serving starts)."""
        torch = self.torch
        g, ys, xs = self.graphs[(batch.net, batch.bucket, batch.slot)]
        st = self.streams[batch.slot]
        with torch.cuda.stream(st):
            row = 0
            for p in batch.pieces:
                ys[row:row + p.count].copy_(p.req.y[p.start:p.start + p.count], non_blocking=True)
                row += p.count
            g.replay()
            row = 0
            for p in batch.pieces:
                p.req.out[p.start:p.start + p.count].copy_(xs[row:row + p.count], non_blocking=True)
                row += p.count
            ev = torch.cuda.Event()
            ev.record(st)
        batch.handle = ev

    def done(self, batch):
        return batch.handle.query()

    def close(self):
        self.graphs.clear()
        for net in self.handles:
            net.free()
        for c in self.ctxs:
            c.close()
        self.arenas = []


# ------------------------------------------------------------ benchmark driver
def make_workload(sizes=(32, 64, 128), ratios=(0.10, 0.25, 0.50), cfg_id=7, device="cuda:0"):
    """One He-initialised network per (image size, ratio), with its own Gaussian Phi."""
    import torch

    import synth
    from paper_1701_03891_amd import NetParams
    nets, phis = [], []
    for q, n in enumerate(sizes):
        for r_i, r in enumerate(ratios):
            M = synth.m_for_ratio(r, n * n)
            cid = cfg_id * 100 + q * 10 + r_i
            phi = synth.make_phi(M, n * n, cfg_id=cid)
            prm = synth.he_init(synth.PAPER_ARCH, n, n, bias_per_pixel=True, cfg_id=cid)
            t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=device)  # noqa: E731
            nets.append(((n, n, M), NetParams(t(phi.T), [t(w) for w in prm.w], [t(b) for b in prm.b]), "bf16"))
            phis.append(t(phi))
    return nets, phis


def make_requests(nets, phis, n_req, qps, max_images=32, cfg_id=7, device="cuda:0"):
    """Poisson arrivals; each request: U{1..max_images} images of a uniformly chosen net,
    measured on the device (y = Phi x, resident in HBM) with its output preallocated."""
    import torch

    import synth
    from paper_1701_03891_amd import Context
    g = synth.rng(cfg_id, synth.STREAM_ARRIVALS)
    t = synth.poisson_arrivals(n_req, qps, cfg_id=cfg_id)
    ctx = Context(int(str(device).split(":")[-1]) if ":" in str(device) else 0)
    reqs = []
    pools = {}
    for i in range(n_req):
        k = int(g.integers(0, len(nets)))
        nimg = int(g.integers(1, max_images + 1))
        n1, n2, M = nets[k][0]
        if k not in pools:   # a pool of synthetic images per net, measured once
            xs = synth.piecewise_smooth_images(64, n1, n2, cfg_id=cfg_id * 1000 + k)
            x = torch.tensor(xs.reshape(64, -1), dtype=torch.float32, device=device)
            pools[k] = ctx.measure(phis[k], x)
        off = int(g.integers(0, 64 - nimg + 1))
        y = pools[k][off:off + nimg].clone()
        out = torch.empty((nimg, n1, n2), dtype=torch.float32, device=device)
        reqs.append(Request(i, k, nimg, float(t[i]), y=y, out=out))
    torch.cuda.synchronize()
    ctx.close()
    return reqs


def run_serving(n_req=2000, qps=2000.0, slots=4, budget_gib=16.0, buckets=DEFAULT_BUCKETS, warmup=200,
                sizes=(32, 64, 128), ratios=(0.10, 0.25, 0.50)):
    """One load point: `warmup` unmeasured requests, then n_req measured ones at `qps`."""
    return sweep_serving((qps,), n_req, slots, budget_gib, buckets, warmup, sizes, ratios,
                         at_fraction=None)["points"][0]


def sweep_serving(qps_list, n_req=10000, slots=4, budget_gib=16.0, buckets=DEFAULT_BUCKETS, warmup=1000,
                  sizes=(32, 64, 128), ratios=(0.10, 0.25, 0.50), at_fraction=0.7, log=None):
    """Latency and throughput over offered loads.  Saturation is the delivered image
    rate at the highest offered load (offered above capacity, the server delivers its
    capacity); with at_fraction set, one more point runs at that fraction of it."""
    import torch
    nets, phis = make_workload(sizes, ratios)
    budget = int(budget_gib * (1 << 30))
    ex = GraphExecutor(nets, n_slots=slots, buckets=buckets, budget=budget)
    Server(ex, len(nets), buckets, budget).run(make_requests(nets, phis, warmup, max(qps_list), cfg_id=8))

    def point(qps, cfg_id=7):
        reqs = make_requests(nets, phis, n_req, qps, cfg_id=cfg_id)
        st = Server(ex, len(nets), buckets, budget).run(reqs)
        torch.cuda.synchronize()
        st.update({"qps": qps, "slots": slots, "budget_bytes": budget, "nets": len(nets),
                   "arena_bytes_per_slot": ex.arena_bytes,
                   "max_bucket_per_net": [max(b for b in buckets if ex.admissible(k, b)) for k in range(len(nets))]})
        del reqs
        if log:
            log(f"serving: {qps:.0f} req/s offered -> {st['images_per_s']:.0f} images/s, "
                f"p50 {st['p50_ms']:.2f} ms, p99 {st['p99_ms']:.2f} ms")
        return st

    pts = [point(q) for q in qps_list]
    out = {"points": pts}
    if at_fraction is not None:
        top = max(pts, key=lambda p: p["qps"])
        sat_img = top["images_per_s"]
        img_per_req = top["images"] / top["requests"]
        q = at_fraction * sat_img / img_per_req
        out["saturation_images_per_s"] = sat_img
        out["at_fraction"] = at_fraction
        out["at_fraction_point"] = point(q, cfg_id=9)
    ex.close()
    return out


if __name__ == "__main__":
    import argparse
    import json
    ap = argparse.ArgumentParser(description="continuous-batching recovery server benchmark")
    ap.add_argument("--requests", type=int, default=3000)
    ap.add_argument("--qps", type=float, default=2000.0)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--budget-gib", type=float, default=16.0)
    a = ap.parse_args()
    print(json.dumps(run_serving(a.requests, a.qps, a.slots, a.budget_gib)))
