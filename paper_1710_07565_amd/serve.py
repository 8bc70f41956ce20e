"""Request server: continuous batching of graph-generation requests.

Requests (n, model, directed, m or p, seed, P) arrive over time.  Every tick
the scheduler admits queued requests in arrival order while their output fits
the HBM budget, packs them into one kg_batch launch (one pass of the
generator over all of them) on the next of S streams, and keeps the edge
lists on the device.  Launches on different streams overlap on the GPU;
requests that arrive while others run are admitted as soon as memory frees
up.  A finished request's latency is completion time minus arrival time;
its memory returns to the budget when the client releases it.

The bytes of a request do not depend on what it was batched with: kg_batch
output for an instance equals kg_gnm / kg_gnp alone (the generator is a pure
function of the instance).
"""
import collections
import threading
import time

from . import _lib
from . import GNM, Instance, KgInstance, _stream


def _edge_bound(spec):
    """Output room for one request: exact for G(n,m); mean + 10 sd + 64 for
    G(n,p) (the slack is returned when the batch completes)."""
    if spec.model == GNM:
        return int(spec.m)
    N = spec.n * (spec.n - 1) // (1 if spec.directed else 2)
    mu = spec.p * N
    sd = (mu * max(1.0 - spec.p, 0.0)) ** 0.5
    return min(N, int(mu + 10.0 * sd + 64))


class Request:
    __slots__ = ("rid", "spec", "arrival", "admitted", "done", "edges", "offset", "batch", "nedges", "bound")

    def __init__(self, rid, spec, arrival):
        self.rid, self.spec, self.arrival = rid, spec, arrival
        self.admitted = self.done = None
        self.edges = None
        self.offset = self.nedges = None
        self.batch = None
        self.bound = _edge_bound(spec)


class _Batch:
    __slots__ = ("reqs", "arena", "offsets", "event", "stream", "ws", "bytes", "reqs_alive")


class Server:
    """Continuous-batching server over one GPU.

    budget_bytes : HBM the in-flight and unreleased outputs may hold
    streams    : launches in flight at once
    max_batch  : requests packed into one launch
    keep       : keep finished edge lists until release() (else release at once)
    on_done    : called with each finished request while its edges are valid
                 (the client's check), before an automatic release
    """

    def __init__(self, budget_bytes, streams=4, max_batch=256, keep=False, on_done=None, device="cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.budget = int(budget_bytes)
        self.used = 0
        self.keep = keep
        self.on_done = on_done
        self.max_batch = max_batch
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(streams)]
        self.next_stream = 0
        self.queue = collections.deque()
        self.inflight = []
        self.finished = []
        self.lock = threading.Lock()
        self.nreq = 0
        self.rejected = 0

    # -- client side -------------------------------------------------------
    def submit(self, spec, arrival=None):
        r = Request(self.nreq, spec, time.perf_counter() if arrival is None else arrival)
        self.nreq += 1
        if 8 * r.bound > self.budget:
            self.rejected += 1
            r.done = r.arrival
            return r
        with self.lock:
            self.queue.append(r)
        return r

    def release(self, req):
        """Client is done with a finished request's edges."""
        if req.edges is not None or req.batch is not None:
            req.edges = None
            b = req.batch
            req.batch = None
            if b is not None:
                b.reqs_alive -= 1
                if b.reqs_alive == 0:
                    self.used -= b.bytes
                    b.arena = None

    # -- scheduler ---------------------------------------------------------
    def _admit(self):
        take = []
        need = 0
        with self.lock:
            while self.queue and len(take) < self.max_batch:
                r = self.queue[0]
                nb = 8 * r.bound
                if self.used + need + nb > self.budget:
                    break
                self.queue.popleft()
                take.append(r)
                need += nb
        return take, need

    def _launch(self, reqs, need):
        import ctypes
        torch = self.torch
        now = time.perf_counter()
        stream = self.streams[self.next_stream]
        self.next_stream = (self.next_stream + 1) % len(self.streams)
        insts = [Instance(r.spec.n, r.spec.model, r.spec.directed, r.spec.m, r.spec.p, r.spec.seed, r.spec.chunks)
                 for r in reqs]
        arr = (KgInstance * len(insts))(*[i.c() for i in insts])
        wsb = ctypes.c_uint64(0)
        _lib.check(_lib.lib().kg_workspace_bytes(arr, len(insts), ctypes.byref(wsb)), "kg_workspace_bytes")
        cap = sum(r.bound for r in reqs)
        with torch.cuda.stream(stream):
            arena = torch.empty((max(cap, 1), 2), dtype=torch.uint32, device=self.device)
            offsets = torch.empty(len(reqs) + 1, dtype=torch.uint64, device=self.device)
            ws = torch.empty(max(wsb.value, 1), dtype=torch.uint8, device=self.device)
            st = _lib.lib().kg_batch(arr, len(insts), arena.data_ptr(), cap, offsets.data_ptr(), ws.data_ptr(),
                                     ws.numel(), _stream(stream))
            _lib.check(st, "kg_batch")
            ev = torch.cuda.Event()
            ev.record(stream)
        b = _Batch()
        b.reqs, b.arena, b.offsets, b.event, b.stream, b.ws, b.bytes = reqs, arena, offsets, ev, stream, ws, need
        self.used += need
        for r in reqs:
            r.admitted = now
            r.batch = b
        self.inflight.append(b)

    def _reap(self):
        torch = self.torch
        still = []
        for b in self.inflight:
            if not b.event.query():
                still.append(b)
                continue
            now = time.perf_counter()
            offs = b.offsets.view(torch.int64).cpu().tolist()
            b.ws = None
            b.reqs_alive = len(b.reqs)
            for i, r in enumerate(b.reqs):
                r.done = now
                r.offset, r.nedges = offs[i], offs[i + 1] - offs[i]
                r.edges = b.arena[offs[i]:offs[i + 1]]
                self.finished.append(r)
                if self.on_done is not None:
                    self.on_done(r)
            if not self.keep:
                for r in b.reqs:
                    self.release(r)
        self.inflight = still

    def step(self):
        """One scheduler tick: reap finished launches, admit and launch."""
        self._reap()
        if len(self.inflight) < len(self.streams):
            reqs, need = self._admit()
            if reqs:
                self._launch(reqs, need)
                return True
        return False

    def drain(self, timeout=600.0):
        t0 = time.perf_counter()
        while (self.queue or self.inflight) and time.perf_counter() - t0 < timeout:
            if not self.step():
                time.sleep(0.0002)
        self._reap()


def run_stream(server, stream, warmup_s=5.0, progress=None):
    """Replay an open-loop arrival stream [(t, spec), ...] in real time.
    Returns per-request records and summary statistics."""
    t0 = time.perf_counter()
    reqs = []
    i = 0
    last = t0
    while i < len(stream) or server.queue or server.inflight:
        now = time.perf_counter() - t0
        while i < len(stream) and stream[i][0] <= now:
            reqs.append(server.submit(stream[i][1], arrival=t0 + stream[i][0]))
            i += 1
        if not server.step():
            time.sleep(0.0001)
        if progress and time.perf_counter() - last > 5.0:
            last = time.perf_counter()
            progress(now, i, len(server.queue), len(server.inflight))
    server._reap()
    span = max(r.done for r in reqs) - t0 if reqs else 0.0
    lat = sorted(r.done - r.arrival for r in reqs if r.arrival - t0 >= warmup_s and r.done is not None)
    edges = sum(r.nedges or 0 for r in reqs)

    def pct(q):
        if not lat:
            return None
        return lat[min(len(lat) - 1, int(q * len(lat)))]
    return reqs, {"requests": len(reqs), "rejected": server.rejected, "edges": edges, "span_s": span,
                  "edges_per_s": edges / span if span > 0 else None, "p50_s": pct(0.50), "p99_s": pct(0.99),
                  "measured_after_s": warmup_s, "latency_samples": len(lat)}
