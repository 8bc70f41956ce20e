"""Request server: continuous batching of graph-generation requests.

Requests (n, model, directed, m or p, seed, P) arrive over time.  Every tick
the scheduler admits queued requests in arrival order while their output fits
the HBM budget, packs them into one kg_batch launch (one pass of the
generator over all of them) on the next of S streams, and keeps the edge
lists on the device.  Output space comes from one device arena of the budget's
size, allocated once; a first-fit range allocator hands out and takes back
contiguous ranges, so a launch never allocates device memory of its own.  Launches on different streams overlap on the GPU;
requests that arrive while others run are admitted as soon as memory frees
up.  A finished request's latency is completion time minus arrival time;
its memory returns to the budget when the client releases it.

The bytes of a request do not depend on what it was batched with: kg_batch
output for an instance equals kg_gnm / kg_gnp alone (the generator is a pure
function of the instance).  With `verify` the client checks every finished
request on the device before releasing it: a 64-bit checksum of its edge
list (kg_edge_hash, on the batch's stream), the edge count (exactly m for
G(n,m)), and for a seeded sample of the requests the checksum of the same
request generated alone.
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
    __slots__ = ("rid", "spec", "arrival", "admitted", "done", "edges", "offset", "batch", "nedges", "bound", "hash")

    def __init__(self, rid, spec, arrival):
        self.rid, self.spec, self.arrival = rid, spec, arrival
        self.admitted = self.done = None
        self.edges = None
        self.offset = self.nedges = None
        self.batch = None
        self.hash = None
        self.bound = _edge_bound(spec)


class _Ranges:
    """First-fit allocator of contiguous edge ranges in [0, cap)."""

    def __init__(self, cap):
        self.free = [(0, cap)]           # sorted, non-adjacent (start, length)

    def alloc(self, n):
        for i, (a, l) in enumerate(self.free):
            if l >= n:
                if l == n:
                    del self.free[i]
                else:
                    self.free[i] = (a + n, l - n)
                return a
        return None

    def release(self, a, n):
        import bisect
        i = bisect.bisect_left(self.free, (a, 0))
        self.free.insert(i, (a, n))
        # merge with the neighbours
        if i + 1 < len(self.free) and self.free[i][0] + self.free[i][1] == self.free[i + 1][0]:
            self.free[i] = (self.free[i][0], self.free[i][1] + self.free[i + 1][1])
            del self.free[i + 1]
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == self.free[i][0]:
            self.free[i - 1] = (self.free[i - 1][0], self.free[i - 1][1] + self.free[i][1])
            del self.free[i]


class _Batch:
    __slots__ = ("reqs", "start", "cap", "offsets", "event", "stream", "si", "ws", "bytes", "reqs_alive")


class Server:
    """Continuous-batching server over one GPU.

    budget_bytes : HBM the in-flight and unreleased outputs may hold
    streams    : launches in flight at once
    max_batch  : requests packed into one launch
    keep       : keep finished edge lists until release() (else release at once)
    on_done    : called with each finished request while its edges are valid
                 (the client's check), before an automatic release
    """

    def __init__(self, budget_bytes, streams=4, max_batch=256, keep=False, on_done=None, device="cuda",
                 verify=False, alone_every=100):
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
        # the output arena and a workspace per stream, allocated once
        self.arena_edges = self.budget // 8
        self.arena = torch.empty((self.arena_edges, 2), dtype=torch.uint32, device=self.device)
        self.ranges = _Ranges(self.arena_edges)
        self.ws = [None] * streams
        self.offsets = [torch.empty(max_batch + 1, dtype=torch.uint64, device=self.device) for _ in range(streams)]
        # client-side checks on the device (checksums, a sample re-generated alone)
        self.verify = verify
        self.alone_every = int(alone_every)
        self.verifying = []
        self.verified = 0
        self.checked_alone = 0
        self.verify_failures = []

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
                    self.ranges.release(b.start, b.cap)

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
        cap = max(sum(r.bound for r in reqs), 1)
        start = self.ranges.alloc(cap)
        if start is None:                    # fragmented: wait for releases
            with self.lock:
                self.queue.extendleft(reversed(reqs))
            return False
        now = time.perf_counter()
        # a stream whose previous batch has been reaped (its offsets buffer and
        # workspace are free again)
        busy = {b.si for b in self.inflight}
        si = next(i for i in range(len(self.streams)) if i not in busy)
        stream = self.streams[si]
        insts = [Instance(r.spec.n, r.spec.model, r.spec.directed, r.spec.m, r.spec.p, r.spec.seed, r.spec.chunks)
                 for r in reqs]
        arr = (KgInstance * len(insts))(*[i.c() for i in insts])
        wsb = ctypes.c_uint64(0)
        _lib.check(_lib.lib().kg_workspace_bytes(arr, len(insts), ctypes.byref(wsb)), "kg_workspace_bytes")
        with torch.cuda.stream(stream):
            if self.ws[si] is None or self.ws[si].numel() < wsb.value:
                self.ws[si] = torch.empty(max(wsb.value, 1 << 20), dtype=torch.uint8, device=self.device)
            ws = self.ws[si]
            offsets = self.offsets[si]
            view = self.arena[start:start + cap]
            st = _lib.lib().kg_batch(arr, len(insts), view.data_ptr(), cap, offsets.data_ptr(), ws.data_ptr(),
                                     ws.numel(), _stream(stream))
            _lib.check(st, "kg_batch")
            ev = torch.cuda.Event()
            ev.record(stream)
        b = _Batch()
        b.reqs, b.start, b.cap, b.offsets, b.event, b.stream, b.si, b.ws, b.bytes = (reqs, start, cap, offsets, ev,
                                                                                   stream, si, ws, need)
        self.used += need
        for r in reqs:
            r.admitted = now
            r.batch = b
        self.inflight.append(b)
        return True

    def _reap(self):
        torch = self.torch
        still = []
        for b in self.inflight:
            if not b.event.query():
                still.append(b)
                continue
            now = time.perf_counter()
            offs = b.offsets[:len(b.reqs) + 1].view(torch.int64).cpu().tolist()
            if offs[-1] > b.cap:
                # a G(n,p) total beyond mean + 10 sd: the launch wrote nothing
                raise RuntimeError("batch of %d requests needs %d edges, reserved %d" % (len(b.reqs), offs[-1], b.cap))
            b.reqs_alive = len(b.reqs)
            for i, r in enumerate(b.reqs):
                r.done = now
                r.offset, r.nedges = offs[i], offs[i + 1] - offs[i]
                r.edges = self.arena[b.start + offs[i]:b.start + offs[i + 1]]
                self.finished.append(r)
                if self.on_done is not None:
                    self.on_done(r)
            if self.verify:
                self._start_verify(b)
            elif not self.keep:
                for r in b.reqs:
                    self.release(r)
        self.inflight = still
        if self.verify:
            self._finish_verify()

    # -- the client's checks -------------------------------------------------
    def _sampled(self, r):
        return self.alone_every > 0 and (r.spec.seed * 0x9E3779B97F4A7C15 >> 7) % self.alone_every == 0

    def _start_verify(self, b):
        """Enqueue the checksums of a finished batch's requests on its stream
        (and, for sampled requests, the request generated alone and its
        checksum); the ranges stay reserved until those kernels are done."""
        from . import edge_hash, gnm, gnp, workspace_bytes
        torch = self.torch
        alone = []
        with torch.cuda.stream(b.stream):
            h = torch.empty(len(b.reqs), dtype=torch.uint64, device=self.device)
            for i, r in enumerate(b.reqs):
                edge_hash(r.edges, out=h[i:i + 1], stream=b.stream)
            for i, r in enumerate(b.reqs):
                if not self._sampled(r):
                    continue
                s = r.spec
                inst = Instance(s.n, s.model, s.directed, s.m, s.p, s.seed, s.chunks)
                buf = torch.empty((max(r.nedges, 1), 2), dtype=torch.uint32, device=self.device)
                ws = torch.empty(max(workspace_bytes([inst]), 1), dtype=torch.uint8, device=self.device)
                if s.model == GNM:
                    gnm(s.n, s.m, s.directed, s.seed, s.chunks, out=buf, workspace=ws, stream=b.stream)
                else:
                    tot = torch.zeros(1, dtype=torch.uint64, device=self.device)
                    gnp(s.n, s.p, s.directed, s.seed, s.chunks, out=buf, total=tot, workspace=ws, stream=b.stream)
                ha = edge_hash(buf[:r.nedges], stream=b.stream)
                alone.append((i, ha, buf, ws))
            ev = torch.cuda.Event()
            ev.record(b.stream)
        self.verifying.append((b, h, alone, ev))

    def _finish_verify(self):
        still = []
        for item in self.verifying:
            b, h, alone, ev = item
            if not ev.query():
                still.append(item)
                continue
            hv = h.view(self.torch.int64).cpu().tolist()
            for i, r in enumerate(b.reqs):
                r.hash = hv[i] & (2**64 - 1)
                if r.spec.model == GNM and r.nedges != r.spec.m:
                    self.verify_failures.append((r.rid, "edge count"))
            for i, ha, _, _ in alone:
                self.checked_alone += 1
                if (int(ha.view(self.torch.int64).item()) & (2**64 - 1)) != b.reqs[i].hash:
                    self.verify_failures.append((b.reqs[i].rid, "checksum differs from the request alone"))
            self.verified += len(b.reqs)
            if not self.keep:
                for r in b.reqs:
                    self.release(r)
        self.verifying = still

    def step(self):
        """One scheduler tick: reap finished launches, admit and launch."""
        self._reap()
        if len(self.inflight) < len(self.streams):
            reqs, need = self._admit()
            if reqs:
                return self._launch(reqs, need)
        return False

    def drain(self, timeout=600.0):
        t0 = time.perf_counter()
        while (self.queue or self.inflight or self.verifying) and time.perf_counter() - t0 < timeout:
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
    while i < len(stream) or server.queue or server.inflight or server.verifying:
        now = time.perf_counter() - t0
        while i < len(stream) and stream[i][0] <= now:
            reqs.append(server.submit(stream[i][1], arrival=t0 + stream[i][0]))
            i += 1
        if not server.step() and not server.inflight and not server.verifying:
            # idle: sleep until the next arrival, in short slices
            if i < len(stream):
                gap = stream[i][0] - (time.perf_counter() - t0)
                if gap > 0:
                    time.sleep(min(gap, 0.0005))
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
                  "measured_after_s": warmup_s, "latency_samples": len(lat),
                  "verified": server.verified, "checked_alone": server.checked_alone,
                  "verify_failures": len(server.verify_failures)}
