"""MI355X generator for Erdos-Renyi graphs G(n,m) / G(n,p), directed or
undirected, by the communication-free method of Funke et al. (arXiv
1710.07565, Sec. 4), and for random geometric graphs in two and three
dimensions by the same paper's cell method (Sec. 5).

The Python layer only marshals arguments: device memory and streams come
from PyTorch, every step of the generator runs in the HIP library
``libkg.so`` (C ABI in include/kg.h).  Importing works without a GPU; calls
need one and raise if the library has not been built.
"""
import ctypes
from dataclasses import dataclass

from . import _lib
from ._lib import KG_GNM, KG_GNP, KgError, KgInstance  # noqa: F401

GNM, GNP = KG_GNM, KG_GNP


@dataclass
class Instance:
    """One graph.  `chunks` is the paper's P: row chunks (directed, Sec. 4.1)
    or sections per matrix dimension (undirected, Sec. 4.2)."""
    n: int
    model: int = GNM
    directed: bool = True
    m: int = 0
    p: float = 0.0
    seed: int = 1
    chunks: int = 1
    view: int = 0        # 0: the whole graph; r + 1: the edges incident to section r (per-PE view)

    def c(self):
        return KgInstance(int(self.n), int(self.model), int(bool(self.directed)), int(self.m), float(self.p),
                          int(self.seed) & (2**64 - 1), int(self.chunks), int(self.view))


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def spec_version():
    return _lib.lib().kg_spec_version()


def instance_seed(base, i):
    """Seed of instance i of a batch with base seed `base`."""
    return _lib.lib().kg_instance_seed(int(base) & (2**64 - 1), int(i))


def set_option(option, value):
    _lib.check(_lib.lib().kg_set_option(int(option), int(value)), "kg_set_option")


def get_option(option):
    return _lib.lib().kg_get_option(int(option))


def workspace_bytes(instances):
    import ctypes
    arr = (KgInstance * len(instances))(*[i.c() for i in instances])
    out = ctypes.c_uint64(0)
    _lib.check(_lib.lib().kg_workspace_bytes(arr, len(instances), ctypes.byref(out)), "kg_workspace_bytes")
    return out.value


def _sync(stream, device):
    """Wait for `stream` (None: the device's current stream) before a host read."""
    torch = _torch()
    if stream is None:
        torch.cuda.current_stream(device).synchronize()
    elif hasattr(stream, "synchronize"):
        stream.synchronize()
    else:
        torch.cuda.synchronize(device)


def _on(stream):
    """Context in which temporaries are allocated on the stream the library
    call runs on, so the caching allocator does not hand them out again
    while that stream still uses them."""
    torch = _torch()
    import contextlib
    if stream is None or not hasattr(stream, "cuda_stream") or not isinstance(stream, torch.cuda.Stream):
        return contextlib.nullcontext()
    return torch.cuda.stream(stream)


def set_workspace(workspace):
    """Register a device uint8 tensor as the current device's workspace for
    calls given none (kg_set_workspace); None removes the registration.  The
    caller keeps the tensor alive while it is registered."""
    if workspace is None:
        _lib.check(_lib.lib().kg_set_workspace(None, 0), "kg_set_workspace")
    else:
        _lib.check(_lib.lib().kg_set_workspace(workspace.data_ptr(), workspace.numel()), "kg_set_workspace")


def _workspace(instances, workspace, device, stream=None):
    torch = _torch()
    need = workspace_bytes(instances)
    if workspace is None:
        with _on(stream):
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=device)
    if workspace.numel() < need:
        raise KgError(_lib.KG_ENOSPC, "workspace")
    return workspace, need


def gnm(n, m, directed=True, seed=1, chunks=1, out=None, workspace=None, stream=None, device="cuda"):
    """Directed (Sec. 4.1) or undirected (Sec. 4.2) G(n,m): an (m, 2) uint32
    tensor of edges on the device, in canonical chunk order."""
    torch = _torch()
    if out is None:
        with _on(stream):
            out = torch.empty((max(int(m), 0), 2), dtype=torch.uint32, device=device)
    inst = Instance(n, GNM, directed, m, 0.0, seed, chunks)
    ws, need = _workspace([inst], workspace, out.device, stream)
    st = _lib.lib().kg_gnm(int(n), int(m), int(bool(directed)), int(seed) & (2**64 - 1), int(chunks),
                           out.data_ptr() if out.numel() else None, out.shape[0], ws.data_ptr(), ws.numel(),
                           _stream(stream))
    _lib.check(st, "kg_gnm")
    return out[:m]


def gnm_static(n, m, directed=True, seed=1, chunks=1, out=None, stream=None, device="cuda"):
    """G(n,m) through kg_gnm_static: the library's static per-device scratch
    is the workspace, so the call allocates nothing but `out` (if not given).
    Same bytes as gnm()."""
    torch = _torch()
    if out is None:
        with _on(stream):
            out = torch.empty((max(int(m), 0), 2), dtype=torch.uint32, device=device)
    st = _lib.lib().kg_gnm_static(int(n), int(m), int(bool(directed)), int(seed) & (2**64 - 1), int(chunks),
                                  out.data_ptr() if out.numel() else None, out.shape[0], _stream(stream))
    _lib.check(st, "kg_gnm_static")
    return out[:m]


def gnp_count(n, p, directed=True, seed=1, chunks=1, workspace=None, stream=None, device="cuda"):
    """Edge total of G(n,p) (synchronises the stream)."""
    import ctypes
    inst = Instance(n, GNP, directed, 0, p, seed, chunks)
    ws, need = _workspace([inst], workspace, device, stream)
    tot = ctypes.c_uint64(0)
    st = _lib.lib().kg_gnp_count(int(n), float(p), int(bool(directed)), int(seed) & (2**64 - 1), int(chunks),
                                 ctypes.byref(tot), ws.data_ptr(), ws.numel(), _stream(stream))
    _lib.check(st, "kg_gnp_count")
    return tot.value


def gnp(n, p, directed=True, seed=1, chunks=1, out=None, total=None, workspace=None, stream=None,
        device="cuda"):
    """G(n,p) (Sec. 4.3).  Without `out` the exact size is found first with
    gnp_count.  With `out`, returns (out, total) where total is a device
    uint64 tensor; if total exceeds out.shape[0] nothing was written."""
    torch = _torch()
    inst = Instance(n, GNP, directed, 0, p, seed, chunks)
    sized = out is None
    if sized:
        E = gnp_count(n, p, directed, seed, chunks, workspace=workspace, stream=stream, device=device)
        with _on(stream):
            out = torch.empty((E, 2), dtype=torch.uint32, device=device)
    if total is None:
        with _on(stream):
            total = torch.zeros(1, dtype=torch.uint64, device=out.device)
    ws, need = _workspace([inst], workspace, out.device, stream)
    st = _lib.lib().kg_gnp(int(n), float(p), int(bool(directed)), int(seed) & (2**64 - 1), int(chunks),
                           out.data_ptr() if out.numel() else None, out.shape[0], total.data_ptr(),
                           ws.data_ptr(), ws.numel(), _stream(stream))
    _lib.check(st, "kg_gnp")
    if sized:
        return out
    return out, total


def chunk_counts(inst, workspace=None, stream=None, device="cuda"):
    """Per-chunk edge counts of one instance (uint64 device tensor)."""
    torch = _torch()
    from . import _lib as L
    C = inst.chunks if inst.directed else inst.chunks * (inst.chunks + 1) // 2
    with _on(stream):
        out = torch.empty(C, dtype=torch.uint64, device=device)
    ws, need = _workspace([inst], workspace, device, stream)
    st = L.lib().kg_chunk_counts(inst.c(), out.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream))
    L.check(st, "kg_chunk_counts")
    return out


def batch(instances, arena=None, offsets=None, workspace=None, stream=None, device="cuda"):
    """Generate many instances in one pass into one arena.  Returns
    (arena, offsets): instance i occupies arena[offsets[i]:offsets[i+1]].
    If the arena is too small nothing is written (offsets[-1] shows the need)."""
    torch = _torch()
    cnt = len(instances)
    arr = (KgInstance * cnt)(*[i.c() for i in instances])
    if arena is None:
        total = 0
        for i in instances:
            if i.model == GNM and not i.view:
                total += int(i.m)
            elif not i.view:
                total += gnp_count(i.n, i.p, i.directed, i.seed, i.chunks, stream=stream, device=device)
            else:
                total += view_count(i, stream=stream, device=device)
        with _on(stream):
            arena = torch.empty((total, 2), dtype=torch.uint32, device=device)
    if offsets is None:
        with _on(stream):
            offsets = torch.empty(cnt + 1, dtype=torch.uint64, device=arena.device)
    ws, need = _workspace(instances, workspace, arena.device, stream)
    st = _lib.lib().kg_batch(arr, cnt, arena.data_ptr() if arena.numel() else None, arena.shape[0],
                             offsets.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream))
    _lib.check(st, "kg_batch")
    return arena, offsets


def view_count(inst, workspace=None, stream=None, device="cuda"):
    """Edges of one instance (whole graph or view) from a counting pass
    (kg_batch with an empty arena; synchronises the stream)."""
    torch = _torch()
    with _on(stream):
        offs = torch.empty(2, dtype=torch.uint64, device=device)
    ws, need = _workspace([inst], workspace, device, stream)
    arr = (KgInstance * 1)(inst.c())
    _lib.check(_lib.lib().kg_batch(arr, 1, None, 0, offs.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream)),
               "kg_batch")
    _sync(stream, device)
    return int(offs.view(torch.int64)[1].item())


def pe_view(n, rank, chunks, directed=True, m=0, p=None, seed=1, out=None, total=None, workspace=None,
            stream=None, device="cuda"):
    """The edges incident to section `rank` of the instance (the per-PE view
    of Sec. 4.1 / 4.2: directed, row chunk `rank`; undirected, the chunk row
    and column of section `rank` of the chunk matrix), in canonical chunk
    order; G(n,m) unless p is given.  Without `out` the exact size is found
    first; with `out`, returns (out, total) as gnp() does."""
    torch = _torch()
    model = GNM if p is None else GNP
    inst = Instance(n, model, directed, m if p is None else 0, 0.0 if p is None else p, seed, chunks)
    view = Instance(n, model, directed, inst.m, inst.p, seed, chunks, view=int(rank) + 1)
    sized = out is None
    if sized:
        E = view_count(view, workspace=workspace, stream=stream, device=device)
        with _on(stream):
            out = torch.empty((E, 2), dtype=torch.uint32, device=device)
    if total is None:
        with _on(stream):
            total = torch.zeros(1, dtype=torch.uint64, device=out.device)
    ws, need = _workspace([view], workspace, out.device, stream)
    st = _lib.lib().kg_pe_view(inst.c(), int(rank), out.data_ptr() if out.numel() else None, out.shape[0],
                               total.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream))
    _lib.check(st, "kg_pe_view")
    if sized:
        return out
    return out, total


def gnp_skip(n, p, directed=True, seed=1, chunks=1, out=None, total=None, workspace=None, stream=None,
             device="cuda"):
    """G(n,p) by geometric skips per tile (kg_gnp_skip): the same law as
    gnp(), other bits.  Without `out` a first call finds the size; with
    `out`, returns (out, total) as gnp() does.  Without `workspace` one of
    gnp_skip_workspace_bytes() is allocated, so that the write pass decodes
    the count pass's stored event positions; a smaller one (at least
    workspace_bytes() of the instance) makes it generate them again."""
    torch = _torch()
    inst = Instance(n, GNP, directed, 0, p, seed, chunks)
    with _on(stream):
        if workspace is None:
            # room for the count pass's event positions (see gnp_skip_workspace_bytes)
            workspace = torch.empty(gnp_skip_workspace_bytes(n, p, directed, chunks), dtype=torch.uint8,
                                    device=device if out is None else out.device)
        ws, need = _workspace([inst], workspace, device if out is None else out.device)
        if total is None:
            total = torch.zeros(1, dtype=torch.uint64, device=ws.device)
    sized = out is None
    if sized:
        st = _lib.lib().kg_gnp_skip(int(n), float(p), int(bool(directed)), int(seed) & (2**64 - 1), int(chunks),
                                    None, 0, total.data_ptr(), ws.data_ptr(), ws.numel(), _stream(stream))
        _lib.check(st, "kg_gnp_skip")
        _sync(stream, ws.device)
        E = int(total.view(torch.int64).cpu()[0])
        with _on(stream):
            out = torch.empty((E, 2), dtype=torch.uint32, device=ws.device)
    st = _lib.lib().kg_gnp_skip(int(n), float(p), int(bool(directed)), int(seed) & (2**64 - 1), int(chunks),
                                out.data_ptr() if out.numel() else None, out.shape[0], total.data_ptr(),
                                ws.data_ptr(), ws.numel(), _stream(stream))
    _lib.check(st, "kg_gnp_skip")
    if sized:
        return out
    return out, total


def gnp_skip_workspace_bytes(n, p, directed=True, chunks=1):
    """Workspace bytes with which gnp_skip keeps the count pass's event
    positions (one row of 32-bit positions per tile), so that the write pass
    only decodes them; a workspace of workspace_bytes() also works, with the
    write pass generating the events again."""
    b = ctypes.c_uint64(0)
    _lib.check(_lib.lib().kg_gnp_skip_workspace_bytes(int(n), float(p), int(bool(directed)), int(chunks),
                                                      ctypes.byref(b)), "kg_gnp_skip_workspace_bytes")
    return int(b.value)


def rgg2d_workspace_bytes(n, r):
    b = ctypes.c_uint64(0)
    _lib.check(_lib.lib().kg_rgg2d_workspace_bytes(int(n), float(r), ctypes.byref(b)), "kg_rgg2d_workspace_bytes")
    return int(b.value)


def rgg2d_expected_edges(n, r):
    """Mean edge count of the two-dimensional RGG: C(n, 2) times the chance
    that two uniform points of the unit square lie closer than r (for r <= 1:
    pi r^2 - 8 r^3 / 3 + r^4 / 2)."""
    import math
    pairs = n * (n - 1) / 2.0
    if r >= math.sqrt(2.0):
        return pairs
    if r <= 1.0:
        return pairs * (math.pi * r * r - 8.0 * r ** 3 / 3.0 + r ** 4 / 2.0)
    return pairs


def rgg2d(n, r, seed=1, points=None, out=None, total=None, workspace=None, stream=None, device="cuda"):
    """Two-dimensional random geometric graph (kg_rgg2d).  Returns
    (points (n, 2) float64, edges (E, 2) uint32).  With `out` given, writes
    into it and returns (points, out, total) without synchronising; if the
    total exceeds out.shape[0] nothing is written to `out`."""
    torch = _torch()
    dev = out.device if out is not None else (points.device if points is not None else torch.device(device))
    with _on(stream):
        if points is None:
            points = torch.empty((int(n), 2), dtype=torch.float64, device=dev)
        if workspace is None:
            workspace = torch.empty(max(rgg2d_workspace_bytes(n, r), 1), dtype=torch.uint8, device=dev)
        if total is None:
            total = torch.zeros(1, dtype=torch.uint64, device=dev)

    def call(edges):
        st = _lib.lib().kg_rgg2d(int(n), float(r), int(seed) & (2**64 - 1),
                                 points.data_ptr() if points.numel() else None,
                                 edges.data_ptr() if edges.numel() else None, edges.shape[0], total.data_ptr(),
                                 workspace.data_ptr(), workspace.numel(), _stream(stream))
        _lib.check(st, "kg_rgg2d")

    if out is not None:
        call(out)
        return points, out, total
    import math
    mu = rgg2d_expected_edges(int(n), float(r))
    cap = int(min(n * (n - 1) // 2, mu * 1.05 + 8.0 * math.sqrt(mu + 1.0) * max(1.0, math.sqrt(n * r * r * 10.0))
                  + 1024))
    with _on(stream):
        edges = torch.empty((max(cap, 0), 2), dtype=torch.uint32, device=dev)
    call(edges)
    _sync(stream, dev)
    E = int(total.view(torch.int64).cpu()[0])
    if E > edges.shape[0]:
        with _on(stream):
            edges = torch.empty((E, 2), dtype=torch.uint32, device=dev)
        call(edges)
    return points, edges[:E]


def rgg3d_workspace_bytes(n, r):
    b = ctypes.c_uint64(0)
    _lib.check(_lib.lib().kg_rgg3d_workspace_bytes(int(n), float(r), ctypes.byref(b)), "kg_rgg3d_workspace_bytes")
    return int(b.value)


def rgg3d_expected_edges(n, r):
    """Mean edge count of the three-dimensional RGG: C(n, 2) times the chance
    that two uniform points of the unit cube lie closer than r (for r <= 1:
    4 pi r^3 / 3 - 3 pi r^4 / 2 + 8 r^5 / 5 - r^6 / 6)."""
    import math
    pairs = n * (n - 1) / 2.0
    if r <= 1.0:
        return pairs * (4.0 * math.pi * r ** 3 / 3.0 - 1.5 * math.pi * r ** 4 + 1.6 * r ** 5 - r ** 6 / 6.0)
    return pairs


def rgg3d(n, r, seed=1, points=None, out=None, total=None, workspace=None, stream=None, device="cuda"):
    """Three-dimensional random geometric graph (kg_rgg3d).  Returns
    (points (n, 3) float64, edges (E, 2) uint32).  With `out` given, writes
    into it and returns (points, out, total) without synchronising; if the
    total exceeds out.shape[0] nothing is written to `out`."""
    torch = _torch()
    dev = out.device if out is not None else (points.device if points is not None else torch.device(device))
    with _on(stream):
        if points is None:
            points = torch.empty((int(n), 3), dtype=torch.float64, device=dev)
        if workspace is None:
            workspace = torch.empty(max(rgg3d_workspace_bytes(n, r), 1), dtype=torch.uint8, device=dev)
        if total is None:
            total = torch.zeros(1, dtype=torch.uint64, device=dev)

    def call(edges):
        st = _lib.lib().kg_rgg3d(int(n), float(r), int(seed) & (2**64 - 1),
                                 points.data_ptr() if points.numel() else None,
                                 edges.data_ptr() if edges.numel() else None, edges.shape[0], total.data_ptr(),
                                 workspace.data_ptr(), workspace.numel(), _stream(stream))
        _lib.check(st, "kg_rgg3d")

    if out is not None:
        call(out)
        return points, out, total
    import math
    mu = rgg3d_expected_edges(int(n), float(r))
    cap = int(min(n * (n - 1) // 2, mu * 1.05 + 8.0 * math.sqrt(mu + 1.0) * max(1.0, (n * r ** 3 * 30.0) ** 0.5)
                  + 1024))
    with _on(stream):
        edges = torch.empty((max(cap, 0), 2), dtype=torch.uint32, device=dev)
    call(edges)
    _sync(stream, dev)
    E = int(total.view(torch.int64).cpu()[0])
    if E > edges.shape[0]:
        with _on(stream):
            edges = torch.empty((E, 2), dtype=torch.uint32, device=dev)
        call(edges)
    return points, edges[:E]


def batch_upload(instances, workspace, stream=None):
    """Write the descriptor table of `instances` into `workspace` (a device
    uint8 tensor of at least workspace_bytes(instances)); synchronises."""
    cnt = len(instances)
    arr = (KgInstance * cnt)(*[i.c() for i in instances])
    _lib.check(_lib.lib().kg_batch_upload(arr, cnt, workspace.data_ptr(), workspace.numel(), _stream(stream)),
               "kg_batch_upload")


def batch_launch(instances, arena, offsets, workspace, stream=None):
    """The kernels of batch() for a list already uploaded to `workspace`:
    enqueues kernels only, so it may run under stream capture."""
    cnt = len(instances)
    arr = (KgInstance * cnt)(*[i.c() for i in instances])
    st = _lib.lib().kg_batch_launch(arr, cnt, arena.data_ptr() if arena.numel() else None, arena.shape[0],
                                    offsets.data_ptr(), workspace.data_ptr(), workspace.numel(), _stream(stream))
    _lib.check(st, "kg_batch_launch")


class BatchGraph:
    """A batch recorded once into a HIP graph (torch.cuda.CUDAGraph) and
    replayed: the arena, offsets and workspace are fixed at construction and
    every replay rewrites the same bytes.  The graph holds kernel launches
    only; the descriptor table is uploaded before the capture."""

    def __init__(self, instances, arena, offsets, workspace):
        torch = _torch()
        self.instances = list(instances)
        self.arena, self.offsets, self.workspace = arena, offsets, workspace
        batch_upload(self.instances, workspace)
        self.graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream(device=arena.device)
        side.wait_stream(torch.cuda.current_stream(arena.device))
        with torch.cuda.graph(self.graph, stream=side):
            batch_launch(self.instances, arena, offsets, workspace)
        torch.cuda.current_stream(arena.device).wait_stream(side)

    def replay(self):
        """Enqueue the recorded kernels on the current stream."""
        self.graph.replay()
        return self.arena, self.offsets


def eval_device(fn, d_in, n, out_dtype, out_width, stream=None):
    """Element-wise evaluation of a device building block (see kg_eval)."""
    torch = _torch()
    out = torch.empty((int(n), out_width), dtype=out_dtype, device=d_in.device)
    st = _lib.lib().kg_eval(int(fn), d_in.data_ptr(), out.data_ptr(), int(n), _stream(stream))
    _lib.check(st, "kg_eval")
    return out


def edge_hash(edges, out=None, stream=None):
    """Order-independent 64-bit checksum of an (E, 2) uint32 edge tensor on
    the device (kg_edge_hash); returns a one-element device uint64 tensor,
    asynchronously on `stream`."""
    torch = _torch()
    if out is None:
        with _on(stream):
            out = torch.empty(1, dtype=torch.uint64, device=edges.device)
    st = _lib.lib().kg_edge_hash(edges.data_ptr() if edges.numel() else None, int(edges.shape[0]),
                                 out.data_ptr(), _stream(stream))
    _lib.check(st, "kg_edge_hash")
    return out


def kernel_time_read(kernel):
    """(summed ms, launches) of kernel `kernel` since the last read, from the
    hipEvents the library records while KG_OPT_TIME_KERNELS is 1."""
    import ctypes
    ms, n = ctypes.c_double(0.0), ctypes.c_uint64(0)
    _lib.check(_lib.lib().kg_kernel_time_read(int(kernel), ctypes.byref(ms), ctypes.byref(n)),
               "kg_kernel_time_read")
    return ms.value, n.value
