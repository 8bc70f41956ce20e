"""ctypes front end of the CPU oracle (kgref.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the GPU library.  It builds
``libkgref.so`` with gcc on first use if it is missing or older than its
source.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kgref.c")
LIB = os.path.join(HERE, "libkgref.so")

GNM, GNP = 0, 1
TAG_DTREE, TAG_UTREE, TAG_CBIN, TAG_TTREE, TAG_TLEAF, TAG_INST = 1, 2, 3, 4, 5, 6
TAG_RTREE, TAG_RPTS = 8, 9
RGG_MAX_LEVEL = 14
RGG3_MAX_LEVEL = 10


def build(force=False):
    """Compile the oracle: plain C11, IEEE binary64 without FMA contraction."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-o", tmp, SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


class Inst(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("m", ctypes.c_uint64), ("p", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("model", ctypes.c_uint32),
                ("directed", ctypes.c_uint32), ("P", ctypes.c_uint32), ("pad", ctypes.c_uint32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        u64, u32, dbl = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double
        vp = ctypes.c_void_p
        ip = ctypes.POINTER(Inst)
        L.kgref_philox.argtypes = [vp, vp, vp]
        L.kgref_log.argtypes = [dbl]; L.kgref_log.restype = dbl
        L.kgref_log1p.argtypes = [dbl]; L.kgref_log1p.restype = dbl
        L.kgref_lnf.argtypes = [u64]; L.kgref_lnf.restype = dbl
        L.kgref_lnf_diff.argtypes = [u64, u64]; L.kgref_lnf_diff.restype = dbl
        L.kgref_hyp.argtypes = [u64, u64, u64, u64, u32, u32, u32]; L.kgref_hyp.restype = u64
        L.kgref_bin.argtypes = [u64, dbl, u64, u32, u32, u32]; L.kgref_bin.restype = u64
        L.kgref_validate.argtypes = [ip]; L.kgref_validate.restype = ctypes.c_int
        L.kgref_tile_exponent.argtypes = [ip]; L.kgref_tile_exponent.restype = u32
        L.kgref_num_chunks.argtypes = [ip]; L.kgref_num_chunks.restype = u64
        L.kgref_chunk_counts.argtypes = [ip, vp]; L.kgref_chunk_counts.restype = ctypes.c_int
        L.kgref_chunk_count_path.argtypes = [ip, u64]; L.kgref_chunk_count_path.restype = u64
        L.kgref_chunk_num_tiles.argtypes = [ip, u64]; L.kgref_chunk_num_tiles.restype = u64
        L.kgref_tile_counts.argtypes = [ip, u64, u64, vp]; L.kgref_tile_counts.restype = u64
        L.kgref_leaf.argtypes = [u64, u64, u64, u32, u32, vp]; L.kgref_leaf.restype = ctypes.c_int
        L.kgref_chunk_edges.argtypes = [ip, u64, vp]; L.kgref_chunk_edges.restype = ctypes.c_int64
        L.kgref_chunk_edges_given.argtypes = [ip, u64, u64, vp]
        L.kgref_chunk_edges_given.restype = ctypes.c_int64
        L.kgref_generate.argtypes = [ip, vp, u64, ctypes.c_int]; L.kgref_generate.restype = ctypes.c_int64
        L.kgref_skip_chunk_edges.argtypes = [ip, u64, vp]; L.kgref_skip_chunk_edges.restype = ctypes.c_int64
        L.kgref_skip_generate.argtypes = [ip, vp, u64, ctypes.c_int]; L.kgref_skip_generate.restype = ctypes.c_int64
        L.kgref_instance_seed.argtypes = [u64, u32]; L.kgref_instance_seed.restype = u64
        L.kgref_max_threads.argtypes = []; L.kgref_max_threads.restype = ctypes.c_int
        L.kgref_eval_many.argtypes = [ctypes.c_int, vp, vp, u64]; L.kgref_eval_many.restype = None
        L.kgref_generate_chunks.argtypes = [ip, vp, u64, u64, vp, u64, ctypes.c_int]
        L.kgref_generate_chunks.restype = ctypes.c_int64
        L.kgref_rgg_level.argtypes = [u64, dbl]; L.kgref_rgg_level.restype = u32
        L.kgref_rgg_cells.argtypes = [u64, dbl, u64, vp]; L.kgref_rgg_cells.restype = ctypes.c_int
        L.kgref_rgg_cell_count_path.argtypes = [u64, dbl, u64, u64]
        L.kgref_rgg_cell_count_path.restype = u64
        L.kgref_rgg2d.argtypes = [u64, dbl, u64, vp, vp, u64]; L.kgref_rgg2d.restype = ctypes.c_int64
        L.kgref_rgg_cell_points.argtypes = [u64, dbl, u64, u64, u64, vp]; L.kgref_rgg_cell_points.restype = None
        L.kgref_rgg3_level.argtypes = [u64, dbl]; L.kgref_rgg3_level.restype = u32
        L.kgref_rgg3_cells.argtypes = [u64, dbl, u64, vp]; L.kgref_rgg3_cells.restype = ctypes.c_int
        L.kgref_rgg3_cell_count_path.argtypes = [u64, dbl, u64, u64]
        L.kgref_rgg3_cell_count_path.restype = u64
        L.kgref_rgg3d.argtypes = [u64, dbl, u64, vp, vp, u64]; L.kgref_rgg3d.restype = ctypes.c_int64
        L.kgref_rgg3_cell_points.argtypes = [u64, dbl, u64, u64, u64, vp]; L.kgref_rgg3_cell_points.restype = None
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def inst(n, m=0, p=0.0, directed=True, seed=1, chunks=1, model=None):
    if model is None:
        model = GNP if (p and not m) else GNM
    return Inst(int(n), int(m), float(p), int(seed) & (2**64 - 1), int(model), int(bool(directed)),
                int(chunks), 0)


def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().kgref_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def log(x):
    return lib().kgref_log(float(x))


def log1p(x):
    return lib().kgref_log1p(float(x))


def lnf(k):
    return lib().kgref_lnf(int(k))


def lnf_diff(x, y):
    return lib().kgref_lnf_diff(int(x), int(y))


def hyp(N, K, k, seed, a=0, b=0, tag=TAG_DTREE):
    return lib().kgref_hyp(int(N), int(K), int(k), int(seed) & (2**64 - 1), a, b, tag)


def bin(N, p, seed, a=0, b=0, tag=TAG_CBIN):  # noqa: A001 - mirrors the variate's name
    return lib().kgref_bin(int(N), float(p), int(seed) & (2**64 - 1), a, b, tag)


def validate(I):
    return lib().kgref_validate(ctypes.byref(I))


def tile_exponent(I):
    return lib().kgref_tile_exponent(ctypes.byref(I))


def num_chunks(I):
    return lib().kgref_num_chunks(ctypes.byref(I))


def chunk_counts(I):
    C = num_chunks(I)
    out = np.zeros(C, dtype=np.uint64)
    st = lib().kgref_chunk_counts(ctypes.byref(I), _ptr(out))
    if st:
        raise ValueError("kgref_chunk_counts status %d" % st)
    return out


def chunk_count_path(I, c):
    return lib().kgref_chunk_count_path(ctypes.byref(I), int(c))


def tile_counts(I, c, Kc):
    T = lib().kgref_chunk_num_tiles(ctypes.byref(I), int(c))
    out = np.zeros(max(T, 1), dtype=np.uint64)
    lib().kgref_tile_counts(ctypes.byref(I), int(c), int(Kc), _ptr(out))
    return out[:T]


def leaf(k, St, seed, ordinal, tile):
    out = np.zeros(max(int(k), 1), dtype=np.uint64)
    st = lib().kgref_leaf(int(k), int(St), int(seed) & (2**64 - 1), int(ordinal), int(tile), _ptr(out))
    if st:
        raise ValueError("kgref_leaf status %d" % st)
    return out[:int(k)]


def chunk_edges(I, c, Kc=None):
    if Kc is None:
        Kc = chunk_count_path(I, c)
    out = np.zeros((max(int(Kc), 1), 2), dtype=np.uint32)
    r = lib().kgref_chunk_edges_given(ctypes.byref(I), int(c), int(Kc), _ptr(out))
    if r < 0:
        raise ValueError("kgref_chunk_edges status %d" % r)
    return out[:r]


def view_chunks(I, rank):
    """Canonical ordinals of the chunks processing element `rank` generates
    in the paper's distributed run: its row chunk (Sec. 4.1, directed), or the
    chunk row and column of its section in the upper-triangular chunk matrix
    (Sec. 4.2, undirected), in row-major order."""
    P = int(I.P)
    rank = int(rank)
    if I.directed:
        return [rank]

    def first(i):          # ordinal of the diagonal chunk (i, i)
        return i * P - i * (i - 1) // 2

    return [first(i) + (rank - i) for i in range(rank)] + [first(rank) + (j - rank) for j in range(rank, P)]


def pe_view(I, rank):
    """The edges PE `rank` generates without communication: for each of its
    chunks the count from the chunk's own root path, then the chunk's edges."""
    parts = [chunk_edges(I, c, chunk_count_path(I, c)) for c in view_chunks(I, rank)]
    return np.concatenate(parts) if parts else np.zeros((0, 2), dtype=np.uint32)


def skip_chunk_edges(I, c):
    """Edges of chunk c under the geometric-skip G(n,p) variant."""
    k = lib().kgref_skip_chunk_edges(ctypes.byref(I), int(c), None)
    if k < 0:
        raise ValueError("kgref_skip_chunk_edges status %d" % k)
    out = np.zeros((max(k, 1), 2), dtype=np.uint32)
    lib().kgref_skip_chunk_edges(ctypes.byref(I), int(c), _ptr(out))
    return out[:k]


def skip_generate(I, threads=0):
    """Whole edge list under the geometric-skip G(n,p) variant."""
    total = sum(int(lib().kgref_skip_chunk_edges(ctypes.byref(I), c, None)) for c in range(num_chunks(I)))
    out = np.zeros((max(total, 1), 2), dtype=np.uint32)
    r = lib().kgref_skip_generate(ctypes.byref(I), _ptr(out), total, int(threads))
    if r < 0:
        raise ValueError("kgref_skip_generate status %d" % r)
    return out[:r]


def generate(I, threads=0, cap=None):
    """Whole edge list as an (E, 2) uint32 array."""
    if cap is None:
        cap = int(chunk_counts(I).sum())
    out = np.zeros((max(cap, 1), 2), dtype=np.uint32)
    r = lib().kgref_generate(ctypes.byref(I), _ptr(out), cap, int(threads))
    if r < 0:
        raise ValueError("kgref_generate status %d" % r)
    return out[:r]


def generate_into(I, out, threads=0):
    """Generate into a preallocated (cap, 2) uint32 array; returns the edge count."""
    r = lib().kgref_generate(ctypes.byref(I), _ptr(out), out.shape[0], int(threads))
    if r < 0:
        raise ValueError("kgref_generate status %d" % r)
    return r


def instance_seed(base, i):
    return lib().kgref_instance_seed(int(base) & (2**64 - 1), int(i))


def max_threads():
    return lib().kgref_max_threads()


def eval_many(fn, records, out_dtype, out_width):
    """Element-wise evaluation (fn: 1 philox, 2 log, 3 log1p, 4 lnf_diff,
    5 hyp, 6 bin) over a contiguous record array."""
    records = np.ascontiguousarray(records)
    n = records.shape[0]
    out = np.zeros((n, out_width), dtype=out_dtype)
    lib().kgref_eval_many(int(fn), _ptr(records), _ptr(out), n)
    return out


def generate_chunks(I, counts, c0, c1, out=None, threads=0):
    """Edges of chunks [c0, c1) given all chunk counts (canonical order)."""
    counts = np.ascontiguousarray(counts, dtype=np.uint64)
    need = int(counts[c0:c1].sum())
    if out is None or out.shape[0] < need:
        out = np.zeros((max(need, 1), 2), dtype=np.uint32)
    r = lib().kgref_generate_chunks(ctypes.byref(I), _ptr(counts), int(c0), int(c1), _ptr(out), out.shape[0],
                                    int(threads))
    if r < 0:
        raise ValueError("kgref_generate_chunks status %d" % r)
    return out[:r]


# ---------------------------------------------------------------------------
# Random geometric graphs in two dimensions (Sec. 2.1.2, Sec. 5)
# ---------------------------------------------------------------------------
def rgg_level(n, r):
    """Cells per side 2^L: the largest L <= RGG_MAX_LEVEL with 2^L r <= 1 and
    4^L <= n (cells of side >= max(r, n^-1/2), Sec. 5)."""
    return int(lib().kgref_rgg_level(int(n), float(r)))


def rgg_cells(n, r, seed):
    """Point count of every cell, Morton order (the quadrant recursion of
    Sec. 5.1 down to the cells)."""
    L = rgg_level(n, r)
    out = np.zeros(1 << (2 * L), dtype=np.uint64)
    lib().kgref_rgg_cells(int(n), float(r), int(seed) & (2**64 - 1), _ptr(out))
    return out


def rgg_cell_count_path(n, r, seed, cell):
    """One cell's count from its root path alone (what a processor owning or
    bordering the cell recomputes, Sec. 5.1)."""
    return int(lib().kgref_rgg_cell_count_path(int(n), float(r), int(seed) & (2**64 - 1), int(cell)))


def rgg_cell_points(n, r, seed, cell, k):
    """The k points of one cell, (k, 2) float64."""
    out = np.zeros((max(int(k), 1), 2), dtype=np.float64)
    lib().kgref_rgg_cell_points(int(n), float(r), int(seed) & (2**64 - 1), int(cell), int(k), _ptr(out))
    return out[:int(k)]


def rgg2d(n, r, seed):
    """(points (n, 2) float64 in vertex order, edges (E, 2) uint32 ascending)."""
    seed = int(seed) & (2**64 - 1)
    pts = np.zeros((max(int(n), 1), 2), dtype=np.float64)
    E = lib().kgref_rgg2d(int(n), float(r), seed, _ptr(pts), None, 0)
    if E < 0:
        raise ValueError("kgref_rgg2d status %d" % E)
    out = np.zeros((max(E, 1), 2), dtype=np.uint32)
    E2 = lib().kgref_rgg2d(int(n), float(r), seed, _ptr(pts), _ptr(out), E)
    assert E2 == E
    return pts[:int(n)], out[:E]


def rgg3_level(n, r):
    """Level L of the 8^L-cell grid of a three-dimensional RGG (Sec. 5, d = 3)."""
    return int(lib().kgref_rgg3_level(int(n), float(r)))


def rgg3_cells(n, r, seed):
    """Point counts of all 8^L cells, Morton order (the octant recursion)."""
    L = rgg3_level(n, r)
    out = np.zeros(max(1, 8 ** L), dtype=np.uint64)
    lib().kgref_rgg3_cells(int(n), float(r), int(seed) & (2**64 - 1), _ptr(out))
    return out


def rgg3_cell_count_path(n, r, seed, cell):
    """One cell's count from its root path only (Sec. 5.1)."""
    return int(lib().kgref_rgg3_cell_count_path(int(n), float(r), int(seed) & (2**64 - 1), int(cell)))


def rgg3_cell_points(n, r, seed, cell, k):
    """The k points (k, 3) of one cell."""
    out = np.zeros((max(int(k), 1), 3), dtype=np.float64)
    lib().kgref_rgg3_cell_points(int(n), float(r), int(seed) & (2**64 - 1), int(cell), int(k), _ptr(out))
    return out[:int(k)]


def rgg3d(n, r, seed):
    """(points (n, 3) float64 in vertex order, edges (E, 2) uint32 ascending)."""
    seed = int(seed) & (2**64 - 1)
    pts = np.zeros((max(int(n), 1), 3), dtype=np.float64)
    E = lib().kgref_rgg3d(int(n), float(r), seed, _ptr(pts), None, 0)
    if E < 0:
        raise ValueError("kgref_rgg3d status %d" % E)
    out = np.zeros((max(E, 1), 2), dtype=np.uint32)
    E2 = lib().kgref_rgg3d(int(n), float(r), seed, _ptr(pts), _ptr(out), E)
    assert E2 == E
    return pts[:int(n)], out[:E]
