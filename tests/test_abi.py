"""The C-ABI library loads on a machine without a GPU, exports every entry
point include/kg.h declares, and rejects bad arguments synchronously (host
logic only: no kernel is launched here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "kg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(kg_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    from paper_1710_07565_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1710_07565_amd import build
        build.build(force=True)
    return _lib.lib()


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 12
    from paper_1710_07565_amd import _lib
    assert sorted(_lib.EXPORTS) == names
    for n in names:
        assert hasattr(L, n), n


def test_one_hip_runtime_in_the_process(L):
    """The binding loads libkg.so after torch, so the library binds to the HIP
    runtime torch holds instead of loading the system copy beside it."""
    maps = open("/proc/self/maps").read().split("\n")
    runtimes = {ln.split()[-1] for ln in maps if "libamdhip64" in ln}
    assert len(runtimes) == 1, runtimes


def test_library_is_built_for_gfx950():
    from paper_1710_07565_amd import _lib
    data = open(_lib.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_host_only_entry_points(L, kgref):
    assert L.kg_spec_version() == 1
    assert L.kg_strerror(0) == b"ok"
    assert L.kg_strerror(-3).startswith(b"output")
    for base in (0, 1, 2**64 - 1):
        for i in (0, 7, 2**32 - 1):
            assert L.kg_instance_seed(base, i) == kgref.instance_seed(base, i)


def _inst(**kw):
    from paper_1710_07565_amd import _lib
    d = dict(n=100, model=0, directed=1, m=10, p=0.0, seed=1, chunks=4, flags=0)
    d.update(kw)
    return _lib.KgInstance(**d)


def test_workspace_bytes_and_validation(L):
    from paper_1710_07565_amd import _lib
    out = ctypes.c_uint64(0)
    assert L.kg_workspace_bytes(ctypes.byref(_inst()), 1, ctypes.byref(out)) == 0 and out.value > 0
    bad = [dict(n=0), dict(chunks=0), dict(chunks=101), dict(m=100 * 99 + 1), dict(model=2), dict(flags=5),
           dict(model=1, p=1.5), dict(model=1, p=-0.1), dict(model=1, p=float("nan"))]
    for kw in bad:
        assert L.kg_workspace_bytes(ctypes.byref(_inst(**kw)), 1, ctypes.byref(out)) == _lib.KG_EINVAL, kw
    N27 = 2**27 * (2**27 - 1)                        # a directed universe above 2^53
    rng = [dict(n=2**32 + 1, chunks=1, m=0),
           dict(n=2**16, directed=0, chunks=2**15 + 1, m=0),
           dict(n=2**27, m=2**53, chunks=2**10),            # N >= 2^53: the count must stay below 2^53
           dict(n=2**27, model=1, p=2.0**52 / N27, chunks=2**10),
           dict(n=2**32, m=0, chunks=1),                    # one chunk of 2^32 - 1 tiles of 2^32 slots
           dict(n=2**32, directed=0, m=0, chunks=1)]
    for kw in rng:
        assert L.kg_workspace_bytes(ctypes.byref(_inst(**kw)), 1, ctypes.byref(out)) == _lib.KG_ERANGE, kw
    # universes of 2^53 slots and more are accepted (n <= 2^32, N < 2^64)
    ok = [dict(n=94906267, m=0, chunks=4), dict(n=134217729, directed=0, m=0, chunks=4),
          dict(n=2**27, m=2**31, chunks=2**10), dict(n=2**27, m=2**53 - 1, chunks=2**16),
          dict(n=2**27, model=1, p=16.0 / (2**27 - 1), chunks=2**10),
          dict(n=2**32, m=2**40, chunks=2**8), dict(n=2**32, directed=0, m=2**40, chunks=2**8)]
    for kw in ok:
        assert L.kg_workspace_bytes(ctypes.byref(_inst(**kw)), 1, ctypes.byref(out)) == 0, kw


def test_view_flags(L):
    """flags = r + 1 selects the view of section r (r < chunks); its
    workspace is that of the chunks incident to the section."""
    out = ctypes.c_uint64(0)
    full = ctypes.c_uint64(0)
    assert L.kg_workspace_bytes(ctypes.byref(_inst(directed=0, chunks=8, m=2000)), 1, ctypes.byref(full)) == 0
    for r in range(8):
        assert L.kg_workspace_bytes(ctypes.byref(_inst(directed=0, chunks=8, m=2000, flags=r + 1)), 1,
                                    ctypes.byref(out)) == 0
        assert 0 < out.value <= full.value
    from paper_1710_07565_amd import _lib
    assert L.kg_workspace_bytes(ctypes.byref(_inst(directed=0, chunks=8, m=2000, flags=9)), 1,
                                ctypes.byref(out)) == _lib.KG_EINVAL
    # kg_pe_view refuses a rank outside [0, chunks) or an instance that is already a view
    assert L.kg_pe_view(ctypes.byref(_inst(chunks=4)), 4, None, 0, None, None, 0, None) == _lib.KG_EINVAL
    assert L.kg_pe_view(ctypes.byref(_inst(chunks=4, flags=1)), 0, None, 0, None, None, 0, None) == _lib.KG_EINVAL


def test_generation_calls_reject_bad_arguments_without_a_device(L):
    from paper_1710_07565_amd import _lib
    # invalid sizes and a too-small capacity return before anything is enqueued
    assert L.kg_gnm(100, 10, 1, 1, 0, None, 10, None, 0, None) == _lib.KG_EINVAL
    assert L.kg_gnm(100, 10**6, 1, 1, 4, None, 10**6, None, 0, None) == _lib.KG_EINVAL
    assert L.kg_gnm(100, 10, 1, 1, 4, 8, 5, None, 0, None) == _lib.KG_ENOSPC
    assert L.kg_gnm(100, 10, 1, 1, 4, 4, 10, None, 0, None) == _lib.KG_EINVAL      # misaligned output
    assert L.kg_gnp(100, 2.0, 1, 1, 4, None, 0, None, None, 0, None) == _lib.KG_EINVAL
    assert L.kg_batch(None, 0, None, 0, None, None, 0, None) == _lib.KG_EINVAL
    assert L.kg_eval(99, None, None, 1, None) == _lib.KG_EINVAL
    assert L.kg_set_option(1, 64) == _lib.KG_ERANGE
    assert L.kg_set_option(1, 4096) == _lib.KG_ERANGE
    assert L.kg_set_option(42, 1) == _lib.KG_EINVAL
    assert L.kg_set_option(2, 8) == 0 and L.kg_get_option(2) == 8
    assert L.kg_set_option(2, 0) == 0 and L.kg_get_option(2) == 0
    assert L.kg_set_option(_lib.KG_OPT_COUNT_LANES, 3) == _lib.KG_ERANGE
    assert L.kg_set_option(_lib.KG_OPT_COUNT_LANES, 8) == 0 and L.kg_get_option(_lib.KG_OPT_COUNT_LANES) == 8
    assert L.kg_set_option(_lib.KG_OPT_COUNT_LANES, 0) == 0 and L.kg_get_option(_lib.KG_OPT_COUNT_LANES) == 0
    assert L.kg_set_option(_lib.KG_OPT_SKIP_ROW, 63) == _lib.KG_ERANGE
    assert L.kg_set_option(_lib.KG_OPT_SKIP_ROW, 1409) == _lib.KG_ERANGE
    assert L.kg_set_option(_lib.KG_OPT_SKIP_ROW, 64) == 0 and L.kg_get_option(_lib.KG_OPT_SKIP_ROW) == 64
    assert L.kg_set_option(_lib.KG_OPT_SKIP_ROW, 0) == 0 and L.kg_get_option(_lib.KG_OPT_SKIP_ROW) == 1408


def test_skip_workspace_holds_a_row_per_tile(L):
    """kg_gnp_skip_workspace_bytes: the G(n,p) workspace (rounded up to 256
    bytes) plus 1408 32-bit positions per tile of the tile bound."""
    from paper_1710_07565_amd import _lib
    b = ctypes.c_uint64(0)
    assert L.kg_gnp_skip_workspace_bytes(2**12, 0.01, 1, 8, None) == _lib.KG_EINVAL
    assert L.kg_gnp_skip_workspace_bytes(2**12, 2.0, 1, 8, ctypes.byref(b)) == _lib.KG_EINVAL
    for n, p, directed, P in [(2**12, 0.01, 1, 8), (2**16, 1e-4, 0, 32), (5000, 0.3516, 1, 3)]:
        assert L.kg_gnp_skip_workspace_bytes(n, p, directed, P, ctypes.byref(b)) == 0
        rows = b.value
        inst = _lib.KgInstance()
        inst.n, inst.model, inst.directed, inst.p, inst.seed, inst.chunks = n, _lib.KG_GNP, directed, p, 1, P
        assert L.kg_workspace_bytes(ctypes.byref(inst), 1, ctypes.byref(b)) == 0
        base = (b.value + 255) // 256 * 256
        assert rows > base and (rows - base) % (1408 * 4) == 0


def test_oracle_tile_exponent_is_minimal(kgref):
    """The tile exponent is the smallest s in [9, 32] with 2^s m >= 560 N
    (tiles hold 560..1120 samples in expectation)."""
    for n, m in [(2**16, 2**20), (2**10, 2**19), (50, 1225), (2**20, 5)]:
        I = kgref.inst(n, m=m, directed=True, seed=1, chunks=1)
        s = kgref.tile_exponent(I)
        N = n * (n - 1)
        assert (m << s) >= 560 * N or s == 32
        assert s == 9 or (m << (s - 1)) < 560 * N


def test_skip_variant_argument_checks(L):
    """kg_gnp_skip refuses bad arguments before touching the device."""
    from paper_1710_07565_amd import _lib
    assert L.kg_gnp_skip(100, 1.5, 1, 1, 4, None, 0, None, None, 0, None) == _lib.KG_EINVAL
    assert L.kg_gnp_skip(100, 0.1, 1, 1, 0, None, 0, None, None, 0, None) == _lib.KG_EINVAL
    assert L.kg_gnp_skip(100, 0.1, 1, 1, 4, 4, 10, None, None, 0, None) == _lib.KG_EINVAL   # misaligned
    assert L.kg_gnp_skip(2**33, 0.1, 1, 1, 4, None, 0, None, None, 0, None) == _lib.KG_ERANGE


def test_rgg_argument_checks_and_workspace(L):
    """kg_rgg2d and its workspace query validate on the host: negative or
    NaN radius, n >= 2^32, too many points per cell, missing or misaligned
    point buffer; the workspace grows with the level rule's cell count."""
    import ctypes
    from paper_1710_07565_amd import _lib
    b = ctypes.c_uint64(0)
    assert L.kg_rgg2d_workspace_bytes(100, -0.1, ctypes.byref(b)) == _lib.KG_EINVAL
    assert L.kg_rgg2d_workspace_bytes(100, float("nan"), ctypes.byref(b)) == _lib.KG_EINVAL
    assert L.kg_rgg2d_workspace_bytes(2**32, 0.001, ctypes.byref(b)) == _lib.KG_ERANGE
    assert L.kg_rgg2d_workspace_bytes(10**6, 0.6, ctypes.byref(b)) == _lib.KG_ERANGE   # one cell
    assert L.kg_rgg2d_workspace_bytes(100, 0.1, None) == _lib.KG_EINVAL
    sizes = []
    for n, r in [(0, 0.5), (1000, 0.5), (1000, 0.1), (1000, 0.01), (10**6, 0.001)]:
        assert L.kg_rgg2d_workspace_bytes(n, r, ctypes.byref(b)) == _lib.KG_OK
        sizes.append(b.value)
    assert sizes[0] > 0 and sizes[1] < sizes[2] < sizes[3] < sizes[4]
    # n = 2^26 at the benchmark radius: 4^11 cells, about 40 B per vertex plus the tree
    import math
    n = 2**26
    assert L.kg_rgg2d_workspace_bytes(n, 0.55 * math.sqrt(math.log(n) / n), ctypes.byref(b)) == _lib.KG_OK
    assert 40 * n < b.value < 40 * n + 64 * 4**11
    assert L.kg_rgg2d(100, -1.0, 1, None, None, 0, None, None, 0, None) == _lib.KG_EINVAL
    assert L.kg_rgg2d(100, 0.1, 1, None, None, 0, None, None, 0, None) == _lib.KG_EINVAL      # no points
    assert L.kg_rgg2d(100, 0.1, 1, 8, None, 0, None, None, 0, None) == _lib.KG_EINVAL         # misaligned
    assert L.kg_rgg2d(2**32, 0.1, 1, None, None, 0, None, None, 0, None) == _lib.KG_ERANGE


def test_static_scratch_entry_point_checks(L, kgref):
    """kg_gnm_static takes kg_gnm's argument checks, and refuses an instance
    whose workspace exceeds the static scratch (96 MiB) with KG_ESCRATCH,
    all before it touches a device; the headline instance fits."""
    import ctypes
    from paper_1710_07565_amd import _lib
    assert _lib.KG_STATIC_SCRATCH_BYTES == 96 << 20
    assert L.kg_gnm_static(100, 10, 1, 1, 0, None, 10, None) == _lib.KG_EINVAL
    assert L.kg_gnm_static(100, 10**6, 1, 1, 4, None, 10**6, None) == _lib.KG_EINVAL
    assert L.kg_gnm_static(100, 10, 1, 1, 4, 8, 5, None) == _lib.KG_ENOSPC
    assert L.kg_gnm_static(100, 10, 1, 1, 4, 4, 10, None) == _lib.KG_EINVAL      # misaligned output
    b = ctypes.c_uint64()
    big = _lib.KgInstance(2**27, 0, 0, 2**32, 0.0, 1, 4096, 0)
    assert L.kg_workspace_bytes(ctypes.byref(big), 1, ctypes.byref(b)) == 0
    assert b.value > _lib.KG_STATIC_SCRATCH_BYTES
    # the output pointer is never used: the size check comes first
    assert L.kg_gnm_static(2**27, 2**32, 0, 1, 4096, 4096, 2**32, None) == _lib.KG_ESCRATCH
    assert b"static scratch" in L.kg_strerror(_lib.KG_ESCRATCH)
    head = _lib.KgInstance(2**26, 0, 0, 2**31, 0.0, 1, 256, 0)
    assert L.kg_workspace_bytes(ctypes.byref(head), 1, ctypes.byref(b)) == 0
    assert b.value <= _lib.KG_STATIC_SCRATCH_BYTES


def test_set_workspace_argument_checks(L):
    """kg_set_workspace refuses a NULL buffer with a size, a buffer without
    one and a pointer that is not 256-byte aligned, before asking for a
    device; removing the registration needs a current device only."""
    from paper_1710_07565_amd import _lib
    assert L.kg_set_workspace(None, 64) == _lib.KG_EINVAL
    assert L.kg_set_workspace(4096, 0) == _lib.KG_EINVAL
    assert L.kg_set_workspace(4096 + 64, 1 << 20) == _lib.KG_EINVAL
    assert L.kg_set_workspace(None, 0) in (_lib.KG_OK, _lib.KG_EDEVICE)


@pytest.mark.parametrize("n,m,p,directed,P,s_want", [
    (2**16, 2**20, 0.0, True, 64, 22),                 # small directed G(n,m)
    (2**26, 2**31, 0.0, False, 256, 30),               # headline undirected G(n,m)
    (2**25, 0, 16.0 / (2**25 - 1), True, 2**16, 31),   # directed G(n,p), mean out-degree 16
    (2**25, 0, 64.0 / (2**25 - 1), False, 256, 29),    # undirected G(n,p), mean degree 64
])
def test_tile_exponent_of_the_workloads(kgref, n, m, p, directed, P, s_want):
    """The tile exponent of each benchmark workload, checked against the
    sampling threshold's definition written out here: the expected samples
    of a full tile, 2^s m / N (G(n,m)) or 2^s p (G(n,p)), reach 560 at s and
    not at s - 1; every one of these workloads lands within 0.02 of 1024."""
    from fractions import Fraction
    model = 0 if p == 0.0 else 1
    I = kgref.inst(n, m=m, p=p, directed=directed, seed=1, chunks=P, model=model)
    s = kgref.tile_exponent(I)
    assert s == s_want
    N = n * (n - 1) // (1 if directed else 2)
    mean = (lambda t: Fraction(m * 2**t, N)) if model == 0 else (lambda t: Fraction(p) * 2**t)
    assert mean(s) >= 560 and mean(s - 1) < 560
    assert abs(float(mean(s)) - 1024.0) < 0.02
