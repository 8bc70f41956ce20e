"""ctypes declarations of the C ABI in include/kg.h (argument marshalling
only: every step of the generator runs in the HIP library)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("KG_LIBRARY") or os.path.join(HERE, "libkg.so")

KG_OK, KG_EINVAL, KG_ERANGE, KG_ENOSPC, KG_EDEVICE, KG_ESCRATCH = 0, -1, -2, -3, -4, -5
KG_STATIC_SCRATCH_BYTES = 96 << 20
KG_GNM, KG_GNP = 0, 1
KG_OPT_LEAF_CAP, KG_OPT_SAMPLE_WAVES, KG_OPT_PLAN_WAVES = 1, 2, 3

EXPORTS = ["kg_spec_version", "kg_strerror", "kg_workspace_bytes", "kg_set_workspace", "kg_gnm", "kg_gnp", "kg_gnp_count",
           "kg_chunk_counts", "kg_batch", "kg_batch_upload", "kg_batch_launch", "kg_pe_view", "kg_gnp_skip",
           "kg_gnp_skip_workspace_bytes",
           "kg_rgg2d_workspace_bytes", "kg_rgg2d", "kg_rgg3d_workspace_bytes", "kg_rgg3d", "kg_instance_seed", "kg_set_option", "kg_get_option", "kg_last_hip_error", "kg_eval",
           "kg_kernel_time_read", "kg_edge_hash", "kg_gnm_static"]
KG_OPT_TIME_KERNELS = 4
KG_OPT_COUNT_LANES = 5
KG_OPT_SKIP_ROW = 6
KG_KERNEL_COUNT, KG_KERNEL_SCAN, KG_KERNEL_PLAN, KG_KERNEL_SAMPLE, KG_KERNEL_QUEUE = 0, 1, 2, 3, 4
KG_EVAL_PHILOX, KG_EVAL_LOG, KG_EVAL_LOG1P, KG_EVAL_LNF_DIFF, KG_EVAL_HYP, KG_EVAL_BIN, KG_EVAL_SQRT_DIV = range(1, 8)


class KgInstance(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("model", ctypes.c_uint32), ("directed", ctypes.c_uint32),
                ("m", ctypes.c_uint64), ("p", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("chunks", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class KgError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        msg = "%s: %s (%d)" % (what, strerror(status), status)
        if status == KG_EDEVICE:
            try:
                msg += ", HIP error %d" % lib().kg_last_hip_error()
            except Exception:
                pass
        super().__init__(msg)


_lib = None


def lib():
    """Load libkg.so; fails loudly if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("HIP library %s is missing: run `python -m paper_1710_07565_amd.build` "
                          "(or __graft_entry__.build())" % LIB_PATH)
    # PyTorch ships its own HIP runtime under the soname libamdhip64.so.7 but
    # asks for it as libamdhip64.so.  Loaded first, libkg.so would pull in the
    # system copy and the process would hold two HIP runtimes, so that the
    # streams and allocations the binding passes in belong to another runtime
    # than the library's launches.  Importing torch first makes libkg.so bind
    # to the runtime torch already holds.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    u64, u32, i32, dbl, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
    ip = ctypes.POINTER(KgInstance)
    L.kg_spec_version.argtypes = []; L.kg_spec_version.restype = u32
    L.kg_strerror.argtypes = [i32]; L.kg_strerror.restype = ctypes.c_char_p
    L.kg_workspace_bytes.argtypes = [ip, u32, ctypes.POINTER(u64)]; L.kg_workspace_bytes.restype = i32
    L.kg_set_workspace.argtypes = [vp, u64]; L.kg_set_workspace.restype = i32
    L.kg_edge_hash.argtypes = [vp, u64, vp, vp]; L.kg_edge_hash.restype = i32
    L.kg_gnm.argtypes = [u64, u64, ctypes.c_int, u64, u32, vp, u64, vp, u64, vp]; L.kg_gnm.restype = i32
    L.kg_gnm_static.argtypes = [u64, u64, ctypes.c_int, u64, u32, vp, u64, vp]; L.kg_gnm_static.restype = i32
    L.kg_gnp.argtypes = [u64, dbl, ctypes.c_int, u64, u32, vp, u64, vp, vp, u64, vp]; L.kg_gnp.restype = i32
    L.kg_gnp_count.argtypes = [u64, dbl, ctypes.c_int, u64, u32, ctypes.POINTER(u64), vp, u64, vp]
    L.kg_gnp_count.restype = i32
    L.kg_chunk_counts.argtypes = [ip, vp, vp, u64, vp]; L.kg_chunk_counts.restype = i32
    L.kg_batch.argtypes = [ip, u32, vp, u64, vp, vp, u64, vp]; L.kg_batch.restype = i32
    L.kg_batch_upload.argtypes = [ip, u32, vp, u64, vp]; L.kg_batch_upload.restype = i32
    L.kg_pe_view.argtypes = [ip, u32, vp, u64, vp, vp, u64, vp]; L.kg_pe_view.restype = i32
    L.kg_gnp_skip.argtypes = [u64, dbl, ctypes.c_int, u64, u32, vp, u64, vp, vp, u64, vp]
    L.kg_gnp_skip.restype = i32
    L.kg_gnp_skip_workspace_bytes.argtypes = [u64, dbl, ctypes.c_int, u32, vp]
    L.kg_gnp_skip_workspace_bytes.restype = i32
    L.kg_rgg2d_workspace_bytes.argtypes = [u64, dbl, vp]; L.kg_rgg2d_workspace_bytes.restype = i32
    L.kg_rgg2d.argtypes = [u64, dbl, u64, vp, vp, u64, vp, vp, u64, vp]; L.kg_rgg2d.restype = i32
    L.kg_rgg3d_workspace_bytes.argtypes = [u64, dbl, vp]; L.kg_rgg3d_workspace_bytes.restype = i32
    L.kg_rgg3d.argtypes = [u64, dbl, u64, vp, vp, u64, vp, vp, u64, vp]; L.kg_rgg3d.restype = i32
    L.kg_batch_launch.argtypes = [ip, u32, vp, u64, vp, vp, u64, vp]; L.kg_batch_launch.restype = i32
    L.kg_instance_seed.argtypes = [u64, u32]; L.kg_instance_seed.restype = u64
    L.kg_set_option.argtypes = [ctypes.c_int, ctypes.c_int64]; L.kg_set_option.restype = i32
    L.kg_get_option.argtypes = [ctypes.c_int]; L.kg_get_option.restype = ctypes.c_int64
    L.kg_last_hip_error.argtypes = []; L.kg_last_hip_error.restype = ctypes.c_int
    L.kg_eval.argtypes = [ctypes.c_int, vp, vp, u64, vp]; L.kg_eval.restype = i32
    L.kg_kernel_time_read.argtypes = [ctypes.c_int, ctypes.POINTER(dbl), ctypes.POINTER(u64)]
    L.kg_kernel_time_read.restype = i32
    _lib = L
    return L


def strerror(status):
    try:
        return lib().kg_strerror(status).decode()
    except Exception:  # the library itself may be what failed to load
        return "status"


def check(status, what):
    if status != KG_OK:
        raise KgError(status, what)
