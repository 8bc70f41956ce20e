"""Helpers shared by the GPU tests (no method arithmetic here)."""
import numpy as np


def to_np_u32(t):
    import torch
    return t.contiguous().view(torch.int32).cpu().numpy().view(np.uint32)


def to_np_u64(t):
    import torch
    return t.contiguous().view(torch.int64).cpu().numpy().view(np.uint64)


def require_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU test on a machine without a GPU"
    import paper_1710_07565_amd as kg
    kg._lib.lib()
    return kg
