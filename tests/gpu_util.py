"""Helpers shared by the GPU tests: device placement and unsigned views."""
import numpy as np
import pytest


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def dev(a, torch):
    """numpy array -> contiguous device tensor (unsigned data in signed dtypes)."""
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    elif a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(a).to("cuda")


def host_u32(t):
    return t.cpu().numpy().view(np.uint32)


def host_u64(t):
    return t.cpu().numpy().view(np.uint64)
