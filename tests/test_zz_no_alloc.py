"""sws_minimizers_noalloc (no workspace argument; scratch in a static device
array) against sws_minimizers with a caller workspace, through the C ABI.

Two calls in a row on one GPU, the second on a smaller input, so the second
runs over the scratch the first left behind."""
import ctypes

import numpy as np
import pytest

from gpu_util import dev, host_u32, host_u64, torch_cuda
from paper_1811_10074_amd import _lib, inputs

pytestmark = pytest.mark.gpu


def _stream(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _with_workspace(torch, lib, seq, k, w, flags):
    n = seq.numel()
    cap = max(1, n - k - w + 2)
    b = ctypes.c_uint64(0)
    assert lib.sws_minimizers_workspace(n, k, w, ctypes.byref(b)) == _lib.SWS_OK
    ws = torch.empty(max(int(b.value), 8), dtype=torch.uint8, device="cuda")
    h = torch.empty(cap, dtype=torch.int64, device="cuda")
    p = torch.empty(cap, dtype=torch.int32, device="cuda")
    c = torch.empty(1, dtype=torch.int64, device="cuda")
    st = lib.sws_minimizers(_p(seq), n, k, w, flags, _p(h), _p(p), cap, _p(c), _p(ws),
                            ws.numel(), _stream(torch))
    assert st == _lib.SWS_OK
    torch.cuda.synchronize()
    m = int(c.item())
    return host_u64(h[:m]), host_u32(p[:m])


def _noalloc(torch, lib, seq, k, w, flags):
    n = seq.numel()
    cap = max(1, n - k - w + 2)
    # outputs start as garbage, so every stored entry must come from the call
    h = torch.full((cap,), 0x5A5A5A5A, dtype=torch.int64, device="cuda")
    p = torch.full((cap,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
    c = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    st = lib.sws_minimizers_noalloc(_p(seq), n, k, w, flags, _p(h), _p(p), cap, _p(c),
                                    _stream(torch))
    assert st == _lib.SWS_OK, _lib.status_str(st)
    torch.cuda.synchronize()
    m = int(c.item())
    assert 0 <= m <= cap
    return host_u64(h[:m]), host_u32(p[:m])


@pytest.mark.parametrize("k,w,flags,n1,n2", [
    (15, 10, 0, 3_000_000, 200_003),                     # wave-tile path, large then small
    (19, 19, 0, 1_000_001, 65_537),
    (21, 100, 0, 2_000_000, 30_011),                     # block path (w > 32)
    (9, 6, _lib.KMER_FORWARD | _lib.HASH_IDENTITY, 500_000, 4_099),
    (15, 10, _lib.SPLIT_AT_INVALID, 1_500_000, 100_000),
])
def test_noalloc_matches_workspace_call(k, w, flags, n1, n2):
    torch = torch_cuda()
    lib = _lib.load()
    print("noalloc k=%d w=%d flags=%d n=%d,%d" % (k, w, flags, n1, n2), flush=True)
    for i, n in enumerate((n1, n2)):
        s = dev(inputs.dna(n, seed=50 + i, n_rate=0.01), torch)
        eh, ep = _with_workspace(torch, lib, s, k, w, flags)
        gh, gp = _noalloc(torch, lib, s, k, w, flags)
        assert len(ep) > 0
        assert np.array_equal(gp, ep), "positions differ (call %d)" % (i + 1)
        assert np.array_equal(gh, eh), "hashes differ (call %d)" % (i + 1)


def test_noalloc_rejects_before_enqueueing():
    torch = torch_cuda()
    lib = _lib.load()
    s = _stream(torch)
    fake = ctypes.c_void_p(0x10000)  # never dereferenced: every call below fails validation
    n = 1000
    bound = n - 15 - 10 + 2
    assert lib.sws_minimizers_noalloc(fake, n, 15, 10, _lib.WORKSPACE_KEPT, fake, fake, bound,
                                      fake, s) == _lib.SWS_ERR_INVALID
    assert lib.sws_minimizers_noalloc(fake, n, 15, 10, 0, fake, fake, bound - 1, fake,
                                      s) == _lib.SWS_ERR_CAPACITY
    assert lib.sws_minimizers_noalloc(fake, n, 15, 10, 0, fake, fake, bound, ctypes.c_void_p(0),
                                      s) == _lib.SWS_ERR_INVALID
    # beyond the scratch array: more look-back participants than it holds
    big = 1 << 30
    b = ctypes.c_uint64(0)
    assert lib.sws_minimizers_workspace(big, 15, 10, ctypes.byref(b)) == _lib.SWS_OK
    assert b.value > _lib.NOALLOC_SCRATCH_BYTES
    assert lib.sws_minimizers_noalloc(fake, big, 15, 10, 0, fake, fake, big, fake,
                                      s) == _lib.SWS_ERR_WORKSPACE
