"""The C-ABI library: it loads, exports every function the header declares,
and validates arguments on the host before anything is enqueued (these calls
return before any device call, so they run without a GPU)."""
import ctypes

import pytest

from paper_1811_10074_amd import _lib

FAKE = ctypes.c_void_p(0x10000)  # never dereferenced: validation fails first
NULL = ctypes.c_void_p(0)


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_exports_every_header_function(lib):
    names = _lib.header_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
        assert name in _lib._SIGNATURES, name


def test_version_and_status(lib):
    assert lib.sws_abi_version() == 5
    for st in (0, -1, -2, -3, -4, -5):
        assert lib.sws_status_str(st)
    assert b"unknown" in lib.sws_status_str(7)


def test_sliding_validation(lib):
    s = NULL
    assert lib.sws_sliding_sum(9, 4, FAKE, 100, FAKE, s) == _lib.SWS_ERR_INVALID
    assert lib.sws_sliding_sum(0, 0, FAKE, 100, FAKE, s) == _lib.SWS_ERR_INVALID
    assert lib.sws_sliding_sum_ex(0, 4, FAKE, 100, FAKE, 2, s) == _lib.SWS_ERR_UNSUPPORTED
    assert lib.sws_sliding_sum_ex(3, 4, FAKE, 100, FAKE, 2, s) == _lib.SWS_ERR_UNSUPPORTED
    assert lib.sws_sliding_sum_ex(1, 4, FAKE, 100, FAKE, 7, s) == _lib.SWS_ERR_INVALID
    # n < w: no outputs, not an error, nothing touched
    assert lib.sws_sliding_sum(0, 10, NULL, 5, NULL, s) == _lib.SWS_OK
    assert lib.sws_sliding_sum(0, 3, NULL, 5, FAKE, s) == _lib.SWS_ERR_INVALID
    assert lib.sws_sliding_sum(0, 3, ctypes.c_void_p(0x10002), 5, FAKE, s) == _lib.SWS_ERR_INVALID
    assert lib.sws_sliding_sum(3, 3, ctypes.c_void_p(0x10004), 5, FAKE, s) == _lib.SWS_ERR_INVALID
    assert lib.sws_sliding_sum(0, 1 << 20, FAKE, 1 << 21, FAKE, s) == _lib.SWS_ERR_UNSUPPORTED


def test_kmer_validation(lib):
    s = NULL
    assert lib.sws_kmers(FAKE, 100, 0, 0, FAKE, s) == _lib.SWS_ERR_INVALID
    assert lib.sws_kmers(FAKE, 100, 32, 0, FAKE, s) == _lib.SWS_ERR_INVALID
    assert lib.sws_kmers(FAKE, 100, 15, 8, FAKE, s) == _lib.SWS_ERR_INVALID
    assert lib.sws_kmers(FAKE, 100, 30, 0, FAKE, s) == _lib.SWS_ERR_UNSUPPORTED
    assert lib.sws_kmers(NULL, 10, 15, 0, NULL, s) == _lib.SWS_OK      # n < k
    assert lib.sws_kmers(NULL, 100, 15, 0, FAKE, s) == _lib.SWS_ERR_INVALID
    assert lib.sws_pack2bit(NULL, 0, NULL, NULL, s) == _lib.SWS_OK
    assert lib.sws_pack2bit(NULL, 10, FAKE, NULL, s) == _lib.SWS_ERR_INVALID


def test_minimizer_validation(lib):
    s = NULL
    b = ctypes.c_uint64(0)
    assert lib.sws_minimizers_workspace(1 << 26, 15, 10, ctypes.byref(b)) == _lib.SWS_OK
    ws = b.value
    assert ws >= 256 + 8 * ((1 << 26) // 2048)
    assert lib.sws_minimizers_workspace(100, 0, 10, ctypes.byref(b)) == _lib.SWS_ERR_INVALID
    assert lib.sws_minimizers_workspace(100, 15, 0, ctypes.byref(b)) == _lib.SWS_ERR_INVALID
    assert lib.sws_minimizers_workspace(100, 15, 2000, ctypes.byref(b)) == _lib.SWS_ERR_UNSUPPORTED
    n = 1000
    bound = n - 15 - 10 + 2
    args = lambda cap, wsb, wsp=FAKE, cnt=FAKE, fl=0: (FAKE, n, 15, 10, fl, FAKE, FAKE, cap, cnt, wsp, wsb, s)
    assert lib.sws_minimizers(*args(bound - 1, 1 << 20)) == _lib.SWS_ERR_CAPACITY
    assert lib.sws_minimizers(*args(bound, 16)) == _lib.SWS_ERR_WORKSPACE
    assert lib.sws_minimizers(*args(bound, 1 << 20, wsp=NULL)) == _lib.SWS_ERR_WORKSPACE
    assert lib.sws_minimizers(*args(bound, 1 << 20, wsp=ctypes.c_void_p(0x10004))) == _lib.SWS_ERR_WORKSPACE
    assert lib.sws_minimizers(*args(bound, 1 << 20, cnt=NULL)) == _lib.SWS_ERR_INVALID
    assert lib.sws_minimizers(*args(bound, 1 << 20, fl=16)) == _lib.SWS_ERR_INVALID
    assert lib.sws_minimizers(NULL, n, 15, 10, 0, FAKE, FAKE, bound, FAKE, FAKE, 1 << 20, s) == _lib.SWS_ERR_INVALID
    assert lib.sws_minimizers(FAKE, 1 << 32, 15, 10, 0, FAKE, FAKE, 1 << 33, FAKE, FAKE, 1 << 30, s) == _lib.SWS_ERR_UNSUPPORTED
    assert lib.sws_minimizers_2bit(ctypes.c_void_p(0x10002), NULL, n, 15, 10, 0, FAKE, FAKE, bound, FAKE, FAKE, 1 << 20, s) == _lib.SWS_ERR_INVALID
    # the batched call's workgroup size is an argument: 0 (default) or 64..512
    for bad in (1, 100, 1024):
        assert lib.sws_minimizers_batch_ex(FAKE, FAKE, 10, 1000, 15, 10, 0, FAKE, FAKE, FAKE,
                                           1 << 20, FAKE, FAKE, 1 << 30, bad, s) == _lib.SWS_ERR_INVALID
    assert not hasattr(lib, "sws_set_minimizer_block")
    assert lib.sws_set_sliding_waves((1 << 24) + 1) == _lib.SWS_ERR_INVALID
    # split semantics: minimizers only, w <= 32
    b2 = ctypes.c_uint64(0)
    assert lib.sws_minimizers_workspace(1000, 15, 33, ctypes.byref(b2)) == _lib.SWS_OK
    assert lib.sws_minimizers(FAKE, 1000, 15, 33, 4, FAKE, FAKE, 1 << 20, FAKE, FAKE, 1 << 30,
                              s) == _lib.SWS_ERR_UNSUPPORTED
    assert lib.sws_kmers(FAKE, 1000, 15, 4, FAKE, s) == _lib.SWS_ERR_INVALID
    assert lib.sws_minimizers(FAKE, 1000, 15, 10, 16, FAKE, FAKE, 1 << 20, FAKE, FAKE, 1 << 30,
                              s) == _lib.SWS_ERR_INVALID
    # a kept workspace is a minimizer option: k-mers refuse it; the batched
    # call takes it (and then stops at the too-small workspace, before any
    # launch), but not with an unknown bit beside it
    kept = _lib.WORKSPACE_KEPT
    assert lib.sws_kmers(FAKE, 1000, 15, kept, FAKE, s) == _lib.SWS_ERR_INVALID
    assert lib.sws_minimizers_batch(FAKE, FAKE, 10, 1000, 15, 10, kept, FAKE, FAKE, FAKE, 1 << 20,
                                    FAKE, FAKE, 8, s) == _lib.SWS_ERR_WORKSPACE
    assert lib.sws_minimizers_batch(FAKE, FAKE, 10, 1000, 15, 10, kept | 16, FAKE, FAKE, FAKE,
                                    1 << 20, FAKE, FAKE, 1 << 30, s) == _lib.SWS_ERR_INVALID
    # the prefix-difference path exists for + only
    for op in (1, 2, 3):
        assert lib.sws_sliding_sum_ex(op, 4, FAKE, 100, FAKE, 3, s) == _lib.SWS_ERR_UNSUPPORTED
    assert lib.sws_sliding_sum_ex(0, 65, FAKE, 100, FAKE, 4, s) == _lib.SWS_ERR_UNSUPPORTED
    assert lib.sws_sliding_sum_ex(0, 4, FAKE, 100, FAKE, 5, s) == _lib.SWS_ERR_INVALID
    # seed table: argument checks happen before anything is enqueued
    b = ctypes.c_uint64(0)
    assert lib.sws_seed_table_workspace(1000, 0, ctypes.byref(b)) == _lib.SWS_ERR_INVALID
    assert lib.sws_seed_table_workspace(1000, 31, ctypes.byref(b)) == _lib.SWS_ERR_INVALID
    assert lib.sws_seed_table_workspace(1 << 32, 16, ctypes.byref(b)) == _lib.SWS_ERR_UNSUPPORTED
    assert lib.sws_seed_table_workspace(1000, 16, ctypes.byref(b)) == _lib.SWS_OK and b.value > 0
    need = b.value
    st = lambda cnt, bits, shift, ws, wsb, h=FAKE, po=FAKE, ptr=FAKE: lib.sws_seed_table(
        h, FAKE, cnt, bits, shift, ptr, po, NULL, ws, wsb, s)
    assert st(1000, 16, 49, FAKE, need) == _lib.SWS_ERR_INVALID          # shift + bits > 64
    assert st(1000, 0, 0, FAKE, need) == _lib.SWS_ERR_INVALID
    assert st(1000, 16, 48, FAKE, need, ptr=NULL) == _lib.SWS_ERR_INVALID
    assert st(1000, 16, 48, FAKE, need, h=NULL) == _lib.SWS_ERR_INVALID
    assert st(1000, 16, 48, FAKE, need, po=NULL) == _lib.SWS_ERR_INVALID
    assert st(1 << 32, 16, 48, FAKE, need) == _lib.SWS_ERR_UNSUPPORTED
    assert st(1000, 16, 48, NULL, need) == _lib.SWS_ERR_WORKSPACE
    assert st(1000, 16, 48, FAKE, need - 1) == _lib.SWS_ERR_WORKSPACE
    assert st(1000, 16, 48, ctypes.c_void_p(0x10008), need) == _lib.SWS_ERR_WORKSPACE
    assert lib.sws_set_sliding_waves(0) == _lib.SWS_OK


def test_binding_rejects_host_buffers():
    """Host memory never reaches a kernel: the binding refuses CPU tensors and
    numpy arrays that report a "cpu" device before calling the library."""
    import numpy as np
    import torch

    import paper_1811_10074_amd as sws
    from paper_1811_10074_amd.batch import BatchRunner

    seq = torch.full((100,), ord("A"), dtype=torch.uint8)
    off = np.array([0, 60, 100], dtype=np.uint64)
    with pytest.raises(ValueError):
        BatchRunner(seq, off, 15, 10, device="cpu")
    with pytest.raises(ValueError):
        sws.minimizers(seq, 15, 10)
    with pytest.raises(ValueError):
        sws.MinimizerRunner(100, 15, 10, device="cpu")
    with pytest.raises(ValueError):
        sws.sliding_sum("add", 4, torch.zeros(100, dtype=torch.int32))
    with pytest.raises(ValueError):
        sws.seed_table(torch.zeros(10, dtype=torch.int64), torch.zeros(10, dtype=torch.int32), 8)


def test_missing_library_fails_loudly(tmp_path):
    """No fallback: without the built library every entry point raises."""
    import subprocess
    import sys
    code = (
        "import sys\n"
        "from paper_1811_10074_amd import _lib\n"
        "_lib.LIB_PATH = %r\n"
        "try:\n"
        "    _lib.load()\n"
        "except ImportError as e:\n"
        "    print('raised:', 'not built' in str(e))\n"
        "    sys.exit(0)\n"
        "sys.exit(1)\n" % str(tmp_path / "absent" / "libsws.so"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       cwd=str(__import__("pathlib").Path(__file__).resolve().parents[1]))
    assert r.returncode == 0 and "raised: True" in r.stdout, r.stdout + r.stderr


def test_wide_window_validation(lib):
    """Windows above 2048 need the workspace call; validation happens on the
    host before anything is enqueued."""
    s = NULL
    b = ctypes.c_uint64(0)
    # no scratch for short windows or for paths that keep their own limits
    assert lib.sws_sliding_sum_workspace(0, 2048, 1 << 20, 0, ctypes.byref(b)) == _lib.SWS_OK
    assert b.value == 0
    assert lib.sws_sliding_sum_workspace(1, 5000, 1 << 20, 2, ctypes.byref(b)) == _lib.SWS_OK
    assert b.value == 0
    assert lib.sws_sliding_sum_workspace(1, 5000, 100, 0, ctypes.byref(b)) == _lib.SWS_OK
    assert b.value == 0  # n < w: no outputs
    # 3 values per chunk of 2048 offsets per segment
    assert lib.sws_sliding_sum_workspace(0, 65537, 1 << 20, 0, ctypes.byref(b)) == _lib.SWS_OK
    nseg, nch = -(-(1 << 20) // 65537), -(-65537 // 2048)
    assert b.value >= 3 * nseg * nch * 4
    assert lib.sws_sliding_sum_workspace(3, 65537, 1 << 20, 1, ctypes.byref(b)) == _lib.SWS_OK
    assert b.value >= 3 * nseg * nch * 8
    assert lib.sws_sliding_sum_workspace(9, 65537, 1 << 20, 0, ctypes.byref(b)) == _lib.SWS_ERR_INVALID
    assert lib.sws_sliding_sum_workspace(0, 0, 1 << 20, 0, ctypes.byref(b)) == _lib.SWS_ERR_INVALID
    # the short-window entry point still refuses wide windows
    assert lib.sws_sliding_sum(0, 4097, FAKE, 1 << 20, FAKE, s) == _lib.SWS_ERR_UNSUPPORTED
    # the wide call: workspace missing or small, explicit paths past their limits
    ws = ctypes.c_uint64(0)
    assert lib.sws_sliding_sum_workspace(0, 4097, 1 << 20, 0, ctypes.byref(ws)) == _lib.SWS_OK
    assert lib.sws_sliding_sum_ws(0, 4097, FAKE, 1 << 20, FAKE, 0, NULL, ws.value, s) == _lib.SWS_ERR_WORKSPACE
    assert lib.sws_sliding_sum_ws(0, 4097, FAKE, 1 << 20, FAKE, 0, FAKE, ws.value - 1, s) == _lib.SWS_ERR_WORKSPACE
    assert lib.sws_sliding_sum_ws(0, 4097, FAKE, 1 << 20, FAKE, 3, FAKE, ws.value, s) == _lib.SWS_ERR_UNSUPPORTED
    assert lib.sws_sliding_sum_ws(1, 5000, FAKE, 1 << 20, FAKE, 2, FAKE, ws.value, s) == _lib.SWS_ERR_UNSUPPORTED
    assert lib.sws_sliding_sum_ws(0, 4097, FAKE, 1 << 20, FAKE, 4, FAKE, ws.value, s) == _lib.SWS_ERR_UNSUPPORTED
    assert lib.sws_sliding_sum_ws(3, 4097, ctypes.c_void_p(0x10004), 1 << 20, FAKE, 0, FAKE, 1 << 30, s) == _lib.SWS_ERR_INVALID
    assert lib.sws_sliding_sum_ws(0, 4097, NULL, 100, NULL, 0, NULL, 0, s) == _lib.SWS_OK  # n < w
