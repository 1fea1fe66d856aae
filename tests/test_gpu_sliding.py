"""Parity of the HIP sliding-sum kernels with the CPU oracle (Eq. 2).

Bit-exact: every operator is integer arithmetic mod 2^32."""
import numpy as np
import pytest

import oracle
from gpu_util import dev, host_u32, torch_cuda
from paper_1811_10074_amd import inputs

pytestmark = pytest.mark.gpu

S16 = 64 * 16  # elements per wavefront slab (16 per lane)


def run(torch, op, w, x, path="auto"):
    import paper_1811_10074_amd as sws
    y = sws.sliding_sum(op, w, dev(x, torch), path=path)
    torch.cuda.synchronize()
    return host_u32(y)


def check(torch, op, w, x, path="auto"):
    got = run(torch, op, w, x, path)
    exp = oracle.sliding_sum(op, w, x)
    assert got.shape == exp.shape, (op, w, path, got.shape, exp.shape)
    if not np.array_equal(got, exp):
        bad = np.nonzero(got.reshape(len(got), -1) != exp.reshape(len(exp), -1))[0]
        raise AssertionError("op=%s w=%d path=%s n=%d: %d mismatches, first at %d"
                             % (op, w, path, len(x), bad.size, bad[0]))


def test_config1_min_and_add():
    """N = 2^20 uniform u32 (seed 0), w = 16, min and + mod 2^32."""
    torch = torch_cuda()
    x = inputs.uniform_u32(1 << 20, seed=0)
    for op in ("min", "add"):
        check(torch, op, 16, x)
    check(torch, "min", 16, x, path="log")


WINDOWS = [1, 2, 3, 4, 5, 7, 10, 15, 16, 17, 31, 33, 64, 100, 255, 256, 1000, 1023, 1024, 1025,
           2047, 2048]


@pytest.mark.parametrize("op", ["add", "min", "max", "affine"])
def test_window_sweep_generic(op):
    torch = torch_cuda()
    rng_seed = {"add": 5, "min": 6, "max": 7, "affine": 8}[op]
    for w in WINDOWS:
        n = 3 * S16 * 2 + 37 + w  # several slabs plus a ragged tail
        x = inputs.affine_pairs(n, rng_seed + w, odd=True) if op == "affine" else \
            inputs.uniform_u32(n, rng_seed + w)
        check(torch, op, w, x, "generic")


def test_window_sweep_prefix():
    """The prefix-difference path (+ only) over the generic sweep's windows."""
    torch = torch_cuda()
    for w in WINDOWS:
        n = 3 * S16 * 2 + 37 + w
        check(torch, "add", w, inputs.uniform_u32(n, 60 + w), "prefix")


@pytest.mark.parametrize("op", ["add", "min", "max", "affine"])
def test_window_sweep_scalar(op):
    """Alg. 1 (scalar input) for every op and w up to 64, over several
    4096-output wavefront runs with a ragged tail."""
    torch = torch_cuda()
    seed = {"add": 70, "min": 71, "max": 72, "affine": 73}[op]
    for w in [1, 2, 3, 5, 10, 16, 17, 31, 32, 33, 63, 64]:
        for n in (w, w + 1, 64 + w, 3 * 4096 + 77 + w):
            x = inputs.affine_pairs(n, seed + w, odd=True) if op == "affine" else \
                inputs.uniform_u32(n, seed + w)
            check(torch, op, w, x, "scalar")


@pytest.mark.parametrize("op", ["min", "max"])
def test_window_sweep_log(op):
    torch = torch_cuda()
    for w in WINDOWS + [4095, 4096]:
        n = 2 * 4096 + 123 + w
        check(torch, op, w, inputs.uniform_u32(n, 40 + w), "log")


@pytest.mark.parametrize("kind", inputs.ADVERSARIAL_KINDS)
def test_adversarial_inputs(kind):
    torch = torch_cuda()
    for w in (4, 16, 17, 64, 1024):
        x = inputs.adversarial(kind, 5000 + w, w, seed=3)
        for op in ("add", "min", "max"):
            check(torch, op, w, x, "generic")
        for op in ("min", "max"):
            check(torch, op, w, x, "log")


def test_affine_uniform_and_many_waves():
    """Uniform a (not forced odd) and an input long enough for many waves,
    each streaming several slabs."""
    torch = torch_cuda()
    for w in (4, 16, 64, 256, 1024):
        x = inputs.affine_pairs(200_003, seed=w)
        check(torch, "affine", w, x)
    x = inputs.uniform_u32(3_000_017, seed=9)
    for w in (16, 1000):
        check(torch, "add", w, x)
        check(torch, "max", w, x)


def test_edges():
    torch = torch_cuda()
    import paper_1811_10074_amd as sws
    for n in (0, 1, 2, 15, 16):
        x = inputs.uniform_u32(n, 1)
        for w in (1, 2, 16, 17):
            for op in ("add", "min"):
                t = dev(x, torch) if n else torch.empty(0, dtype=torch.int32, device="cuda")
                y = sws.sliding_sum(op, w, t)
                torch.cuda.synchronize()
                assert y.numel() == max(0, n - w + 1)
                if y.numel():
                    assert np.array_equal(host_u32(y), oracle.sliding_sum(op, w, x))
    with pytest.raises(ValueError):
        sws.sliding_sum("add", 0, dev(inputs.uniform_u32(10, 1), torch))
    with pytest.raises(ValueError):
        sws.sliding_sum("add", 4, dev(inputs.uniform_u32(10, 1), torch), path="log")


def test_unaligned_pointers():
    """Views starting 1..3 elements into a buffer take the unaligned path."""
    torch = torch_cuda()
    import paper_1811_10074_amd as sws
    base = inputs.uniform_u32(70_001, 2)
    t = dev(base, torch)
    for off in (1, 2, 3):
        for w in (5, 16, 300):
            for op in ("add", "min", "max"):
                y = sws.sliding_sum(op, w, t[off:])
                torch.cuda.synchronize()
                assert np.array_equal(host_u32(y), oracle.sliding_sum(op, w, base[off:])), (off, w, op)
    tp = dev(inputs.affine_pairs(50_001, 3, odd=True), torch)
    y = sws.sliding_sum("affine", 9, tp[1:])
    torch.cuda.synchronize()
    assert np.array_equal(host_u32(y), oracle.sliding_sum("affine", 9, host_u32(tp[1:])))


def test_paths_agree_and_repeat():
    """Generic and log paths agree bit for bit; repeated calls are identical."""
    torch = torch_cuda()
    x = inputs.uniform_u32(500_000, 11)
    for w in (3, 16, 100, 1024):
        for op in ("min", "max"):
            a = run(torch, op, w, x, "generic")
            b = run(torch, op, w, x, "log")
            c = run(torch, op, w, x, "generic")
            assert np.array_equal(a, b) and np.array_equal(a, c)


def _sample_check(torch, op, w, x, y, samples, rng):
    idx = np.concatenate([[0, y.shape[0] - 1], rng.integers(0, y.shape[0], samples)])
    for i in idx:
        exp = oracle.sliding_sum(op, w, x[i:i + w])
        assert np.array_equal(y[i], exp[0]), (op, w, int(i))


@pytest.mark.parametrize("op", ["add", "min", "max", "affine"])
def test_config3_full_size(op):
    """N = 2^28 at every window of the sweep, in the bench's launch
    configuration, every output compared: min and max against the oracle's
    O(N) deque, + against the prefix-difference identity, affine (odd
    multipliers, so every map is invertible) against prefix compositions;
    and 300 sampled outputs against the fold of Eq. 2 itself."""
    torch = torch_cuda()
    import paper_1811_10074_amd as sws
    n = 1 << 28
    rng = np.random.default_rng(99)
    x = inputs.affine_pairs(n, seed=2, odd=True) if op == "affine" else inputs.uniform_u32(n, seed=2)
    t = dev(x, torch)
    paths = {"min": ["auto", "generic", "log"], "max": ["auto", "generic", "log"],
             "add": ["auto", "generic", "prefix"], "affine": ["auto", "generic"]}[op]
    pfx = None
    if op == "add":
        pfx = np.zeros(n + 1, dtype=np.uint64)
        np.cumsum(x, dtype=np.uint64, out=pfx[1:])
    for w in (4, 16, 64, 256, 1024):
        print("config 3 full size: op=%s w=%d" % (op, w), flush=True)
        if op in ("min", "max"):
            exp = oracle.sliding_extremum_deque(op, w, x)
        elif op == "affine":
            exp = oracle.affine_windows_by_prefix(w, x)
        else:
            exp = ((pfx[w:] - pfx[:-w]) & np.uint64(0xFFFFFFFF)).astype(np.uint32)
        for path in paths:
            y = sws.sliding_sum(op, w, t, path=path)
            torch.cuda.synchronize()
            yh = host_u32(y)
            del y
            if not np.array_equal(yh, exp):
                bad = np.nonzero(yh.reshape(len(yh), -1) != exp.reshape(len(exp), -1))[0]
                raise AssertionError("op=%s w=%d path=%s: %d mismatches, first at %d"
                                     % (op, w, path, bad.size, bad[0]))
            _sample_check(torch, op, w, x, yh, 100, rng)
        del exp


def _slab(op, w):
    """Elements per wavefront slab of the generic kernel for (op, w)."""
    if op == "affine":
        r = 8 if w <= 512 else (16 if w <= 1024 else 32)
    else:
        r = 16 if w <= 1024 else 32
    return 64 * r


@pytest.fixture
def few_waves():
    import paper_1811_10074_amd as sws
    yield sws.set_sliding_waves
    sws.set_sliding_waves(0)


@pytest.mark.parametrize("waves", [1, 2, 3, 5])
@pytest.mark.parametrize("op", ["add", "min", "max", "affine"])
def test_long_streams_per_wave(few_waves, waves, op):
    """Few wavefronts, each streaming many slabs: the unchecked steady-state
    loop, its peeled first step, the step that prefetches the next wave's
    first slab, the last in-range steps of a wave and the checked steps at
    the end, with n on either side of the slab boundaries that decide between
    them; waves of one slab, of fewer slabs than are in flight, and of odd and
    even slab counts (two register buffers alternate).  Windows from 128 on
    load the next wave's first slab at the wave's start instead (w = 127 and
    128 on either side of that, 512 the last such window of 8-element affine
    runs)."""
    torch = torch_cuda()
    few_waves(waves)
    seed = {"add": 21, "min": 22, "max": 23, "affine": 24}[op]
    for w in (1, 16, 17, 127, 128, 512, 1024, 1025, 2048):
        S = _slab(op, w)
        for n in (2 * S + w, 3 * S - 1, 3 * S + w - 1, 4 * S + w, 5 * S + w - 2, 7 * S + w + 1,
                  12 * S + 3):
            if n < w:
                continue
            x = inputs.affine_pairs(n, seed + n, odd=True) if op == "affine" else \
                inputs.uniform_u32(n, seed + n)
            check(torch, op, w, x, "generic")
            if op == "add":
                check(torch, op, w, x, "prefix")


@pytest.mark.parametrize("waves", [1, 3])
def test_long_streams_unaligned(few_waves, waves):
    """As above on views 1..3 elements into a buffer (the checked path for
    every step)."""
    torch = torch_cuda()
    import paper_1811_10074_amd as sws
    few_waves(waves)
    base = inputs.uniform_u32(9 * S16 + 77, 31)
    t = dev(base, torch)
    for off in (0, 1, 3):
        for w in (16, 300):
            for op in ("add", "max"):
                y = sws.sliding_sum(op, w, t[off:], path="generic")
                torch.cuda.synchronize()
                assert np.array_equal(host_u32(y), oracle.sliding_sum(op, w, base[off:])), (off, w, op)


@pytest.mark.parametrize("op", ["add", "min"])
def test_beyond_2p32_elements_sampled(op):
    """n = 2^32 + 4099 (past 32-bit element indices, ragged tail), made on the
    device by a seeded generator; outputs around index 2^32, the last ones and
    random ones against the oracle, on every path of the op."""
    torch = torch_cuda()
    import paper_1811_10074_amd as sws
    n = (1 << 32) + 4099
    g = torch.Generator(device="cuda")
    g.manual_seed(4242)
    t = torch.randint(-(1 << 31), 1 << 31, (n,), dtype=torch.int32, device="cuda", generator=g)
    rng = np.random.default_rng(5)
    for w in (16, 1000):
        m = n - w + 1
        idx = np.unique(np.concatenate([np.arange((1 << 32) - w - 3, (1 << 32) + 3),
                                        np.arange(m - 5, m), rng.integers(0, m, 200)]))
        it = torch.from_numpy(idx).to("cuda")
        win = host_u32(t[(it[:, None] + torch.arange(w, device="cuda")).flatten()]).reshape(-1, w)
        exp = np.array([oracle.sliding_sum(op, w, row)[0] for row in win], dtype=np.uint32)
        for path in (["generic", "prefix"] if op == "add" else ["generic", "log"]):
            y = sws.sliding_sum(op, w, t, path=path)
            got = host_u32(y[it])
            bad = np.nonzero(got != exp)[0]
            assert bad.size == 0, (op, w, path, idx[bad[:5]].tolist())
            del y
    del t
    torch.cuda.empty_cache()


def _wide_expected(op, w, x):
    """O(N) expectations: the deque (min, max), the prefix identity (+), the
    prefix compositions (affine with odd multipliers)."""
    if op in ("min", "max"):
        return oracle.sliding_extremum_deque(op, w, x)
    if op == "affine":
        return oracle.affine_windows_by_prefix(w, x)
    pfx = np.zeros(x.size + 1, dtype=np.uint64)
    np.cumsum(x, dtype=np.uint64, out=pfx[1:])
    return ((pfx[w:] - pfx[:-w]) & np.uint64(0xFFFFFFFF)).astype(np.uint32)


@pytest.mark.parametrize("op", ["add", "min", "max", "affine"])
def test_wide_windows(op):
    """Windows past one slab (Eq. 2 holds for every w): w in {2049, 4097,
    65537} and a window of 2^22 + 3, with n from exactly w (one output) to
    several segments with a ragged last chunk; every output against an O(N)
    oracle and sampled outputs against the fold itself, on AUTO and GENERIC."""
    torch = torch_cuda()
    import paper_1811_10074_amd as sws
    rng = np.random.default_rng({"add": 1, "min": 2, "max": 3, "affine": 4}[op])
    cases = [(2049, 2049), (2049, 2050), (2049, 3 * 2049 + 777), (4097, 100_003),
             (65537, 65537 + 1), (65537, 1_000_000), (65537, 1 << 22), ((1 << 22) + 3, 1 << 24)]
    for w, n in cases:
        print("wide window: op=%s w=%d n=%d" % (op, w, n), flush=True)
        x = inputs.affine_pairs(n, seed=w % 1000, odd=True) if op == "affine" else \
            inputs.uniform_u32(n, seed=w % 1000)
        if op in ("min", "max") and n > 5000:
            x[rng.integers(0, n, 50)] = 0 if op == "min" else 0xFFFFFFFF  # extremes to carry far
        exp = _wide_expected(op, w, x)
        t = dev(x, torch)
        for path in ("auto", "generic"):
            y = sws.sliding_sum(op, w, t, path=path)
            torch.cuda.synchronize()
            got = host_u32(y)
            assert got.shape == exp.shape, (op, w, n, path)
            if not np.array_equal(got, exp):
                bad = np.nonzero(got.reshape(len(got), -1) != exp.reshape(len(exp), -1))[0]
                raise AssertionError("op=%s w=%d n=%d path=%s: %d mismatches, first at %d"
                                     % (op, w, n, path, bad.size, bad[0]))
        if w <= 65537:
            idx = np.concatenate([[0, exp.shape[0] - 1], rng.integers(0, exp.shape[0], 5)])
            for i in idx:
                assert np.array_equal(exp[i], oracle.sliding_sum(op, w, x[i:i + w])[0]), (op, w, i)


def test_wide_windows_beyond_other_paths():
    """LOG serves min and max up to 4096 only; PREFIX (+) and SCALAR keep
    their limits; n < w gives no outputs."""
    torch = torch_cuda()
    import paper_1811_10074_amd as sws
    x = dev(inputs.uniform_u32(10_000, seed=5), torch)
    with pytest.raises(ValueError):
        sws.sliding_sum("min", 4097, x, path="log")
    with pytest.raises(ValueError):
        sws.sliding_sum("add", 4097, x, path="prefix")
    with pytest.raises(ValueError):
        sws.sliding_sum("add", 4097, x, path="scalar")
    assert sws.sliding_sum("max", 10_001, x).numel() == 0
