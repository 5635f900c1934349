"""GPU parity of the rANS coder (tpc_rans_encode through the C-ABI): the
stream must be byte-identical to the oracle's for the same array and
parameters (integer arithmetic on both sides), and the oracle's decoder must
give the array back."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _gpu(x, L, B, cap=None):
    import torch
    from paper_2412_13755_amd.reco import rans_encode
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.int32)).cuda()
    out = None if cap is None else torch.empty(cap, dtype=torch.uint8, device="cuda")
    out, size, status = rans_encode(t, L, B, out=out)
    torch.cuda.synchronize()
    n = int(size.item())
    st = int(status.item())
    return (out[:n].cpu().numpy().tobytes() if st == 0 else None), n, st


def _check(x, L, B, label):
    print("[rans] %s: n=%d L=%d B=%d" % (label, len(x), L, B), flush=True)
    g, n, st = _gpu(x, L, B)
    assert st == 0, st
    r = oracle.rans_encode(x, L, B)
    assert len(g) == len(r), (len(g), len(r))
    assert g == r, "streams differ at byte %d" % next(i for i in range(len(r)) if g[i] != r[i])
    np.testing.assert_array_equal(oracle.rans_decode(g), x)
    return len(g)


@pytest.mark.parametrize("L,B", [(16, 64), (12, 4096), (11, 32768), (16, 1 << 20)])
def test_geometric_symbols(torch_dev, L, B):
    rng = np.random.default_rng(L * 7 + B)
    x = (rng.geometric(0.05, 1_000_003) - 20).astype(np.int32)
    size = _check(x, L, B, "geometric")
    if B >= 4096:                      # 256 bytes of coder states per block
        assert size < 2 * len(x)


def test_ragged_small_and_degenerate(torch_dev):
    rng = np.random.default_rng(3)
    for n in (0, 1, 2, 63, 64, 65, 64 * 37 + 13):
        _check(rng.integers(-3, 9, n).astype(np.int32), 12, 128, "ragged %d" % n)
    _check(np.full(10_000, -7, np.int32), 12, 1024, "one symbol")
    _check((np.int32(-2**31) + rng.integers(0, 5, 5000)).astype(np.int32), 16, 256, "int32 minimum")
    _check(np.array([7], np.int32), 16, 64, "single value")


def test_wide_range_uses_global_histogram(torch_dev):
    rng = np.random.default_rng(4)
    x = rng.integers(0, 16000, 500_000).astype(np.int32)        # range above the LDS histogram
    _check(x, 16, 8192, "wide")
    y = np.concatenate([rng.integers(0, 50, 100_000), [1 << 19]]).astype(np.int32)   # sparse wide range
    _check(y, 12, 4096, "sparse range")


def test_errors_and_capacity(torch_dev):
    _, _, st = _gpu(np.arange(300, dtype=np.int32), 8, 64)             # 300 symbols, M = 256
    assert st == -1
    _, _, st = _gpu(np.array([0, 1 << 21], np.int32), 16, 64)           # range beyond 2^20
    assert st == -1
    x = np.random.default_rng(6).integers(0, 40, 50_000).astype(np.int32)
    want = len(oracle.rans_encode(x, 12, 4096))
    g, n, st = _gpu(x, 12, 4096, cap=want - 1)
    assert st == -2 and n == want
    g, n, st = _gpu(x, 12, 4096, cap=want)
    assert st == 0 and n == want


def test_large_array(torch_dev):
    rng = np.random.default_rng(9)
    x = np.round(rng.normal(0.0, 12.0, 1 << 24)).astype(np.int32)
    _check(x, 14, 1 << 15, "2^24 normal")


def test_large_arrays_counted_in_one_pass(torch_dev):
    """Arrays of 2^22 symbols or more count their histogram in the range pass,
    relative to a window of 2^20 around the first symbol: in the window (the
    first symbol at the range's low end), one symbol beyond it (the two-pass
    path takes over), and a range wider than 2^20 (refused)."""
    rng = np.random.default_rng(12)
    x = np.abs(np.round(rng.normal(0.0, 300.0, 1 << 22))).astype(np.int32)
    x[0] = 0                                                   # the window's centre at the minimum
    _check(x, 14, 1 << 15, "2^22, first symbol at the minimum")
    y = x.copy()
    y[12345] = 900_000                                         # range < 2^20, beyond the window
    _check(y, 14, 1 << 15, "2^22, one symbol beyond the window")
    z = x.copy()
    z[777] = 1 << 21                                           # range beyond 2^20
    _, _, st = _gpu(z, 14, 1 << 15)
    assert st == -1


def test_repeat_is_identical(torch_dev):
    x = np.random.default_rng(10).integers(-100, 100, 300_000).astype(np.int32)
    a, _, _ = _gpu(x, 12, 4096)
    b, _, _ = _gpu(x, 12, 4096)
    assert a == b


def test_batch_equals_single_calls_and_device_counts(torch_dev):
    import torch
    from paper_2412_13755_amd.reco import rans_encode_batch
    rng = np.random.default_rng(11)
    xs = [rng.integers(-5, 30, n).astype(np.int32) for n in (0, 1, 63, 5000, 70_000, 300_001)]
    xs.append(rng.integers(0, 15000, 100_000).astype(np.int32))          # global histogram path
    jobs = []
    for x in xs:
        cap = np.concatenate([x, rng.integers(-9, 9, 77).astype(np.int32)])   # spare entries past n
        t = torch.from_numpy(cap).cuda()
        jobs.append({"symbols": t, "n_device": torch.tensor([len(x)], dtype=torch.int64, device="cuda")})
    rans_encode_batch(jobs, 16, 4096)
    torch.cuda.synchronize()
    for x, j in zip(xs, jobs):
        assert int(j["status"].item()) == 0
        got = j["out"][:int(j["out_size"].item())].cpu().numpy().tobytes()
        assert got == oracle.rans_encode(x, 16, 4096)


def _decode(stream: bytes, cap):
    import torch
    from paper_2412_13755_amd.reco import rans_decode
    buf = torch.from_numpy(np.frombuffer(stream, dtype=np.uint8).copy()).cuda()
    out, n, st = rans_decode(buf, len(stream), cap)
    torch.cuda.synchronize()
    return out.cpu().numpy(), int(n.item()), int(st.item())


def test_decoder_round_trips(torch_dev):
    rng = np.random.default_rng(21)
    cases = [(np.zeros(0, np.int32), 12, 64), (np.array([5], np.int32), 16, 64),
             (rng.integers(-3, 9, 64 * 37 + 13).astype(np.int32), 12, 128),
             (np.full(10_000, -7, np.int32), 12, 1024),
             (rng.integers(0, 16000, 200_000).astype(np.int32), 16, 8192),
             ((rng.geometric(0.05, 1_000_003) - 20).astype(np.int32), 11, 32768),
             ((np.int32(-2**31) + rng.integers(0, 5, 5000)).astype(np.int32), 16, 256)]
    for x, L, B in cases:
        s = oracle.rans_encode(x, L, B)
        got, n, st = _decode(s, len(x) + 7)
        assert st == 0 and n == len(x)
        np.testing.assert_array_equal(got[:n], x)
    x = np.round(np.random.default_rng(9).normal(0.0, 12.0, 1 << 22)).astype(np.int32)
    g, _, _ = _gpu(x, 14, 1 << 15)                      # GPU-coded stream
    got, n, st = _decode(g, len(x))
    assert st == 0 and n == len(x)
    np.testing.assert_array_equal(got, x)


def test_decoder_refuses_bad_streams(torch_dev):
    x = np.random.default_rng(22).integers(0, 40, 50_000).astype(np.int32)
    s = oracle.rans_encode(x, 12, 4096)
    _, n, st = _decode(s, len(x) - 1)
    assert st == -2 and n == len(x)                      # capacity
    bad = bytearray(s); bad[0] ^= 1
    assert _decode(bytes(bad), len(x))[2] == -1          # magic
    assert _decode(s[:-10], len(x))[2] == -1             # truncated words
    assert _decode(s[:100], len(x))[2] == -1             # truncated tables
    bad = bytearray(s); bad[-101] ^= 0x40
    assert _decode(bytes(bad), len(x))[2] == -1          # a flipped word
    # the compressed table: (run, f - 1) varints from byte 40, T bytes (header word 9)
    T = int.from_bytes(s[36:40], "little")
    assert 80 <= T <= 160                                # 40 symbols, f - 1 below 2^14
    bad = bytearray(s); bad[41] = 0x7F
    assert _decode(bytes(bad), len(x))[2] == -1          # frequencies summing past 2^L
    bad = bytearray(s); bad[40:43] = b"\x80\x80\x80"
    assert _decode(bytes(bad), len(x))[2] == -1          # a varint of 4 bytes or more
    bad = bytearray(s); bad[40] = 0x7F
    assert _decode(bytes(bad), len(x))[2] == -1          # a symbol past the range
    bad = bytearray(s); bad[36:40] = (T - 1).to_bytes(4, "little")
    assert _decode(bytes(bad), len(x))[2] == -1          # a table cut inside a pair
    bad = bytearray(s); bad[36:40] = (10**6).to_bytes(4, "little")
    assert _decode(bytes(bad), len(x))[2] == -1          # a table past its bound
    bad = bytearray(s); bad[4] = 1
    assert _decode(bytes(bad), len(x))[2] == -1          # version 1
