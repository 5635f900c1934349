"""Pins of the oracle's rANS coder (the entropy coding of compressed time
frames, Sec. 4.1 of the paper: every integer array coded on its own with
rANS, frequencies counted per frame, several coders interleaved).

The expected values come from outside the coder: closed forms of the coder
state where one step or the binary expansion of the input gives it, the
information content of the symbols under the coded frequencies (the size a
correct coder reaches within a fraction of a percent), and properties of the
frequency scaling.  Round trips through the oracle's decoder cover the rest.
"""
import struct

import numpy as np
import pytest

import oracle

HEAD = 40


def _varints(b):
    """Unsigned LEB128 values of a byte string."""
    out, v, sh = [], 0, 0
    for x in b:
        v |= (x & 0x7F) << sh
        sh += 7
        if not x & 0x80:
            out.append(v)
            v, sh = 0, 0
    assert sh == 0
    return out


def _parse(stream):
    magic, ver, n, lo, R, L, B, nb, T = struct.unpack_from("<IIQiIIIII", stream, 0)
    p = HEAD
    table = bytes(stream[p:p + T])
    v = _varints(table)
    f = np.zeros(R, np.uint32)
    s = -1
    for gap, fm1 in zip(v[0::2], v[1::2]):
        s += gap + 1
        f[s] = fm1 + 1
    p += (T + 3) // 4 * 4
    starts = np.frombuffer(stream, np.uint32, nb + 1, p)
    p += 4 * (nb + 1)
    states = np.frombuffer(stream, np.uint32, 64 * nb, p).reshape(nb, 64)
    p += 256 * nb
    words = np.frombuffer(stream, np.uint16, (len(stream) - p) // 2, p)
    return dict(magic=magic, ver=ver, n=n, lo=lo, R=R, L=L, B=B, nb=nb, f=f, starts=starts,
                states=states, words=words, table=table)


def test_one_symbol_per_coder_is_one_step_from_the_start_state():
    # symbols 0, 1, 1, 2 (counts 1, 2, 1), L = 4: f = floor(c (16 - 3) / 4) + 1 = (4, 7, 4),
    # the missing 1 goes to the most frequent symbol: f = (4, 8, 4), cum = (0, 4, 12);
    # coder k codes only symbol k from x = 2^16: x' = (2^16 div f) 2^4 + (2^16 mod f) + cum
    st = _parse(oracle.rans_encode(np.array([0, 1, 1, 2]), 4, 64))
    assert (st["magic"], st["ver"], st["n"], st["lo"], st["R"], st["L"], st["B"], st["nb"]) == (
        0x534E4152, 2, 4, 0, 3, 4, 64, 1)
    np.testing.assert_array_equal(st["f"], [4, 8, 4])
    # the table: (run of absent symbols, f - 1) per present symbol
    assert st["table"] == bytes([0, 3, 0, 7, 0, 3])
    want = np.full(64, 1 << 16)
    want[:4] = [(65536 // 4) * 16 + 0, (65536 // 8) * 16 + 4, (65536 // 8) * 16 + 4,
                (65536 // 4) * 16 + 12]
    np.testing.assert_array_equal(st["states"][0], want)
    assert st["words"].size == 0 and list(st["starts"]) == [0, 0]


def test_two_equal_symbols_code_to_their_binary_expansion():
    # alphabet {0, 1} with 2^L = 2: f = (1, 1) whatever the counts, so coding a
    # bit b is x <- 2x + b.  Each coder takes 16 bits b_0..b_15 (symbol 64 j + k
    # is bit j of coder k); coded backwards from 2^16, after b_15..b_1 the state
    # is 2^31 + sum_{j>=1} b_j 2^(j-1) >= 2^31, so before b_0 it emits those low
    # 16 bits and keeps 2^15, ending at 2^16 + b_0.
    rng = np.random.default_rng(5)
    bits = rng.integers(0, 2, (16, 64))
    bits[:, 0] = [0, 1] * 8          # both symbols present
    st = _parse(oracle.rans_encode(bits.reshape(-1), 1, 1024))
    np.testing.assert_array_equal(st["states"][0], (1 << 16) + bits[0])
    word = (bits[1:] * (1 << np.arange(15))[:, None]).sum(axis=0)
    # pushed by coders 63 .. 0 in the last coded round, stored last pushed first
    np.testing.assert_array_equal(st["words"], word)


def test_a_certain_source_costs_nothing():
    st = _parse(oracle.rans_encode(np.full(5000, -7), 12, 1024))
    assert st["R"] == 1 and st["lo"] == -7 and list(st["f"]) == [4096]
    assert st["words"].size == 0 and np.all(st["states"] == 1 << 16)


@pytest.mark.parametrize("L,p", [(11, 0.35), (14, 0.08), (16, 0.02)])
def test_size_matches_the_information_content(L, p):
    rng = np.random.default_rng(L)
    x = (rng.geometric(p, 300_000) - 1).astype(np.int32)
    s = oracle.rans_encode(x, L, 8192)
    st = _parse(s)
    M = 1 << L
    f = st["f"].astype(np.float64)
    info = float(np.sum(-np.log2(f[x - st["lo"]] / M)))       # bits under the coded frequencies
    held = 16.0 * st["words"].size + float(np.sum(np.log2(st["states"] / 65536.0)))
    assert abs(held - info) <= 1e-3 * info + 64 * st["nb"], (held, info)
    np.testing.assert_array_equal(oracle.rans_decode(s), x)


def test_frequency_scaling_properties():
    rng = np.random.default_rng(2)
    for R, L in ((1, 1), (7, 3), (300, 12), (5000, 16)):
        c = rng.integers(0, 50, R).astype(np.uint32)
        c[rng.integers(0, R)] += 1
        n = int(c.sum())
        f = oracle.rans_freqs(c, n, L)
        D = int((c > 0).sum())
        if D > (1 << L):
            assert f is None
            continue
        assert int(f.sum()) == 1 << L
        np.testing.assert_array_equal(f > 0, c > 0)
        # a smaller count never gets a larger frequency
        vals = np.unique(c[c > 0])
        hi_f = [int(f[c == v].max()) for v in vals]
        lo_f = [int(f[c == v].min()) for v in vals]
        assert all(hi_f[k] <= lo_f[k + 1] for k in range(len(vals) - 1))
    assert oracle.rans_freqs(np.ones(9, np.uint32), 9, 3) is None        # 9 symbols, M = 8


CASES = ["empty", "one", "ragged", "wide", "extreme", "single_block"]


@pytest.mark.parametrize("case", CASES)
def test_round_trips(case):
    rng = np.random.default_rng(CASES.index(case))
    x = {"empty": np.zeros(0, np.int32), "one": np.array([123456], np.int32),
         "ragged": rng.integers(-3, 9, 64 * 37 + 13).astype(np.int32),
         "wide": rng.integers(0, 16000, 200_000).astype(np.int32),
         "extreme": (np.int32(-2**31) + rng.integers(0, 5, 1000)).astype(np.int32),
         "single_block": rng.integers(0, 2, 63).astype(np.int32)}[case]
    for L, B in ((16, 64), (12, 4096), (16, 65536)):
        if case == "wide" and L < 16:
            continue
        s = oracle.rans_encode(x, L, B)
        np.testing.assert_array_equal(oracle.rans_decode(s), x)


def test_rejects_too_many_symbols_and_corruption():
    with pytest.raises(ValueError):
        oracle.rans_encode(np.arange(300), 8, 64)                       # 300 symbols, M = 256
    with pytest.raises(ValueError):
        oracle.rans_encode(np.array([0, 2**21]), 16, 64)                # range beyond 2^20
    x = np.random.default_rng(1).integers(0, 40, 20000).astype(np.int32)
    s = bytearray(oracle.rans_encode(x, 12, 4096))
    s[-7] ^= 0x5A
    with pytest.raises(ValueError):
        oracle.rans_decode(bytes(s))


def test_the_table_is_compressed():
    # symbols 0 (3 times) and 1000 (once), L = 12: f = floor(c (4096 - 2) / 4) + 1 =
    # (3071, 1024), the shortfall 1 to symbol 0: (3072, 1024); pairs (0, 3071) and
    # (999, 1023): 3071 = 0x0BFF -> FF 17, 999 = 0x3E7 -> E7 07, 1023 -> FF 07
    s = oracle.rans_encode(np.array([0, 0, 1000, 0]), 12, 64)
    st = _parse(s)
    assert st["R"] == 1001
    assert st["table"] == bytes([0x00, 0xFF, 0x17, 0xE7, 0x07, 0xFF, 0x07])
    assert list(np.nonzero(st["f"])[0]) == [0, 1000] and list(st["f"][[0, 1000]]) == [3072, 1024]
    # 7 table bytes (padded to 8) against 4 R = 4004 raw
    assert len(s) == HEAD + 8 + 4 * 2 + 256 + 2 * st["words"].size
    # a dense alphabet: at most 2 + 3 bytes per present symbol, far below 4 bytes per entry
    x = np.random.default_rng(4).integers(0, 16000, 200_000).astype(np.int32)
    st = _parse(oracle.rans_encode(x, 16, 65536))
    D = int((st["f"] > 0).sum())
    assert len(st["table"]) <= 3 * D + 16 and len(st["table"]) < 0.8 * 4 * st["R"]
    np.testing.assert_array_equal(st["f"] > 0, np.bincount(x - x.min(), minlength=st["R"]) > 0)


def test_malformed_tables_are_refused():
    x = np.random.default_rng(3).integers(0, 40, 5000).astype(np.int32)
    s = bytearray(oracle.rans_encode(x, 12, 1024))
    T = struct.unpack_from("<I", s, 36)[0]
    for what, mutate in [("a 4-byte varint", lambda b: b.__setitem__(slice(HEAD, HEAD + 3), b"\x80\x80\x80")),
                         ("a symbol past the range", lambda b: b.__setitem__(HEAD + T - 2, 0x7F)),
                         ("a table length short of a pair", lambda b: struct.pack_into("<I", b, 36, T - 1)),
                         ("a table length past the bound", lambda b: struct.pack_into("<I", b, 36, 10**6)),
                         ("version 1", lambda b: struct.pack_into("<I", b, 4, 1))]:
        b = bytearray(s)
        mutate(b)
        with pytest.raises(ValueError):
            oracle.rans_decode(bytes(b))
