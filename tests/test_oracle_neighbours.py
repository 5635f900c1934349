"""Pins of the oracle's neighbour search (CPU only).

The oracle loops over up candidates, then down candidates, and keeps the first
strict minimum.  These tests pin it against an independent formulation: every
(d, h, u) triple is scored at once in numpy float32 (each operation rounded,
no fused multiply-add) and the lexicographic minimum of (q, u, d) is taken
explicitly; plus hand-derived cases (ties, inclusive edges, NaN).
"""
import json
import os

import numpy as np
import pytest

import oracle
from tests.conftest import NB

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "neighbour_cases.json")


def brute_neighbours(off, y, z, n_rows, win_y, win_z, cut_y, cut_z):
    f32 = np.float32
    wy, wz, ty, tz = f32(win_y), f32(win_z), f32(cut_y), f32(cut_z)
    n = int(off[-1])
    up = np.full(n, -1, np.int32)
    dn = np.full(n, -1, np.int32)
    for seg in range(len(off) - 1):
        r = seg % n_rows
        if r == 0 or r == n_rows - 1:
            continue
        H = np.arange(off[seg], off[seg + 1])
        U = np.arange(off[seg + 1], off[seg + 2])
        D = np.arange(off[seg - 1], off[seg])
        if H.size == 0 or U.size == 0 or D.size == 0:
            continue
        yh, zh = y[H][:, None, None], z[H][:, None, None]
        yu, zu = y[U][None, :, None], z[U][None, :, None]
        yd, zd = y[D][None, None, :], z[D][None, None, :]
        with np.errstate(invalid="ignore", over="ignore"):
            ay, az = yu - yh, zu - zh
            by, bz = yh - yd, zh - zd
            dy, dz = ay - by, az - bz
            ok = ((np.abs(ay) <= wy) & (np.abs(az) <= wz) & (np.abs(by) <= wy) & (np.abs(bz) <= wz)
                  & (np.abs(dy) <= ty) & (np.abs(dz) <= tz))
            q = dy * dy + dz * dz
        assert q.dtype == np.float32
        for i, h in enumerate(H):
            iu, idd = np.nonzero(ok[i])
            if iu.size == 0:
                continue
            qq = q[i][iu, idd]
            uu, dd = U[iu], D[idd]
            k = np.lexsort((dd, uu, qq))[0]
            up[h], dn[h] = uu[k], dd[k]
    return up, dn


def _random_rows(rng, n_seg_rows, per_row, spread, quant):
    counts = rng.integers(0, per_row + 1, n_seg_rows)
    off = np.zeros(n_seg_rows + 1, np.int32)
    np.cumsum(counts, out=off[1:])
    n = int(off[-1])
    y = (np.round(rng.uniform(-spread, spread, n) / quant) * quant).astype(np.float32)
    z = (np.round(rng.uniform(-spread, spread, n) / quant) * quant).astype(np.float32)
    return off, y, z


@pytest.mark.parametrize("seed", range(6))
def test_oracle_matches_brute_force_quantised(seed):
    """Coarse 1/8 cm grid: many exact score ties, window and cut edges hit exactly."""
    rng = np.random.default_rng(100 + seed)
    n_rows = 7
    off, y, z = _random_rows(rng, 2 * n_rows, 25, 3.0, 0.125)
    if seed == 5:
        y[::7] = np.nan
        z[3::11] = np.inf
    up, dn = oracle.neighbours(off, y, z, n_rows, **NB)
    bu, bd = brute_neighbours(off, y, z, n_rows, **NB)
    assert (up >= 0).sum() > 10
    np.testing.assert_array_equal(up, bu)
    np.testing.assert_array_equal(dn, bd)


@pytest.mark.parametrize("seed", range(3))
def test_oracle_matches_brute_force_continuous(seed):
    rng = np.random.default_rng(200 + seed)
    n_rows = 6
    off, y, z = _random_rows(rng, 3 * n_rows, 40, 4.0, 1e-6)
    up, dn = oracle.neighbours(off, y, z, n_rows, **NB)
    bu, bd = brute_neighbours(off, y, z, n_rows, **NB)
    np.testing.assert_array_equal(up, bu)
    np.testing.assert_array_equal(dn, bd)


def test_oracle_matches_brute_force_on_generated_rows():
    """A few rows of the single-sector workload, sliced out with their offsets."""
    from tpcsynth import make_config
    fr = make_config(0)
    rows = slice(60, 72)
    off = fr.row_offsets[rows.start:rows.stop + 1]
    a, b = int(off[0]), int(off[-1])
    off = (off - a).astype(np.int32)
    y, z = fr.y[a:b], fr.z[a:b]
    n_rows = rows.stop - rows.start
    up, dn = oracle.neighbours(off, y, z, n_rows, **NB)
    bu, bd = brute_neighbours(off, y, z, n_rows, **NB)
    assert (up >= 0).sum() > 0.5 * len(y)
    np.testing.assert_array_equal(up, bu)
    np.testing.assert_array_equal(dn, bd)


def _golden_cases():
    with open(GOLDEN) as f:
        d = json.load(f)
    return d["params"], d["cases"]


@pytest.mark.parametrize("case", _golden_cases()[1], ids=lambda c: c["name"])
def test_oracle_golden_cases(case):
    params, _ = _golden_cases()
    rows = case["rows"]
    n_rows = len(rows)
    off = np.zeros(n_rows + 1, np.int32)
    np.cumsum([len(r) for r in rows], out=off[1:])
    y = np.array([float(c[0]) for r in rows for c in r], dtype=np.float32)
    z = np.array([float(c[1]) for r in rows for c in r], dtype=np.float32)
    up, dn = oracle.neighbours(off, y, z, n_rows, **params)
    assert up.tolist() == case["up"]
    assert dn.tolist() == case["dn"]
    bu, bd = brute_neighbours(off, y, z, n_rows, **params)
    assert bu.tolist() == case["up"] and bd.tolist() == case["dn"]


def test_oracle_empty_frame():
    off = np.zeros(6, np.int32)                      # one sector of five empty rows
    up, dn = oracle.neighbours(off, np.zeros(0, np.float32), np.zeros(0, np.float32), 5, **NB)
    assert up.size == 0 and dn.size == 0


def test_oracle_refuses_partial_sectors():
    """Row offsets that are not whole sectors would make the search of the
    last interior row read past the offsets: refused."""
    with pytest.raises(ValueError):
        oracle.neighbours(np.zeros(5, np.int32), np.zeros(0, np.float32), np.zeros(0, np.float32), 5, **NB)


def test_order_of_clusters_only_relabels():
    """Permuting clusters within rows permutes the result (ties aside, via ids)."""
    rng = np.random.default_rng(7)
    n_rows = 6
    off, y, z = _random_rows(rng, n_rows, 30, 3.0, 1e-6)   # continuous: no exact ties
    up, dn = oracle.neighbours(off, y, z, n_rows, **NB)
    perm = np.arange(len(y))
    for s in range(n_rows):
        a, b = off[s], off[s + 1]
        perm[a:b] = a + rng.permutation(b - a)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm))
    up2, dn2 = oracle.neighbours(off, y[perm], z[perm], n_rows, **NB)
    # cluster perm[i] is now at i; its partners map back through perm
    np.testing.assert_array_equal(np.where(up2 >= 0, perm[np.maximum(up2, 0)], -1), up[perm])
    np.testing.assert_array_equal(np.where(dn2 >= 0, perm[np.maximum(dn2, 0)], -1), dn[perm])
