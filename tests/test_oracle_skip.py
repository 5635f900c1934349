"""Pins of the oracle's neighbour search across a missing pad row.

The definition (partners one or two rows away, the triplet spanning the
fewest rows first, then the normalised second difference q, then ids) is
pinned by
* exhaustive enumeration on tiny frames, written here as a sort of every
  candidate triplet by (rows spanned, q, u, d) in numpy single precision;
* closed forms: noise-free straight lines across a missing row give D = 0
  and link at any slope inside the window; an exact parabola gives the same
  D = 2k for every (a, b), so a cut just above 2k links it across the gap;
* the adjacent-row result is kept wherever it exists;
* physics: a dead pad row no longer splits the seeds, and on a frame with
  10% pad-row inefficiency the seeds are several times longer while the new
  links join clusters of one track.
"""
import numpy as np
import pytest

import oracle
from tests.conftest import NB, MIN_HITS
from tpcsynth import make_config, drop_clusters

f32 = np.float32


def brute(off, y, z, R, win_y, win_z, cut_y, cut_z):
    n = int(off[-1])
    up = np.full(n, -1, np.int32)
    dn = np.full(n, -1, np.int32)
    y = y.astype(np.float32)
    z = z.astype(np.float32)
    wy, wz, cy, cz = f32(win_y), f32(win_z), f32(cut_y), f32(cut_z)
    with np.errstate(all="ignore"):
        for seg in range(off.size - 1):
            r = seg % R
            if r == 0 or r == R - 1:
                continue
            for h in range(off[seg], off[seg + 1]):
                cands = []
                for a in (1, 2):
                    for b in (1, 2):
                        if r - a < 0 or r + b > R - 1:
                            continue
                        fa, fb = f32(a), f32(b)
                        g = f32(2) / f32(a + b)
                        for u in range(off[seg + b], off[seg + b + 1]):
                            Ay, Az = y[u] - y[h], z[u] - z[h]
                            for d in range(off[seg - a], off[seg - a + 1]):
                                By, Bz = y[h] - y[d], z[h] - z[d]
                                if not (abs(Ay) <= fb * wy and abs(Az) <= fb * wz and
                                        abs(By) <= fa * wy and abs(Bz) <= fa * wz):
                                    continue
                                Dy = g * (Ay / fb - By / fa)
                                Dz = g * (Az / fb - Bz / fa)
                                if not (abs(Dy) <= cy and abs(Dz) <= cz):
                                    continue
                                cands.append((a + b, f32(Dy * Dy) + f32(Dz * Dz), u, d))
                if cands:
                    best = min(cands)
                    up[h], dn[h] = best[2], best[3]
    return up, dn


def tiny_frame(rng, R):
    """A few lines on a 0.25 grid (each cluster kept with probability 0.7,
    so rows go missing) plus random clusters; coarse values make ties."""
    ys, zs, rows = [], [], []
    for _ in range(int(rng.integers(1, 4))):
        y0, z0 = rng.integers(-4, 5, 2) * 0.25
        my, mz = rng.integers(-2, 3, 2) * 0.25
        for r in range(R):
            if rng.random() < 0.7:
                rows.append(r)
                ys.append(y0 + my * r + rng.integers(-1, 2) * 0.25)
                zs.append(z0 + mz * r + rng.integers(-1, 2) * 0.25)
    for _ in range(int(rng.integers(0, 2 * R))):
        rows.append(int(rng.integers(0, R)))
        ys.append(rng.integers(-8, 9) * 0.25)
        zs.append(rng.integers(-8, 9) * 0.25)
    rows = np.array(rows, np.int64)
    order = np.argsort(rows, kind="stable")
    off = np.zeros(R + 1, np.int32)
    off[1:] = np.cumsum(np.bincount(rows, minlength=R))
    y = np.array(ys, np.float32)[order]
    z = np.array(zs, np.float32)[order]
    if y.size:
        y[rng.random(y.size) < 0.03] = np.nan
    return off, y, z


@pytest.mark.parametrize("seed", range(6))
def test_tiny_frames_match_exhaustive_enumeration(seed):
    rng = np.random.default_rng(100 + seed)
    prm = dict(win_y=1.0, win_z=1.25, cut_y=0.3, cut_z=0.4)
    spans = set()
    nlinks = 0
    for _ in range(120):
        R = int(rng.integers(3, 9))
        off, y, z = tiny_frame(rng, R)
        up, dn = oracle.neighbours_skip(off, y, z, R, **prm)
        bu, bd = brute(off, y, z, R, **prm)
        np.testing.assert_array_equal(up, bu)
        np.testing.assert_array_equal(dn, bd)
        nlinks += int((up >= 0).sum())
        seg = np.repeat(np.arange(R), np.diff(off))
        k = np.flatnonzero(up >= 0)
        spans |= set(zip((seg[k] - seg[dn[k]]).tolist(), (seg[up[k]] - seg[k]).tolist()))
    assert nlinks > 300
    assert spans == {(1, 1), (1, 2), (2, 1), (2, 2)}


def _line_frame(R, lines, drop_rows):
    """One sector, clusters of the given lines y = y0 + m r, z = z0 + k r
    (noise-free), none in drop_rows; returns (off, y, z, line_of)."""
    rows, ys, zs, lid = [], [], [], []
    for i, (y0, m, z0, k) in enumerate(lines):
        for r in range(R):
            if r in drop_rows:
                continue
            rows.append(r)
            ys.append(y0 + m * r)
            zs.append(z0 + k * r)
            lid.append(i)
    rows = np.array(rows)
    order = np.argsort(rows, kind="stable")
    off = np.zeros(R + 1, np.int32)
    off[1:] = np.cumsum(np.bincount(rows, minlength=R))
    return (off, np.array(ys, np.float32)[order], np.array(zs, np.float32)[order],
            np.array(lid)[order], rows[order])


def test_straight_lines_link_across_a_missing_row():
    # slopes up to ~0.9 of the window per row: a wrongly normalised second
    # difference (e.g. A/a - B/b) would be of the order of the slope, far
    # above the cuts
    R = 24
    lines = [(-40.0 + 8.0 * i, 0.5 * (i - 5) * 0.4, 100.0 + 3.0 * i, 0.2 * (4 - i)) for i in range(11)]
    off, y, z, lid, rows = _line_frame(R, lines, drop_rows={12})
    up, dn = oracle.neighbours_skip(off, y, z, R, **NB)
    for i in range(len(lines)):
        at = {int(rows[j]): j for j in np.flatnonzero(lid == i)}
        assert up[at[11]] == at[13] and dn[at[11]] == at[10], i
        assert dn[at[13]] == at[11] and up[at[13]] == at[14], i
    sd = oracle.ca_seed(off, up, dn, 1, R, MIN_HITS)
    assert np.diff(sd["offsets"]).tolist() == [R - 1] * len(lines)
    # the adjacent-row search cannot cross the gap
    a_up, a_dn = oracle.neighbours(off, y, z, R, **NB)
    assert (a_up[rows == 11] < 0).all() and (a_dn[rows == 13] < 0).all()


def test_two_missing_rows_are_not_crossed():
    R = 20
    off, y, z, lid, rows = _line_frame(R, [(0.0, 0.3, 50.0, 0.1)], drop_rows={9, 10})
    up, dn = oracle.neighbours_skip(off, y, z, R, **NB)
    assert up[rows == 8][0] == -1 and dn[rows == 11][0] == -1
    assert (up[(rows > 0) & (rows < 7)] >= 0).all()


def test_parabola_has_one_second_difference_for_every_span():
    # y = k r^2 with k a power of two: every value and difference is exact;
    # the normalised D is 2k for (1,1), (1,2), (2,1) and (2,2) alike, so a
    # cut of 2.25 k links the whole track across the gap (an unscaled or
    # otherwise normalised D would be at least 3k there)
    k = 2.0 ** -4
    R = 20
    prm = dict(win_y=30.0, win_z=1.0, cut_y=2.25 * k, cut_z=0.1)
    for gap in (5, 10, 14):
        rows = np.array([r for r in range(R) if r != gap])
        y = (k * rows.astype(np.float64) ** 2).astype(np.float32)
        z = np.full(rows.size, 7.0, np.float32)
        off = np.zeros(R + 1, np.int32)
        off[1:] = np.cumsum(np.bincount(rows, minlength=R))
        up, dn = oracle.neighbours_skip(off, y, z, R, **prm)
        j = {int(r): i for i, r in enumerate(rows)}
        assert up[j[gap - 1]] == j[gap + 1] and dn[j[gap + 1]] == j[gap - 1], gap
        sd = oracle.ca_seed(off, up, dn, 1, R, MIN_HITS)
        assert np.diff(sd["offsets"]).tolist() == [R - 1], gap
        # just below 2k nothing links at all
        up2, _ = oracle.neighbours_skip(off, y, z, R, **{**prm, "cut_y": 1.75 * k})
        assert (up2 < 0).all()


@pytest.fixture(scope="module")
def inefficient():
    fr = make_config(1, scale=0.1, hit_eff=0.9)
    a = oracle.neighbours(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)
    s = oracle.neighbours_skip(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)
    return fr, a, s


def test_adjacent_result_is_kept(inefficient):
    fr, (a_up, a_dn), (s_up, s_dn) = inefficient
    m = a_up >= 0
    assert m.sum() > 50000
    np.testing.assert_array_equal(s_up[m], a_up[m])
    np.testing.assert_array_equal(s_dn[m], a_dn[m])
    seg = np.repeat(np.arange(fr.row_offsets.size - 1), np.diff(fr.row_offsets))
    row, sec = seg % fr.n_rows, seg // fr.n_rows
    new = ~m & (s_up >= 0)
    assert (s_dn[new] >= 0).all()
    du = row[s_up[new]] - row[new]
    dd = row[new] - row[s_dn[new]]
    assert set(zip(dd.tolist(), du.tolist())) == {(1, 2), (2, 1), (2, 2)}
    assert (sec[s_up[new]] == sec[new]).all() and (sec[s_dn[new]] == sec[new]).all()


def test_new_links_join_one_track_and_lengthen_seeds(inefficient):
    fr, (a_up, a_dn), (s_up, s_dn) = inefficient
    t = fr.track_of
    new = (a_up < 0) & (s_up >= 0)
    assert new.sum() > 10000
    same = (t[new] >= 0) & (t[s_up[new]] == t[new]) & (t[s_dn[new]] == t[new])
    assert same.mean() > 0.95
    la = np.diff(oracle.ca_seed(fr.row_offsets, a_up, a_dn, fr.n_sectors, fr.n_rows, MIN_HITS)["offsets"])
    ls = np.diff(oracle.ca_seed(fr.row_offsets, s_up, s_dn, fr.n_sectors, fr.n_rows, MIN_HITS)["offsets"])
    assert ls.mean() > 2.5 * la.mean()
    assert ls.sum() > la.sum()


def test_dead_row_does_not_split_seeds():
    fr0 = make_config(1, scale=0.05)
    seg = np.repeat(np.arange(fr0.row_offsets.size - 1), np.diff(fr0.row_offsets))
    dead = 70
    fr = drop_clusters(fr0, seg % fr0.n_rows != dead)
    seg = np.repeat(np.arange(fr.row_offsets.size - 1), np.diff(fr.row_offsets))
    row = seg % fr.n_rows
    # track segments with clusters on rows 68, 69, 71, 72 of one sector
    t = fr.track_of
    keys = {}
    for rr in (68, 69, 71, 72):
        sel = (row == rr) & (t >= 0)
        keys[rr] = set(zip(t[sel].tolist(), (seg[sel] // fr.n_rows).tolist()))
    crossing = keys[68] & keys[69] & keys[71] & keys[72]
    assert len(crossing) > 200

    def bridging(up, dn):
        sd = oracle.ca_seed(fr.row_offsets, up, dn, fr.n_sectors, fr.n_rows, MIN_HITS)
        c = 0
        for i in range(len(sd["offsets"]) - 1):
            r = row[sd["hits"][sd["offsets"][i]:sd["offsets"][i + 1]]]
            c += bool((r < dead).any() and (r > dead).any())
        return c

    assert bridging(*oracle.neighbours(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)) == 0
    assert bridging(*oracle.neighbours_skip(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)) > 0.8 * len(crossing)
