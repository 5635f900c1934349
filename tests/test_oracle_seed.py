"""Pins of the oracle's seeding (CPU only).

Independent formulation: the mutual-link graph is split into connected
components with a union-find; each component must be a path over consecutive
rows; claims and seeds are then resolved per component.  Invariants are
checked on the workload-shaped inputs, and an isolated clean track must give
exactly one seed that holds all of its hits.
"""
import numpy as np
import pytest

import oracle
from tests.conftest import NB, MIN_HITS
from tpcsynth import make_config, make_frames, Tracks


def _uf_find(par, i):
    while par[i] != i:
        par[i] = par[par[i]]
        i = par[i]
    return i


def component_seeds(off, up, dn, n_sectors, n_rows, min_hits):
    n = int(off[-1])
    seg = np.repeat(np.arange(len(off) - 1), np.diff(off))
    row = seg % n_rows
    mutual = [(h, int(up[h])) for h in range(n) if up[h] >= 0 and dn[up[h]] == h]
    par = list(range(n))
    deg = np.zeros(n, int)
    for a, b in mutual:
        deg[a] += 1
        deg[b] += 1
        ra, rb = _uf_find(par, a), _uf_find(par, b)
        if ra != rb:
            par[max(ra, rb)] = min(ra, rb)
    comps = {}
    for h in range(n):
        if deg[h]:
            comps.setdefault(_uf_find(par, h), []).append(h)
    chains = []
    for members in comps.values():
        members = sorted(members, key=lambda h: row[h])
        rows = [row[h] for h in members]
        assert rows == list(range(rows[0], rows[0] + len(rows))), "component is not a row path"
        chains.append(members)
    linked = deg > 0
    claims = {}
    for ch in chains:
        m = len(ch)
        if m < min_hits - 2:
            continue
        key = (-m, ch[0])
        for e in (int(dn[ch[0]]), int(up[ch[-1]])):
            if e >= 0 and not linked[e]:
                claims[e] = min(claims.get(e, key), key)
    seeds = []
    for ch in chains:
        m = len(ch)
        key = (-m, ch[0])
        eb, et = int(dn[ch[0]]), int(up[ch[-1]])
        wb = m >= min_hits - 2 and claims.get(eb) == key
        wt = m >= min_hits - 2 and claims.get(et) == key
        s = ([eb] if wb else []) + ch + ([et] if wt else [])
        if len(s) >= min_hits:
            seeds.append(s)
    seeds.sort(key=lambda s: s[0])
    return seeds, seg


def _oracle_seed_lists(sd):
    o = sd["offsets"]
    return [sd["hits"][o[i]:o[i + 1]].tolist() for i in range(len(o) - 1)]


def _check(fr):
    up, dn = oracle.neighbours(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)
    sd = oracle.ca_seed(fr.row_offsets, up, dn, fr.n_sectors, fr.n_rows, MIN_HITS)
    ref, seg = component_seeds(fr.row_offsets, up, dn, fr.n_sectors, fr.n_rows, MIN_HITS)
    got = _oracle_seed_lists(sd)
    assert got == ref
    # invariants
    allh = np.concatenate([np.array(s) for s in got]) if got else np.zeros(0, int)
    assert len(np.unique(allh)) == len(allh), "a cluster is in two seeds"
    firsts = [s[0] for s in got]
    assert firsts == sorted(firsts)
    for i, s in enumerate(got):
        assert len(s) >= MIN_HITS
        sg = seg[np.array(s)]
        assert np.all(np.diff(sg) == 1), "rows of a seed are not consecutive in one sector"
        assert sd["first_row"][i] == sg[0] % fr.n_rows
        assert sd["sector"][i] == (sg[0] // fr.n_rows) % fr.n_sectors
        assert sd["frame"][i] == sg[0] // (fr.n_rows * fr.n_sectors)
    return sd


def test_seeds_single_sector_workload():
    fr = make_config(0)
    sd = _check(fr)
    assert len(sd["offsets"]) - 1 > 20


def test_seeds_full_tpc_scaled():
    fr = make_config(1, scale=0.05)
    sd = _check(fr)
    assert len(sd["offsets"]) - 1 > 100


def test_seeds_batched_frames_scaled():
    fr = make_config(3, scale=0.005)
    sd = _check(fr)
    assert fr.n_frames == 64 and np.unique(sd["frame"]).size > 10


def _one_track(phi0, inv_pt, q, tgl, nmax=1 << 30):
    return Tracks(np.array([q], np.int8), np.array([inv_pt]), np.array([phi0]), np.array([tgl]),
                  np.array([nmax]), np.array([0], np.int32), np.array([0.0]))


@pytest.mark.parametrize("trk", [(0.02, 0.3, 1, 0.2), (-0.05, 2.0, -1, -0.6), (0.0, 1.0, 1, 0.05),
                                 (0.1, 0.5, 1, 0.3, 40)])
def test_isolated_clean_track_gives_one_full_seed(trk):
    fr = make_frames(n_sectors=1, tracks_per_frame=(1,), seed=0, smear=False,
                     tracks=_one_track(*trk))
    n = fr.n_clusters
    assert n >= 5
    up, dn = oracle.neighbours(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)
    sd = oracle.ca_seed(fr.row_offsets, up, dn, fr.n_sectors, fr.n_rows, MIN_HITS)
    assert len(sd["offsets"]) == 2
    assert sorted(sd["hits"].tolist()) == list(range(n))


def test_short_chain_claims_both_ends_or_is_dropped():
    """Five clusters on a line in rows 0..4: core rows 1..3 (m=3) claims both ends -> 5 hits;
    with min_hits 6 the same chain is dropped."""
    off = np.arange(6, dtype=np.int32)
    y = np.zeros(5, np.float32)
    z = np.zeros(5, np.float32)
    up, dn = oracle.neighbours(off, y, z, 5, **NB)
    assert up.tolist() == [-1, 2, 3, 4, -1] and dn.tolist() == [-1, 0, 1, 2, -1]
    sd = oracle.ca_seed(off, up, dn, 1, 5, 5)
    assert sd["hits"].tolist() == [0, 1, 2, 3, 4]
    sd6 = oracle.ca_seed(off, up, dn, 1, 5, 6)
    assert len(sd6["offsets"]) == 1


def test_contested_end_goes_to_longer_chain():
    """Two chains want the same unlinked cluster: the longer core wins it."""
    # hand-built links (not from a neighbour search): rows 0..6, one frame, one sector
    # chain A: ids in rows 1..5 (m=5) bottom claims id 0 (row 0)
    # chain B: rows 1..3 (m=3) whose bottom also points down to id 0
    n_rows = 7
    rows = [[0], [1, 2], [3, 4], [5, 6], [7], [8], [9]]
    off = np.zeros(n_rows + 1, np.int32)
    np.cumsum([len(r) for r in rows], out=off[1:])
    n = int(off[-1])
    up = np.full(n, -1, np.int32)
    dn = np.full(n, -1, np.int32)
    def link(a, b):   # a below b
        up[a] = b
        dn[b] = a
    for a, b in [(1, 3), (3, 5), (5, 7), (7, 8)]:
        link(a, b)
    for a, b in [(2, 4), (4, 6)]:
        link(a, b)
    dn[1] = 0
    dn[2] = 0
    up[8] = 9
    up[6] = 7     # B's top points at a linked cluster: not claimable
    sd = oracle.ca_seed(off, up, dn, 1, n_rows, 5)
    ref, _ = component_seeds(off, up, dn, 1, n_rows, 5)
    assert _oracle_seed_lists(sd) == ref == [[0, 1, 3, 5, 7, 8, 9]]
