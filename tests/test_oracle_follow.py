"""Pins of the oracle's track following against generator truth.

The oracle's following and duplicate removal are checked against facts that do
not come from its own arithmetic: clusters of one simulated particle, with
gaps planted by removing its clusters from chosen pad rows, must come back as
exactly one track per particle when every gap is at most max_miss rows, and
as separate tracks where a gap is wider; a cluster displaced off the helix by
3 sigma is taken up and one displaced by 8 sigma is not (the gate is a chi2
of the predicted residual with the cluster resolution in it); of two
clusters at the same place the one with the smaller id is taken; a cluster
that two tracks take stays with the longer one and the shorter, owning the
rest of its clusters, is kept too; with a zero gate nothing is taken up and
the refit is the seed fit.
"""
import numpy as np
import pytest

import oracle
from tests.conftest import NB, FIT, MIN_HITS
from tpcsynth import make_frames, drop_clusters, add_clusters
from tpcsynth.generator import Tracks

GATE = 25.0
MAX_MISS = 3


def _reco(fr, gate=GATE, max_miss=MAX_MISS):
    up, dn = oracle.neighbours(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)
    sd = oracle.ca_seed(fr.row_offsets, up, dn, fr.n_sectors, fr.n_rows, MIN_HITS)
    out = oracle.follow(sd, fr.row_offsets, fr.y, fr.z, fr.row_x, fr.n_sectors, fr.n_rows,
                        gate=gate, max_miss=max_miss, **FIT)
    return sd, out


def _row_of(fr):
    seg = np.repeat(np.arange(fr.row_offsets.size - 1), np.diff(fr.row_offsets))
    return seg % fr.n_rows


def _truth_groups(fr, max_miss):
    """Cluster sets of each particle, split where more than max_miss rows in a row are empty."""
    row = _row_of(fr)
    groups = []
    for t in np.unique(fr.track_of[fr.track_of >= 0]):
        ids = np.nonzero(fr.track_of == t)[0]
        ids = ids[np.argsort(row[ids])]
        r = row[ids]
        assert np.all(np.diff(r) > 0), "a particle crosses a row twice"
        cut = np.nonzero(np.diff(r) > max_miss + 1)[0] + 1
        groups.extend(frozenset(g.tolist()) for g in np.split(ids, cut))
    return groups


def _kept_sets(out):
    ok = np.nonzero(out["status"] == 0)[0]
    return [frozenset(out["rows"][i][out["rows"][i] >= 0].tolist()) for i in ok]


def _tracks(n, seed, inv_pt=(0.2, 1.5)):
    rng = np.random.default_rng(seed)
    return Tracks(q=np.where(rng.random(n) < 0.5, -1, 1).astype(np.int8),
                  inv_pt=rng.uniform(*inv_pt, n), phi0=rng.uniform(-0.1, 0.1, n),
                  tgl=np.linspace(-0.9, 0.9, n) + rng.uniform(-0.02, 0.02, n),
                  nmax=np.full(n, 1 << 30), frame=np.zeros(n, np.int32), t0=np.zeros(n))


def _planted_frame():
    fr = make_frames(n_sectors=1, tracks_per_frame=(12,), seed=21, keep_truth=True,
                     tracks=_tracks(12, 21))
    row = _row_of(fr)
    t = fr.track_of
    p = int(t[row == fr.n_rows - 1].min())                 # a particle crossing every row
    drop = np.isin(row, (40, 41, 42, 90)) & (t >= 0)      # gaps of max_miss rows and of 1 row
    drop |= (t == p) & (row >= 110) & (row <= 113)        # one of max_miss + 1 rows in particle p
    return drop_clusters(fr, ~drop), p


def test_planted_gaps_merge_into_one_track_per_particle():
    fr, p = _planted_frame()
    sd, out = _reco(fr)
    T = len(sd["offsets"]) - 1
    n_part = np.unique(fr.track_of).size
    assert T >= 2 * n_part, "the gaps must break the chains into several seeds"
    kept = _kept_sets(out)
    groups = _truth_groups(fr, MAX_MISS)
    big = [g for g in groups if len(g) >= 10]
    # every kept track is exactly one truth group ...
    for k in kept:
        assert k in groups, sorted(set(fr.track_of[list(k)]))
    # ... and every sizeable group is found exactly once
    for g in big:
        assert kept.count(g) == 1
    # particle p ends as two tracks, split at its wider gap
    gp = [g for g in groups if fr.track_of[next(iter(g))] == p]
    assert len(gp) == 2 and all(g in kept for g in gp)
    # the other pieces were merged away
    assert (out["status"] == 4).sum() == T - len(kept) - np.isin(out["status"], (1, 2, 3)).sum()


def _one_track_frame(shift_sigma):
    tr = Tracks(q=np.array([1], np.int8), inv_pt=np.array([1.0]), phi0=np.array([0.02]),
                tgl=np.array([0.3]), nmax=np.array([1 << 30]), frame=np.array([0], np.int32),
                t0=np.zeros(1))
    fr = make_frames(n_sectors=1, tracks_per_frame=(1,), seed=5, keep_truth=True, tracks=tr)
    row = _row_of(fr)
    fr = drop_clusters(fr, ~np.isin(row, (59, 61)))         # row 60 is left without links
    row = _row_of(fr)
    (c60,) = np.nonzero(row == 60)[0]
    y = fr.y.copy()
    z = fr.z.copy()
    y[c60] = np.float32(fr.y_true[c60] + shift_sigma * fr.sigma_y)
    z[c60] = np.float32(fr.z_true[c60])
    fr.y, fr.z = y, z
    return fr, int(c60)


@pytest.mark.parametrize("shift,taken", [(3.0, True), (8.0, False)])
def test_gate_takes_a_displaced_cluster_only_within_the_chi2_gate(shift, taken):
    fr, c60 = _one_track_frame(shift)
    sd, out = _reco(fr)
    assert len(sd["offsets"]) - 1 == 2, "the empty rows 59 and 61 split the chain in two seeds"
    seed_hits = set(sd["hits"].tolist())
    assert c60 not in seed_hits
    kept = _kept_sets(out)
    assert len(kept) == 1
    others = set(range(fr.n_clusters)) - {c60}
    assert kept[0] == frozenset(others | ({c60} if taken else set()))


def test_equal_chi2_goes_to_the_smaller_id():
    fr, c60 = _one_track_frame(0.0)
    fr = add_clusters(fr, [0], [0], [60], [fr.y[c60]], [fr.z[c60]])   # an exact copy, next id
    sd, out = _reco(fr)
    kept = _kept_sets(out)
    assert len(kept) == 1
    assert c60 in kept[0] and c60 + 1 not in kept[0]


def test_a_shared_cluster_stays_with_the_longer_track_and_both_are_kept():
    # particle A crosses every row; B is a straight line through A's cluster
    # of row 120 that has no cluster of its own there
    tr = Tracks(q=np.array([1], np.int8), inv_pt=np.array([0.5]), phi0=np.array([0.0]),
                tgl=np.array([0.2]), nmax=np.array([1 << 30]), frame=np.array([0], np.int32),
                t0=np.zeros(1))
    fr = make_frames(n_sectors=1, tracks_per_frame=(1,), seed=9, keep_truth=True, tracks=tr)
    row = _row_of(fr)
    (a120,) = np.nonzero(row == 120)[0]
    rows_b = np.array([r for r in range(100, fr.n_rows) if r != 120])
    dx = fr.row_x[rows_b].astype(np.float64) - float(fr.row_x[120])
    yb = fr.y[a120] + 0.45 * dx
    zb = fr.z[a120] + 0.35 * dx
    n = rows_b.size
    fr = add_clusters(fr, np.zeros(n, int), np.zeros(n, int), rows_b, yb, zb, np.ones(n, np.int32))
    row = _row_of(fr)
    (a120,) = np.nonzero((row == 120) & (fr.track_of == 0))[0]
    sd, out = _reco(fr)
    kept = _kept_sets(out)
    set_a = frozenset(np.nonzero(fr.track_of == 0)[0].tolist())
    set_b = frozenset(np.nonzero(fr.track_of == 1)[0].tolist()) | {int(a120)}
    assert sorted(kept, key=len) == [set_b, set_a]


def test_zero_gate_takes_nothing_and_refits_the_seed():
    fr = make_frames(n_sectors=1, tracks_per_frame=(60,), seed=3, phi_range=(-0.1, 0.1), noise_frac=0.05)
    sd, out = _reco(fr, gate=0.0, max_miss=0)
    ref = oracle.fit(sd, fr.y, fr.z, fr.row_x, fr.n_rows, **FIT)
    T = len(sd["offsets"]) - 1
    for i in range(T):
        r = out["rows"][i]
        a, b = sd["offsets"][i], sd["offsets"][i + 1]
        np.testing.assert_array_equal(r[r >= 0], sd["hits"][a:b])
    np.testing.assert_array_equal(out["status"], ref["status"])     # disjoint seeds: no duplicates
    ok = ref["status"] == 0
    np.testing.assert_array_equal(out["par"][ok], ref["par"][ok])
    np.testing.assert_array_equal(out["cov"][ok], ref["cov"][ok])
    np.testing.assert_array_equal(out["chi2"][ok], ref["chi2"][ok])


def test_kept_tracks_are_distinct_and_hits_ascend():
    fr = make_frames(n_sectors=1, tracks_per_frame=(150,), seed=8, phi_range=(-0.17, 0.17),
                     noise_frac=0.05, hit_eff=0.95)
    sd, out = _reco(fr)
    kept = _kept_sets(out)
    assert len(kept) == len(set(kept))
    row = _row_of(fr)
    ok = out["status"] == 0
    for i in np.nonzero(ok)[0]:
        r = out["rows"][i]
        on = np.nonzero(r >= 0)[0]
        assert np.all(row[r[on]] == on), "rows[i][r] must be a cluster of pad row r"
        assert np.all(np.diff(on) <= MAX_MISS + 1)
        assert out["ndf"][i] == 2 * on.size - 5
    seg = np.repeat(np.arange(fr.row_offsets.size - 1), np.diff(fr.row_offsets))
    for i in np.nonzero(ok)[0]:
        c = out["rows"][i][out["rows"][i] >= 0]
        assert np.unique(seg[c] // fr.n_rows).size == 1, "a track stays in its (frame, sector)"


def test_following_seeds_that_skip_rows():
    # seeds from links across a missing row: every seed hit stays at its own
    # row, and following reaches the completeness of adjacent-row seeds from
    # fewer seeds (the inefficiency no longer splits them)
    from tpcsynth import make_config
    fr = make_config(1, scale=0.1, hit_eff=0.9)
    t = fr.track_of
    sec = np.repeat(np.arange(fr.row_offsets.size - 1), np.diff(fr.row_offsets)) // fr.n_rows
    row = np.repeat(np.arange(fr.row_offsets.size - 1), np.diff(fr.row_offsets)) % fr.n_rows
    piece = t.astype(np.int64) * 4096 + sec
    pk, pn = np.unique(piece[t >= 0], return_counts=True)
    res = {}
    for name, nbf in (("adjacent", oracle.neighbours), ("skip", oracle.neighbours_skip)):
        up, dn = nbf(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)
        sd = oracle.ca_seed(fr.row_offsets, up, dn, fr.n_sectors, fr.n_rows, MIN_HITS)
        fo = oracle.follow(sd, fr.row_offsets, fr.y, fr.z, fr.row_x, fr.n_sectors, fr.n_rows,
                           gate=25.0, max_miss=3, **FIT)
        assert (fo["status"] == 1).mean() < 0.01          # start failures only
        for i in np.flatnonzero(fo["status"] != 1):
            h = sd["hits"][sd["offsets"][i]:sd["offsets"][i + 1]]
            np.testing.assert_array_equal(fo["rows"][i][row[h]], h)
        best = {}
        for r in fo["rows"][fo["status"] == 0]:
            c = r[r >= 0]
            c = c[t[c] >= 0]
            u, n = np.unique(piece[c], return_counts=True)
            for a, b in zip(u.tolist(), n.tolist()):
                best[a] = max(best.get(a, 0), b)
        big = pn >= 20
        res[name] = (len(sd["offsets"]) - 1,
                     np.mean([best.get(a, 0) >= 0.8 * b for a, b in zip(pk[big].tolist(), pn[big].tolist())]))
    assert res["skip"][0] < 0.5 * res["adjacent"][0]
    assert res["skip"][1] > 0.93 and abs(res["skip"][1] - res["adjacent"][1]) < 0.01


def test_following_refuses_malformed_seeds():
    from tpcsynth import make_config
    fr = make_config(0)
    up, dn = oracle.neighbours(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)
    sd = oracle.ca_seed(fr.row_offsets, up, dn, 1, fr.n_rows, MIN_HITS)
    o = sd["offsets"]
    h = sd["hits"][o[0]:o[1]].copy()
    bad = np.concatenate([h[:2], h[3:4], h[2:3], h[4:]])          # two rows swapped
    s2 = dict(offsets=np.array([0, len(h), 2 * len(h)], np.int32), hits=np.concatenate([h, bad]).astype(np.int32),
              frame=np.zeros(2, np.int32), sector=np.zeros(2, np.int32), first_row=np.full(2, sd["first_row"][0], np.int32))
    fo = oracle.follow(s2, fr.row_offsets, fr.y, fr.z, fr.row_x, 1, fr.n_rows, gate=25.0, max_miss=3, **FIT)
    assert fo["status"][0] == 0 and fo["status"][1] == 1
    assert (fo["rows"][1] == -1).all()
    s3 = dict(s2, frame=np.ones(2, np.int32))
    assert (oracle.follow(s3, fr.row_offsets, fr.y, fr.z, fr.row_x, 1, fr.n_rows, gate=25.0, max_miss=3,
                          **FIT)["status"] == 1).all()
