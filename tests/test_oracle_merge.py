"""Pins of the oracle's merging of track segments across sector edges:

* the transfer of a state into a neighbouring sector's frame and on to a
  plane there, and back, returns the state (closed form: rotations and
  helix steps compose); its Jacobian equals finite differences;
* against the generator's truth: a particle's true state at a cluster of
  one sector, transferred to the plane of one of its clusters in the next
  sector, equals its true state there (the generator intersects global
  circles with each sector's planes; nothing is shared with the transfer);
* on a full-TPC event (workload 1 x 0.3): the chi2 of linked segment pairs
  of one particle has the mean of a chi2 with 5 degrees of freedom; every
  link between pure segments joins one particle; at least 88 % of the
  sector-edge junctions (a particle's outermost piece in one sector and
  its innermost in the next) are linked; links are mutual, chi2 <= cut,
  and a single-sector frame has none; the two segments combined at the
  outer one's plane have unit pulls against the truth there, no variance
  above the outer segment's alone and a smaller q/pT variance.
"""
import numpy as np
import pytest

import oracle
from tests.conftest import NB, FIT, MIN_HITS
from tpcsynth import make_config

BZ, MS = FIT["bz"], FIT["max_sin"]
CUT = 30.0


def test_transfer_round_trip_and_jacobian():
    rng = np.random.default_rng(8)
    for _ in range(20):
        p = np.array([rng.uniform(-10, 10), rng.uniform(-50, 50), rng.uniform(-0.3, 0.3),
                      rng.uniform(-1, 1), rng.uniform(-2, 2)])
        x, xt = rng.uniform(90, 200), rng.uniform(90, 240)
        da = np.radians(20.0) * rng.choice([-1, 1])
        st, q, J = oracle.transfer(p, x, da, xt, BZ, MS)
        if st:
            continue
        st2, r, _ = oracle.transfer(q, xt, -da, x, BZ, MS)
        assert st2 == 0
        np.testing.assert_allclose(r, p, rtol=0, atol=1e-10)
        h = 1e-6
        fd = np.zeros((5, 5))
        for j in range(5):
            e = np.zeros(5)
            e[j] = h
            fd[:, j] = (oracle.transfer(p + e, x, da, xt, BZ, MS)[1] - oracle.transfer(p - e, x, da, xt, BZ, MS)[1]) / (2 * h)
        np.testing.assert_allclose(J, fd, rtol=1e-6, atol=1e-7)


def test_transfer_matches_the_generator_truth():
    fr = make_config(1, scale=0.05, keep_truth=True)
    seg = np.repeat(np.arange(fr.row_offsets.size - 1), np.diff(fr.row_offsets))
    sec, row = seg // fr.n_rows % fr.n_sectors, seg % fr.n_rows
    alpha = lambda s: np.radians((s % 18 + 0.5) * 20.0)
    checked = 0
    t = fr.track_of
    for p in np.unique(t[t >= 0])[:400]:
        c = np.nonzero(t == p)[0]
        secs = np.unique(sec[c])
        for sa in secs:
            for sb in secs:
                if sa // 18 != sb // 18 or (sb % 18 - sa % 18) % 18 != 1:
                    continue
                a = c[sec[c] == sa][np.argmax(row[c[sec[c] == sa]])]       # outermost in sa
                b = c[sec[c] == sb][np.argmin(row[c[sec[c] == sb]])]       # innermost in sb
                pa = np.array([fr.y_true[a], fr.z_true[a], fr.s_true[a], fr.t_true[a], fr.w_true[a]])
                pb = np.array([fr.y_true[b], fr.z_true[b], fr.s_true[b], fr.t_true[b], fr.w_true[b]])
                if abs(pa[4]) > 2.0 or abs(pb[4]) > 2.0:
                    continue                    # loopers: legs that come back inwards
                st, q, _ = oracle.transfer(pa, fr.row_x[row[a]], alpha(sb) - alpha(sa), fr.row_x[row[b]], BZ, MS)
                if st:
                    continue
                np.testing.assert_allclose(q, pb, rtol=0, atol=2e-4)
                checked += 1
    assert checked > 50


@pytest.fixture(scope="module")
def event():
    fr = make_config(1, scale=0.3, keep_truth=True)
    up, dn = oracle.neighbours(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)
    sd = oracle.ca_seed(fr.row_offsets, up, dn, fr.n_sectors, fr.n_rows, MIN_HITS)
    o = oracle.fit(sd, fr.y, fr.z, fr.row_x, fr.n_rows, **FIT)
    nxt, prv, chi, mp, mc = oracle.merge(o, sd["frame"], sd["sector"], fr.n_sectors, bz=BZ, max_sin=MS, cut=CUT)
    off = sd["offsets"]
    tid = np.full(len(off) - 1, -1)
    for i in range(len(off) - 1):
        tt = fr.track_of[sd["hits"][off[i]:off[i + 1]]]
        if tt[0] >= 0 and (tt == tt[0]).all():
            tid[i] = tt[0]
    return fr, sd, o, nxt, prv, chi, tid, mp, mc


def test_links_are_mutual_and_within_the_cut(event):
    fr, sd, o, nxt, prv, chi, tid, mp, mc = event
    L = np.nonzero(nxt >= 0)[0]
    assert L.size > 1000
    np.testing.assert_array_equal(prv[nxt[L]], L)
    assert (prv >= 0).sum() == L.size
    assert np.all(chi[L] <= CUT) and np.all(chi[L] > 0) and np.all(chi[nxt < 0] == 0)
    assert np.all(o["status"][L] == 0) and np.all(o["status"][nxt[L]] == 0)
    assert np.all(sd["frame"][L] == sd["frame"][nxt[L]])
    d = (sd["sector"][nxt[L]] % 18 - sd["sector"][L] % 18) % 18
    assert np.all((d == 1) | (d == 17)) and np.all(sd["sector"][L] // 18 == sd["sector"][nxt[L]] // 18)


def test_links_join_one_particle_with_chi2_of_five_dof(event):
    fr, sd, o, nxt, prv, chi, tid, mp, mc = event
    L = np.nonzero(nxt >= 0)[0]
    pure = (tid[L] >= 0) & (tid[nxt[L]] >= 0)
    assert pure.sum() > 1000
    assert np.all(tid[L][pure] == tid[nxt[L]][pure])
    assert abs(chi[L][pure].mean() - 5.0) < 0.4, chi[L][pure].mean()


def test_sector_edge_junctions_are_linked(event):
    fr, sd, o, nxt, prv, chi, tid, mp, mc = event
    ok = (o["status"] == 0) & (tid >= 0)
    r = np.hypot(o["x"], o["par"][:, 0])
    idx = np.nonzero(ok)[0]
    key = sd["frame"][idx].astype(np.int64) * 1000000 + tid[idx]
    junctions = 0
    linked = 0
    for k in np.unique(key):
        segs = idx[key == k]
        for sa in np.unique(sd["sector"][segs]):
            for sb in np.unique(sd["sector"][segs]):
                if sa // 18 != sb // 18 or (sb % 18 - sa % 18) % 18 not in (1, 17):
                    continue
                A = segs[sd["sector"][segs] == sa]
                B = segs[sd["sector"][segs] == sb]
                a, b = A[np.argmax(r[A])], B[np.argmin(r[B])]
                if r[a] < r[b]:
                    junctions += 1
                    linked += nxt[a] == b
    assert junctions > 1000
    assert linked / junctions >= 0.88, linked / junctions


def test_combined_pairs_have_unit_pulls_and_gain_information(event):
    # the fused state of a linked pure pair at the outer segment's innermost
    # plane against the generator's truth at that cluster
    fr, sd, o, nxt, prv, chi, tid, mp, mc = event
    L = np.nonzero(nxt >= 0)[0]
    L = L[(tid[L] >= 0) & (tid[nxt[L]] == tid[L])]
    h = sd["hits"][sd["offsets"][nxt[L]]]
    tru = np.stack([fr.y_true[h], fr.z_true[h], fr.s_true[h], fr.t_true[h], fr.w_true[h]], 1)
    C = oracle.unpack_cov(mc[L])
    var = np.einsum("tii->ti", C)
    pulls = (mp[L] - tru) / np.sqrt(var)
    width = np.quantile(np.abs(pulls), 0.683, axis=0)
    assert len(L) > 1000
    assert np.all(np.abs(width - 1.0) < 0.1), width
    assert np.all(np.abs(np.median(pulls, 0)) < 0.1)
    vb = np.einsum("tii->ti", oracle.unpack_cov(o["cov"][nxt[L]]))
    assert np.all(var <= vb * (1 + 1e-9))
    assert np.median(var[:, 4] / vb[:, 4]) < 0.9                # q/pT gains from the inner segment
    assert not mp[nxt < 0].any() and not mc[nxt < 0].any()


def test_single_sector_has_no_links():
    fr = make_config(0)
    up, dn = oracle.neighbours(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)
    sd = oracle.ca_seed(fr.row_offsets, up, dn, fr.n_sectors, fr.n_rows, MIN_HITS)
    o = oracle.fit(sd, fr.y, fr.z, fr.row_x, fr.n_rows, **FIT)
    nxt, prv, chi, _, _ = oracle.merge(o, sd["frame"], sd["sector"], 1, bz=BZ, max_sin=MS, cut=CUT)
    assert np.all(nxt == -1) and np.all(prv == -1)
