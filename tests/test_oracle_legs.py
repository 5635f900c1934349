"""Pins of the oracle's pairing of the legs of loopers (a particle whose
circle stays inside the TPC turns back; its returning leg is fitted as a
track running outwards along the same circle in the other sense):

* against the generator's truth: the true states of a looper's outgoing and
  returning legs (the generator reports the returning leg in the outward
  orientation, as the fit sees it) give the same circle centre in global
  coordinates, and curvatures and tan(lambda) of opposite signs;
* the circle's Jacobian equals finite differences;
* on a full-TPC event (workload 1 x 0.3): the pairs are mutual and within
  the cut; at least 95 % of the pairs of pure segments join one particle,
  whose legs run in opposite senses (opposite fitted q/pT); one sector has
  no pairs.
"""
import numpy as np
import pytest

import oracle
from tests.conftest import NB, FIT, MIN_HITS
from tpcsynth import make_config

BZ = FIT["bz"]
CUT = 30.0
alpha = lambda s: np.radians((s % 18 + 0.5) * 20.0)


def test_both_legs_of_a_looper_share_their_circle():
    fr = make_config(1, scale=0.3, keep_truth=True)
    seg = np.repeat(np.arange(fr.row_offsets.size - 1), np.diff(fr.row_offsets))
    sec, row = seg // fr.n_rows % fr.n_sectors, seg % fr.n_rows
    t = fr.track_of
    checked = 0
    for p in np.unique(t[t >= 0]):
        c = np.nonzero(t == p)[0]
        wt = fr.w_true[c]
        if (wt > 0).all() or (wt < 0).all():
            continue
        m = []
        for h in (c[wt > 0][0], c[wt < 0][0]):
            st, mh, _ = oracle.leg_circle(np.array([fr.y_true[h], fr.z_true[h], fr.s_true[h], fr.t_true[h],
                                                    fr.w_true[h]]), fr.row_x[row[h]], alpha(sec[h]), BZ)
            m.append(mh if st == 0 else None)
        if m[0] is None or m[1] is None:
            continue
        np.testing.assert_allclose(m[0], m[1] * np.array([1, 1, -1, -1]), rtol=0, atol=1e-9)
        checked += 1
    assert checked > 100


def test_circle_jacobian():
    rng = np.random.default_rng(4)
    for _ in range(20):
        p = np.array([rng.uniform(-20, 20), rng.uniform(-50, 50), rng.uniform(-0.8, 0.8), rng.uniform(-1, 1),
                      rng.choice([-1, 1]) * rng.uniform(3, 8)])
        x, a = rng.uniform(90, 240), alpha(int(rng.integers(0, 18)))
        st, m, J = oracle.leg_circle(p, x, a, BZ)
        assert st == 0
        h = 1e-6
        fd = np.zeros((4, 5))
        for j in range(5):
            e = np.zeros(5)
            e[j] = h
            fd[:, j] = (oracle.leg_circle(p + e, x, a, BZ)[1] - oracle.leg_circle(p - e, x, a, BZ)[1]) / (2 * h)
        np.testing.assert_allclose(J, fd, rtol=1e-6, atol=1e-6)
    # a circle larger than the TPC is no looper
    assert oracle.leg_circle(np.array([0, 0, 0.1, 0.2, 1.0]), 100.0, 0.3, BZ)[0] == 1


def test_legs_pair_one_particle():
    fr = make_config(1, scale=0.3, keep_truth=True)
    up, dn = oracle.neighbours(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)
    sd = oracle.ca_seed(fr.row_offsets, up, dn, fr.n_sectors, fr.n_rows, MIN_HITS)
    o = oracle.fit(sd, fr.y, fr.z, fr.row_x, fr.n_rows, **FIT)
    leg, chi = oracle.legs(o, sd["frame"], sd["sector"], fr.n_sectors, bz=BZ, cut=CUT)
    L = np.nonzero(leg >= 0)[0]
    assert L.size > 200
    np.testing.assert_array_equal(leg[leg[L]], L)
    assert np.all(chi[L] <= CUT) and np.all(chi[L] > 0) and np.all(chi[leg < 0] == 0)
    assert np.all(sd["frame"][L] == sd["frame"][leg[L]])
    off = sd["offsets"]
    tid = np.full(len(off) - 1, -1)
    for i in range(len(off) - 1):
        tt = fr.track_of[sd["hits"][off[i]:off[i + 1]]]
        if tt[0] >= 0 and (tt == tt[0]).all():
            tid[i] = tt[0]
    pure = (tid[L] >= 0) & (tid[leg[L]] >= 0)
    same = tid[L][pure] == tid[leg[L]][pure]
    assert same.mean() >= 0.95, same.mean()
    w = o["par"][:, 4]
    assert np.all(np.sign(w[L][pure][same]) != np.sign(w[leg[L]][pure][same]))


def test_single_sector_has_no_legs():
    fr = make_config(0)
    up, dn = oracle.neighbours(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)
    sd = oracle.ca_seed(fr.row_offsets, up, dn, fr.n_sectors, fr.n_rows, MIN_HITS)
    o = oracle.fit(sd, fr.y, fr.z, fr.row_x, fr.n_rows, **FIT)
    leg, chi = oracle.legs(o, sd["frame"], sd["sector"], 1, bz=BZ, cut=CUT)
    assert np.all(leg == -1)
