"""Pins of the oracle's assembly of tracks from linked segments and their
refit over all hits:

* a chain of one segment is that segment's seed fit, bit for bit;
* noise-free helices crossing sector edges, cut into per-sector segments
  linked by the generator's truth: the refit of each chain returns the true
  state at its innermost hit to round-off, with chi2 ~ 0 (the rotation into
  each sector's frame and the transfer across the boundaries are exact);
* with Gaussian smearing the refits' pulls against the truth have zero mean
  and unit width, chi2/ndf averages 1 and the chi2 probabilities are flat
  (the covariance is carried through the boundaries correctly);
* a two-segment chain refitted over its hits agrees with the two segment
  fits combined at the outer segment's plane (the linearised joint fit):
  the same variances, states within a fraction of a standard deviation;
* a refit with a map equals the refit of clusters corrected beforehand;
* the track ids are the connected components of the link graph (breadth-
  first search), named by their smallest segment;
* the joint circle of two looper legs that are single segments has the
  chi2 of the legs' pairing; the gain form of the fusion equals the
  information form (S_i^-1 + S_j^-1)^-1 (S_i^-1 m_i + S_j^-1 m_j) and its
  chi2 the weighted least-squares minimum; on particles of the full event
  the joint circle lies much closer to the true circle than either leg's.
"""
from collections import deque

import numpy as np
import pytest

import oracle
from tests.conftest import NB, FIT, MIN_HITS
from tests.test_oracle_fit import truth_runs, FLOOR
from tpcsynth import make_config, make_frames

BZ, MS = FIT["bz"], FIT["max_sin"]
CUT = 30.0
alpha = lambda s: np.radians((np.asarray(s) % 18 + 0.5) * 20.0)
D = np.diag([1.0, 1.0, -1.0, -1.0])


def truth_links(fr, sd):
    """next/prev between a particle's consecutive truth segments in
    neighbouring sectors of one side (particles that do not turn back)."""
    T = len(sd["offsets"]) - 1
    first = sd["hits"][sd["offsets"][:-1]]
    p = fr.track_of[first]
    r = np.hypot(fr.row_x[sd["first_row"]], fr.y_true[first])
    nxt = np.full(T, -1, np.int32)
    prv = np.full(T, -1, np.int32)
    for q in np.unique(p):
        idx = np.nonzero(p == q)[0]
        c = fr.track_of == q
        if not ((fr.w_true[c] > 0).all() or (fr.w_true[c] < 0).all()):
            continue
        idx = idx[np.argsort(r[idx])]
        for a, b in zip(idx[:-1], idx[1:]):
            sa, sb = sd["sector"][a], sd["sector"][b]
            if sa // 18 == sb // 18 and (sb % 18 - sa % 18) % 18 in (1, 17):
                nxt[a], prv[b] = b, a
    return nxt, prv


def truth_state(fr, h):
    return np.stack([fr.y_true[h], fr.z_true[h], fr.s_true[h], fr.t_true[h], fr.w_true[h]], -1)


def multi_heads(r, nxt):
    return np.nonzero((r["status"] != 5) & (nxt >= 0))[0]


@pytest.fixture(scope="module")
def truth_chains():
    out = {}
    for smear in (False, True):
        fr = make_frames(n_sectors=36, tracks_per_frame=(3000,), seed=21, smear=smear, keep_truth=True)
        sd = truth_runs(fr, 6)
        y, z = (fr.y, fr.z) if smear else (fr.y_true, fr.z_true)
        o = oracle.fit(sd, y, z, fr.row_x, fr.n_rows, **FIT)
        nxt, prv = truth_links(fr, sd)
        r = oracle.refit(sd, o, nxt, prv, None, y, z, fr.row_x, fr.n_rows, fr.n_sectors, **FIT)
        out[smear] = (fr, sd, o, nxt, prv, r, y, z)
    return out


@pytest.fixture(scope="module")
def event():
    fr = make_config(1, scale=0.3, keep_truth=True)
    up, dn = oracle.neighbours(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)
    sd = oracle.ca_seed(fr.row_offsets, up, dn, fr.n_sectors, fr.n_rows, MIN_HITS)
    o = oracle.fit(sd, fr.y, fr.z, fr.row_x, fr.n_rows, **FIT)
    nxt, prv, _, _, _ = oracle.merge(o, sd["frame"], sd["sector"], fr.n_sectors, bz=BZ, max_sin=MS, cut=CUT)
    leg, lchi = oracle.legs(o, sd["frame"], sd["sector"], fr.n_sectors, bz=BZ, cut=CUT)
    r = oracle.refit(sd, o, nxt, prv, leg, fr.y, fr.z, fr.row_x, fr.n_rows, fr.n_sectors, **FIT)
    return fr, sd, o, nxt, prv, leg, lchi, r


def test_chain_of_one_segment_is_its_seed_fit(event):
    fr, sd, o, nxt, prv, leg, lchi, r = event
    single = (o["status"] == 0) & (prv < 0) & (nxt < 0)
    assert single.sum() > 1000
    for k in ("x", "par", "cov", "chi2", "ndf", "status"):
        np.testing.assert_array_equal(r[k][single], o[k][single], err_msg=k)


def test_heads_and_members(event):
    fr, sd, o, nxt, prv, leg, lchi, r = event
    head = (o["status"] == 0) & (prv < 0)
    np.testing.assert_array_equal(r["status"] != 5, head)
    assert (nxt[head] >= 0).sum() > 1000
    m = ~head
    assert not r["par"][m].any() and not r["cov"][m].any() and not r["x"][m].any() and not r["chi2"][m].any()
    np.testing.assert_array_equal(r["ndf"][m], 0)
    # ndf counts every hit of the chain
    off = sd["offsets"]
    for h in np.nonzero(head & (nxt >= 0))[0][:200]:
        n, s = 0, h
        while s >= 0:
            n += off[s + 1] - off[s]
            s = nxt[s]
        assert r["ndf"][h] == 2 * n - 5


def test_noise_free_chains_are_exact(truth_chains):
    fr, sd, o, nxt, prv, r, y, z = truth_chains[False]
    H = multi_heads(r, nxt)
    assert H.size > 1500
    assert np.all(r["status"][H] == 0)
    # chains of three or more segments are among them
    assert (nxt[nxt[H]] >= 0).sum() > 50
    tru = truth_state(fr, sd["hits"][sd["offsets"][H]])
    err = np.abs(r["par"][H] - tru) / np.maximum(np.abs(tru), FLOOR)
    assert err.max() <= 1e-11, err.max(axis=0)
    assert r["chi2"][H].max() <= 1e-15
    np.testing.assert_array_equal(r["x"][H], fr.row_x[sd["first_row"][H]].astype(np.float64))


def test_pulls_and_chi2_of_chain_refits(truth_chains):
    from scipy import stats
    fr, sd, o, nxt, prv, r, y, z = truth_chains[True]
    H = multi_heads(r, nxt)
    assert np.all(r["status"][H] == 0) and H.size > 1500
    tru = truth_state(fr, sd["hits"][sd["offsets"][H]])
    sig = np.sqrt(np.einsum("tii->ti", oracle.unpack_cov(r["cov"][H])))
    pull = (r["par"][H] - tru) / sig
    assert np.all(np.abs(pull.mean(axis=0)) < 0.06), pull.mean(axis=0)
    assert np.all(np.abs(pull.std(axis=0) - 1.0) < 0.05), pull.std(axis=0)
    assert abs((r["chi2"][H] / r["ndf"][H]).mean() - 1.0) < 0.02
    prob = stats.chi2.sf(r["chi2"][H], r["ndf"][H])
    assert stats.kstest(prob, "uniform").pvalue > 1e-3
    # a chain measures q/pT better than its head segment alone
    v0 = np.einsum("tii->ti", oracle.unpack_cov(o["cov"][H]))
    assert np.median(sig[:, 4] ** 2 / v0[:, 4]) < 0.5


def test_two_segment_refit_agrees_with_pair_fusion(truth_chains):
    fr, sd, o, nxt, prv, r, y, z = truth_chains[True]
    H = multi_heads(r, nxt)
    two = H[nxt[nxt[H]] < 0]
    mn, _, _, mp, mc = oracle.merge(o, sd["frame"], sd["sector"], fr.n_sectors, bz=BZ, max_sin=MS, cut=1e9)
    two = two[mn[two] == nxt[two]]
    assert two.size > 1000
    b = nxt[two]
    da = alpha(sd["sector"][b]) - alpha(sd["sector"][two])
    da = (da + np.pi) % (2 * np.pi) - np.pi
    dev, ratio = [], []
    for a_, bb, d in zip(two, b, da):
        st, q, J = oracle.transfer(r["par"][a_], r["x"][a_], d, o["x"][bb], BZ, MS)
        assert st == 0
        Cq = J @ oracle.unpack_cov(r["cov"][a_][None])[0] @ J.T
        s_m = np.sqrt(np.diag(oracle.unpack_cov(mc[a_][None])[0]))
        dev.append(np.abs(q - mp[a_]) / s_m)
        ratio.append(np.sqrt(np.diag(Cq)) / s_m)
    dev, ratio = np.array(dev), np.array(ratio)
    assert np.all(np.abs(np.median(ratio, axis=0) - 1.0) < 1e-3), np.median(ratio, axis=0)
    assert np.all(np.quantile(dev, 0.95, axis=0) < 0.5), np.quantile(dev, 0.95, axis=0)


def test_map_equals_corrected_clusters(truth_chains):
    fr, sd, o, nxt, prv, r, y, z = truth_chains[True]
    rng = np.random.default_rng(5)
    mp = rng.normal(0, 0.2, (fr.n_sectors, fr.n_rows, 2))
    seg = np.repeat(np.arange(len(fr.row_offsets) - 1), np.diff(fr.row_offsets))
    sec, row = seg // fr.n_rows % fr.n_sectors, seg % fr.n_rows
    r1 = oracle.refit(sd, o, nxt, prv, None, y, z, fr.row_x, fr.n_rows, fr.n_sectors, map_=mp, **FIT)
    r2 = oracle.refit(sd, o, nxt, prv, None, y - mp[sec, row, 0], z - mp[sec, row, 1], fr.row_x, fr.n_rows,
                      fr.n_sectors, **FIT)
    H = multi_heads(r1, nxt)
    np.testing.assert_array_equal(r1["status"], r2["status"])
    np.testing.assert_allclose(r1["par"][H], r2["par"][H], rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(r1["chi2"][H], r2["chi2"][H], rtol=1e-7)


def test_track_ids_are_components(event):
    fr, sd, o, nxt, prv, leg, lchi, r = event
    T = len(nxt)
    adj = [[] for _ in range(T)]
    for i in range(T):
        for j in (nxt[i], leg[i]):
            if j >= 0:
                adj[i].append(j)
                adj[j].append(i)
    want = np.full(T, -1)
    for s in range(T):
        if o["status"][s] != 0 or want[s] >= 0:
            continue
        comp, dq = [s], deque([s])
        want[s] = s
        while dq:
            u = dq.popleft()
            for v in adj[u]:
                if want[v] < 0:
                    want[v] = s
                    comp.append(v)
                    dq.append(v)
        want[comp] = min(comp)
    np.testing.assert_array_equal(r["track_id"], want)
    assert np.unique(want[want >= 0]).size < (o["status"] == 0).sum() - 1000


def test_chain_longer_than_a_side_is_refused(event):
    fr, sd, o, nxt, prv, leg, lchi, r = event
    ok = np.nonzero(o["status"] == 0)[0][:19]
    n2, p2 = np.full(len(nxt), -1, np.int32), np.full(len(nxt), -1, np.int32)
    n2[ok[:-1]], p2[ok[1:]] = ok[1:], ok[:-1]
    r2 = oracle.refit(sd, o, n2, p2, None, fr.y, fr.z, fr.row_x, fr.n_rows, fr.n_sectors, **FIT)
    assert r2["status"][ok[0]] == 6 and np.all(r2["status"][ok[1:]] == 5)
    assert "loop_par" not in r2
    # one segment fewer is a chain
    n2[ok[-2]] = -1
    p2[ok[-1]] = -1
    r3 = oracle.refit(sd, o, n2, p2, None, fr.y, fr.z, fr.row_x, fr.n_rows, fr.n_sectors, **FIT)
    assert r3["status"][ok[0]] != 6


def _circle(fr, sd, r, h):
    st, m, J = oracle.leg_circle(r["par"][h], r["x"][h], alpha(sd["sector"][h]), BZ)
    return st, m, J @ oracle.unpack_cov(r["cov"][h][None])[0] @ J.T


def _cov4(c10):
    C = np.zeros((4, 4))
    q = 0
    for a in range(4):
        for b in range(a + 1):
            C[a, b] = C[b, a] = c10[q]
            q += 1
    return C


def _head(prv, i):
    while prv[i] >= 0:
        i = prv[i]
    return i


def test_looper_circles_single_legs_and_information_form(event):
    fr, sd, o, nxt, prv, leg, lchi, r = event
    L = np.nonzero(r["loop_chi2"] >= 0)[0]
    assert L.size > 100
    assert np.all(leg[L] > L)
    rest = np.ones(len(leg), bool)
    rest[L] = False
    assert np.all(r["loop_chi2"][rest] == -1) and not r["loop_par"][rest].any() and not r["loop_cov"][rest].any()
    singles = 0
    for i in L:
        j = leg[i]
        hi, hj = _head(prv, i), _head(prv, j)
        if hi == i and hj == j and nxt[i] < 0 and nxt[j] < 0:
            np.testing.assert_allclose(r["loop_chi2"][i], lchi[i], rtol=1e-9)
            singles += 1
        st1, mi, Si = _circle(fr, sd, r, hi)
        st2, mj, Sj = _circle(fr, sd, r, hj)
        assert st1 == 0 and st2 == 0
        mj, Sj = D @ mj, D @ Sj @ D
        Wi, Wj = np.linalg.inv(Si), np.linalg.inv(Sj)
        C = np.linalg.inv(Wi + Wj)
        x = C @ (Wi @ mi + Wj @ mj)
        obj = (mi - x) @ Wi @ (mi - x) + (mj - x) @ Wj @ (mj - x)
        sx = np.sqrt(np.diag(C))
        assert np.all(np.abs(r["loop_par"][i] - x) <= 1e-4 * sx), (r["loop_par"][i] - x) / sx
        np.testing.assert_allclose(_cov4(r["loop_cov"][i]), C, rtol=1e-5, atol=1e-12 * np.abs(C).max())
        np.testing.assert_allclose(r["loop_chi2"][i], obj, rtol=1e-6)
    assert singles > 10


def test_looper_circle_against_the_truth():
    fr = make_config(1, scale=1.0, keep_truth=True)
    up, dn = oracle.neighbours(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)
    sd = oracle.ca_seed(fr.row_offsets, up, dn, fr.n_sectors, fr.n_rows, MIN_HITS)
    o = oracle.fit(sd, fr.y, fr.z, fr.row_x, fr.n_rows, **FIT)
    nxt, prv, _, _, _ = oracle.merge(o, sd["frame"], sd["sector"], fr.n_sectors, bz=BZ, max_sin=MS, cut=CUT)
    leg, _ = oracle.legs(o, sd["frame"], sd["sector"], fr.n_sectors, bz=BZ, cut=CUT)
    r = oracle.refit(sd, o, nxt, prv, leg, fr.y, fr.z, fr.row_x, fr.n_rows, fr.n_sectors, **FIT)
    off, hits = sd["offsets"], sd["hits"]

    def pure_chain(h):
        t = fr.track_of[hits[off[h]:off[h + 1]]]
        c = [h]
        while nxt[c[-1]] >= 0:
            c.append(nxt[c[-1]])
        ts = np.concatenate([fr.track_of[hits[off[s]:off[s + 1]]] for s in c])
        return t[0] if t[0] >= 0 and (ts == t[0]).all() else -1

    ef, ei, ej = [], [], []
    for i in np.nonzero(r["loop_chi2"] >= 0)[0]:
        hi, hj = _head(prv, i), _head(prv, leg[i])
        pi_, pj_ = pure_chain(hi), pure_chain(hj)
        if pi_ < 0 or pi_ != pj_:
            continue
        h = hits[off[hi]]
        st, mt, _ = oracle.leg_circle(truth_state(fr, h), fr.row_x[sd["first_row"][hi]], alpha(sd["sector"][hi]), BZ)
        assert st == 0
        _, mi, Si = _circle(fr, sd, r, hi)
        _, mj, Sj = _circle(fr, sd, r, hj)
        ef.append(np.abs(r["loop_par"][i] - mt))
        ei.append(np.abs(mi - mt))
        ej.append(np.abs(D @ mj - mt))
        # no joint variance above either leg's
        v = np.diag(_cov4(r["loop_cov"][i]))
        assert np.all(v <= np.minimum(np.diag(Si), np.diag(Sj)) * (1 + 1e-9))
    assert len(ef) > 300
    ef, ei, ej = np.median(ef, 0), np.median(ei, 0), np.median(ej, 0)
    assert np.all(ef[:3] < 0.3 * np.minimum(ei, ej)[:3]), (ef, ei, ej)
    assert ef[3] < np.minimum(ei, ej)[3]
