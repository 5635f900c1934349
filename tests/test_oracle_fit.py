"""Pins of the oracle's Kalman helix fit (CPU only).

* the exact helix step reproduces the generator's crossing points, which the
  generator computes independently as circle/plane intersections in global
  coordinates (<= 1e-10 cm);
* the analytic propagation Jacobian equals central finite differences;
* noise-free helices are recovered to round-off, with chi2 ~ 0;
* with Gaussian smearing the pulls have zero mean and unit width and
  chi2/ndf averages 1 (statistics over 1e4 tracks);
* the map gradient of the summed chi2 from finite differences of the C oracle
  equals reverse-mode autograd of an independent float64 torch implementation.
"""
import math

import numpy as np
import pytest

import oracle
from tests.conftest import FIT
from tpcsynth import make_frames

FLOOR = np.array([1.0, 1.0, 1e-2, 1e-2, 1e-2])


def truth_runs(fr, min_len=10):
    """Seeds built from truth: per track and sector, the longest run of
    consecutive rows with exactly one cluster of that track per row."""
    seg = np.repeat(np.arange(len(fr.row_offsets) - 1), np.diff(fr.row_offsets))
    row = seg % fr.n_rows
    fs = seg // fr.n_rows                      # frame * n_sectors + sector
    tr = fr.track_of.astype(np.int64)
    key = tr * (fs.max() + 1 if len(fs) else 1) + fs
    order = np.lexsort((row, key))
    order = order[tr[order] >= 0]
    seeds_h, first_rows, secs = [], [], []
    k_sorted = key[order]
    starts = np.r_[0, np.nonzero(np.diff(k_sorted))[0] + 1, len(order)]
    for a, b in zip(starts[:-1], starts[1:]):
        ids = order[a:b]
        rw = row[ids]
        uniq, cnt = np.unique(rw, return_counts=True)
        good = set(uniq[cnt == 1].tolist())
        best, cur = [], []
        for i, r in zip(ids, rw):
            if r not in good:
                cur = []
                continue
            if cur and row[cur[-1]] == r - 1:
                cur.append(i)
            elif not cur or row[cur[-1]] != r:
                cur = [i]
            if len(cur) > len(best):
                best = list(cur)
        if len(best) >= min_len:
            seeds_h.append(best)
            first_rows.append(int(row[best[0]]))
            secs.append(int(fs[best[0]] % fr.n_sectors))
    offs = np.zeros(len(seeds_h) + 1, np.int32)
    np.cumsum([len(s) for s in seeds_h], out=offs[1:])
    hits = np.concatenate(seeds_h).astype(np.int32)
    T = len(seeds_h)
    return dict(offsets=offs, hits=hits, frame=np.zeros(T, np.int32),
                sector=np.array(secs, np.int32), first_row=np.array(first_rows, np.int32))


def _clean_frames(n_tracks, seed, smear, inv_pt=(0.2, 5.0)):
    fr = make_frames(n_sectors=1, tracks_per_frame=(n_tracks,), seed=seed,
                     phi_range=(-math.radians(10), math.radians(10)), smear=smear, keep_truth=True)
    return fr


def test_helix_step_reproduces_generator_crossings():
    fr = _clean_frames(300, 11, smear=False)
    sd = truth_runs(fr, 10)
    worst = 0.0
    for i in range(len(sd["offsets"]) - 1):
        h = sd["hits"][sd["offsets"][i]:sd["offsets"][i + 1]]
        r0 = sd["first_row"][i]
        for k in range(len(h) - 1):
            a, b = h[k + 1], h[k]
            p = np.array([fr.y_true[a], fr.z_true[a], fr.s_true[a], fr.t_true[a], fr.w_true[a]])
            dx = float(fr.row_x[r0 + k]) - float(fr.row_x[r0 + k + 1])
            st, po, _ = oracle.propagate(p, dx, FIT["bz"], FIT["max_sin"])
            assert st == 0
            want = np.array([fr.y_true[b], fr.z_true[b], fr.s_true[b], fr.t_true[b], fr.w_true[b]])
            worst = max(worst, float(np.max(np.abs(po - want))))
    assert len(sd["offsets"]) > 50
    assert worst <= 1e-10, worst


@pytest.mark.parametrize("seed", range(4))
def test_propagation_jacobian_matches_central_differences(seed):
    rng = np.random.default_rng(seed)
    for _ in range(50):
        p = np.array([rng.uniform(-30, 30), rng.uniform(-200, 200), rng.uniform(-0.8, 0.8),
                      rng.uniform(-1, 1), rng.uniform(-8, 8) * rng.choice([1e-3, 1.0])])
        dx = rng.choice([-1.0596, 1.0596, -7.3, 12.0])
        st, po, F = oracle.propagate(p, dx, FIT["bz"], FIT["max_sin"])
        if st:
            continue
        Fd = np.zeros((5, 5))
        for j in range(5):            # five-point central stencil
            h = 1e-3 * max(abs(p[j]), 0.1)
            vals = []
            for m in (2, 1, -1, -2):
                pq = p.copy()
                pq[j] += m * h
                vals.append(oracle.propagate(pq, dx, FIT["bz"], FIT["max_sin"])[1])
            Fd[:, j] = (-vals[0] + 8 * vals[1] - 8 * vals[2] + vals[3]) / (12 * h)
        np.testing.assert_allclose(F, Fd, rtol=1e-7, atol=1e-7)


def test_noise_free_helices_recovered_to_round_off():
    fr = _clean_frames(400, 12, smear=False)
    sd = truth_runs(fr, 10)
    r = oracle.fit(sd, fr.y_true, fr.z_true, fr.row_x, fr.n_rows, **FIT)
    assert np.all(r["status"] == 0)
    first = sd["hits"][sd["offsets"][:-1]]
    truth = np.stack([fr.y_true[first], fr.z_true[first], fr.s_true[first], fr.t_true[first],
                      fr.w_true[first]], axis=1)
    err = np.abs(r["par"] - truth) / np.maximum(np.abs(truth), FLOOR)
    assert err.max() <= 1e-9, err.max(axis=0)
    assert r["chi2"].max() <= 1e-12
    np.testing.assert_array_equal(r["x"], fr.row_x[sd["first_row"]].astype(np.float64))
    np.testing.assert_array_equal(r["ndf"], 2 * np.diff(sd["offsets"]) - 5)


def test_pulls_and_chi2_under_gaussian_smearing():
    fr = _clean_frames(24000, 13, smear=True)
    sd = truth_runs(fr, 10)
    T = len(sd["offsets"]) - 1
    assert T >= 10000
    r = oracle.fit(sd, fr.y, fr.z, fr.row_x, fr.n_rows, **FIT)
    ok = r["status"] == 0
    assert ok.mean() > 0.999
    first = sd["hits"][sd["offsets"][:-1]]
    truth = np.stack([fr.y_true[first], fr.z_true[first], fr.s_true[first], fr.t_true[first],
                      fr.w_true[first]], axis=1)
    C = oracle.unpack_cov(r["cov"])
    sig = np.sqrt(np.stack([C[:, i, i] for i in range(5)], axis=1))
    pull = ((r["par"] - truth) / sig)[ok]
    mu = pull.mean(axis=0)
    sd_ = pull.std(axis=0)
    assert np.all(np.abs(mu) < 0.03), mu
    assert np.all(np.abs(sd_ - 1.0) < 0.03), sd_
    cn = (r["chi2"] / r["ndf"])[ok]
    assert abs(cn.mean() - 1.0) < 0.02, cn.mean()
    # chi2 probabilities are flat
    from scipy import stats
    prob = stats.chi2.sf(r["chi2"][ok], r["ndf"][ok])
    assert stats.kstest(prob, "uniform").pvalue > 1e-3


def test_map_shift_is_equivalent_to_shifting_clusters():
    """Subtracting a map from the clusters equals fitting pre-corrected clusters."""
    fr = _clean_frames(100, 14, smear=True)
    sd = truth_runs(fr, 10)
    rng = np.random.default_rng(3)
    mp = rng.normal(0, 0.2, (1, fr.n_rows, 2))
    seg = np.repeat(np.arange(len(fr.row_offsets) - 1), np.diff(fr.row_offsets))
    y2 = fr.y.astype(np.float64) - mp[0, seg, 0]
    z2 = fr.z.astype(np.float64) - mp[0, seg, 1]
    a = oracle.fit(sd, fr.y, fr.z, fr.row_x, fr.n_rows, map_=mp, **FIT)
    b = oracle.fit(sd, y2, z2, fr.row_x, fr.n_rows, **FIT)
    np.testing.assert_allclose(a["par"], b["par"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(a["chi2"], b["chi2"], rtol=1e-12)


def test_fd_gradient_matches_independent_autograd():
    from oracle import ref_autograd
    fr = make_frames(n_sectors=36, tracks_per_frame=(60,), seed=15, smear=True, keep_truth=True,
                     distortion_amp=0.3, phi_range=(0.0, math.radians(40.0)))
    seeds = truth_runs(fr, 8)
    T = len(seeds["offsets"]) - 1
    assert T >= 20 and np.unique(seeds["sector"]).size >= 2
    mp = np.random.default_rng(4).normal(0, 0.1, (fr.n_sectors, fr.n_rows, 2))
    r = oracle.fit(seeds, fr.y, fr.z, fr.row_x, fr.n_rows, map_=mp, **FIT)
    assert np.all(r["status"] == 0)
    L, g = ref_autograd.map_gradient(mp, seeds, fr.y, fr.z, fr.row_x, **FIT)
    assert abs(L - r["chi2"].sum()) <= 1e-9 * abs(L)
    rng = np.random.default_rng(5)
    covered = np.argwhere(np.abs(g).sum(axis=2) > 0)
    pick = covered[rng.choice(len(covered), size=min(60, len(covered)), replace=False)]
    entries = [(int(s), int(rr), int(a)) for s, rr in pick for a in (0, 1)]
    fd = oracle.fd_map_gradient(seeds, fr.y, fr.z, fr.row_x, fr.n_rows, mp, entries, h=1e-3, **FIT)
    ag = np.array([g[s, rr, a] for s, rr, a in entries])
    scale = np.abs(ag).max()
    np.testing.assert_allclose(fd, ag, rtol=1e-6, atol=1e-6 * scale)
    # entries no seed covers have zero gradient
    assert np.all(g[np.abs(g).sum(axis=2) == 0] == 0)


def test_direction_margin_is_the_distance_to_the_threshold():
    """The oracle's sin_margin report: a track that passed its fit with the
    smallest margins fails when max_sin drops by a little more than the
    margin and passes when it drops by a little less; failed steps report a
    negative margin."""
    fr = make_frames(n_sectors=1, tracks_per_frame=(3000,), seed=31, smear=True, keep_truth=True,
                     phi_range=(-math.radians(40), math.radians(40)), looper_frac=0.3)
    sd = truth_runs(fr, 10)
    prm = dict(FIT, max_sin=0.8)
    r = oracle.fit(sd, fr.y, fr.z, fr.row_x, fr.n_rows, **prm)
    ok = r["status"] == 0
    assert np.all(r["sin_margin"][ok] > 0)
    assert np.all(r["sin_margin"][r["status"] == 2] <= 0)
    assert (r["status"] == 2).sum() > 5
    # the closest passes whose binding threshold is max_sin (not cos phi at the start)
    cand = np.nonzero(ok & (r["sin_margin"] < 0.05))[0]
    assert cand.size >= 10
    checked = 0
    for i in cand[np.argsort(r["sin_margin"][cand])][:20]:
        one = oracle.subset_seeds(sd, np.array([i]))
        m = r["sin_margin"][i]
        lo = oracle.fit(one, fr.y, fr.z, fr.row_x, fr.n_rows, **dict(prm, max_sin=prm["max_sin"] - m * (1 + 1e-6)))
        hi = oracle.fit(one, fr.y, fr.z, fr.row_x, fr.n_rows, **dict(prm, max_sin=prm["max_sin"] - m * (1 - 1e-6)))
        if hi["status"][0] == 0:
            assert lo["status"][0] != 0
            checked += 1
    assert checked >= 10
