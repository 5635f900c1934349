"""Pins of the oracle's fit with material (multiple scattering as process
noise, rejection of outlying hits), against a stepping simulation with
scattering kicks in global coordinates (tpcsynth.make_scattering_frame,
which shares nothing with the fit's x-parametrised helix step):

* with the simulation's radiation length in the fit, the five parameters'
  pulls at the innermost hit have unit width and chi2/ndf is 1;
* the same tracks fitted without scattering have chi2/ndf well above 1 and
  pulls several times too wide (the noise term matters);
* an infinite radiation length and no cut reduce to the plain fit exactly;
* hits displaced by 12 sigma after seeding are rejected, clean ones are kept.
"""
import numpy as np
import pytest

import oracle
from tests.conftest import NB, FIT, MIN_HITS
from tpcsynth import make_scattering_frame, PION_MASS

X0 = 50.0          # cm: scattering well above the measurement error at these momenta


def _seeds(fr):
    up, dn = oracle.neighbours(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)
    return oracle.ca_seed(fr.row_offsets, up, dn, 1, fr.n_rows, MIN_HITS)


def _pulls(fr, sd, x0, full=False):
    o = oracle.fit_material(sd, fr.y, fr.z, fr.row_x, x0=x0, mass=PION_MASS, chi2_cut=1e30, **FIT)
    T = len(sd["offsets"]) - 1
    first = sd["hits"][sd["offsets"][:-1]]
    tru = np.stack([fr.y_true[first], fr.z_true[first], fr.s_true[first], fr.t_true[first],
                    fr.w_true[first]], 1)
    pure = np.array([np.unique(fr.track_of[sd["hits"][sd["offsets"][i]:sd["offsets"][i + 1]]]).size == 1
                     for i in range(T)])
    sel = (o["status"] == 0) & pure & (np.diff(sd["offsets"]) >= 20)
    cv = oracle.unpack_cov(o["cov"][sel])
    pulls = (o["par"][sel] - tru[sel]) / np.sqrt(np.einsum("tii->ti", cv))
    if full:
        return pulls, tru[sel], o["chi2"][sel], o["ndf"][sel]
    return pulls, o["chi2"][sel].sum() / o["ndf"][sel].sum(), int(sel.sum())


@pytest.fixture(scope="module")
def scattered():
    frames = [make_scattering_frame(n_tracks=400, seed=s, x0_cm=X0, inv_pt=(0.5, 5.0))
              for s in range(11, 19)]
    return [(fr, _seeds(fr)) for fr in frames]


def test_scattering_noise_gives_unit_pulls(scattered):
    P, num, den = [], 0.0, 0
    for fr, sd in scattered:
        p, q, n = _pulls(fr, sd, X0)
        P.append(p)
        num += q * n
        den += n
    pulls = np.concatenate(P)
    assert pulls.shape[0] > 700
    assert np.all(np.abs(pulls.mean(0)) < 0.1), pulls.mean(0)
    assert np.all(np.abs(pulls.std(0) - 1.0) < 0.1), pulls.std(0)
    assert abs(num / den - 1.0) < 0.03


def test_pulls_of_steep_and_slow_tracks(scattered):
    # the noise grows with the path (dip angle) and falls with beta p: these
    # subsets test the path and velocity factors and the tan(lambda) terms
    P, TR = [], []
    for fr, sd in scattered:
        p, tru, _, _ = _pulls(fr, sd, X0, full=True)
        P.append(p)
        TR.append(tru)
    pulls, tru = np.concatenate(P), np.concatenate(TR)
    mom = np.sqrt(1 + tru[:, 3] ** 2) / np.abs(tru[:, 4])
    for name, sel in (("steep", np.abs(tru[:, 3]) > 0.5), ("slow", mom < 0.7)):
        assert sel.sum() > 250, (name, sel.sum())
        sd_ = pulls[sel].std(0)
        assert np.all(np.abs(sd_[2:] - 1.0) < 0.1), (name, sd_)


def test_without_the_noise_term_the_fit_is_inconsistent(scattered):
    fr, sd = scattered[0]
    pulls, chi, _ = _pulls(fr, sd, np.inf)
    assert chi > 1.2
    assert np.all(pulls.std(0)[1:] > 2.0)


def test_no_material_and_no_cut_is_the_plain_fit():
    fr = make_scattering_frame(n_tracks=150, seed=4, x0_cm=300.0)
    sd = _seeds(fr)
    a = oracle.fit_material(sd, fr.y, fr.z, fr.row_x, x0=np.inf, mass=PION_MASS, chi2_cut=np.inf, **FIT)
    b = oracle.fit(sd, fr.y, fr.z, fr.row_x, fr.n_rows, **FIT)
    np.testing.assert_array_equal(a["status"], b["status"])
    ok = b["status"] == 0
    for k in ("par", "cov", "chi2", "x", "ndf"):
        np.testing.assert_array_equal(a[k][ok], b[k][ok], err_msg=k)
    assert not a["rejected"].any()


def test_displaced_hits_are_rejected():
    fr = make_scattering_frame(n_tracks=300, seed=5, x0_cm=300.0)
    sd = _seeds(fr)
    rng = np.random.default_rng(6)
    off = sd["offsets"]
    planted = []
    for i in range(len(off) - 1):
        n = off[i + 1] - off[i]
        if n < 20:
            continue
        k = int(rng.integers(1, n // 2 - 1))       # neither a start point nor the innermost
        planted.append(off[i] + k)
    planted = np.array(planted)
    y = fr.y.astype(np.float64).copy()
    y[sd["hits"][planted]] += 12 * fr.sigma_y          # chi2 mostly 60..120, cut 30
    o = oracle.fit_material(sd, y, fr.z, fr.row_x, x0=300.0, mass=PION_MASS, chi2_cut=30.0, **FIT)
    clean = oracle.fit_material(sd, fr.y, fr.z, fr.row_x, x0=300.0, mass=PION_MASS, chi2_cut=30.0, **FIT)
    ok = o["status"][np.searchsorted(off, planted, side="right") - 1] == 0
    assert planted.size > 100
    assert o["rejected"][planted[ok]].all()
    assert clean["rejected"].mean() < 2e-3
    others = np.ones(o["rejected"].size, bool)
    others[planted] = False
    assert o["rejected"][others].mean() < 5e-3
