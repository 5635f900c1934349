"""Pins of the oracle's smoother (the state at every hit's plane from all
hits: a Kalman filter of the deviation from the fit's trajectory, then the
Rauch-Tung-Striebel pass):

* without process noise the smoothed states are one helix: the state at
  every plane equals the smoothed innermost state carried there by the
  exact helix step, and its covariance that state's covariance carried by
  the step's Jacobian (an independent closed form: the smoother never calls
  the step from the innermost plane outwards);
* at the innermost plane the smoothed covariance equals the fit's (the fit
  has already seen every hit there);
* against the generator's truth at every hit, pulls of all five parameters
  have unit width -- on tracks without material and on the stepping
  simulation with scattering, where the fit's final state carried outwards
  (what the smoother reduces to without process noise) is inconsistent.
Widths are the 68.3 % quantile of |pull| (robust to the few badly measured
tracks whose pulls are large at every hit).
"""
import numpy as np
import pytest

import oracle
from tests.conftest import NB, FIT, MIN_HITS
from tpcsynth import make_config, make_scattering_frame, PION_MASS


def _seeds(fr):
    up, dn = oracle.neighbours(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)
    return oracle.ca_seed(fr.row_offsets, up, dn, fr.n_sectors, fr.n_rows, MIN_HITS)


def _smooth(fr, sd, x0=np.inf):
    return oracle.fit_rows(sd, fr.row_offsets, fr.y, fr.z, fr.row_x, fr.n_sectors, fr.n_rows, err=None,
                           x0=x0, mass=PION_MASS, chi2_cut=np.inf, smooth=True, **FIT)


def _rows(fr):
    return np.repeat(np.arange(fr.row_offsets.size - 1), np.diff(fr.row_offsets)) % fr.n_rows


def _width(p):
    return np.quantile(np.abs(p), 0.683, axis=0)


def _hit_pulls(fr, sd, o, min_hits=20):
    P = []
    for i in range(len(sd["offsets"]) - 1):
        a, b = sd["offsets"][i], sd["offsets"][i + 1]
        h = sd["hits"][a:b]
        if o["status"][i] or b - a < min_hits or fr.track_of[h[0]] < 0 or np.unique(fr.track_of[h]).size != 1:
            continue
        tru = np.stack([fr.y_true[h], fr.z_true[h], fr.s_true[h], fr.t_true[h], fr.w_true[h]], 1)
        cv = oracle.unpack_cov(o["hit_cov"][a:b])
        P.append((o["hit_par"][a:b] - tru) / np.sqrt(np.einsum("tii->ti", cv)))
    return np.concatenate(P)


def test_without_process_noise_the_smoothed_states_are_one_helix():
    fr = make_config(0)
    sd = _seeds(fr)
    o = _smooth(fr, sd)
    row = _rows(fr)
    worst_p = worst_c = 0.0
    checked = 0
    for i in range(len(sd["offsets"]) - 1):
        if o["status"][i]:
            continue
        a, b = sd["offsets"][i], sd["offsets"][i + 1]
        xs = fr.row_x[row[sd["hits"][a:b]]].astype(np.float64)
        S0 = oracle.unpack_cov(o["hit_cov"][a:a + 1])[0]
        for k in range(b - a):
            st, pk, F = oracle.propagate(o["hit_par"][a], xs[k] - xs[0], FIT["bz"], FIT["max_sin"])
            assert st == 0
            Ck = F @ S0 @ F.T
            sig = np.sqrt(np.diag(Ck))
            sc = oracle.unpack_cov(o["hit_cov"][a + k:a + k + 1])[0]
            worst_p = max(worst_p, np.max(np.abs(o["hit_par"][a + k] - pk) / sig))
            worst_c = max(worst_c, np.max(np.abs(sc - Ck) / np.outer(sig, sig)))
            checked += 1
    assert checked > 2000
    assert worst_p < 0.05, worst_p
    assert worst_c < 0.1, worst_c


def test_innermost_smoothed_covariance_is_the_fits():
    fr = make_config(1, scale=0.05)
    sd = _seeds(fr)
    o = _smooth(fr, sd)
    ok = o["status"] == 0
    a0 = sd["offsets"][:-1][ok]
    vs = np.einsum("tii->ti", oracle.unpack_cov(o["hit_cov"][a0]))
    vf = np.einsum("tii->ti", oracle.unpack_cov(o["cov"][ok]))
    np.testing.assert_allclose(np.median(vs / vf, 0), 1.0, atol=2e-3)


def test_pulls_at_every_hit_without_material():
    fr = make_config(1, scale=0.1, keep_truth=True)
    sd = _seeds(fr)
    p = _hit_pulls(fr, sd, _smooth(fr, sd))
    assert len(p) > 40000
    assert np.all(np.abs(_width(p) - 1.0) < 0.08), _width(p)
    assert np.all(np.abs(np.median(p, 0)) < 0.1), np.median(p, 0)


@pytest.fixture(scope="module")
def scattered():
    out = []
    for s in range(11, 19):
        fr = make_scattering_frame(n_tracks=400, seed=s, x0_cm=50.0, inv_pt=(0.5, 5.0))
        sd = _seeds(fr)
        out.append((fr, sd, _smooth(fr, sd, 50.0)))
    return out


def test_pulls_at_every_hit_with_scattering(scattered):
    p = np.concatenate([_hit_pulls(fr, sd, o) for fr, sd, o in scattered])
    assert len(p) > 40000
    assert np.all(np.abs(_width(p) - 1.0) < 0.08), _width(p)
    assert np.all(np.abs(np.median(p, 0)) < 0.1), np.median(p, 0)


def test_without_the_noise_term_the_trajectory_is_inconsistent(scattered):
    # the fit's final state carried outwards (the smoother without process
    # noise) misses the kinks: its pulls at the outer half are far from unit
    P = []
    for fr, sd, o in scattered:
        row = _rows(fr)
        for i in range(len(sd["offsets"]) - 1):
            a, b = sd["offsets"][i], sd["offsets"][i + 1]
            h = sd["hits"][a:b]
            if o["status"][i] or b - a < 40 or np.unique(fr.track_of[h]).size != 1:
                continue
            xs = fr.row_x[row[h]].astype(np.float64)
            C0 = oracle.unpack_cov(o["cov"][i:i + 1])[0]
            for k in range((b - a) // 2, b - a, 5):
                st, pk, F = oracle.propagate(o["par"][i], xs[k] - xs[0], FIT["bz"], FIT["max_sin"])
                tru = np.array([fr.y_true[h[k]], fr.z_true[h[k]], fr.s_true[h[k]], fr.t_true[h[k]],
                                fr.w_true[h[k]]])
                P.append((pk - tru) / np.sqrt(np.diag(F @ C0 @ F.T)))
    P = np.array(P)
    assert len(P) > 1000
    assert np.max(np.abs(_width(P) - 1.0)) > 0.5, _width(P)
