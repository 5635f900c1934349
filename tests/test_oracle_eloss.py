"""Pins of the oracle's energy loss (the fit with material and the smoother
in a gas of density rho, Z/A and mean excitation energy I):

* the mean loss per density at minimum ionisation equals the tabulated
  values of the Particle Data Group's atomic and nuclear properties tables
  for argon, neon, helium and nitrogen gas (1.519, 1.724, 1.937 and
  1.825 MeV cm^2/g; the tables use the Bethe formula with the density
  effect, which vanishes at minimum ionisation in a gas);
* a gas of zero density changes nothing;
* the map of a step (w' = w P/P', the loss given back at fixed direction)
  against its closed form, its Jacobian against finite differences of that
  form with the loss held fixed, the straggling against Bohr's variance
  carried by dw/dE; a segment past the cap is left alone;
* on a stepping simulation that loses energy without scattering (the loss
  integrated in sub-steps, with Bohr straggling), the q/pT pulls at the
  innermost hit have unit width and the same mean (signed by the charge)
  as on the same tracks without any gas, while the fit without the loss
  is grossly off; the smoother's pulls at every hit have unit width, and
  without the loss are off; where the straggling dominates (pions in a gas
  120 times denser than argon) the q/pT pulls have unit width;
* with scattering and energy loss together (protons, a gas 30 times denser
  than argon) all five pulls have unit width, chi2/ndf is 1, and no long
  seed's q/pT is locked far off (the fit starts with a wide q/pT variance
  from a start state that can be far from the truth).
"""
import numpy as np
import pytest

import oracle
from tests.conftest import NB, FIT, MIN_HITS
from tpcsynth import make_scattering_frame, PROTON_MASS, PION_MASS, ARGON_GAS

MUON_MASS = 0.1056583755
RHO = 0.05
GAS = (RHO, ARGON_GAS[1], ARGON_GAS[2])
X0_GAS = 19.55 / RHO                          # argon's radiation length, 19.55 g/cm^2


@pytest.mark.parametrize("zoa,exc,dedx_min", [(0.45059, 188.0e-9, 1.519), (0.49555, 137.0e-9, 1.724),
                                              (0.49967, 41.8e-9, 1.937), (0.49976, 82.0e-9, 1.825)])
def test_minimum_ionisation_matches_the_tables(zoa, exc, dedx_min):
    bg = np.geomspace(1.0, 30.0, 3000)
    v = np.array([oracle.bethe(b, MUON_MASS, zoa, exc) for b in bg]) * 1e3
    i = int(v.argmin())
    assert 2.5 < bg[i] < 4.5
    assert abs(v[i] - dedx_min) < 2e-3 * dedx_min, v[i]


def _frozen_map(w, t, s, dx, dE, mass):
    """w after a step inwards that gives back the energy dE: the momentum
    P = sqrt(1+t^2)/|w| grows to sqrt((E+dE)^2 - m^2) at fixed direction."""
    P = np.sqrt(1.0 + t * t) / abs(w)
    E = np.hypot(P, mass)
    return np.sign(w) * np.sqrt(1.0 + t * t) / np.sqrt((E + dE) ** 2 - mass * mass)


@pytest.mark.parametrize("w,t,s", [(1.3, 0.4, 0.2), (-0.6, -0.9, -0.5), (3.0, 0.05, 0.0)])
def test_energy_loss_map_and_its_jacobian(w, t, s):
    dx = 1.5
    state = np.array([1.0, 2.0, s, t, w])
    st, w1, j43, j44, vw = oracle.eloss(state, dx, PROTON_MASS, GAS)
    assert st == 0
    P = np.sqrt(1 + t * t) / abs(w)
    E = np.hypot(P, PROTON_MASS)
    ds = dx * np.sqrt(1 + t * t) / np.sqrt(1 - s * s)
    dE = ds * RHO * oracle.bethe(P / PROTON_MASS, PROTON_MASS, GAS[1], GAS[2])
    assert 0 < dE < 0.01 * E
    assert w1 == pytest.approx(_frozen_map(w, t, s, dx, dE, PROTON_MASS), rel=1e-12)
    assert abs(w1) < abs(w)
    h = 1e-6
    fd_w = (_frozen_map(w + h, t, s, dx, dE, PROTON_MASS) - _frozen_map(w - h, t, s, dx, dE, PROTON_MASS)) / (2 * h)
    fd_t = (_frozen_map(w, t + h, s, dx, dE, PROTON_MASS) - _frozen_map(w, t - h, s, dx, dE, PROTON_MASS)) / (2 * h)
    assert j44 == pytest.approx(fd_w, rel=1e-6)
    assert j43 == pytest.approx(fd_t, rel=1e-5, abs=1e-12)
    # the straggling of E, carried to w by dw/dE at the start
    b2 = (P / E) ** 2
    var_e = 0.307075e-3 * GAS[1] * RHO * ds * 0.51099895e-3 * (1 - b2 / 2) / (1 - b2)
    assert vw == pytest.approx(var_e * (w * E / P ** 2) ** 2, rel=1e-12)
    # outwards the loss is taken away; a segment past the cap is left alone
    st, w2, _, _, _ = oracle.eloss(state, dx, PROTON_MASS, GAS, direction=-1.0)
    assert st == 0 and abs(w2) > abs(w)
    st, w3, j43, j44, vw = oracle.eloss(np.array([0, 0, s, t, 40.0]), dx, PROTON_MASS, GAS)
    assert (st, w3, j43, j44, vw) == (0, 40.0, 0.0, 1.0, 0.0)


def _seeds(fr):
    up, dn = oracle.neighbours(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)
    return oracle.ca_seed(fr.row_offsets, up, dn, fr.n_sectors, fr.n_rows, MIN_HITS)


def _frames(gas, x0, seeds=range(11, 15)):
    return [make_scattering_frame(n_tracks=400, seed=s, x0_cm=x0, mass=PROTON_MASS, inv_pt=(0.7, 2.0),
                                  gas=gas) for s in seeds]


def _first_pulls(frames, fit_gas, x0):
    """Pulls at the innermost hit of pure seeds of >= 20 hits (q/pT signed by
    the charge) and chi2/ndf."""
    P, ch, nd = [], 0.0, 0
    for fr in frames:
        sd = _seeds(fr)
        o = oracle.fit_material(sd, fr.y, fr.z, fr.row_x, x0=x0, mass=PROTON_MASS, chi2_cut=np.inf,
                                gas=fit_gas, **FIT)
        first = sd["hits"][sd["offsets"][:-1]]
        n = np.diff(sd["offsets"])
        t = fr.track_of
        pure = np.array([t[first[i]] >= 0 and (t[sd["hits"][sd["offsets"][i]:sd["offsets"][i + 1]]]
                                               == t[first[i]]).all() for i in range(n.size)])
        sel = (o["status"] == 0) & pure & (n >= 20)
        tru = np.stack([fr.y_true[first], fr.z_true[first], fr.s_true[first], fr.t_true[first],
                        fr.w_true[first]], 1)[sel]
        p = (o["par"][sel] - tru) / np.sqrt(np.einsum("tii->ti", oracle.unpack_cov(o["cov"][sel])))
        p[:, 4] *= np.sign(tru[:, 4])
        P.append(p)
        ch += o["chi2"][sel].sum()
        nd += o["ndf"][sel].sum()
    P = np.concatenate(P)
    return P, ch / nd


def _width(p):
    return np.quantile(np.abs(p), 0.683, axis=0)


def test_zero_density_changes_nothing():
    fr = _frames(GAS, X0_GAS, seeds=[3])[0]
    sd = _seeds(fr)
    kw = dict(x0=X0_GAS, mass=PROTON_MASS, chi2_cut=30.0, **FIT)
    a = oracle.fit_material(sd, fr.y, fr.z, fr.row_x, gas=None, **kw)
    b = oracle.fit_material(sd, fr.y, fr.z, fr.row_x, gas=(0.0, 0.5, 1e-7), **kw)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


@pytest.fixture(scope="module")
def lossy():
    """Protons losing energy in the gas without scattering, and the same
    tracks in no gas."""
    return _frames(GAS, 1e9), _frames(None, 1e9)


def test_fit_with_energy_loss_has_unit_pulls(lossy):
    frames, control = lossy
    P, chi = _first_pulls(frames, GAS, np.inf)
    C, _ = _first_pulls(control, None, np.inf)
    assert len(P) > 1000
    assert np.all(np.abs(_width(P) - 1.0) < 0.08), _width(P)
    assert abs(P[:, 4].mean() - C[:, 4].mean()) < 0.06, (P[:, 4].mean(), C[:, 4].mean())
    assert np.all(np.abs(P[:, :4].mean(0)) < 0.1)
    assert abs(chi - 1.0) < 0.03
    N, _ = _first_pulls(frames, None, np.inf)             # the loss ignored
    assert N[:, 4].mean() - C[:, 4].mean() > 1.0
    assert _width(N)[4] > 1.5


def _hit_pulls(frames, fit_gas, x0):
    P = []
    for fr in frames:
        sd = _seeds(fr)
        o = oracle.fit_rows(sd, fr.row_offsets, fr.y, fr.z, fr.row_x, fr.n_sectors, fr.n_rows, err=None,
                            x0=x0, mass=PROTON_MASS, chi2_cut=np.inf, gas=fit_gas, smooth=True, **FIT)
        for i in range(len(sd["offsets"]) - 1):
            a, b = sd["offsets"][i], sd["offsets"][i + 1]
            h = sd["hits"][a:b]
            if o["status"][i] or b - a < 20 or fr.track_of[h[0]] < 0 or np.unique(fr.track_of[h]).size != 1:
                continue
            tru = np.stack([fr.y_true[h], fr.z_true[h], fr.s_true[h], fr.t_true[h], fr.w_true[h]], 1)
            p = (o["hit_par"][a:b] - tru) / np.sqrt(np.einsum("tii->ti", oracle.unpack_cov(o["hit_cov"][a:b])))
            p[:, 4] *= np.sign(tru[:, 4])
            P.append(p)
    return np.concatenate(P)


def test_straggling_dominated_fit_has_unit_pulls():
    # pions in a gas 120 times denser than argon, no scattering: the loss
    # fluctuations dominate the q/pT resolution of long tracks
    gas = (0.2, ARGON_GAS[1], ARGON_GAS[2])
    P = []
    for s in range(11, 15):
        fr = make_scattering_frame(n_tracks=400, seed=s, x0_cm=1e9, mass=PION_MASS, inv_pt=(0.5, 1.5), gas=gas)
        sd = _seeds(fr)
        o = oracle.fit_material(sd, fr.y, fr.z, fr.row_x, x0=np.inf, mass=PION_MASS, chi2_cut=np.inf, gas=gas,
                                **FIT)
        first = sd["hits"][sd["offsets"][:-1]]
        sel = (o["status"] == 0) & (np.diff(sd["offsets"]) >= 20) & (fr.track_of[first] >= 0)
        sw = np.sqrt(oracle.unpack_cov(o["cov"][sel])[:, 4, 4])
        P.append((o["par"][sel, 4] - fr.w_true[first][sel]) / sw)
    P = np.concatenate(P)
    assert len(P) > 1000
    assert abs(_width(P) - 1.0) < 0.08, _width(P)


def test_smoother_with_energy_loss_has_unit_pulls(lossy):
    frames, _ = lossy
    P = _hit_pulls(frames[:2], GAS, np.inf)
    assert len(P) > 40000
    assert np.all(np.abs(_width(P) - 1.0) < 0.08), _width(P)
    assert np.all(np.abs(np.median(P, 0)) < 0.1), np.median(P, 0)
    N = _hit_pulls(frames[:2], None, np.inf)
    assert _width(N)[4] > 1.4, _width(N)


def test_scattering_and_energy_loss_together():
    frames = _frames(GAS, X0_GAS)
    P, chi = _first_pulls(frames, GAS, X0_GAS)
    assert len(P) > 1000
    assert np.all(np.abs(_width(P) - 1.0) < 0.1), _width(P)
    assert abs(chi - 1.0) < 0.05, chi
    assert np.abs(P[:, 4]).max() < 10.0, np.abs(P[:, 4]).max()
