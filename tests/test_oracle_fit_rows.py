"""Pins of the oracle's fit of seeds whose hits may skip pad rows, with
per-cluster errors (each hit's row found from the cluster layout):

* on seeds without gaps, no per-cluster errors and no material it is the
  plain fit bit for bit; with material, the fit with material bit for bit;
  errors equal to the constants change nothing;
* on seeds that bridge missing rows (skip links on a frame with 10%
  pad-row inefficiency) the pulls at the innermost hit have unit width and
  chi2/ndf is 1, while the same seeds fitted as if their rows were
  consecutive are grossly inconsistent;
* with a resolution drawn per cluster (independently in y and z, 0.5-2x the
  nominal) and passed in, unit pulls and chi2/ndf 1; the nominal errors in
  its place, or errors of the wrong cluster, are far off;
* seeds that leave their (frame, sector), repeat or reverse a row, or hold
  an id outside the clusters are refused.
"""
import numpy as np
import pytest

import oracle
from tests.conftest import NB, FIT, MIN_HITS
from tpcsynth import make_config, PION_MASS

NOMAT = dict(x0=np.inf, mass=PION_MASS, chi2_cut=np.inf)


def _rows_fit(fr, sd, err=None, **kw):
    m = {**NOMAT, **kw}
    fit = {k: v for k, v in FIT.items() if k not in kw}
    return oracle.fit_rows(sd, fr.row_offsets, fr.y, fr.z, fr.row_x, fr.n_sectors, fr.n_rows,
                           err=err, **m, **fit)


def _seeds(fr, skip):
    f = oracle.neighbours_skip if skip else oracle.neighbours
    up, dn = f(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)
    return oracle.ca_seed(fr.row_offsets, up, dn, fr.n_sectors, fr.n_rows, MIN_HITS)


def _pulls(fr, sd, o):
    T = len(sd["offsets"]) - 1
    n = np.diff(sd["offsets"])
    first = sd["hits"][sd["offsets"][:-1]]
    tru = np.stack([fr.y_true[first], fr.z_true[first], fr.s_true[first], fr.t_true[first],
                    fr.w_true[first]], 1)
    t = fr.track_of
    pure = np.array([t[first[i]] >= 0 and
                     (t[sd["hits"][sd["offsets"][i]:sd["offsets"][i + 1]]] == t[first[i]]).all()
                     for i in range(T)])
    sel = (o["status"] == 0) & pure & (n >= 20)
    cv = oracle.unpack_cov(o["cov"][sel])
    pulls = (o["par"][sel] - tru[sel]) / np.sqrt(np.einsum("tii->ti", cv))
    return sel, pulls, o["chi2"][sel].sum() / o["ndf"][sel].sum()


def test_contiguous_seeds_are_the_plain_and_material_fits():
    fr = make_config(0)
    sd = _seeds(fr, skip=False)
    a = _rows_fit(fr, sd)
    b = oracle.fit(sd, fr.y, fr.z, fr.row_x, fr.n_rows, **FIT)
    np.testing.assert_array_equal(a["status"], b["status"])
    ok = b["status"] == 0
    assert ok.sum() > 50
    for k in ("x", "par", "cov", "chi2", "ndf"):
        np.testing.assert_array_equal(a[k][ok], b[k][ok], err_msg=k)
    c = _rows_fit(fr, sd, x0=300.0, chi2_cut=30.0)
    d = oracle.fit_material(sd, fr.y, fr.z, fr.row_x, x0=300.0, mass=PION_MASS, chi2_cut=30.0, **FIT)
    for k in d:
        np.testing.assert_array_equal(c[k], d[k], err_msg=k)


def test_errors_equal_to_the_constants_change_nothing():
    fr = make_config(0, hit_eff=0.9)
    sd = _seeds(fr, skip=True)
    sy, sz = np.float32(FIT["sigma_y"]), np.float32(FIT["sigma_z"])
    err = np.tile(np.array([sy, sz], np.float32), (fr.n_clusters, 1))
    kw = dict(sigma_y=float(sy), sigma_z=float(sz))
    a = _rows_fit(fr, sd, err=err, **kw)
    b = _rows_fit(fr, sd, err=None, **kw)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


@pytest.fixture(scope="module")
def gapped():
    fr = make_config(1, scale=0.1, keep_truth=True, hit_eff=0.9)
    return fr, _seeds(fr, skip=True)


def test_seeds_across_missing_rows_have_unit_pulls(gapped):
    fr, sd = gapped
    o = _rows_fit(fr, sd)
    sel, pulls, chi = _pulls(fr, sd, o)
    seg = np.repeat(np.arange(fr.row_offsets.size - 1), np.diff(fr.row_offsets))
    row = seg % fr.n_rows
    gaps = np.array([np.diff(row[sd["hits"][sd["offsets"][i]:sd["offsets"][i + 1]]]).max() > 1
                     for i in range(len(sd["offsets"]) - 1)])
    assert sel.sum() > 1000 and gaps[sel].mean() > 0.8
    assert np.all(np.abs(pulls.mean(0)) < 0.1), pulls.mean(0)
    assert np.all(np.abs(pulls.std(0) - 1.0) < 0.08), pulls.std(0)
    assert abs(chi - 1.0) < 0.03
    # the rows matter: the same seeds fitted on consecutive rows
    b = oracle.fit(sd, fr.y, fr.z, fr.row_x, fr.n_rows, **FIT)
    s2 = sel & gaps & (b["status"] == 0)
    assert b["chi2"][s2].sum() / b["ndf"][s2].sum() > 10.0


def test_per_cluster_errors_give_unit_pulls():
    fr = make_config(1, scale=0.1, keep_truth=True, err_scale=(0.5, 2.0))
    sd = _seeds(fr, skip=False)
    sel, pulls, chi = _pulls(fr, sd, _rows_fit(fr, sd, err=fr.err))
    assert sel.sum() > 1000
    assert np.all(np.abs(pulls.mean(0)) < 0.1), pulls.mean(0)
    assert np.all(np.abs(pulls.std(0) - 1.0) < 0.08), pulls.std(0)
    assert abs(chi - 1.0) < 0.03
    _, _, chi_nominal = _pulls(fr, sd, _rows_fit(fr, sd, err=None))
    assert chi_nominal > 1.5
    _, _, chi_shifted = _pulls(fr, sd, _rows_fit(fr, sd, err=np.roll(fr.err, 1, 0)))
    assert chi_shifted > 1.3
    _, _, chi_swapped = _pulls(fr, sd, _rows_fit(fr, sd, err=fr.err[:, ::-1] * np.float32(
        [FIT["sigma_y"] / FIT["sigma_z"], FIT["sigma_z"] / FIT["sigma_y"]])))
    assert chi_swapped > 1.3


def test_malformed_seeds_are_refused():
    fr = make_config(0)
    sd = _seeds(fr, skip=False)
    off = sd["offsets"]
    i = int(np.argmax(np.diff(off)))                  # a long seed
    h = sd["hits"][off[i]:off[i + 1]].copy()
    seg = np.repeat(np.arange(fr.row_offsets.size - 1), np.diff(fr.row_offsets))
    low = int(fr.row_offsets[seg[h[2]]])              # a cluster of the row of the third hit
    s5 = seg[h[5]]
    mate = [c for c in range(fr.row_offsets[s5], fr.row_offsets[s5 + 1]) if c != h[5]][0]
    cases = {
        "ok": h,
        "reversed pair": np.concatenate([h[:3], h[4:5], h[3:4], h[5:]]),
        "row repeated": np.concatenate([h[:5], [min(mate, h[5]), max(mate, h[5])], h[6:]]),
        "lower row last": np.concatenate([h, [low]]),
        "negative id": np.concatenate([h[:-1], [-1]]),
        "id past the end": np.concatenate([h[:-1], [fr.n_clusters]]),
    }
    hits = np.concatenate(list(cases.values())).astype(np.int32)
    offs = np.concatenate([[0], np.cumsum([len(v) for v in cases.values()])]).astype(np.int32)
    n = len(cases)
    sds = dict(offsets=offs, hits=hits, frame=np.zeros(n, np.int32), sector=np.zeros(n, np.int32),
               first_row=np.zeros(n, np.int32))
    o = _rows_fit(fr, sds)
    st = dict(zip(cases, o["status"].tolist()))
    assert st.pop("ok") == 0
    assert all(v == 1 for v in st.values()), st
    bad = dict(sds, frame=np.full(n, 1, np.int32))
    assert (_rows_fit(fr, bad)["status"] == 1).all()
    bad = dict(sds, sector=np.full(n, -1, np.int32))
    assert (_rows_fit(fr, bad)["status"] == 1).all()


def test_seed_of_another_sector_is_refused():
    fr = make_config(1, scale=0.02)
    sd = _seeds(fr, skip=True)
    o = _rows_fit(fr, sd)
    moved = dict(sd, sector=(sd["sector"] + 1) % fr.n_sectors)
    m = _rows_fit(fr, moved)
    assert (o["status"] == 0).mean() > 0.95
    assert (m["status"] == 1).all()
