"""Comparison helpers for GPU-vs-oracle parity (shared by the GPU tests)."""
import numpy as np

import oracle

# per-component floors for the parameter tolerance (y, z in cm; sin phi,
# tan lambda; q/pT in 1/GeV)
PAR_FLOOR = np.array([1.0, 1.0, 1e-2, 1e-2, 1e-2])
PAR_RTOL = 1e-4
COV_RTOL = 1e-3
CHI2_RTOL = 1e-3


def seed_lists(sd):
    o = np.asarray(sd["offsets"])
    h = np.asarray(sd["hits"])
    return [h[o[i]:o[i + 1]] for i in range(len(o) - 1)]


def assert_seeds_equal(got: dict, ref: dict):
    for k in ("offsets", "hits", "frame", "sector", "first_row"):
        a, b = np.asarray(got[k]), np.asarray(ref[k])
        assert a.shape == b.shape, (k, a.shape, b.shape)
        np.testing.assert_array_equal(a, b, err_msg=k)


def compare_fit(gpu: dict, ref: dict, max_fail_frac=1e-4):
    """Fit parity against the float64 oracle on the same seeds.

    Returns a dict of statistics; raises AssertionError on violation.
    Tracks that either side flags as failed are excluded; at most
    ``max_fail_frac`` of the tracks (and at least one) may be flagged by one
    side only.
    """
    st_g = np.asarray(gpu["status"])
    st_r = np.asarray(ref["status"])
    T = len(st_r)
    mism = int(np.sum((st_g == 0) != (st_r == 0)))
    assert mism <= max(1, int(max_fail_frac * T)), "status mismatches: %d of %d" % (mism, T)
    ok = (st_g == 0) & (st_r == 0)
    pg = np.asarray(gpu["par"], np.float64)[ok]
    pr = np.asarray(ref["par"])[ok]
    tol = PAR_RTOL * np.maximum(np.abs(pr), PAR_FLOOR)
    dpar = np.abs(pg - pr) / np.maximum(np.abs(pr), PAR_FLOOR)
    bad = np.abs(pg - pr) > tol
    assert not bad.any(), "parameter mismatch: %d entries, worst rel %.3g (component %s)" % (
        bad.sum(), dpar.max(), np.unravel_index(dpar.argmax(), dpar.shape)[1])
    cg = oracle.unpack_cov(np.asarray(gpu["cov"], np.float64)[ok])
    cr = oracle.unpack_cov(np.asarray(ref["cov"])[ok])
    dg = np.sqrt(np.einsum("tii->ti", cr))
    scale = dg[:, :, None] * dg[:, None, :]
    dcov = np.abs(cg - cr) / scale
    assert dcov.max() <= COV_RTOL, "covariance mismatch: worst %.3g" % dcov.max()
    xg = np.asarray(gpu["x"], np.float64)[ok]
    np.testing.assert_allclose(xg, np.asarray(ref["x"])[ok], rtol=1e-6)
    chig = np.asarray(gpu["chi2"], np.float64)[ok]
    chir = np.asarray(ref["chi2"])[ok]
    dchi = np.abs(chig - chir) / np.maximum(chir, 1.0)
    assert dchi.max() <= CHI2_RTOL, "chi2 mismatch: worst %.3g" % dchi.max()
    np.testing.assert_array_equal(np.asarray(gpu["ndf"])[ok], np.asarray(ref["ndf"])[ok])
    return dict(tracks=T, compared=int(ok.sum()), status_mismatch=mism,
                worst_par=float(dpar.max()) if dpar.size else 0.0,
                worst_cov=float(dcov.max()) if dcov.size else 0.0,
                worst_chi2=float(dchi.max()) if dchi.size else 0.0)
