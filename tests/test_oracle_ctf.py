"""Pins of the oracle's track-model residual transform (the flat integer
arrays a time frame is reduced to before entropy coding, Sec. 4.1).

The transform must be lossless up to the quantisation: an inverse written
here from the arrays' definitions (not from the oracle's code) rebuilds, for
every (frame, sector, pad row), exactly the multiset of quantised (y, z) of
its clusters -- every cluster once, whether it lies on a track or not.
"""
import numpy as np
import pytest

import oracle
from tests.conftest import NB, FIT, MIN_HITS
from tpcsynth import make_config

Q = 0.01


def _quant(v, q):
    s = np.asarray(v, np.float32) * np.float32(1.0 / q)
    ok = np.isfinite(s) & (s > -2.0**30) & (s < 2.0**30)
    return np.where(ok, np.rint(np.where(ok, s, 0)), 0).astype(np.int64)


def _inverse(a, n_rows, NR):
    """segment -> sorted list of (qy, qz) from the arrays alone"""
    out = {s: [] for s in range(NR)}
    h = 0                              # cursor into hit_drow
    g = 0                              # cursor into hit_ry / hit_rz
    for t in range(a["trk_seg"].size):
        m = int(a["trk_n"][t])
        if m == 0:
            continue
        y = [int(a["trk_y0h"][t]) * 256 + int(a["trk_y0l"][t])]
        z = [int(a["trk_z0h"][t]) * 256 + int(a["trk_z0l"][t])]
        r = [int(a["trk_row0"][t])]
        for k in range(1, m):
            r.append(r[-1] + 1 + int(a["hit_drow"][h]))
            h += 1
            if k == 1:
                y.append(y[0] + int(a["trk_dy1"][t]))
                z.append(z[0] + int(a["trk_dz1"][t]))
            else:
                y.append(int(a["hit_ry"][g]) + 2 * y[-1] - y[-2])
                z.append(int(a["hit_rz"][g]) + 2 * z[-1] - z[-2])
                g += 1
        base = int(a["trk_seg"][t]) * n_rows
        for k in range(m):
            out[base + r[k]].append((y[k], z[k]))
    assert h == a["hit_drow"].size and g == a["hit_ry"].size == a["hit_rz"].size
    f = 0
    for s in range(NR):
        for _ in range(int(a["seg_nfree"][s])):
            out[s].append((int(a["free_yh"][f]) * 256 + int(a["free_yl"][f]),
                           int(a["free_zh"][f]) * 256 + int(a["free_zl"][f])))
            f += 1
    assert f == a["free_yh"].size
    return {s: sorted(v) for s, v in out.items()}


def _frame_arrays(fr, gate=25.0, max_miss=3):
    up, dn = oracle.neighbours(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)
    sd = oracle.ca_seed(fr.row_offsets, up, dn, fr.n_sectors, fr.n_rows, MIN_HITS)
    fo = oracle.follow(sd, fr.row_offsets, fr.y, fr.z, fr.row_x, fr.n_sectors, fr.n_rows,
                       gate=gate, max_miss=max_miss, **FIT)
    a = oracle.ctf_build(fr.row_offsets, fr.y, fr.z, fr.n_sectors, fr.n_rows, fo["rows"],
                         fo["status"], sd["frame"], sd["sector"], Q, Q)
    return a, fo


@pytest.mark.parametrize("k,scale", [(0, 1.0), (1, 0.15), (3, 0.01)])
def test_inverse_rebuilds_every_segment(k, scale):
    fr = make_config(k, scale=scale, hit_eff=0.97)
    a, fo = _frame_arrays(fr)
    NR = fr.row_offsets.size - 1
    got = _inverse(a, fr.n_rows, NR)
    qy, qz = _quant(fr.y, Q), _quant(fr.z, Q)
    for s in range(NR):
        c0, c1 = fr.row_offsets[s], fr.row_offsets[s + 1]
        assert got[s] == sorted(zip(qy[c0:c1].tolist(), qz[c0:c1].tolist())), s
    assert a["trk_seg"].size == int((fo["status"] == 0).sum())
    # clusters on tracks are coded as residuals, not as raw values
    assert a["free_yh"].size < fr.n_clusters // 4


def test_non_finite_and_far_values_quantise_to_zero():
    fr = make_config(0)
    y, z = fr.y.copy(), fr.z.copy()
    y[:3] = [np.nan, np.inf, 3e7]
    z[3:5] = [-np.inf, -5e8]
    fr.y, fr.z = y, z
    a, _ = _frame_arrays(fr)
    got = _inverse(a, fr.n_rows, fr.row_offsets.size - 1)
    flat = sorted(p for v in got.values() for p in v)
    want = sorted(zip(_quant(y, Q).tolist(), _quant(z, Q).tolist()))
    assert flat == want


def test_residuals_are_small_on_tracks():
    # smeared helices: the second difference over one pad pitch is the
    # measurement noise, sqrt(6) sigma, far below a row's raw coordinate range
    fr = make_config(1, scale=0.1)
    a, _ = _frame_arrays(fr)
    assert np.std(a["hit_ry"]) < 4 * np.sqrt(6) * fr.sigma_y / Q
    assert np.std(a["hit_rz"]) < 4 * np.sqrt(6) * fr.sigma_z / Q
    assert np.mean(a["hit_drow"] == 0) > 0.95
