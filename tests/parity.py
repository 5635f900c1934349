"""Comparison helpers for GPU-vs-oracle parity (shared by the GPU tests)."""
import numpy as np

import oracle

# per-component floors for the parameter tolerance (y, z in cm; sin phi,
# tan lambda; q/pT in 1/GeV)
PAR_FLOOR = np.array([1.0, 1.0, 1e-2, 1e-2, 1e-2])
PAR_RTOL = 1e-4
COV_RTOL = 1e-3
CHI2_RTOL = 1e-3
SIN_MARGIN = 1e-5      # a status may differ only this close to a direction threshold


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
    side only, and where the oracle reports its fits' closest approach to
    the direction thresholds (``sin_margin``) each such track must have come
    within SIN_MARGIN of one: a decision the two precisions may take
    differently.
    """
    st_g = np.asarray(gpu["status"])
    st_r = np.asarray(ref["status"])
    T = len(st_r)
    mis = (st_g == 0) != (st_r == 0)
    mism = int(np.sum(mis))
    assert mism <= max(1, int(max_fail_frac * T)), "status mismatches: %d of %d" % (mism, T)
    if "sin_margin" in ref and mism:
        m = np.abs(np.asarray(ref["sin_margin"])[mis])
        assert (m <= SIN_MARGIN).all(), "status mismatch away from a threshold: margins %s" % m
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


def sector_results(fr, s, up, dn, seeds, tracks=None, f=0):
    """The GPU results of sector ``s`` of frame ``f`` rebased as a one-sector
    frame (ids minus the sector's first id), in the layout the oracle
    returns for ``fr.sector_view(f, s)``.  Reconstruction within a sector
    reads no other sector, so these are that view's results.  ``seeds`` is
    a dict of host arrays (Seeds.to_numpy()); ``tracks`` a dict of host
    arrays indexed by seed, or None."""
    sv = fr.sector_view(f, s)
    a = fr.first_id(f, s)
    b = a + sv.n_clusters
    gu = np.array(up[a:b], dtype=np.int64)
    gd = np.array(dn[a:b], dtype=np.int64)
    gu[gu >= 0] -= a
    gd[gd >= 0] -= a
    o = np.asarray(seeds["offsets"])
    h = np.asarray(seeds["hits"])
    first = h[o[:-1]] if len(o) > 1 else np.zeros(0, np.int64)
    i0, i1 = np.searchsorted(first, a), np.searchsorted(first, b)
    sd = dict(offsets=o[i0:i1 + 1] - o[i0], hits=h[o[i0]:o[i1]] - a,
              frame=np.zeros(i1 - i0, np.int32), sector=np.zeros(i1 - i0, np.int32),
              first_row=np.asarray(seeds["first_row"])[i0:i1])
    assert np.all(np.asarray(seeds["sector"])[i0:i1] == s) and np.all(np.asarray(seeds["frame"])[i0:i1] == f)
    tr = None if tracks is None else {k: np.asarray(v)[i0:i1] for k, v in tracks.items()}
    return sv, gu.astype(np.int32), gd.astype(np.int32), sd, tr


def check_sector(fr, s, up, dn, seeds, tracks, nb, min_hits, fit_prm, f=0):
    """Oracle on one sector of a frame against the GPU's results for it:
    identical links and seeds, fit within tolerance.  Returns statistics."""
    sv, gu, gd, gs, gt = sector_results(fr, s, up, dn, seeds, tracks, f)
    ru, rd = oracle.neighbours(sv.row_offsets, sv.y, sv.z, sv.n_rows, **nb)
    np.testing.assert_array_equal(gu, ru, err_msg="up links differ in sector %d" % s)
    np.testing.assert_array_equal(gd, rd, err_msg="down links differ in sector %d" % s)
    rs = oracle.ca_seed(sv.row_offsets, ru, rd, 1, sv.n_rows, min_hits)
    assert_seeds_equal(gs, rs)
    st = dict(sector=s, clusters=sv.n_clusters, linked=int((ru >= 0).sum()), seeds=len(rs["offsets"]) - 1)
    if gt is not None:
        rt = oracle.fit(rs, sv.y, sv.z, sv.row_x, sv.n_rows, **fit_prm)
        st["fit"] = compare_fit(gt, rt)
    return st


def check_link_invariants(row_offsets, n_rows, up, dn):
    """Properties of the links that hold at any size: a partner lies in the
    adjacent row of the same (frame, sector), clusters of the first and last
    rows have none, and up and down partners come together."""
    off = np.asarray(row_offsets, np.int64)
    up = np.asarray(up, np.int64)
    dn = np.asarray(dn, np.int64)
    N = off[-1]
    seg = np.repeat(np.arange(off.size - 1), np.diff(off))
    r = seg % n_rows
    has = up >= 0
    assert np.array_equal(has, dn >= 0), "up and down partners must come together"
    assert not has[(r == 0) | (r == n_rows - 1)].any(), "edge rows have no partners"
    assert up.max(initial=-1) < N and dn.max(initial=-1) < N
    assert np.array_equal(seg[up[has]], seg[has] + 1), "up partner not in the next row"
    assert np.array_equal(seg[dn[has]], seg[has] - 1), "down partner not in the previous row"
    return int(has.sum())


def check_seed_invariants(row_offsets, n_sectors, n_rows, seeds, min_hits):
    """Properties of the seeds that hold at any size: at least min_hits
    hits each, one hit per row in consecutive rows of one (frame, sector)
    from first_row up, no cluster in two seeds, seeds ordered by first hit."""
    off = np.asarray(row_offsets, np.int64)
    o = np.asarray(seeds["offsets"], np.int64)
    h = np.asarray(seeds["hits"], np.int64)
    T = len(o) - 1
    ln = np.diff(o)
    assert (ln >= min_hits).all(), "seed shorter than min_hits"
    seg = np.repeat(np.arange(off.size - 1), np.diff(off))
    hs = seg[h]
    inner = np.ones(h.size, bool)
    inner[o[1:] - 1] = False                    # last hit of each seed
    assert np.array_equal(hs[1:][inner[:-1]], hs[:-1][inner[:-1]] + 1), "hits not in consecutive rows"
    first = hs[o[:-1]]
    assert np.array_equal(first % n_rows, np.asarray(seeds["first_row"])), "first_row"
    fs = first // n_rows
    assert np.array_equal(fs % n_sectors, np.asarray(seeds["sector"])), "sector"
    assert np.array_equal(fs // n_sectors, np.asarray(seeds["frame"])), "frame"
    assert np.unique(h).size == h.size, "a cluster in two seeds"
    assert (np.diff(h[o[:-1]]) > 0).all(), "seeds not ordered by first hit"
    return T


def capped_fraction(fr, seeds, mass, gas):
    """Fraction of the inward fit steps whose energy loss in `gas` (density,
    Z/A, mean excitation) would change the momentum by more than 1 % and is
    therefore not applied, evaluated on the generator's true state at the
    step's outer cluster: the share of steps that take the cap branch."""
    o = np.asarray(seeds["offsets"])
    h = np.asarray(seeds["hits"])
    seg = np.repeat(np.arange(len(fr.row_offsets) - 1), np.diff(fr.row_offsets))
    row = seg % fr.n_rows
    capped = total = 0
    for i in range(len(o) - 1):
        hh = h[o[i]:o[i + 1]]
        for k in range(len(hh) - 2, -1, -1):
            a, b = hh[k + 1], hh[k]
            p = np.array([fr.y_true[a], fr.z_true[a], fr.s_true[a], fr.t_true[a], fr.w_true[a]])
            st, w1, _, _, vw = oracle.eloss(p, fr.row_x[row[b]] - fr.row_x[row[a]], mass, gas, 1.0)
            if st:
                continue
            total += 1
            capped += w1 == p[4] and vw == 0.0
    return capped / max(total, 1)


def oracle_chain(fr, nb, min_hits, fit_prm, cut, legs=True):
    """The oracle's own chain on a frame: neighbours, seeds, float64 fits,
    the merging links and (with legs) the pairing of looper legs."""
    ru, rd = oracle.neighbours(fr.row_offsets, fr.y, fr.z, fr.n_rows, **nb)
    rs = oracle.ca_seed(fr.row_offsets, ru, rd, fr.n_sectors, fr.n_rows, min_hits)
    ro = oracle.fit(rs, fr.y, fr.z, fr.row_x, fr.n_rows, **fit_prm)
    rn, rp, rc, rmp, rmc = oracle.merge(ro, rs["frame"], rs["sector"], fr.n_sectors, bz=fit_prm["bz"],
                                        max_sin=fit_prm["max_sin"], cut=cut)
    out = dict(up=ru, dn=rd, seeds=rs, fit=ro, next=rn, prev=rp, chi2=rc, mpar=rmp, mcov=rmc)
    if legs:
        out["leg"], out["leg_chi2"] = oracle.legs(ro, rs["frame"], rs["sector"], fr.n_sectors, bz=fit_prm["bz"],
                                                  cut=cut)
    return out


MERGE_DIFF = 2e-3       # share of the links a marginal decision may change


def compare_merge(g, r):
    """Merging of the GPU's chain (dict: next, prev, chi2, mpar, mcov and
    optionally leg, leg_chi2; host arrays) against the oracle's own chain
    (oracle_chain).  The GPU compares chi2 of float fits with the cut, the
    oracle of float64 fits, so a link or pairing may differ where that
    decision is marginal: at most MERGE_DIFF of the links.  Where they agree
    the chi2 is within 10x the fit's chi2 tolerance and the combined state
    within 10x the fit tolerances.  Returns statistics."""
    gn, gp = np.asarray(g["next"]), np.asarray(g["prev"])
    rn = np.asarray(r["next"])
    T = rn.size
    nl = max(int((rn >= 0).sum()), 1)
    # the GPU's links are mutual
    L = np.nonzero(gn >= 0)[0]
    np.testing.assert_array_equal(gp[gn[L]], L)
    assert (gp >= 0).sum() == L.size
    dn_ = int((gn != rn).sum())
    assert dn_ <= max(2, MERGE_DIFF * nl), "links differ at %d of %d" % (dn_, nl)
    A = (gn == rn) & (rn >= 0)
    gc = np.asarray(g["chi2"], np.float64)
    np.testing.assert_allclose(gc[A], r["chi2"][A], rtol=10 * CHI2_RTOL, atol=1e-4)
    assert np.all(gc[gn < 0] == 0)
    gmp, gmc = np.asarray(g["mpar"], np.float64), np.asarray(g["mcov"], np.float64)
    tol = 10 * PAR_RTOL * np.maximum(np.abs(r["mpar"][A]), PAR_FLOOR)
    assert not (np.abs(gmp[A] - r["mpar"][A]) > tol).any(), np.abs(gmp[A] - r["mpar"][A]).max(axis=0)
    if A.any():
        C1, C2 = oracle.unpack_cov(gmc[A]), oracle.unpack_cov(r["mcov"][A])
        sd_ = np.sqrt(np.einsum("tii->ti", C2))
        assert (np.abs(C1 - C2) / (sd_[:, :, None] * sd_[:, None, :])).max() <= 10 * COV_RTOL
    assert not gmp[gn < 0].any() and not gmc[gn < 0].any()
    st = dict(segments=T, links=int((rn >= 0).sum()), links_differ=dn_)
    if "leg" in g and g["leg"] is not None:
        gl, rl = np.asarray(g["leg"]), np.asarray(r["leg"])
        P = np.nonzero(gl >= 0)[0]
        np.testing.assert_array_equal(gl[gl[P]], P)
        dl_ = int((gl != rl).sum())
        assert dl_ <= max(2, MERGE_DIFF * nl), "leg pairs differ at %d" % dl_
        B = (gl == rl) & (rl >= 0)
        glc = np.asarray(g["leg_chi2"], np.float64)
        np.testing.assert_allclose(glc[B], r["leg_chi2"][B], rtol=10 * CHI2_RTOL, atol=1e-4)
        assert np.all(glc[gl < 0] == 0)
        st.update(leg_pairs=int((rl >= 0).sum()) // 2, legs_differ=dl_)
    return st


def link_components(status, nxt, leg=None):
    """Connected components of the segments of status 0 under the mutual
    next/prev and leg links (breadth-first search), each named by its
    smallest segment; -1 for the others."""
    from collections import deque
    status = np.asarray(status)
    nxt = np.asarray(nxt)
    T = status.size
    adj = [[] for _ in range(T)]
    for i in range(T):
        for j in (nxt[i], -1 if leg is None else np.asarray(leg)[i]):
            if j >= 0 and status[i] == 0 and status[j] == 0:
                adj[i].append(int(j))
                adj[j].append(i)
    out = np.full(T, -1, np.int64)
    for s in range(T):
        if status[s] != 0 or out[s] >= 0:
            continue
        comp, dq = [s], deque([s])
        out[s] = s
        while dq:
            u = dq.popleft()
            for v in adj[u]:
                if out[v] < 0:
                    out[v] = s
                    comp.append(v)
                    dq.append(v)
        out[comp] = min(comp)
    return out
