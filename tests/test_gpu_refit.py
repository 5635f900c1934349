"""GPU parity of the assembly of tracks and their refit over all hits
(tpc_track_refit through the C-ABI), and of the merging links it reads,
against the oracle's own chain: the oracle finds its neighbours, seeds,
fits (float64), merges and pairs looper legs, and refits, all from the
same clusters; the GPU does the same in its kernels.

* links and seeds are bit-exact; a merging link or leg pairing may differ
  only where the decision is marginal (the GPU compares chi2 of float fits
  with the cut, the oracle of float64 fits): at most 0.2 % of the links;
* on links that agree the link chi2 and the combined pair state are within
  the fit tolerances; each chain that is the same on both sides is
  refitted within the fit tolerances (parameters 1e-4 relative with
  floors, covariance 1e-3 of the standard deviations, chi2 1e-3); heads,
  members and ndf equal;
* the track ids equal the oracle's component ids of the GPU's own links
  (integers, exact), and so do the refits of every chain against the
  oracle refitting the GPU's chains; the joint looper circles are within
  the same tolerances where both sides formed them;
* on 64 uneven frames (no link crosses a frame) and on one sector (no
  links: every refit is its seed fit)."""
import numpy as np
import pytest

import oracle
from tests.conftest import NB, FIT, MIN_HITS
from tests import parity
from tpcsynth import make_config

pytestmark = pytest.mark.gpu
CUT = 30.0
MAX_LINK_DIFF = 2e-3


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _host(tr, T):
    return {k: getattr(tr, k)[:T].cpu().numpy() for k in ("x", "par", "cov", "chi2", "ndf", "status")}


def _chains(nxt, prv, heads):
    out = {}
    for h in heads:
        c, s = [], h
        while s >= 0 and len(c) < 19:
            c.append(int(s))
            s = nxt[s]
        out[int(h)] = tuple(c)
    return out


def _compare_circles(gp, gc, rp, rc):
    tol = parity.PAR_RTOL * np.maximum(np.abs(rp), np.array([1.0, 1.0, 1e-4, 1e-2]))
    assert not (np.abs(gp - rp) > tol).any(), np.abs(gp - rp).max(axis=0)
    C1 = np.zeros((len(gc), 4, 4))
    C2 = np.zeros_like(C1)
    q = 0
    for a in range(4):
        for b in range(a + 1):
            C1[:, a, b] = C1[:, b, a] = gc[:, q]
            C2[:, a, b] = C2[:, b, a] = rc[:, q]
            q += 1
    sd = np.sqrt(np.einsum("tii->ti", C2))
    assert (np.abs(C1 - C2) / (sd[:, :, None] * sd[:, None, :])).max() <= parity.COV_RTOL


def check(fr, label, expect_links=True):
    import torch
    from paper_2412_13755_amd.reco import Reco, RecoConfig
    print("[refit] %s: N=%d frames=%d" % (label, fr.n_clusters, fr.n_frames), flush=True)
    reco = Reco(RecoConfig(row_x=fr.row_x, n_sectors=fr.n_sectors, min_hits=MIN_HITS, **NB, **FIT), "cuda:0")
    dfr = reco.upload(fr)
    up, dn = reco.neighbours(dfr)
    seeds = reco.seed(dfr, up, dn)
    tr = reco.fit(dfr, seeds)
    nxt, prv, chi, mp, mc, leg, lchi = reco.merge(seeds, tr, CUT)
    out = reco.refit(dfr, seeds, tr, nxt, prv, leg)
    torch.cuda.synchronize()
    T = int(seeds.n_seeds.item())
    # the oracle's own chain
    ru, rd = oracle.neighbours(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)
    np.testing.assert_array_equal(up.cpu().numpy(), ru)
    np.testing.assert_array_equal(dn.cpu().numpy(), rd)
    rs = oracle.ca_seed(fr.row_offsets, ru, rd, fr.n_sectors, fr.n_rows, MIN_HITS)
    parity.assert_seeds_equal(seeds.to_numpy(), rs)
    ro = oracle.fit(rs, fr.y, fr.z, fr.row_x, fr.n_rows, **FIT)
    g = _host(tr, T)
    parity.compare_fit(g, ro)
    rn, rp, rc, rmp, rmc = oracle.merge(ro, rs["frame"], rs["sector"], fr.n_sectors, bz=FIT["bz"],
                                        max_sin=FIT["max_sin"], cut=CUT)
    rl, rlc = oracle.legs(ro, rs["frame"], rs["sector"], fr.n_sectors, bz=FIT["bz"], cut=CUT)
    gn, gp_, gc = nxt[:T].cpu().numpy(), prv[:T].cpu().numpy(), chi[:T].cpu().numpy()
    gl, glc = leg[:T].cpu().numpy(), lchi[:T].cpu().numpy()
    # merging decisions: equal but for marginal ones
    dn_ = int((gn != rn).sum())
    dl_ = int((gl != rl).sum())
    nl = max(int((rn >= 0).sum()), 1)
    print("[refit] %s: seeds %d links %d (differ %d) legs %d (differ %d)" % (
        label, T, int((rn >= 0).sum()), dn_, int((rl >= 0).sum()) // 2, dl_), flush=True)
    assert dn_ <= max(2, MAX_LINK_DIFF * nl) and dl_ <= max(2, MAX_LINK_DIFF * nl)
    L = (gn == rn) & (rn >= 0)
    np.testing.assert_allclose(gc[L], rc[L], rtol=parity.CHI2_RTOL * 10, atol=1e-4)
    gmp, gmc = mp[:T].cpu().numpy().astype(np.float64), mc[:T].cpu().numpy().astype(np.float64)
    tol = 10 * parity.PAR_RTOL * np.maximum(np.abs(rmp[L]), parity.PAR_FLOOR)
    assert not (np.abs(gmp[L] - rmp[L]) > tol).any(), np.abs(gmp[L] - rmp[L]).max(axis=0)
    P = (gl == rl) & (rl >= 0)
    np.testing.assert_allclose(glc[P], rlc[P], rtol=parity.CHI2_RTOL * 10, atol=1e-4)
    # refits of the oracle's own chains where both sides built the same chain
    rr = oracle.refit(rs, ro, rn, rp, rl, fr.y, fr.z, fr.row_x, fr.n_rows, fr.n_sectors, **FIT)
    gr = _host(out["refit"], T)
    hg = np.nonzero(gr["status"] != 5)[0]
    hr = np.nonzero(rr["status"] != 5)[0]
    cg, cr = _chains(gn, gp_, hg), _chains(rn, rp, hr)
    same = np.array(sorted(h for h in cg if h in cr and cg[h] == cr[h]), dtype=np.int64)
    assert same.size >= 0.995 * max(len(cr), 1)
    np.testing.assert_array_equal(gr["ndf"][same], rr["ndf"][same])
    st = parity.compare_fit({k: v[same] for k, v in gr.items()}, {k: v[same] for k, v in rr.items()})
    multi = int((gn[same] >= 0).sum())
    print("[refit] %s: chains %d (multi-segment %d) refits compared %d, worst par %.2g cov %.2g" % (
        label, len(cr), multi, st["compared"], st["worst_par"], st["worst_cov"]), flush=True)
    if expect_links:
        assert multi > 500
    # the GPU's own links through the oracle: ids exact, every chain within tolerance
    ro_g = {k: v.astype(np.float64) if v.dtype.kind == "f" else v for k, v in g.items()}
    rr2 = oracle.refit(rs, ro_g, gn, gp_, gl, fr.y, fr.z, fr.row_x, fr.n_rows, fr.n_sectors, **FIT)
    np.testing.assert_array_equal(out["track_id"][:T].cpu().numpy(), rr2["track_id"])
    np.testing.assert_array_equal(gr["status"] == 5, rr2["status"] == 5)
    parity.compare_fit(gr, rr2)
    lg = out["loop_chi2"][:T].cpu().numpy()
    lr = rr2["loop_chi2"]
    both = (lg >= 0) & (lr >= 0)
    assert (lg >= 0).sum() - both.sum() <= max(1, 1e-3 * len(lg))
    assert (lr >= 0).sum() - both.sum() <= max(1, 1e-3 * len(lg))
    if both.any():
        np.testing.assert_allclose(lg[both], lr[both], rtol=1e-2, atol=1e-3)
        _compare_circles(out["loop_par"][:T].cpu().numpy().astype(np.float64)[both], out["loop_cov"][:T].cpu()
                         .numpy().astype(np.float64)[both], rr2["loop_par"][both], rr2["loop_cov"][both])
    assert not out["loop_par"][:T].cpu().numpy()[lg < 0].any()
    return multi, int(both.sum())


def test_headline_event(torch_dev):
    multi, loops = check(make_config(1), "full-tpc-event-1e4")
    assert loops > 200


def test_uneven_frames(torch_dev):
    check(make_config(3, scale=0.02), "batched-64-uneven x0.02")


def test_single_sector_refits_are_seed_fits(torch_dev):
    multi, loops = check(make_config(0), "single sector", expect_links=False)
    assert multi == 0 and loops == 0


def test_refit_with_map_and_without_legs(torch_dev):
    import torch
    from paper_2412_13755_amd.reco import Reco, RecoConfig
    fr = make_config(1, scale=0.2)
    reco = Reco(RecoConfig(row_x=fr.row_x, n_sectors=fr.n_sectors, min_hits=MIN_HITS, **NB, **FIT), "cuda:0")
    dfr = reco.upload(fr)
    up, dn = reco.neighbours(dfr)
    seeds = reco.seed(dfr, up, dn)
    tr = reco.fit(dfr, seeds)
    nxt, prv, *_ = reco.merge(seeds, tr, CUT, legs=False)
    rng = np.random.default_rng(9)
    mp = rng.normal(0, 0.05, (fr.n_sectors, fr.n_rows, 2)).astype(np.float32)
    out = reco.refit(dfr, seeds, tr, nxt, prv, None, torch.from_numpy(mp).to("cuda:0"))
    torch.cuda.synchronize()
    assert "loop_par" not in out
    T = int(seeds.n_seeds.item())
    sd = seeds.to_numpy()
    g = _host(tr, T)
    ref = oracle.refit(sd, g, nxt[:T].cpu().numpy(), prv[:T].cpu().numpy(), None, fr.y, fr.z, fr.row_x,
                       fr.n_rows, fr.n_sectors, map_=mp.astype(np.float64), **FIT)
    np.testing.assert_array_equal(out["track_id"][:T].cpu().numpy(), ref["track_id"])
    parity.compare_fit(_host(out["refit"], T), ref)


def test_refit_arguments_refused(torch_dev):
    import ctypes
    import torch
    from paper_2412_13755_amd import _capi as C
    from paper_2412_13755_amd.reco import Reco, RecoConfig
    fr = make_config(0)
    reco = Reco(RecoConfig(row_x=fr.row_x, n_sectors=fr.n_sectors, min_hits=MIN_HITS, **NB, **FIT), "cuda:0")
    dfr = reco.upload(fr)
    up, dn = reco.neighbours(dfr)
    seeds = reco.seed(dfr, up, dn)
    tr = reco.fit(dfr, seeds)
    nxt, prv, chi, mp, mc, leg, lchi = reco.merge(seeds, tr, CUT)
    out = reco.refit(dfr, seeds, tr, nxt, prv, leg)
    sc, gc, rc = seeds.c(), tr.c(), out["refit"].c()
    lib = C.lib()
    # loop outputs without leg links, and a partial set of loop outputs
    st = lib.tpc_track_refit(reco._ctx, ctypes.byref(dfr.c), ctypes.byref(sc), ctypes.byref(gc), nxt.data_ptr(),
                             prv.data_ptr(), None, None, out["track_id"].data_ptr(), ctypes.byref(rc),
                             out["loop_par"].data_ptr(), out["loop_cov"].data_ptr(), out["loop_chi2"].data_ptr(),
                             None)
    assert st == C.TPC_ERR_ARG
    st = lib.tpc_track_refit(reco._ctx, ctypes.byref(dfr.c), ctypes.byref(sc), ctypes.byref(gc), nxt.data_ptr(),
                             prv.data_ptr(), leg.data_ptr(), None, out["track_id"].data_ptr(), ctypes.byref(rc),
                             out["loop_par"].data_ptr(), None, out["loop_chi2"].data_ptr(), None)
    assert st == C.TPC_ERR_ARG
    st = lib.tpc_track_refit(reco._ctx, ctypes.byref(dfr.c), ctypes.byref(sc), ctypes.byref(gc), None,
                             prv.data_ptr(), leg.data_ptr(), None, out["track_id"].data_ptr(), ctypes.byref(rc),
                             None, None, None, None)
    assert st == C.TPC_ERR_ARG
    torch.cuda.synchronize()
