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
* the track ids are the connected components of the GPU's own links (a
  breadth-first search in the test), and equal the oracle's where the links
  agree; the joint looper circles are within the same tolerances where
  both sides paired the same legs over the same chains;
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
    # the oracle's own chain from the same clusters
    r = parity.oracle_chain(fr, NB, MIN_HITS, FIT, CUT)
    rs, ro = r["seeds"], r["fit"]
    np.testing.assert_array_equal(up.cpu().numpy(), r["up"])
    np.testing.assert_array_equal(dn.cpu().numpy(), r["dn"])
    parity.assert_seeds_equal(seeds.to_numpy(), rs)
    g = _host(tr, T)
    parity.compare_fit(g, ro)
    gn, gp_ = nxt[:T].cpu().numpy(), prv[:T].cpu().numpy()
    gl = leg[:T].cpu().numpy()
    mst = parity.compare_merge(dict(next=gn, prev=gp_, chi2=chi[:T].cpu().numpy(), mpar=mp[:T].cpu().numpy(),
                                    mcov=mc[:T].cpu().numpy(), leg=gl, leg_chi2=lchi[:T].cpu().numpy()), r)
    rn, rp, rl = r["next"], r["prev"], r["leg"]
    print("[refit] %s: %s" % (label, mst), flush=True)
    # refits of the chains both sides built the same way
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
    # heads and members: a segment is a head exactly when its fit succeeded
    # and no counted prev link reaches it (a property of the GPU's own links)
    head = (g["status"] == 0) & (gp_ < 0)
    np.testing.assert_array_equal(gr["status"] != 5, head)
    # track ids: the components of the GPU's own links; equal to the
    # oracle's where both sides linked the same way
    gid = out["track_id"][:T].cpu().numpy()
    np.testing.assert_array_equal(gid, parity.link_components(g["status"], gn, gl))
    if np.array_equal(gn, rn) and np.array_equal(gl, rl) and np.array_equal(g["status"] == 0, ro["status"] == 0):
        np.testing.assert_array_equal(gid, rr["track_id"])
    # joint looper circles of the pairs both sides formed over the same chains
    lg, lr = out["loop_chi2"][:T].cpu().numpy(), rr["loop_chi2"]
    def heads_of(p, i):
        while p[i] >= 0:
            i = p[i]
        return i
    both = np.array([i for i in np.nonzero((lg >= 0) & (lr >= 0))[0]
                     if gl[i] == rl[i] and cg.get(heads_of(gp_, i)) == cr.get(heads_of(rp, i))
                     and cg.get(heads_of(gp_, gl[i])) == cr.get(heads_of(rp, rl[i]))], dtype=np.int64)
    assert ((lg >= 0) != (lr >= 0)).sum() <= max(2, parity.MERGE_DIFF * max(int((rl >= 0).sum()), 1))
    if both.size:
        np.testing.assert_allclose(lg[both], lr[both], rtol=1e-2, atol=1e-3)
        _compare_circles(out["loop_par"][:T].cpu().numpy().astype(np.float64)[both], out["loop_cov"][:T].cpu()
                         .numpy().astype(np.float64)[both], rr["loop_par"][both], rr["loop_cov"][both])
    assert not out["loop_par"][:T].cpu().numpy()[lg < 0].any()
    return multi, int(both.size)


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
    # the oracle's own chain, its refit with the same map
    r = parity.oracle_chain(fr, NB, MIN_HITS, FIT, CUT, legs=False)
    parity.assert_seeds_equal(seeds.to_numpy(), r["seeds"])
    gn, gp_ = nxt[:T].cpu().numpy(), prv[:T].cpu().numpy()
    ref = oracle.refit(r["seeds"], r["fit"], r["next"], r["prev"], None, fr.y, fr.z, fr.row_x, fr.n_rows,
                       fr.n_sectors, map_=mp.astype(np.float64), **FIT)
    g = _host(tr, T)
    np.testing.assert_array_equal(out["track_id"][:T].cpu().numpy(), parity.link_components(g["status"], gn))
    gr = _host(out["refit"], T)
    cg = _chains(gn, gp_, np.nonzero(gr["status"] != 5)[0])
    cr = _chains(r["next"], r["prev"], np.nonzero(ref["status"] != 5)[0])
    same = np.array(sorted(h for h in cg if h in cr and cg[h] == cr[h]), dtype=np.int64)
    assert same.size >= 0.995 * max(len(cr), 1) and (gn[same] >= 0).sum() > 100
    parity.compare_fit({k: v[same] for k, v in gr.items()}, {k: v[same] for k, v in ref.items()})


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


def test_chain_longer_than_a_side(torch_dev):
    """Links that chain 19 segments (more than the 18 sectors of a side) are
    refused at the head with TPC_REFIT_LONG_CHAIN, the shorter chain of 18
    is refitted, and every non-head gets TPC_REFIT_NOT_HEAD -- as the
    oracle on its own seeds and fits with the same (test-made) links."""
    import torch
    from paper_2412_13755_amd import _capi as C
    from paper_2412_13755_amd.reco import Reco, RecoConfig
    fr = make_config(1, scale=0.05)
    reco = Reco(RecoConfig(row_x=fr.row_x, n_sectors=fr.n_sectors, min_hits=MIN_HITS, **NB, **FIT), "cuda:0")
    dfr = reco.upload(fr)
    up, dn = reco.neighbours(dfr)
    seeds = reco.seed(dfr, up, dn)
    tr = reco.fit(dfr, seeds)
    torch.cuda.synchronize()
    T = int(seeds.n_seeds.item())
    r = parity.oracle_chain(fr, NB, MIN_HITS, FIT, CUT, legs=False)
    parity.assert_seeds_equal(seeds.to_numpy(), r["seeds"])
    g = _host(tr, T)
    ok = np.nonzero((g["status"] == 0) & (r["fit"]["status"] == 0))[0]
    for length, want in ((19, C.TPC_REFIT_LONG_CHAIN), (18, None)):
        c = ok[:length]
        nxt = np.full(seeds.frame.numel(), -1, np.int32)
        prv = np.full(seeds.frame.numel(), -1, np.int32)
        nxt[c[:-1]], prv[c[1:]] = c[1:], c[:-1]
        out = reco.refit(dfr, seeds, tr, torch.from_numpy(nxt).cuda(), torch.from_numpy(prv).cuda())
        torch.cuda.synchronize()
        st = out["refit"].status[:T].cpu().numpy()
        ref = oracle.refit(r["seeds"], r["fit"], nxt[:T], prv[:T], None, fr.y, fr.z, fr.row_x, fr.n_rows,
                           fr.n_sectors, **FIT)
        both = (g["status"] == 0) == (r["fit"]["status"] == 0)
        np.testing.assert_array_equal(st[both], ref["status"][both])
        assert np.all(st[c[1:]] == C.TPC_REFIT_NOT_HEAD)
        if want is not None:
            assert st[c[0]] == want
        else:
            assert st[c[0]] != C.TPC_REFIT_LONG_CHAIN and out["refit"].ndf[c[0]].item() == ref["ndf"][c[0]]
        np.testing.assert_array_equal(out["track_id"][:T].cpu().numpy(), parity.link_components(g["status"], nxt[:T]))
