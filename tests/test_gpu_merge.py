"""GPU parity of the merging of fitted segments across sector edges
(tpc_track_merge through the C-ABI) against the oracle run on the same
fitted tracks (the GPU fit's float outputs): the links (next, prev) equal,
the chi2 of every link within 1e-6 (relative; the GPU reports it in float),
the combined state of every linked pair within the fit's tolerances, the
pairing of looper legs equal and its chi2 within 1e-6.
On the headline event (26 707 seeds, 36 sectors), on 64 uneven frames
(links never cross frames) and on a single sector (no links)."""
import numpy as np
import pytest

import oracle
from tests.conftest import NB, FIT, MIN_HITS
from tests import parity
from tpcsynth import make_config

pytestmark = pytest.mark.gpu
CUT = 30.0


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def check(fr, label):
    import torch
    from paper_2412_13755_amd.reco import Reco, RecoConfig
    print("[merge] %s: N=%d frames=%d" % (label, fr.n_clusters, fr.n_frames), flush=True)
    reco = Reco(RecoConfig(row_x=fr.row_x, n_sectors=fr.n_sectors, min_hits=MIN_HITS, **NB, **FIT), "cuda:0")
    dfr = reco.upload(fr)
    up, dn = reco.neighbours(dfr)
    seeds = reco.seed(dfr, up, dn)
    tr = reco.fit(dfr, seeds)
    nxt, prv, chi, mp, mc, leg, lchi = reco.merge(seeds, tr, CUT)
    torch.cuda.synchronize()
    T = int(seeds.n_seeds.item())
    g = {k: getattr(tr, k)[:T].cpu().numpy() for k in ("x", "par", "cov", "status")}
    frame = seeds.frame[:T].cpu().numpy()
    sector = seeds.sector[:T].cpu().numpy()
    key = frame.astype(np.int64) * fr.n_sectors + sector
    assert np.all(np.diff(key) >= 0)
    rn, rp, rc, rmp, rmc = oracle.merge({k: v.astype(np.float64) for k, v in g.items()}, frame, sector, fr.n_sectors,
                              bz=FIT["bz"], max_sin=FIT["max_sin"], cut=CUT)
    gn, gp, gc = nxt[:T].cpu().numpy(), prv[:T].cpu().numpy(), chi[:T].cpu().numpy()
    np.testing.assert_array_equal(gn, rn)
    np.testing.assert_array_equal(gp, rp)
    L = rn >= 0
    np.testing.assert_allclose(gc[L], rc[L], rtol=1e-6)
    assert np.all(gc[~L] == 0)
    # the combined states of linked pairs: the fit tolerances (reading of the fit parity)
    gmp, gmc = mp[:T].cpu().numpy().astype(np.float64), mc[:T].cpu().numpy().astype(np.float64)
    assert not gmp[~L].any() and not gmc[~L].any()
    tol = parity.PAR_RTOL * np.maximum(np.abs(rmp[L]), parity.PAR_FLOOR)
    assert not (np.abs(gmp[L] - rmp[L]) > tol).any(), np.abs(gmp[L] - rmp[L]).max()
    if L.any():
        C1, C2 = oracle.unpack_cov(gmc[L]), oracle.unpack_cov(rmc[L])
        sd_ = np.sqrt(np.einsum("tii->ti", C2))
        assert (np.abs(C1 - C2) / (sd_[:, :, None] * sd_[:, None, :])).max() <= parity.COV_RTOL
    # the legs of loopers
    rl, rlc = oracle.legs({k: v.astype(np.float64) for k, v in g.items()}, frame, sector, fr.n_sectors,
                          bz=FIT["bz"], cut=CUT)
    gl, glc = leg[:T].cpu().numpy(), lchi[:T].cpu().numpy()
    np.testing.assert_array_equal(gl, rl)
    P = rl >= 0
    np.testing.assert_allclose(glc[P], rlc[P], rtol=1e-6)
    assert np.all(glc[~P] == 0)
    print("[merge] %s: seeds %d links %d looper legs paired %d" % (label, T, int(L.sum()), int(P.sum()) // 2),
          flush=True)
    return int(L.sum()), T


def test_headline_event(torch_dev):
    links, T = check(make_config(1), "full-tpc-event-1e4")
    assert links > 5000


def test_uneven_frames(torch_dev):
    links, T = check(make_config(3, scale=0.02), "batched-64-uneven x0.02")
    assert links > 1000


def test_single_sector_has_no_links(torch_dev):
    links, T = check(make_config(0), "single sector")
    assert links == 0 and T > 50
