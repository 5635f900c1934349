"""GPU parity of the merging of fitted segments across sector edges and of
the pairing of looper legs (tpc_track_merge through the C-ABI) against the
oracle's own chain from the same clusters (its neighbours, seeds, float64
fits, merge and legs): links and seeds exact, fits within tolerance; the
merging links and leg pairs equal except where a decision is marginal (the
GPU decides on chi2 of float fits, the oracle on float64 fits: at most
0.2 % of the links), the chi2 of agreeing links and pairs and the combined
states within 10x the fit tolerances, the GPU's links mutual.
On the headline event (26 707 seeds, 36 sectors), on 64 uneven frames
(links never cross frames) and on a single sector (no links); the
links-only form writes no leg outputs."""
import numpy as np
import pytest

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


def check(fr, label, legs=True):
    import torch
    from paper_2412_13755_amd.reco import Reco, RecoConfig
    print("[merge] %s: N=%d frames=%d" % (label, fr.n_clusters, fr.n_frames), flush=True)
    reco = Reco(RecoConfig(row_x=fr.row_x, n_sectors=fr.n_sectors, min_hits=MIN_HITS, **NB, **FIT), "cuda:0")
    dfr = reco.upload(fr)
    up, dn = reco.neighbours(dfr)
    seeds = reco.seed(dfr, up, dn)
    tr = reco.fit(dfr, seeds)
    nxt, prv, chi, mp, mc, leg, lchi = reco.merge(seeds, tr, CUT, legs=legs)
    torch.cuda.synchronize()
    T = int(seeds.n_seeds.item())
    r = parity.oracle_chain(fr, NB, MIN_HITS, FIT, CUT, legs=legs)
    np.testing.assert_array_equal(up.cpu().numpy(), r["up"])
    np.testing.assert_array_equal(dn.cpu().numpy(), r["dn"])
    parity.assert_seeds_equal(seeds.to_numpy(), r["seeds"])
    g = {k: getattr(tr, k)[:T].cpu().numpy() for k in ("x", "par", "cov", "chi2", "ndf", "status")}
    parity.compare_fit(g, r["fit"])
    gm = dict(next=nxt[:T].cpu().numpy(), prev=prv[:T].cpu().numpy(), chi2=chi[:T].cpu().numpy(),
              mpar=mp[:T].cpu().numpy(), mcov=mc[:T].cpu().numpy())
    if legs:
        gm.update(leg=leg[:T].cpu().numpy(), leg_chi2=lchi[:T].cpu().numpy())
    else:
        assert leg is None and lchi is None
    st = parity.compare_merge(gm, r)
    print("[merge] %s: %s" % (label, st), flush=True)
    return st


def test_headline_event(torch_dev):
    st = check(make_config(1), "full-tpc-event-1e4")
    assert st["links"] > 5000 and st["leg_pairs"] > 400


def test_headline_event_links_only(torch_dev):
    st = check(make_config(1, scale=0.3), "full-tpc-event-1e4 x0.3, links only", legs=False)
    assert st["links"] > 1000 and "leg_pairs" not in st


def test_uneven_frames(torch_dev):
    st = check(make_config(3, scale=0.02), "batched-64-uneven x0.02")
    assert st["links"] > 1000


def test_single_sector_has_no_links(torch_dev):
    st = check(make_config(0), "single sector")
    assert st["links"] == 0 and st["links_differ"] == 0 and st["segments"] > 50
