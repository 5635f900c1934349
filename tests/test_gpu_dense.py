"""GPU parity on the continuous-readout time frame at full size: 50
collisions spread over a 100 us drift window, 5x10^5 tracks, 6.4x10^7
clusters, every pad row holding 4x10^3 to 1.7x10^4 clusters (the regime
where neighbouring rows are searched in z-sorted slabs staged through LDS).

The whole frame is reconstructed on the GPU in the launch form the bench
times.  Two full-density sectors (one per side of the central membrane) are
checked against the oracle exactly: reconstruction within a sector reads no
other sector, so their links and seeds are those of the oracle on that
sector alone (bit-exact), and their fitted tracks must agree within the fit
tolerance.  Every link and seed of the frame is checked against properties
that hold at any size.  The persistent form must reproduce the staged form
bit for bit.
"""
import os

import numpy as np
import pytest

from tests import parity
from tests.conftest import NB, FIT, MIN_HITS

pytestmark = pytest.mark.gpu

SECTORS = (7, 26)


@pytest.fixture(scope="module")
def frame():
    import torch
    from tpcsynth import make_config
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    print("[dense] generating the continuous-readout frame", flush=True)
    fr = make_config(2)
    print("[dense] %d clusters" % fr.n_clusters, flush=True)
    return fr


@pytest.fixture(scope="module")
def staged(frame):
    import torch
    from paper_2412_13755_amd.reco import Reco, RecoConfig
    reco = Reco(RecoConfig(row_x=frame.row_x, n_sectors=frame.n_sectors, min_hits=MIN_HITS, **NB, **FIT),
                "cuda:0")
    dfr = reco.upload(frame)
    up, dn, seeds, tracks = reco.reconstruct(dfr, "staged")
    torch.cuda.synchronize()
    assert int(seeds.status.item()) == 0
    sd = seeds.to_numpy()
    T = len(sd["offsets"]) - 1
    tr = {k: getattr(tracks, k)[:T].cpu().numpy() for k in ("x", "par", "cov", "chi2", "ndf", "status")}
    return reco, dfr, up.cpu().numpy(), dn.cpu().numpy(), sd, tr


def test_rows_are_dense(frame):
    n = np.diff(frame.row_offsets)
    assert frame.n_clusters > 6e7
    assert (n > 4096).all() and n.max() > 16000


def test_frame_invariants(frame, staged):
    _, _, up, dn, sd, _ = staged
    linked = parity.check_link_invariants(frame.row_offsets, frame.n_rows, up, dn)
    T = parity.check_seed_invariants(frame.row_offsets, frame.n_sectors, frame.n_rows, sd, MIN_HITS)
    print("[dense] %d linked clusters, %d seeds" % (linked, T), flush=True)
    assert linked > 0.8 * frame.n_clusters and T > 10 ** 6


@pytest.mark.parametrize("s", SECTORS)
def test_sector_matches_oracle(frame, staged, s):
    import oracle
    oracle.set_threads(min(16, len(os.sched_getaffinity(0))))
    _, _, up, dn, sd, tr = staged
    st = parity.check_sector(frame, s, up, dn, sd, tr, NB, MIN_HITS, FIT)
    print("[dense] sector %d: %s" % (s, st), flush=True)
    assert st["clusters"] > 10 ** 6 and st["fit"]["compared"] > 5 * 10 ** 4


def test_persistent_matches_staged(frame, staged):
    import torch
    reco, dfr, up, dn, sd, tr = staged
    pu, pd, ps, pt = reco.reconstruct(dfr, "persistent")
    torch.cuda.synchronize()
    assert int(ps.status.item()) == 0
    np.testing.assert_array_equal(pu.cpu().numpy(), up)
    np.testing.assert_array_equal(pd.cpu().numpy(), dn)
    parity.assert_seeds_equal(ps.to_numpy(), sd)
    T = len(sd["offsets"]) - 1
    for k in ("par", "cov", "chi2", "status"):
        np.testing.assert_array_equal(getattr(pt, k)[:T].cpu().numpy(), tr[k], err_msg=k)
