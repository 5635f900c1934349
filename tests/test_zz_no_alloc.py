"""tpc_ca_seed_noalloc (seeding with the library's built-in device scratch,
no allocation in the call) against tpc_ca_seed with a caller workspace:
identical seeds on two calls in a row, the second on a smaller frame (the
scratch keeps the first call's contents), and frames too large for the
scratch refused before anything is enqueued."""
import ctypes

import numpy as np
import pytest

from tests import parity
from tests.conftest import NB, FIT, MIN_HITS

pytestmark = pytest.mark.gpu


def _reco(fr):
    from paper_2412_13755_amd.reco import Reco, RecoConfig
    return Reco(RecoConfig(row_x=fr.row_x, n_sectors=fr.n_sectors, min_hits=MIN_HITS, **NB, **FIT), "cuda:0")


def _both(fr):
    import torch
    reco = _reco(fr)
    dfr = reco.upload(fr)
    up, dn = reco.neighbours(dfr)
    ref = reco.seed(dfr, up, dn)
    got = reco.seed_noalloc(dfr, up, dn, reco.alloc_seeds(dfr))
    torch.cuda.synchronize()
    assert int(ref.status.item()) == 0 and int(got.status.item()) == 0
    a, b = got.to_numpy(), ref.to_numpy()
    parity.assert_seeds_equal(a, b)
    H = len(b["hits"])
    np.testing.assert_array_equal(got.hit_yz[:H].cpu().numpy(), ref.hit_yz[:H].cpu().numpy())
    return len(b["offsets"]) - 1


def test_two_calls_second_smaller():
    from tpcsynth import make_config
    big = make_config(1)
    small = make_config(1, scale=0.3)
    assert small.n_clusters < big.n_clusters
    t1 = _both(big)
    t2 = _both(small)
    print("[noalloc] %d then %d seeds" % (t1, t2), flush=True)
    assert t1 > t2 > 1000


def test_too_large_is_refused():
    import torch
    from paper_2412_13755_amd import _capi as C
    from paper_2412_13755_amd.reco import DeviceFrames
    from tpcsynth import make_config
    fr = make_config(0)
    reco = _reco(fr)
    # a frame header claiming far more clusters than the scratch holds; the
    # size check comes before any use of the pointers
    n = 4_000_000
    off = torch.zeros(fr.n_sectors * fr.n_rows + 1, dtype=torch.int32, device="cuda")
    off[-1] = n
    y = torch.zeros(n, dtype=torch.float32, device="cuda")
    dfr = DeviceFrames(off, y, y, 1)
    up = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    seeds = reco.alloc_seeds(dfr, cap_seeds=16, cap_hits=16)
    sc = seeds.c()
    rc = C.lib().tpc_ca_seed_noalloc(reco._ctx, ctypes.byref(dfr.c), up.data_ptr(), up.data_ptr(),
                                     ctypes.byref(sc), seeds.status.data_ptr(), None)
    assert rc == C.TPC_ERR_WORKSPACE
    assert b"scratch" in C.lib().tpc_last_error()
