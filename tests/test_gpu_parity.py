"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

Links and seeds must be identical (bit-exact integer output); fitted tracks
must agree with the float64 oracle on the same seeds within 1e-4 relative on
parameters (floors 1 cm, 1 cm, 1e-2, 1e-2, 1e-2 /GeV), 1e-3 on covariance
(relative to sqrt(C_ii C_jj)) and 1e-3 on chi2.
"""
import json
import os

import numpy as np
import pytest

import oracle
from tests.conftest import NB, MIN_HITS, FIT
from tests import parity
from tpcsynth import make_config, make_frames

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def make_reco(fr, n_sectors=None):
    from paper_2412_13755_amd.reco import Reco, RecoConfig
    cfg = RecoConfig(row_x=fr.row_x, n_sectors=fr.n_sectors if n_sectors is None else n_sectors,
                     min_hits=MIN_HITS, **NB, **FIT)
    return Reco(cfg, "cuda:0")


def run_gpu(fr):
    import torch
    reco = make_reco(fr)
    dfr = reco.upload(fr)
    up, dn = reco.neighbours(dfr)
    seeds = reco.seed(dfr, up, dn)
    tracks = reco.fit(dfr, seeds)
    torch.cuda.synchronize()
    assert int(seeds.status.item()) == 0
    sd = seeds.to_numpy()
    T = len(sd["offsets"]) - 1
    tr = dict(x=tracks.x[:T].cpu().numpy(), par=tracks.par[:T].cpu().numpy(),
              cov=tracks.cov[:T].cpu().numpy(), chi2=tracks.chi2[:T].cpu().numpy(),
              ndf=tracks.ndf[:T].cpu().numpy(), status=tracks.status[:T].cpu().numpy())
    return up.cpu().numpy(), dn.cpu().numpy(), sd, tr


def run_oracle(fr):
    up, dn = oracle.neighbours(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)
    sd = oracle.ca_seed(fr.row_offsets, up, dn, fr.n_sectors, fr.n_rows, MIN_HITS)
    tr = oracle.fit(sd, fr.y, fr.z, fr.row_x, fr.n_rows, **FIT)
    return up, dn, sd, tr


def check_all(fr, label):
    print("[parity] %s: N=%d" % (label, fr.n_clusters), flush=True)
    gu, gd, gs, gt = run_gpu(fr)
    ru, rd, rs, rt = run_oracle(fr)
    np.testing.assert_array_equal(gu, ru, err_msg="up links differ")
    np.testing.assert_array_equal(gd, rd, err_msg="down links differ")
    parity.assert_seeds_equal(gs, rs)
    stats = parity.compare_fit(gt, rt)
    print("[parity] %s: %s" % (label, stats), flush=True)
    return stats


def test_single_sector_workload(torch_dev):
    fr = make_config(0)
    st = check_all(fr, "single-sector-200")
    assert st["tracks"] > 20


def test_full_tpc_event(torch_dev):
    fr = make_config(1)
    st = check_all(fr, "full-tpc-event-1e4")
    assert st["tracks"] > 10000


def test_batched_frames_scaled(torch_dev):
    fr = make_config(3, scale=0.02)
    assert fr.n_frames == 64
    check_all(fr, "batched-64-uneven x0.02")


def test_continuous_tf_scaled(torch_dev):
    """Dense rows (many candidates per window) at 5% of the track count."""
    fr = make_config(2, scale=0.05)
    check_all(fr, "continuous-tf x0.05")


def test_quantised_ties_and_nan(torch_dev):
    """Coarse grid: exact score ties everywhere; NaN and inf sprinkled in."""
    rng = np.random.default_rng(1)
    n_rows = 9
    counts = rng.integers(0, 40, n_rows)
    off = np.zeros(n_rows + 1, np.int32)
    np.cumsum(counts, out=off[1:])
    n = int(off[-1])
    y = (np.round(rng.uniform(-3, 3, n) * 8) / 8).astype(np.float32)
    z = (np.round(rng.uniform(-3, 3, n) * 8) / 8).astype(np.float32)
    y[::13] = np.nan
    z[5::17] = np.inf

    class F:
        pass
    fr = F()
    fr.row_offsets, fr.y, fr.z, fr.n_frames, fr.n_sectors, fr.n_rows = off, y, z, 1, 1, n_rows
    fr.row_x = np.linspace(85, 93, n_rows).astype(np.float32)
    reco = make_reco(fr)
    dfr = reco.upload(fr)
    up, dn = reco.neighbours(dfr)
    ru, rd = oracle.neighbours(off, y, z, n_rows, **NB)
    np.testing.assert_array_equal(up.cpu().numpy(), ru)
    np.testing.assert_array_equal(dn.cpu().numpy(), rd)
    seeds = reco.seed(dfr, up, dn)
    rs = oracle.ca_seed(off, ru, rd, 1, n_rows, MIN_HITS)
    parity.assert_seeds_equal(seeds.to_numpy(), rs)


def test_golden_neighbour_cases(torch_dev):
    path = os.path.join(os.path.dirname(__file__), "golden", "neighbour_cases.json")
    with open(path) as f:
        d = json.load(f)
    for case in d["cases"]:
        rows = case["rows"]
        n_rows = len(rows)
        off = np.zeros(n_rows + 1, np.int32)
        np.cumsum([len(r) for r in rows], out=off[1:])

        class F:
            pass
        fr = F()
        fr.row_offsets = off
        fr.y = np.array([float(c[0]) for r in rows for c in r], dtype=np.float32)
        fr.z = np.array([float(c[1]) for r in rows for c in r], dtype=np.float32)
        fr.n_frames, fr.n_sectors, fr.n_rows = 1, 1, n_rows
        fr.row_x = np.arange(85, 85 + n_rows, dtype=np.float32)
        reco = make_reco(fr)
        up, dn = reco.neighbours(reco.upload(fr))
        assert up.cpu().numpy().tolist() == case["up"], case["name"]
        assert dn.cpu().numpy().tolist() == case["dn"], case["name"]


def test_empty_frame_and_empty_rows(torch_dev):
    import torch
    fr = make_config(0)
    # keep only every third row populated
    seg = np.repeat(np.arange(fr.n_rows), np.diff(fr.row_offsets))
    keep = (seg % 3) == 0
    fr2 = make_config(0)
    fr2.y, fr2.z = fr.y[keep], fr.z[keep]
    cnt = np.bincount(seg[keep], minlength=fr.n_rows)
    fr2.row_offsets = np.r_[0, np.cumsum(cnt)].astype(np.int32)
    gu, gd, gs, gt = run_gpu(fr2)
    assert np.all(gu == -1) and np.all(gd == -1) and len(gs["offsets"]) == 1
    # no clusters at all
    fr3 = make_config(0)
    fr3.y = fr3.y[:0]
    fr3.z = fr3.z[:0]
    fr3.row_offsets = np.zeros_like(fr.row_offsets)
    reco = make_reco(fr3)
    dfr = reco.upload(fr3)
    up, dn = reco.neighbours(dfr)
    seeds = reco.seed(dfr, up, dn)
    tracks = reco.fit(dfr, seeds)
    torch.cuda.synchronize()
    assert int(seeds.n_seeds.item()) == 0 and int(seeds.status.item()) == 0


def test_capacity_overflow_reports_required_size(torch_dev):
    import torch
    fr = make_config(0)
    reco = make_reco(fr)
    dfr = reco.upload(fr)
    up, dn = reco.neighbours(dfr)
    full = reco.seed(dfr, up, dn)
    torch.cuda.synchronize()
    ns, nh = int(full.n_seeds.item()), int(full.n_hits.item())
    small = reco.alloc_seeds(dfr, cap_seeds=ns // 2, cap_hits=nh)
    reco.seed(dfr, up, dn, seeds=small)
    torch.cuda.synchronize()
    from paper_2412_13755_amd._capi import TPC_ERR_CAPACITY
    assert int(small.status.item()) == TPC_ERR_CAPACITY
    assert int(small.n_seeds.item()) == ns and int(small.n_hits.item()) == nh
    # the stored prefix is the oracle's prefix
    ref = full.to_numpy()
    k = ns // 2
    got_off = small.offsets[:k].cpu().numpy()
    np.testing.assert_array_equal(got_off, ref["offsets"][:k])
    exact = reco.alloc_seeds(dfr, cap_seeds=ns, cap_hits=nh)
    reco.seed(dfr, up, dn, seeds=exact)
    torch.cuda.synchronize()
    assert int(exact.status.item()) == 0
    parity.assert_seeds_equal(exact.to_numpy(), ref)


def test_repeat_runs_identical(torch_dev):
    import torch
    fr = make_config(1, scale=0.2)
    reco = make_reco(fr)
    dfr = reco.upload(fr)
    outs = []
    for _ in range(3):
        up, dn = reco.neighbours(dfr)
        seeds = reco.seed(dfr, up, dn)
        tr = reco.fit(dfr, seeds)
        torch.cuda.synchronize()
        T = int(seeds.n_seeds.item())
        outs.append((up.cpu().numpy(), seeds.to_numpy(), tr.par[:T].cpu().numpy().copy()))
    for o in outs[1:]:
        np.testing.assert_array_equal(o[0], outs[0][0])
        parity.assert_seeds_equal(o[1], outs[0][1])
        np.testing.assert_array_equal(o[2], outs[0][2])


def test_fit_with_map_matches_oracle(torch_dev):
    import torch
    fr = make_config(4, scale=0.02)
    reco = make_reco(fr)
    dfr = reco.upload(fr)
    up, dn = reco.neighbours(dfr)
    seeds = reco.seed(dfr, up, dn)
    mp = np.random.default_rng(0).normal(0, 0.2, (fr.n_sectors, fr.n_rows, 2)).astype(np.float32)
    tr = reco.fit(dfr, seeds, torch.from_numpy(mp).cuda())
    torch.cuda.synchronize()
    # the oracle fits its own seeds, equal to the GPU's
    ru, rd = oracle.neighbours(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)
    sd = oracle.ca_seed(fr.row_offsets, ru, rd, fr.n_sectors, fr.n_rows, MIN_HITS)
    parity.assert_seeds_equal(seeds.to_numpy(), sd)
    T = len(sd["offsets"]) - 1
    gt = dict(x=tr.x[:T].cpu().numpy(), par=tr.par[:T].cpu().numpy(), cov=tr.cov[:T].cpu().numpy(),
              chi2=tr.chi2[:T].cpu().numpy(), ndf=tr.ndf[:T].cpu().numpy(),
              status=tr.status[:T].cpu().numpy())
    rt = oracle.fit(sd, fr.y, fr.z, fr.row_x, fr.n_rows, map_=mp.astype(np.float64), **FIT)
    parity.compare_fit(gt, rt)


def test_seed_hit_coordinates_and_gather_path(torch_dev):
    """The coordinates stored by the seeding are the frames' coordinates of
    the seed hits, and the fit gives bit-identical tracks whether it reads
    them or gathers them by id (seeds without coordinates)."""
    import torch
    fr = make_config(1, scale=0.2)
    reco = make_reco(fr)
    dfr = reco.upload(fr)
    up, dn = reco.neighbours(dfr)
    with_yz = reco.seed(dfr, up, dn)
    without = reco.seed(dfr, up, dn, seeds=reco.alloc_seeds(dfr, hit_yz=False))
    ta = reco.fit(dfr, with_yz)
    tb = reco.fit(dfr, without)
    torch.cuda.synchronize()
    sd = with_yz.to_numpy()
    parity.assert_seeds_equal(sd, without.to_numpy())
    H, T = len(sd["hits"]), len(sd["offsets"]) - 1
    yz = with_yz.hit_yz[:H].cpu().numpy()
    np.testing.assert_array_equal(yz[:, 0], fr.y[sd["hits"]])
    np.testing.assert_array_equal(yz[:, 1], fr.z[sd["hits"]])
    for k in ("x", "par", "cov", "chi2", "ndf", "status"):
        np.testing.assert_array_equal(getattr(ta, k)[:T].cpu().numpy(), getattr(tb, k)[:T].cpu().numpy(),
                                      err_msg=k)


def test_dense_rows_every_neighbour_and_ranking_form(torch_dev):
    """Two frames dense enough that rows go through all three neighbour forms
    (small LDS, large LDS for 513..1024 clusters, cell-sorted global copy
    above 1024) and some 16-row blocks exceed the LDS chain-ranking
    capacity (8192 clusters): bit-exact links and seeds, fit within
    tolerance."""
    from tpcsynth import make_frames
    fr = make_frames(n_sectors=36, n_rows=48, tracks_per_frame=(2600, 6500), seed=7,
                     phi_range=(0.03, 0.32), looper_frac=0.05, trunc_frac=0.3, noise_frac=0.1)
    n = np.diff(fr.row_offsets)
    assert (n > 1024).sum() > 0 and ((n > 512) & (n <= 1024)).sum() > 0 and (n <= 512).sum() > 0
    seg0 = np.arange(0, len(n), 16)
    blocks = fr.row_offsets[np.minimum(seg0 + 16, len(n))] - fr.row_offsets[seg0]
    assert (blocks > 8192).any()
    check_all(fr, "dense rows (48 rows, 2 frames)")


def test_sixteen_bit_row_ids(torch_dev):
    """Rows at the width of the dense search's relative ids (16 bits, the
    all-ones pattern reserved for no partner): an h-row between two rows of
    65 535 clusters is searched in LDS slabs with ids up to 65 534, one next
    to a row of 65 536 clusters in the global copies.  Clusters uniform over
    the rows (6.5 per cm^2), every link and seed exact."""
    from tpcsynth.generator import Frames, make_row_x
    rng = np.random.default_rng(65535)
    sizes = np.array([65535, 3000, 65535, 3000, 65536])
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    y = rng.uniform(-20.0, 20.0, off[-1]).astype(np.float32)
    z = rng.uniform(0.0, 250.0, off[-1]).astype(np.float32)
    fr = Frames(1, 1, 5, make_row_x(5), off, y, z)
    gu, gd, _, _ = run_gpu(fr)
    ru, rd = oracle.neighbours(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)
    np.testing.assert_array_equal(gu, ru, err_msg="up links differ")
    np.testing.assert_array_equal(gd, rd, err_msg="down links differ")
    # partners with the largest ids of the 65 535-cluster rows are found
    linked = rd[off[1]:off[2]]
    assert (linked >= 0).mean() > 0.9 and linked.max() >= off[0] + 65000
    assert (gu[off[3]:off[4]] >= off[4]).any()


def test_non_uniform_row_pitch_refused(torch_dev):
    """The neighbour predicate's second difference assumes equally spaced
    pad-row planes: a pitch more than 1e-3 off the mean is refused, float32
    rounding of a uniform table is accepted."""
    from paper_2412_13755_amd.reco import Reco, RecoConfig
    from paper_2412_13755_amd._capi import TpcError
    from tpcsynth import make_row_x
    rx = make_row_x(152)
    Reco(RecoConfig(row_x=rx, min_hits=MIN_HITS, **NB, **FIT), "cuda:0").close()
    bad = rx.copy()
    bad[70:] += np.float32(0.01)                    # one pitch 1% longer
    with pytest.raises(TpcError, match="pitch"):
        Reco(RecoConfig(row_x=bad, min_hits=MIN_HITS, **NB, **FIT), "cuda:0")
