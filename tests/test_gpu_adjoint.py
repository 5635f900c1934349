"""GPU adjoint of the summed fit chi2 w.r.t. the per-(sector, row) map,
through the C-ABI, against the float64 references on the oracle's own
seeds (checked equal to the GPU's first): central finite differences of
the C oracle and reverse-mode autograd of the independent torch
implementation, on the differentiable workload at x0.05 (autograd, 11 368
seeds) and at full size (finite differences of 64 sampled entries, 645 424
seeds).  Bar: relative L2 error <= 1e-3 and per entry
|d| <= 1e-3 * max(|g|, 1e-3 * max|g|).  Map recovery with Adam to 0.01 cm
after projecting out the modes the tracks absorb."""
import math

import numpy as np
import pytest

import oracle
from oracle import ref_autograd
from tests.conftest import NB, MIN_HITS, FIT
from tests import parity
from tpcsynth import make_config

pytestmark = pytest.mark.gpu

GRAD_RTOL = 1e-3


def _setup(scale=0.003, seed_map=0, amp=0.05):
    import torch
    from paper_2412_13755_amd.reco import Reco, RecoConfig
    fr = make_config(4, scale=scale)
    reco = Reco(RecoConfig(row_x=fr.row_x, n_sectors=fr.n_sectors, min_hits=MIN_HITS, **NB, **FIT),
                "cuda:0")
    dfr = reco.upload(fr)
    up, dn = reco.neighbours(dfr)
    seeds = reco.seed(dfr, up, dn)
    torch.cuda.synchronize()
    print("[adjoint] workload 4 x%g: N=%d" % (scale, fr.n_clusters), flush=True)
    # the references run on the oracle's own seeds, equal to the GPU's
    ru, rd = oracle.neighbours(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)
    sd = oracle.ca_seed(fr.row_offsets, ru, rd, fr.n_sectors, fr.n_rows, MIN_HITS)
    parity.assert_seeds_equal(seeds.to_numpy(), sd)
    mp = np.random.default_rng(seed_map).normal(0, amp, (fr.n_sectors, fr.n_rows, 2)).astype(np.float32)
    return fr, reco, dfr, seeds, mp, sd


def _grad_gpu(reco, dfr, seeds, mp, dloss=1.0):
    import torch
    from paper_2412_13755_amd.reco import KalmanChi2
    m = torch.from_numpy(mp).cuda().requires_grad_(True)
    loss = KalmanChi2.apply(m, reco, dfr, seeds)
    (loss * dloss).backward()
    torch.cuda.synchronize()
    return float(loss.item()), m.grad.cpu().numpy().astype(np.float64)


def _check(g, ref, label):
    err = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    floor = 1e-3 * np.abs(ref).max()
    worst = np.max(np.abs(g - ref) / np.maximum(np.abs(ref), floor))
    print("[adjoint] %s: rel L2 %.3g, worst entry %.3g" % (label, err, worst), flush=True)
    assert err <= GRAD_RTOL, err
    assert worst <= GRAD_RTOL, worst


def test_adjoint_matches_autograd_reference(torch_dev=None):
    fr, reco, dfr, seeds, mp, sd = _setup(scale=0.05)
    L, g = _grad_gpu(reco, dfr, seeds, mp)
    ref_fit = oracle.fit(sd, fr.y, fr.z, fr.row_x, fr.n_rows, map_=mp.astype(np.float64), **FIT)
    ok = ref_fit["status"] == 0
    Lr, gr = ref_autograd.map_gradient(mp.astype(np.float64), sd, fr.y, fr.z, fr.row_x, include=ok, **FIT)
    assert abs(L - Lr) <= 1e-5 * abs(Lr), (L, Lr)
    assert np.abs(gr).max() > 0
    _check(g, gr, "vs float64 autograd, %d seeds" % ok.sum())


@pytest.mark.parametrize("scale", [0.002, 1.0])
def test_adjoint_matches_finite_differences(scale):
    fr, reco, dfr, seeds, mp, sd = _setup(scale=scale, seed_map=1)
    L, g = _grad_gpu(reco, dfr, seeds, mp)
    rng = np.random.default_rng(2)
    covered = np.argwhere(np.abs(g).sum(axis=2) > 0)
    pick = covered[rng.choice(len(covered), size=min(128, len(covered)), replace=False)]
    entries = [(int(s), int(r), int(a)) for s, r in pick for a in (0, 1)]
    fd = oracle.fd_map_gradient(sd, fr.y, fr.z, fr.row_x, fr.n_rows, mp.astype(np.float64), entries,
                                h=1e-3, **FIT)
    gg = np.array([g[s, r, a] for s, r, a in entries])
    _check(gg, fd, "x%g vs oracle finite differences, %d entries" % (scale, len(entries)))


def test_adjoint_scales_with_dloss_and_is_deterministic():
    fr, reco, dfr, seeds, mp, sd = _setup(scale=0.002, seed_map=3)
    _, g1 = _grad_gpu(reco, dfr, seeds, mp, dloss=1.0)
    _, g2 = _grad_gpu(reco, dfr, seeds, mp, dloss=1.0)
    _, g3 = _grad_gpu(reco, dfr, seeds, mp, dloss=-2.5)
    np.testing.assert_array_equal(g1, g2)
    np.testing.assert_allclose(g3, -2.5 * g1, rtol=1e-6, atol=1e-6 * np.abs(g1).max())


def _project_gauge(d, row_x):
    """Remove, per sector, the modes the track parameters absorb:
    dy in span{1, x, x^2}, dz in span{1, x}."""
    x = row_x.astype(np.float64)
    x = (x - x.mean()) / x.std()
    out = d.copy()
    for a, deg in ((0, 2), (1, 1)):
        V = np.stack([x ** k for k in range(deg + 1)], axis=1)
        Q, _ = np.linalg.qr(V)
        for s in range(d.shape[0]):
            v = d[s, :, a]
            out[s, :, a] = v - Q @ (Q.T @ v)
    return out


def _seed_subset(seeds, sel):
    """The seeds `sel` (host indices) as a new device Seeds."""
    import torch
    from paper_2412_13755_amd.reco import Seeds
    sd = seeds.to_numpy()
    o, h = sd["offsets"], sd["hits"]
    n = np.diff(o)[sel]
    no = np.zeros(len(sel) + 1, np.int64)
    np.cumsum(n, out=no[1:])
    nh = np.concatenate([h[o[i]:o[i + 1]] for i in sel])
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(seeds.offsets.device)
    return Seeds(t([len(sel)]), t([nh.size]), t(no), t(nh), t(sd["frame"][sel]), t(sd["sector"][sel]),
                 t(sd["first_row"][sel]), t([0]), None)


def _adam(m, reco, dfr, seeds, its, lr0, lr1):
    import torch
    from paper_2412_13755_amd.reco import KalmanChi2
    opt = torch.optim.Adam([m], lr=lr0)
    sch = torch.optim.lr_scheduler.ExponentialLR(opt, gamma=(lr1 / lr0) ** (1.0 / its))
    losses = []
    for it in range(its):
        opt.zero_grad()
        loss = KalmanChi2.apply(m, reco, dfr, seeds)
        loss.backward()
        opt.step()
        sch.step()
        if it % 100 == 0 or it == its - 1:
            losses.append(float(loss.item()))
            print("[adam] it %d loss %.6g" % (it, losses[-1]), flush=True)
    return losses


def test_adam_recovers_injected_distortion():
    """Minimise the summed chi2 over the map with Adam (seeds fixed from the
    distorted clusters), in two passes: all seeds, then the seeds whose
    chi2/ndf at the first pass's map is below 3 (about 1 % of the seeds hold
    clusters of other particles or noise, and their chi2 pulls a plain sum
    off the injected map by about 0.02 cm).  The recovered map equals the
    injected distortion to 0.01 cm rms after projecting out the modes the
    track parameters absorb."""
    import torch
    fr = make_config(4, scale=0.1)
    D = fr.distortion.astype(np.float64)
    from paper_2412_13755_amd.reco import Reco, RecoConfig
    reco = Reco(RecoConfig(row_x=fr.row_x, n_sectors=fr.n_sectors, min_hits=MIN_HITS, **NB, **FIT),
                "cuda:0")
    dfr = reco.upload(fr)
    up, dn = reco.neighbours(dfr)
    seeds = reco.seed(dfr, up, dn)
    m = torch.zeros(fr.n_sectors, fr.n_rows, 2, device="cuda", requires_grad=True)
    l1 = _adam(m, reco, dfr, seeds, 400, 0.02, 2e-4)
    assert l1[-1] < l1[0]
    tr = reco.fit(dfr, seeds, m.detach().contiguous())
    T = int(seeds.n_seeds.item())
    st, c2, nd = (getattr(tr, k)[:T].cpu().numpy() for k in ("status", "chi2", "ndf"))
    keep = np.nonzero((st == 0) & (c2 < 3.0 * nd))[0]
    assert 0.95 * T < keep.size < T
    _adam(m, reco, dfr, _seed_subset(seeds, keep), 400, 0.005, 5e-5)
    M = m.detach().cpu().numpy().astype(np.float64)
    r0 = _project_gauge(D, fr.row_x)
    r1 = _project_gauge(M - D, fr.row_x)
    rms0 = float(np.sqrt(np.mean(r0 ** 2)))
    rms1 = float(np.sqrt(np.mean(r1 ** 2)))
    print("[adam] projected rms: injected %.4f cm, residual %.5f cm (%d of %d seeds in the second pass)" % (
        rms0, rms1, keep.size, T), flush=True)
    assert rms1 <= 0.01
