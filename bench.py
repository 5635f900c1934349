"""Throughput of the TPC tracking path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--legs main,event,batched,...]

One step = neighbour finding + cellular-automaton seeding + Kalman fit of one
synthetic time frame whose clusters are already resident in device memory
(no host transfer inside the timed region).  The headline workload is a
continuous-readout time frame: 50 Pb-Pb-like collisions spread uniformly
over a 100 us drift window (z shifted by the drift), 5x10^5 helix tracks (8%
low-pT loopers, half truncated), 10% noise, 6.4x10^7 clusters over 36
sectors x 152 pad rows (4x10^3 to 1.7x10^4 clusters per row).  The launch
form (staged kernels or one persistent kernel, grid, fit order) is the
autotuner's choice for this workload.  The oracle runs on one sector of the
frame (cpu_baseline) and its results gate the reported value.

Extra legs, reported beside the headline value:
  event    the same path on one central event over the full TPC (10^4 tracks,
           1.3x10^6 clusters)
  batched  64 time frames of uneven size (log-uniform 100..20000 tracks):
           plain per-frame calls vs all frames in one persistent launch
           replayed as a graph
  adjoint  10^5 tracks with an injected distortion map: full gradient
           evaluations per second (fit with checkpoints + chi2 sum + adjoint)
  follow   track following after the fit on the full-TPC event: every seed
           prolonged with chi2-gated cluster pickup (gate 25, up to 3 empty
           rows crossed), refitted, duplicates removed; the oracle is timed
           on the same seeds
  rans     rANS coding of a 2^28-symbol int32 array (rounded normal, sigma 12,
           about 5.6 bits of entropy per symbol; scale 2^14, blocks of 2^15
           symbols): symbols/s of tpc_rans_encode with the array resident in
           HBM, against the paper's CPU figure of 10^9 symbols/s; the oracle
           coder is timed on 2^24 of the symbols
  ctf      compression of the full-TPC event: track following, then (timed)
           the track-model residual transform into 17 integer arrays and the
           rANS coding of all of them in one batch (scale 2^14, blocks of
           2^13, counts read on the device), eagerly and as a graph;
           clusters/s and bits per cluster
  merge    the full-TPC event's fitted segments linked across sector edges,
           each linked pair combined, and the legs of loopers paired
           (tpc_track_merge, chi2 cut 30): ms per call, links, segments/s
  material the fit with multiple scattering (radiation length 2870 cm, pion
           mass), energy loss in the TPC's Ne-CO2-N2 gas and outlier
           rejection (chi2 > 30) on the headline seeds, and the same fit over
           rows followed by the smoother (tpc_kalman_smooth)
  skip     the headline event with 10% pad-row inefficiency: neighbours across
           one missing row + seeding + the fit over the hits' own rows, against
           the adjacent-row path on the same frame (times per call, seed
           lengths, track pieces found in one seed); the oracle chain is
           timed on the same frame
  copy     a 1 GiB device copy (reference for the HBM traffic counters; run
           alone with --legs copy)
  stages   the three stage calls on the headline workload, --steps times,
           nothing else (the launch sequence the counter profiles use; run
           alone with --legs stages)
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Method parameters of the workloads (cm, GeV/c, T).
NB = dict(win_y=2.5, win_z=2.5, cut_y=0.6, cut_z=0.75)
FIT = dict(bz=0.5, sigma_y=0.05, sigma_z=0.06, max_sin=0.999, var_sin0=1.0, var_tgl0=1.0,
           var_qpt0=100.0)
MIN_HITS = 5

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
VALU_PEAK_TFLOPS = 78.6        # MI355X vector FMA, FP64 (= non-packed FP32), TFLOP/s
ALU_PEAK_TOPS = 39.3           # one FP32 VALU operation per lane per clock: 256 CU x 64 lanes x 2.4 GHz

# Algorithmic work per unit: the method's own inputs and outputs per stage.
B_NB_PER_CLUSTER = 16          # read y, z; write up, dn
B_SEED_PER_CLUSTER = 8         # read up, dn
B_SEED_PER_HIT = 4             # write seed hit id
B_SEED_PER_SEED = 16           # write offset, frame, sector, first row
B_FIT_PER_HIT = 8              # read the hit's y, z
B_FIT_PER_TRACK = 24 + 96      # read seed record; write 24 words
FLOP_FIT_PER_HIT = 300         # helix step ~35, Jacobian ~30, F C F^T ~110, update ~125
NB_OPS_DENSE = 200             # FP32 operations per cluster of the neighbour search by predicted
                               # position at the continuous frame's density: window tests of the
                               # up candidates, then the down candidates around each prediction
FOLLOW_GATE, FOLLOW_MAX_MISS = 25.0, 3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--legs", default="main,event,batched,adjoint,follow,rans,ctf,material,skip,merge")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--stages-workload", type=int, default=2,
                    help="workload of the stages leg (2: continuous time frame, 1: full-TPC event, "
                         "3: 64 uneven frames)")
    return ap.parse_args()


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def make_reco(fr):
    from paper_2412_13755_amd.reco import Reco, RecoConfig
    return Reco(RecoConfig(row_x=fr.row_x, n_sectors=fr.n_sectors, min_hits=MIN_HITS, **NB, **FIT),
                "cuda:0")


CPU_SECTOR = 7                 # sector of the headline frame the oracle runs on


def cpu_baseline(fr, host, budget_s):
    """The oracle (as it stands) on one full-density sector of the headline
    frame, repeated within a time budget; its results are also compared with
    the GPU's for that sector (a sector reads no other sector), which gates
    the reported value.  Returns (baseline, parity)."""
    import oracle
    from tests import parity
    cores = len(os.sched_getaffinity(0))
    oracle.set_threads(cores)
    up, dn, sd, tr = host
    sv, gu, gd, gs, gt = parity.sector_results(fr, CPU_SECTOR, up, dn, sd, tr)
    times = []
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        ru, rd = oracle.neighbours(sv.row_offsets, sv.y, sv.z, sv.n_rows, **NB)
        rs = oracle.ca_seed(sv.row_offsets, ru, rd, 1, sv.n_rows, MIN_HITS)
        rt = oracle.fit(rs, sv.y, sv.z, sv.row_x, sv.n_rows, **FIT)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() - t_start > budget_s or len(times) >= 20:
            break
    t = float(np.median(times))
    check = {"sector": CPU_SECTOR, "clusters": sv.n_clusters}
    try:
        np.testing.assert_array_equal(gu, ru)
        np.testing.assert_array_equal(gd, rd)
        parity.assert_seeds_equal(gs, rs)
        check["fit"] = parity.compare_fit(gt, rt)
        check["links_seeds_identical"] = True
        check["ok"] = True
    except AssertionError as e:
        check["ok"] = False
        check["error"] = str(e)[:300]
    base = {"value": round(sv.n_clusters / t / 1e6, 4), "unit": "M clusters/s",
            "cores": int(oracle.max_threads()), "kind": "oracle",
            "sample": "sector %d of the headline frame (%d clusters at full density), %d runs, median "
                      "%.3f s; FP32 neighbours, integer seeding, FP64 fit" % (CPU_SECTOR, sv.n_clusters,
                                                                            len(times), t)}
    return base, check


def batched_cpu_check(fr, out, frames=(0, 40)):
    """The oracle on sector CPU_SECTOR of a few frames of the batched input
    against a batched run's results for them (frames and sectors are
    independent units).  `out` = (up, dn, seeds, tracks) on the device."""
    from tests import parity
    up, dn, seeds, tracks = out
    T = int(seeds.n_seeds.item())
    sd = seeds.to_numpy()
    tr = {k: getattr(tracks, k)[:T].cpu().numpy() for k in ("x", "par", "cov", "chi2", "ndf", "status")}
    hu, hd = up.cpu().numpy(), dn.cpu().numpy()
    check = {"sector": CPU_SECTOR, "frames": list(frames)}
    try:
        st = [parity.check_sector(fr, CPU_SECTOR, hu, hd, sd, tr, NB, MIN_HITS, FIT, f) for f in frames]
        check["clusters"] = int(sum(x["clusters"] for x in st))
        check["worst_par"] = max(x["fit"]["worst_par"] for x in st)
        check["ok"] = True
    except AssertionError as e:
        check["ok"] = False
        check["error"] = str(e)[:300]
    return check


def adjoint_cpu_check(fr, seeds, grad, n_entries=16):
    """The adjoint at map 0 against central finite differences of the oracle
    on sector CPU_SECTOR of the frame (its map entries depend on that sector's
    seeds only), on the oracle's own seeds for it, which must equal the
    GPU's."""
    import oracle
    sd = seeds.to_numpy()
    sv = fr.sector_view(0, CPU_SECTOR)
    check = {"sector": CPU_SECTOR, "clusters": sv.n_clusters}
    try:
        ru, rd = oracle.neighbours(sv.row_offsets, sv.y, sv.z, sv.n_rows, **NB)
        rs = oracle.ca_seed(sv.row_offsets, ru, rd, 1, sv.n_rows, MIN_HITS)
        a, b = fr.first_id(0, CPU_SECTOR), fr.first_id(0, CPU_SECTOR) + sv.n_clusters
        o, h = np.asarray(sd["offsets"]), np.asarray(sd["hits"])
        first = h[o[:-1]]
        i0, i1 = np.searchsorted(first, a), np.searchsorted(first, b)
        np.testing.assert_array_equal(o[i0:i1 + 1] - o[i0], rs["offsets"])
        np.testing.assert_array_equal(h[o[i0]:o[i1]] - a, rs["hits"])
        g = grad[CPU_SECTOR]
        cov = np.argwhere(np.abs(g).sum(axis=1) > 0)[:, 0]
        rng = np.random.default_rng(7)
        rows = rng.choice(cov, size=min(n_entries // 2, cov.size), replace=False)
        entries = [(0, int(r), ax) for r in rows for ax in (0, 1)]
        fd = oracle.fd_map_gradient(rs, sv.y, sv.z, sv.row_x, sv.n_rows, np.zeros((1, sv.n_rows, 2)), entries,
                                    h=1e-3, **FIT)
        gg = np.array([g[r, ax] for _, r, ax in entries], dtype=np.float64)
        err = float(np.linalg.norm(gg - fd) / np.linalg.norm(fd))
        floor = 1e-3 * np.abs(fd).max()
        worst = float(np.max(np.abs(gg - fd) / np.maximum(np.abs(fd), floor)))
        check.update(entries=len(entries), rel_l2=err, worst_entry=worst, seeds_identical=True)
        check["ok"] = err <= 1e-3 and worst <= 1e-3
    except AssertionError as e:
        check["ok"] = False
        check["error"] = str(e)[:300]
    return check


# HBM traffic per launch from the committed counter profiles; used only
# while the kernel sources are those the counters were taken on.
FIT_SOURCES = ("tpc_fit.hip", "tpc_fit_common.hpp", "tpc_fit_math.hpp", "tpc_internal.hpp")
FIT_PROFILE = os.path.join(ROOT, "profiles", "path_full_tpc_event_1e4.txt")
NB_SOURCES = ("tpc_neighbours.hip", "tpc_nb_device.hpp", "tpc_internal.hpp")
NB_PROFILE = os.path.join(ROOT, "profiles", "path_continuous_tf_50x1e4.txt")


def source_sha(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2412_13755_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def fit_source_sha():
    return source_sha(FIT_SOURCES)


def profile_keys(path, files):
    """The key = value lines of a profile summary, or None if it is missing or
    was taken on other kernel sources."""
    try:
        with open(path) as f:
            kv = dict(l.split(" = ", 1) for l in f.read().splitlines() if " = " in l and not l.startswith("#"))
    except OSError:
        return None
    if kv.get("source_sha256", "").strip() != source_sha(files):
        return None
    return kv


def profile_traffic(path, files):
    """Calibrated HBM bytes per launch recorded in a profile summary, or None."""
    kv = profile_keys(path, files)
    return None if kv is None else int(float(kv["traffic_bytes_per_launch"]))


def profile_valu(path, files, ms):
    """Executed VALU lane operations per launch from the profile's counters
    (SQ_INSTS_VALU x 64 x the active-lane fraction) and their rate over a
    launch of ms, against the issue peak of one lane operation per lane per
    clock (ALU_PEAK_TOPS); None without a matching profile."""
    kv = profile_keys(path, files)
    if kv is None or "valu_lane_ops_per_launch" not in kv:
        return None
    ops = float(kv["valu_lane_ops_per_launch"])
    rate = ops / (ms * 1e-3) / 1e12
    return {"lane_ops_per_launch": int(ops), "achieved": round(rate, 4), "peak": ALU_PEAK_TOPS,
            "unit": "Top/s", "frac": round(rate / ALU_PEAK_TOPS, 5)}


def fit_profile_traffic():
    return profile_traffic(FIT_PROFILE, FIT_SOURCES)


def nb_profile_traffic():
    return profile_traffic(NB_PROFILE, NB_SOURCES)


def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3


def stage_events(reco, dfr, out, ws, steps):
    """Mean HIP-event time of each stage call of the staged path, recorded on
    the launch stream (the current torch stream)."""
    import torch
    up, dn, sd, tr = out
    stream = torch.cuda.current_stream()
    evs = []
    for _ in range(steps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        e[0].record(stream)
        reco.neighbours(dfr, up, dn, ws)
        e[1].record(stream)
        reco.seed(dfr, up, dn, sd, ws)
        e[2].record(stream)
        reco.fit(dfr, sd, None, tr, ws)
        e[3].record(stream)
        evs.append(e)
    torch.cuda.synchronize()
    return np.array([[e[j].elapsed_time(e[j + 1]) for j in range(3)] for e in evs]).mean(axis=0)


def fit_roofline(n_hits, n_seeds, fit_ms, traffic=None):
    """Roofline of tpc_kalman_fit (the length order of the seeds, four small
    kernels, then fit_tracks_ordered, when the seeds carry their hit
    coordinates) against the FP64 vector peak; fit_ms is the whole call."""
    flops = FLOP_FIT_PER_HIT * n_hits
    achieved = flops / (fit_ms * 1e-3) / 1e12
    nbytes = B_FIT_PER_HIT * n_hits + B_FIT_PER_TRACK * n_seeds
    return {"bound": "alu", "achieved": round(achieved, 4), "peak": VALU_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / VALU_PEAK_TFLOPS, 5), "traffic": traffic,
            "kernel": "tpc_kalman_fit (fit_order_* + fit_tracks_ordered)", "avg_ms": round(fit_ms, 5),
            "algorithmic_flops": int(flops),
            "algorithmic_bytes": int(nbytes),
            "hbm_frac": round(nbytes / (fit_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 6)}


def leg_path(args, k):
    """The whole path (neighbours + seeding + fit) on workload k: the
    autotuner's launch form, eagerly and as a graph replay, then each stage
    of the staged path timed with HIP events.  Returns (result, frames,
    host copies of the staged outputs)."""
    import torch
    from paper_2412_13755_amd import tune
    from paper_2412_13755_amd.reco import ReconstructGraph
    from tpcsynth import make_config
    t0 = time.perf_counter()
    fr = make_config(k)
    log("workload %s: %d clusters (generated in %.1f s)" % (fr.meta["name"], fr.n_clusters,
                                                           time.perf_counter() - t0))
    reco = make_reco(fr)
    dfr = reco.upload(fr)
    best = tune.autotune(reco, dfr, use_cache=False, repeats=5 if k != 2 else 3)
    log("autotune: %s" % json.dumps(best))
    out = reco.reconstruct(dfr, best["mode"], best["tune"])
    torch.cuda.synchronize()
    seeds = out[2]
    n_seeds, n_hits = int(seeds.n_seeds.item()), int(seeds.n_hits.item())
    assert int(seeds.status.item()) == 0
    steps = args.steps if k != 2 else max(5, args.steps // 5)
    ms_eager = timed(lambda: reco.reconstruct(dfr, best["mode"], best["tune"], out), steps, args.warmup)
    g = ReconstructGraph(reco, dfr, best["mode"], best["tune"])
    ms_graph = timed(g.replay, steps, args.warmup)
    del g
    ms = min(ms_eager, ms_graph)
    log("path: eager %.3f ms, graph %.3f ms" % (ms_eager, ms_graph))
    # per-stage event timing of the staged path on the launch stream
    ws = reco.workspace(dfr)
    st_out = reco.reconstruct(dfr, "staged")
    stage_ms = stage_events(reco, dfr, st_out, ws, steps)
    N = dfr.n_clusters
    names = ["tpc_neighbours", "tpc_ca_seed", "tpc_kalman_fit"]
    nb_gbs = B_NB_PER_CLUSTER * N / (stage_ms[0] * 1e-3) / 1e9
    seed_bytes = B_SEED_PER_CLUSTER * N + B_SEED_PER_HIT * n_hits + B_SEED_PER_SEED * n_seeds
    if k == 2:
        # neighbour search on dense rows (nb_bin + nb_query_dense, ~95% of
        # the stage): plain FP32 ALU work, NB_OPS_DENSE operations per cluster
        ops = NB_OPS_DENSE * N
        achieved = ops / (stage_ms[0] * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": round(achieved, 4), "peak": ALU_PEAK_TOPS, "unit": "Top/s",
                "frac": round(achieved / ALU_PEAK_TOPS, 5), "traffic": nb_profile_traffic(),
                "kernel": "tpc_neighbours (nb_dense_order + nb_bin + nb_query_dense)", "avg_ms": round(float(stage_ms[0]), 5),
                "algorithmic_ops": int(ops), "algorithmic_bytes": int(B_NB_PER_CLUSTER * N),
                "hbm_frac": round(nb_gbs / HBM_PEAK_GBS, 6),
                "executed_valu": profile_valu(NB_PROFILE, NB_SOURCES, float(stage_ms[0]))}
    else:
        roof = fit_roofline(n_hits, n_seeds, float(stage_ms[2]), fit_profile_traffic())
    res = {
        "value": round(N / (ms * 1e-3) / 1e6, 3), "ms_per_step": round(ms, 5),
        "config": {"workload": fr.meta["name"], "clusters": N, "tracks_generated": fr.meta["n_tracks"],
                   "collisions": 50 if k == 2 else 1,
                   "seeds": n_seeds, "seed_hits": n_hits, "sectors": fr.n_sectors, "rows": fr.n_rows,
                   "max_row_clusters": int(np.diff(fr.row_offsets).max()),
                   "mode": best["mode"], "tune": best["tune"],
                   "graph": ms_graph <= ms_eager},
        "tracks_per_s": round(n_seeds / (ms * 1e-3), 1),
        "ms_eager": round(ms_eager, 5), "ms_graph": round(ms_graph, 5),
        "autotune_table": best["table"],
        "stage_ms_staged": {n: round(float(v), 5) for n, v in zip(names, stage_ms)},
        "stage_hbm_frac": {"tpc_neighbours": round(nb_gbs / HBM_PEAK_GBS, 5),
                           "tpc_ca_seed": round(seed_bytes / (stage_ms[1] * 1e-3) / 1e9 / HBM_PEAK_GBS, 5)},
        "stage_fit_roofline": fit_roofline(n_hits, n_seeds, float(stage_ms[2])),
        "roofline": roof,
    }
    up, dn, sd, tr = st_out
    T = n_seeds
    host = (up.cpu().numpy(), dn.cpu().numpy(), sd.to_numpy(),
            {k2: getattr(tr, k2)[:T].cpu().numpy() for k2 in ("x", "par", "cov", "chi2", "ndf", "status")})
    # the autotuner's form must give the staged form's results
    same = (np.array_equal(out[0].cpu().numpy(), host[0]) and np.array_equal(out[1].cpu().numpy(), host[1])
            and int(out[2].n_seeds.item()) == T)
    res["launch_form_matches_staged"] = bool(same)
    del out, st_out, ws
    reco.close()
    torch.cuda.empty_cache()
    return res, fr, host


def leg_batched(args):
    import torch
    from paper_2412_13755_amd import tune
    from paper_2412_13755_amd.reco import ReconstructGraph
    from tpcsynth import make_config
    fr = make_config(3)
    log("batched workload: %d frames, %d clusters" % (fr.n_frames, fr.n_clusters))
    reco = make_reco(fr)
    dfr = reco.upload(fr)
    SR = fr.n_sectors * fr.n_rows
    views = [dfr.frame_view(f, SR) for f in range(fr.n_frames)]
    outs = [reco.reconstruct(v, "staged") for v in views]
    wsz = max(reco.workspace_bytes(v) for v in views)
    ws = torch.empty(wsz, dtype=torch.uint8, device="cuda")

    def plain():
        for v, o in zip(views, outs):
            reco.reconstruct(v, "staged", None, o, ws)
    steps = max(3, args.steps // 10)
    ms_plain = timed(plain, steps, 2)
    best = tune.autotune(reco, dfr, use_cache=False, repeats=3)
    log("batched autotune: %s" % json.dumps({k: best[k] for k in ("mode", "tune", "ms")}))
    pers = min((e for e in best["table"] if e["mode"] == "persistent"), key=lambda e: e["ms"])
    ptune = tuple(pers["tune"])
    g = ReconstructGraph(reco, dfr, "persistent", ptune)
    ms_persist = timed(g.replay, steps, 2)
    gs = ReconstructGraph(reco, dfr, "staged")
    ms_staged_batched = timed(gs.replay, steps, 2)
    N = dfr.n_clusters
    checks = {}
    if not args.no_cpu:
        checks = {"persistent": batched_cpu_check(fr, g.replay()), "staged": batched_cpu_check(fr, gs.replay())}
    ok = all(c["ok"] for c in checks.values())
    return {"workload": fr.meta["name"], "frames": fr.n_frames, "clusters": N,
            "parity": checks if checks else {"ok": None, "note": "not checked (--no-cpu)"},
            "plain_per_frame": {"ms": round(ms_plain, 4), "M_clusters_per_s": round(N / ms_plain / 1e3, 3)},
            "batched_persistent_graph": {"ms": round(ms_persist, 4),
                                         "M_clusters_per_s": round(N / ms_persist / 1e3, 3),
                                         "tune": list(ptune)},
            "batched_staged_graph": {"ms": round(ms_staged_batched, 4),
                                     "M_clusters_per_s": round(N / ms_staged_batched / 1e3, 3)},
            "autotune_choice": {"mode": best["mode"], "tune": best["tune"]},
            "speedup_persistent_vs_plain": round(ms_plain / ms_persist, 3) if ok else None,
            "speedup_batched_vs_plain": round(ms_plain / min(ms_persist, ms_staged_batched), 3) if ok else None}


def leg_adjoint(args):
    import torch
    from paper_2412_13755_amd.reco import KalmanChi2
    from tpcsynth import make_config
    fr = make_config(4)
    log("adjoint workload: %d clusters" % fr.n_clusters)
    reco = make_reco(fr)
    dfr = reco.upload(fr)
    up, dn = reco.neighbours(dfr)
    seeds = reco.seed(dfr, up, dn)
    torch.cuda.synchronize()
    T = int(seeds.n_seeds.item())
    H = int(seeds.n_hits.item())
    m = torch.zeros(fr.n_sectors, fr.n_rows, 2, device="cuda", requires_grad=True)

    def step():
        m.grad = None
        loss = KalmanChi2.apply(m, reco, dfr, seeds)
        loss.backward()
    steps = max(3, args.steps // 5)
    ms = timed(step, steps, 2)
    res = {"workload": fr.meta["name"], "clusters": dfr.n_clusters, "seeds": T, "seed_hits": H,
           "ms_per_gradient": round(ms, 4), "grads_per_s": round(1e3 / ms, 3),
           "tracks_per_s": round(T / ms * 1e3, 1), "ckpt_rows": reco.cfg.ckpt_rows}
    if not args.no_cpu:
        res["parity"] = adjoint_cpu_check(fr, seeds, m.grad.cpu().numpy())
        if not res["parity"]["ok"]:
            res["grads_per_s"] = None            # no number for a run that fails parity
    return res


def leg_follow(args, with_cpu=True):
    """tpc_track_follow on the headline workload's seeds, timed with HIP events
    on the launch stream; the oracle's following timed on the same seeds."""
    import torch
    from tpcsynth import make_config
    fr = make_config(1)
    reco = make_reco(fr)
    dfr = reco.upload(fr)
    ws = reco.workspace(dfr)
    up, dn = reco.neighbours(dfr, ws=ws)
    seeds = reco.seed(dfr, up, dn, ws=ws)
    rows, tr = reco.follow(dfr, seeds, FOLLOW_GATE, FOLLOW_MAX_MISS, ws=ws)
    torch.cuda.synchronize()
    T, H = int(seeds.n_seeds.item()), int(seeds.n_hits.item())
    stream = torch.cuda.current_stream()
    steps = max(5, args.steps)
    for _ in range(2):
        reco.follow(dfr, seeds, FOLLOW_GATE, FOLLOW_MAX_MISS, rows, tr, ws)
    evs = []
    for _ in range(steps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record(stream)
        reco.follow(dfr, seeds, FOLLOW_GATE, FOLLOW_MAX_MISS, rows, tr, ws)
        e[1].record(stream)
        evs.append(e)
    torch.cuda.synchronize()
    ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    st = tr.status[:T].cpu().numpy()
    rw = rows[:T].cpu().numpy()
    final_hits = int((rw >= 0).sum())
    kept_hits = int((rw[st == 0] >= 0).sum())
    # seed fit over the seed hits, outward pass and refit over the final hits
    flops = FLOP_FIT_PER_HIT * (H + 2 * final_hits)
    achieved = flops / (ms * 1e-3) / 1e12
    res = {"workload": fr.meta["name"], "clusters": dfr.n_clusters, "seeds": T, "seed_hits": H,
           "gate_chi2": FOLLOW_GATE, "max_miss": FOLLOW_MAX_MISS,
           "kept": int((st == 0).sum()), "duplicates": int((st == 4).sum()),
           "hits_kept": kept_hits, "ms": round(ms, 5), "seeds_per_s": round(T / ms * 1e3, 1),
           "M_clusters_per_s": round(dfr.n_clusters / ms / 1e3, 3),
           "roofline": {"bound": "alu", "achieved": round(achieved, 4), "peak": VALU_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(achieved / VALU_PEAK_TFLOPS, 5),
                        "algorithmic_flops": int(flops),
                        "calls": "fl_index, fl_tracks, fl_owner_init, fl_claim, fl_keep"}}
    if with_cpu:
        import oracle
        oracle.set_threads(len(os.sched_getaffinity(0)))
        up_r, dn_r = oracle.neighbours(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)
        sd = oracle.ca_seed(fr.row_offsets, up_r, dn_r, fr.n_sectors, fr.n_rows, MIN_HITS)
        times = []
        for _ in range(5):
            t0 = time.perf_counter()
            oracle.follow(sd, fr.row_offsets, fr.y, fr.z, fr.row_x, fr.n_sectors, fr.n_rows,
                          gate=FOLLOW_GATE, max_miss=FOLLOW_MAX_MISS, **FIT)
            times.append(time.perf_counter() - t0)
        t = float(np.median(times))
        res["cpu_oracle"] = {"ms": round(t * 1e3, 3), "cores": int(oracle.max_threads()),
                             "seeds_per_s": round(T / t, 1)}
    return res


RANS_L, RANS_B, RANS_N = 14, 1 << 15, 1 << 28
RANS_PAPER_SYMBOLS_PER_S = 1e9      # the paper's AVX2 coder, 16 interleaved encoders


def leg_rans(args, with_cpu=True):
    """tpc_rans_encode of a large resident array, HIP events on the launch stream."""
    import torch
    from paper_2412_13755_amd.reco import rans_encode, rans_max_bytes, rans_workspace
    g = torch.Generator(device="cuda").manual_seed(28)
    x = torch.round(torch.randn(RANS_N, device="cuda", generator=g) * 12.0).to(torch.int32)
    out = torch.empty(rans_max_bytes(RANS_N, 1 << 20, RANS_L, RANS_B), dtype=torch.uint8, device="cuda")
    ws = rans_workspace(RANS_N, RANS_L, RANS_B)
    size = torch.zeros(1, dtype=torch.int64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    for _ in range(2):
        rans_encode(x, RANS_L, RANS_B, out, ws, size, status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    stream = torch.cuda.current_stream()
    steps = max(3, args.steps // 5)
    evs = []
    for _ in range(steps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record(stream)
        rans_encode(x, RANS_L, RANS_B, out, ws, size, status)
        e[1].record(stream)
        evs.append(e)
    torch.cuda.synchronize()
    ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    nbytes = int(size.item())
    sps = RANS_N / (ms * 1e-3)
    # the decoder on the same stream
    from paper_2412_13755_amd.reco import rans_decode
    dec = torch.empty(RANS_N, dtype=torch.int32, device="cuda")
    dws = None
    for _ in range(2):
        _, dn, dst = rans_decode(out, nbytes, RANS_N, out=dec, ws=dws)
    torch.cuda.synchronize()
    assert int(dst.item()) == 0 and int(dn.item()) == RANS_N and bool(torch.equal(dec, x))
    devs = []
    for _ in range(steps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record(stream)
        rans_decode(out, nbytes, RANS_N, out=dec, ws=dws)
        e[1].record(stream)
        devs.append(e)
    torch.cuda.synchronize()
    ms_dec = float(np.mean([e[0].elapsed_time(e[1]) for e in devs]))
    alg = 4 * RANS_N + nbytes                      # read the symbols, write the stream
    res = {"workload": "normal-sigma12-2^28", "symbols": RANS_N, "scale_bits": RANS_L,
           "block_symbols": RANS_B, "stream_bytes": nbytes,
           "bits_per_symbol": round(8.0 * nbytes / RANS_N, 4), "ms": round(ms, 4),
           "G_symbols_per_s": round(sps / 1e9, 3),
           "vs_paper_cpu": round(sps / RANS_PAPER_SYMBOLS_PER_S, 2),
           "decode_ms": round(ms_dec, 4), "decode_G_symbols_per_s": round(RANS_N / ms_dec / 1e6, 3),
           "roofline": {"bound": "hbm", "achieved": round(alg / (ms * 1e-3) / 1e9, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                        "algorithmic_bytes": alg,
                        "calls": "rs_init, rs_window, rs_minmax, rs_clear, rs_hist, rs_freq, rs_table, rs_encode, rs_scan, rs_pack"}}
    if with_cpu:
        import oracle
        xs = x[:1 << 24].cpu().numpy()
        times = []
        for _ in range(3):
            t0 = time.perf_counter()
            oracle.rans_encode(xs, RANS_L, RANS_B)
            times.append(time.perf_counter() - t0)
        t = float(np.median(times))
        res["cpu_oracle"] = {"symbols": int(xs.size), "ms": round(t * 1e3, 2), "cores": 1,
                             "G_symbols_per_s": round(xs.size / t / 1e9, 4)}
    return res


CTF_Q = 0.01                      # quantisation step of y and z, cm
CTF_B = 1 << 13                   # coding block of the frame's arrays


def leg_ctf(args):
    """Transform + coding of every array of the headline frame's CTF."""
    import torch
    from paper_2412_13755_amd import _capi as C
    from paper_2412_13755_amd.reco import rans_encode_batch, rans_batch_workspace
    from tpcsynth import make_config
    fr = make_config(1)
    reco = make_reco(fr)
    dfr = reco.upload(fr)
    ws = reco.workspace(dfr)
    up, dn = reco.neighbours(dfr, ws=ws)
    seeds = reco.seed(dfr, up, dn, ws=ws)
    rows, tr = reco.follow(dfr, seeds, FOLLOW_GATE, FOLLOW_MAX_MISS, ws=ws)
    arr = reco.ctf_build(dfr, seeds, rows, tr, CTF_Q, CTF_Q, ws=ws)
    torch.cuda.synchronize()
    counts = [int(v) for v in arr["counts"].cpu()]
    # all 17 arrays coded by one batch; counts read on the device (no host sync)
    jobs = [{"symbols": arr[k], "n_device": arr["counts"][i:i + 1]} for i, k in enumerate(C.CTF_ARRAYS)]
    rans_encode_batch(jobs, RANS_L, CTF_B)
    rws = rans_batch_workspace(jobs, RANS_L, CTF_B)

    def step():
        reco.ctf_build(dfr, seeds, rows, tr, CTF_Q, CTF_Q, out=arr, ws=ws)
        rans_encode_batch(jobs, RANS_L, CTF_B, rws)
    step()
    torch.cuda.synchronize()
    assert all(int(j["status"].item()) == 0 for j in jobs)
    total = sum(int(j["out_size"].item()) for j in jobs)
    stream = torch.cuda.current_stream()
    steps = max(5, args.steps // 2)

    def event_ms(fn):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps
    ms_eager = event_ms(step)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    ms_graph = event_ms(g.replay)
    torch.cuda.synchronize()
    assert sum(int(j["out_size"].item()) for j in jobs) == total
    ms = min(ms_eager, ms_graph)
    N = dfr.n_clusters
    return {"workload": fr.meta["name"], "clusters": N, "q_cm": CTF_Q, "arrays": len(counts),
            "scale_bits": RANS_L, "block_symbols": CTF_B,
            "symbols": int(sum(counts)), "stream_bytes": total,
            "bits_per_cluster": round(8.0 * total / N, 3),
            "ratio_vs_float_yz": round(8.0 * N / total, 3),
            "ms_eager": round(ms_eager, 4), "ms_graph": round(ms_graph, 4),
            "M_clusters_per_s": round(N / ms / 1e3, 2),
            "G_symbols_per_s": round(sum(counts) / ms / 1e6, 3)}


MAT_X0, MAT_CUT = 2870.0, 30.0


def leg_material(args):
    """tpc_kalman_fit_material (scattering, energy loss in the TPC gas, outlier
    cut) on the headline seeds, then the fit over rows with the smoother; HIP
    events on the launch stream."""
    import torch
    from tpcsynth import make_config, PION_MASS, TPC_GAS
    fr = make_config(1)
    reco = make_reco(fr)
    dfr = reco.upload(fr)
    ws = reco.workspace(dfr)
    up, dn = reco.neighbours(dfr, ws=ws)
    seeds = reco.seed(dfr, up, dn, ws=ws)
    tr, rej = reco.fit_material(dfr, seeds, MAT_X0, PION_MASS, MAT_CUT, ws=ws, gas=TPC_GAS)
    torch.cuda.synchronize()
    T, H = int(seeds.n_seeds.item()), int(seeds.n_hits.item())
    stream = torch.cuda.current_stream()
    steps = max(5, args.steps)
    for _ in range(2):
        reco.fit_material(dfr, seeds, MAT_X0, PION_MASS, MAT_CUT, tr, rej, ws, gas=TPC_GAS)
    evs = []
    for _ in range(steps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record(stream)
        reco.fit_material(dfr, seeds, MAT_X0, PION_MASS, MAT_CUT, tr, rej, ws, gas=TPC_GAS)
        e[1].record(stream)
        evs.append(e)
    torch.cuda.synchronize()
    ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    flops = (FLOP_FIT_PER_HIT + 80) * H            # the fit's step and update, plus scattering and energy loss
    # the fit over rows followed by the smoother, same seeds and material
    mat = (MAT_X0, PION_MASS, MAT_CUT) + TPC_GAS
    out = reco.smooth(dfr, seeds, material=mat, ws=ws)
    torch.cuda.synchronize()
    evs = []
    for _ in range(steps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record(stream)
        out = reco.smooth(dfr, seeds, material=mat, tracks=out[0], ws=ws)
        e[1].record(stream)
        evs.append(e)
    torch.cuda.synchronize()
    ms_s = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    return {"workload": fr.meta["name"], "seeds": T, "seed_hits": H, "x0_cm": MAT_X0, "chi2_cut": MAT_CUT,
            "gas": {"rho": TPC_GAS[0], "z_over_a": TPC_GAS[1], "mean_exc_gev": TPC_GAS[2]},
            "rejected_hits": int(rej[:H].sum()), "ms": round(ms, 5),
            "tracks_per_s": round(T / ms * 1e3, 1),
            "fit_and_smoother_ms": round(ms_s, 5), "smoothed_hits_per_s": round(H / ms_s * 1e3, 1),
            "roofline": {"bound": "alu", "achieved": round(flops / (ms * 1e-3) / 1e12, 4),
                         "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(flops / (ms * 1e-3) / 1e12 / VALU_PEAK_TFLOPS, 5),
                         "kernel": "fit_ms_tracks", "algorithmic_flops": int(flops)}}


SKIP_EFF = 0.9                 # pad-row efficiency of the row-skipping workload


def _one_seed_coverage(fr, sd, min_clusters=20, frac=0.8):
    """Fraction of (track, sector) pieces with >= min_clusters clusters of
    which at least frac land in a single seed."""
    t = fr.track_of
    seg = np.repeat(np.arange(fr.row_offsets.size - 1), np.diff(fr.row_offsets))
    sec = seg // fr.n_rows
    sig = t >= 0
    piece = t.astype(np.int64) * 4096 + sec
    pk, pn = np.unique(piece[sig], return_counts=True)
    big = pk[pn >= min_clusters]
    nbig = pn[pn >= min_clusters]
    h = sd["hits"]
    sid = np.repeat(np.arange(len(sd["offsets"]) - 1), np.diff(sd["offsets"]))
    ok = t[h] >= 0
    key = sid[ok].astype(np.int64) * (1 << 40) + piece[h[ok]]
    uk, un = np.unique(key, return_counts=True)
    upiece = uk % (1 << 40)
    best = {}
    for p_, n_ in zip(upiece.tolist(), un.tolist()):
        if n_ > best.get(p_, 0):
            best[p_] = n_
    got = np.array([best.get(p_, 0) for p_ in big.tolist()])
    return float(np.mean(got >= frac * nbig)) if big.size else 0.0


def leg_merge(args):
    """tpc_track_merge on the headline event's fitted seeds (links only, then
    links and looper legs) and tpc_track_refit on its links: each C-ABI call
    between HIP events on the launch stream, into preallocated outputs."""
    import torch
    from tpcsynth import make_config
    fr = make_config(1)
    reco = make_reco(fr)
    dfr = reco.upload(fr)
    ws = reco.workspace(dfr)
    up, dn = reco.neighbours(dfr, ws=ws)
    seeds = reco.seed(dfr, up, dn, ws=ws)
    tr = reco.fit(dfr, seeds)
    out = reco.alloc_merge(seeds, legs=True)
    nxt, prv, chi, mp, mc, leg, lchi = reco.merge(seeds, tr, MERGE_CUT, out=out)
    rf = reco.refit(dfr, seeds, tr, nxt, prv, leg)
    torch.cuda.synchronize()
    T = int(seeds.n_seeds.item())
    stream = torch.cuda.current_stream()

    def timed_events(fn):
        evs = []
        for _ in range(max(5, args.steps)):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            e[0].record(stream)
            fn()
            e[1].record(stream)
            evs.append(e)
        torch.cuda.synchronize()
        return float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))

    ms_links = timed_events(lambda: reco.merge(seeds, tr, MERGE_CUT, out=out, legs=False))
    ms_legs = timed_events(lambda: reco.merge(seeds, tr, MERGE_CUT, out=out, legs=True))
    ms_refit = timed_events(lambda: reco.refit(dfr, seeds, tr, nxt, prv, leg, out=rf))
    links = int((nxt[:T] >= 0).sum().item())
    legs = int((leg[:T] >= 0).sum().item()) // 2
    st = rf["refit"].status[:T]
    heads = int((st != 5).sum().item())
    multi = int(((st != 5) & (nxt[:T] >= 0)).sum().item())
    tracks = int(torch.unique(rf["track_id"][:T][rf["track_id"][:T] >= 0]).numel())
    return {"workload": fr.meta["name"], "seeds": T, "chi2_cut": MERGE_CUT, "links": links, "looper_leg_pairs": legs,
            "ms_links": round(ms_links, 5), "ms_links_and_legs": round(ms_legs, 5),
            "ms_refit": round(ms_refit, 5), "chains": heads, "multi_segment_chains": multi, "tracks": tracks,
            "segments_per_s": round(T / ms_legs * 1e3, 1)}


MERGE_CUT = 30.0


def leg_skip(args, with_cpu=True):
    """Row-skipping path on the headline frame with 10% pad-row inefficiency
    (neighbours across a missing row, seeding, the fit over the hits' rows)
    against the adjacent-row path on the same frame; HIP events per call on
    the launch stream."""
    import torch
    from tpcsynth import make_config
    fr = make_config(1, hit_eff=SKIP_EFF)
    N = fr.n_clusters
    reco = make_reco(fr)
    dfr = reco.upload(fr)
    ws = reco.workspace(dfr)
    up, dn = reco.neighbours_skip(dfr, ws=ws)
    seeds = reco.seed(dfr, up, dn, ws=ws)
    tr, rej = reco.fit_rows(dfr, seeds, ws=ws)
    up0, dn0 = reco.neighbours(dfr, ws=ws)
    seeds0 = reco.seed(dfr, up0, dn0, ws=ws)
    tr0 = reco.fit(dfr, seeds0, ws=ws)
    torch.cuda.synchronize()
    assert int(seeds.status.item()) == 0 and int(seeds0.status.item()) == 0
    stream = torch.cuda.current_stream()
    steps = max(5, args.steps)

    def run(calls):
        for _ in range(2):
            for c in calls:
                c()
        ev = []
        for _ in range(steps):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(len(calls) + 1)]
            e[0].record(stream)
            for k, c in enumerate(calls):
                c()
                e[k + 1].record(stream)
            ev.append(e)
        torch.cuda.synchronize()
        t = np.array([[e[k].elapsed_time(e[k + 1]) for k in range(len(calls))] for e in ev]).mean(0)
        return [round(float(v), 5) for v in t]

    ts = run([lambda: reco.neighbours_skip(dfr, up, dn, ws), lambda: reco.seed(dfr, up, dn, seeds, ws),
              lambda: reco.fit_rows(dfr, seeds, tracks=tr, rejected=rej, ws=ws)])
    ta = run([lambda: reco.neighbours(dfr, up0, dn0, ws), lambda: reco.seed(dfr, up0, dn0, seeds0, ws),
              lambda: reco.fit(dfr, seeds0, tracks=tr0, ws=ws)])
    sd, sd0 = seeds.to_numpy(), seeds0.to_numpy()
    T, H = len(sd["offsets"]) - 1, sd["hits"].size
    ms = sum(ts)
    flops = FLOP_FIT_PER_HIT * H
    res = {"workload": fr.meta["name"] + " with 10% pad-row inefficiency", "clusters": N,
           "hit_efficiency": SKIP_EFF,
           "skip": {"ms": round(ms, 5), "M_clusters_per_s": round(N / ms / 1e3, 3),
                    "stage_ms": dict(zip(("tpc_neighbours_skip", "tpc_ca_seed", "tpc_kalman_fit_rows"), ts)),
                    "linked_frac": round(float((up >= 0).float().mean().item()), 4),
                    "seeds": T, "seed_hits": H, "mean_seed_hits": round(H / max(T, 1), 2),
                    "pieces_80pct_in_one_seed": round(_one_seed_coverage(fr, sd), 4)},
           "adjacent": {"ms": round(sum(ta), 5), "M_clusters_per_s": round(N / sum(ta) / 1e3, 3),
                        "stage_ms": dict(zip(("tpc_neighbours", "tpc_ca_seed", "tpc_kalman_fit"), ta)),
                        "linked_frac": round(float((up0 >= 0).float().mean().item()), 4),
                        "seeds": len(sd0["offsets"]) - 1, "seed_hits": int(sd0["hits"].size),
                        "mean_seed_hits": round(sd0["hits"].size / max(len(sd0["offsets"]) - 1, 1), 2),
                        "pieces_80pct_in_one_seed": round(_one_seed_coverage(fr, sd0), 4)},
           "skip_pass_ms": round(ts[0] - ta[0], 5),
           "roofline": {"bound": "alu", "kernel": "fit_ms_tracks (rows)", "avg_ms": ts[2],
                        "achieved": round(flops / (ts[2] * 1e-3) / 1e12, 4), "peak": VALU_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(flops / (ts[2] * 1e-3) / 1e12 / VALU_PEAK_TFLOPS, 5),
                        "algorithmic_flops": int(flops)}}
    if with_cpu:
        import oracle
        oracle.set_threads(len(os.sched_getaffinity(0)))
        inf = float("inf")
        t0 = time.perf_counter()
        u, d = oracle.neighbours_skip(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)
        s = oracle.ca_seed(fr.row_offsets, u, d, fr.n_sectors, fr.n_rows, MIN_HITS)
        oracle.fit_rows(s, fr.row_offsets, fr.y, fr.z, fr.row_x, fr.n_sectors, fr.n_rows, err=None,
                        x0=inf, mass=0.0, chi2_cut=inf, **FIT)
        t = time.perf_counter() - t0
        res["cpu_oracle"] = {"ms": round(t * 1e3, 3), "cores": int(oracle.max_threads()),
                             "M_clusters_per_s": round(N / t / 1e6, 3)}
    return res


def leg_copy(args):
    """A plain device copy of known size (calibrates the HBM traffic counters)."""
    import torch
    n = 1 << 28                                   # 1 GiB of float32
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    ms = timed(lambda: b.copy_(a), 5, 1)
    return {"bytes_read": 4 * n, "bytes_written": 4 * n, "ms": round(ms, 4),
            "GB_per_s": round(8 * n / (ms * 1e-3) / 1e9, 1)}


def leg_stages(args):
    """Only the staged stage calls on one workload (for profilers)."""
    import torch
    from tpcsynth import make_config
    fr = make_config(args.stages_workload)
    reco = make_reco(fr)
    dfr = reco.upload(fr)
    ws = reco.workspace(dfr)
    up, dn, sd, tr = reco.reconstruct(dfr, "staged")
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        e[0].record(stream)
        reco.neighbours(dfr, up, dn, ws)
        e[1].record(stream)
        reco.seed(dfr, up, dn, sd, ws)
        e[2].record(stream)
        reco.fit(dfr, sd, None, tr, ws)
        e[3].record(stream)
        evs.append(e)
    torch.cuda.synchronize()
    st = np.array([[e[j].elapsed_time(e[j + 1]) for j in range(3)] for e in evs]).mean(axis=0)
    return {"workload": fr.meta["name"], "clusters": dfr.n_clusters, "steps": args.steps,
            "ms_per_step": round((time.perf_counter() - t0) / max(args.steps, 1) * 1e3, 5),
            "stage_ms": {"tpc_neighbours": round(float(st[0]), 5), "tpc_ca_seed": round(float(st[1]), 5),
                         "tpc_kalman_fit": round(float(st[2]), 5)}}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    legs = set(args.legs.split(","))
    if legs == {"copy"}:
        print(json.dumps({"copy": leg_copy(args)}), flush=True)
        return
    if legs == {"event"}:
        print(json.dumps({"event": leg_path(args, 1)[0]}), flush=True)
        return
    if legs == {"batched"}:
        print(json.dumps({"batched": leg_batched(args)}), flush=True)
        return
    if legs == {"adjoint"}:
        print(json.dumps({"adjoint": leg_adjoint(args)}), flush=True)
        return
    if legs == {"stages"}:
        print(json.dumps({"stages": leg_stages(args)}), flush=True)
        return
    if legs == {"follow"}:
        print(json.dumps({"follow": leg_follow(args, not args.no_cpu)}), flush=True)
        return
    if legs == {"material"}:
        print(json.dumps({"material": leg_material(args)}), flush=True)
        return
    if legs == {"ctf"}:
        print(json.dumps({"ctf": leg_ctf(args)}), flush=True)
        return
    if legs == {"skip"}:
        print(json.dumps({"skip": leg_skip(args, not args.no_cpu)}), flush=True)
        return
    if legs == {"rans"}:
        print(json.dumps({"rans": leg_rans(args, not args.no_cpu)}), flush=True)
        return
    if legs == {"merge"}:
        print(json.dumps({"merge": leg_merge(args)}), flush=True)
        return
    main_res, fr, host = leg_path(args, 2)
    out = {
        "metric": "M clusters/s through CA seed+Kalman fit (plain vs batched); adjoint grads/s",
        "value": main_res.pop("value"), "unit": "M clusters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": main_res.pop("ms_per_step"), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": main_res.pop("config"),
    }
    out.update(main_res)
    if "event" in legs:
        ev, _, _ = leg_path(args, 1)
        out["event"] = ev
    if "batched" in legs:
        out["batched"] = leg_batched(args)
    if "adjoint" in legs:
        out["adjoint"] = leg_adjoint(args)
    if "follow" in legs:
        out["follow"] = leg_follow(args, not args.no_cpu)
    if "rans" in legs:
        out["rans"] = leg_rans(args, not args.no_cpu)
    if "ctf" in legs:
        out["ctf"] = leg_ctf(args)
    if "material" in legs:
        out["material"] = leg_material(args)
    if "skip" in legs:
        out["skip"] = leg_skip(args, not args.no_cpu)
    if "merge" in legs:
        out["merge"] = leg_merge(args)
    if "copy" in legs:
        out["copy"] = leg_copy(args)
    if not args.no_cpu:
        out["cpu_baseline"], out["parity"] = cpu_baseline(fr, host, args.cpu_seconds)
        if not out["parity"]["ok"]:
            out["value"] = None              # no number for a run that fails parity
    else:
        out["parity"] = {"ok": None, "note": "not checked (--no-cpu)"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
