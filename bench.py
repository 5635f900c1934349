"""Throughput of the TPC tracking path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

One step = neighbour finding + cellular-automaton seeding + Kalman fit of one
synthetic time frame whose clusters are already resident in device memory
(no host transfer inside the timed region).  The default workload is one
central Pb-Pb-like event over the full TPC: 36 sectors x 152 pad rows,
10^4 helix tracks (8% low-pT loopers, half truncated), 10% noise, about
1.3 M clusters.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Method parameters of the workload (cm, GeV/c, T).
NB = dict(win_y=2.5, win_z=2.5, cut_y=0.6, cut_z=0.75)
FIT = dict(bz=0.5, sigma_y=0.05, sigma_z=0.06, max_sin=0.999, var_sin0=1.0, var_tgl0=1.0,
           var_qpt0=100.0)
MIN_HITS = 5

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_VECTOR_PEAK = 157.3       # MI355X FP32 vector TFLOP/s

# Algorithmic traffic per unit (bytes): the method's own inputs and outputs at
# each stage boundary.
B_NB_PER_CLUSTER = 16          # read y, z; write up, dn
B_SEED_PER_CLUSTER = 8         # read up, dn
B_SEED_PER_HIT = 4             # write seed hit id
B_SEED_PER_SEED = 16           # write offset, frame, sector, first row
B_FIT_PER_HIT = 12             # read hit id, y, z
B_FIT_PER_TRACK = 24 + 96      # read seed record (offsets, first row, sector) + write 24 words


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="full-tpc-event-1e4")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    return ap.parse_args()


def cpu_baseline(fr, budget_s):
    """The oracle (as it stands) on the same frame, repeated within a time budget."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    oracle.set_threads(cores)
    times = []
    t_start = time.perf_counter()
    while True:
        t0 = time.perf_counter()
        up, dn = oracle.neighbours(fr.row_offsets, fr.y, fr.z, fr.n_rows, **NB)
        sd = oracle.ca_seed(fr.row_offsets, up, dn, fr.n_sectors, fr.n_rows, MIN_HITS)
        oracle.fit(sd, fr.y, fr.z, fr.row_x, fr.n_rows, **FIT)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() - t_start > budget_s or len(times) >= 20:
            break
    t = float(np.median(times))
    return {"value": fr.n_clusters / t / 1e6, "unit": "M clusters/s", "cores": int(oracle.max_threads()),
            "kind": "oracle",
            "sample": "whole frame (%d clusters), %d runs, median %.3f s; FP32 neighbours, "
                      "integer seeding, FP64 fit" % (fr.n_clusters, len(times), t)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2412_13755_amd.reco import Reco, RecoConfig
    from tpcsynth import make_config, CONFIG_NAMES

    k = CONFIG_NAMES.index(args.workload)
    fr = make_config(k)
    reco = Reco(RecoConfig(row_x=fr.row_x, n_sectors=fr.n_sectors, min_hits=MIN_HITS, **NB, **FIT),
                "cuda:0")
    dfr = reco.upload(fr)
    ws = reco.workspace(dfr)
    up = torch.empty(dfr.n_clusters, dtype=torch.int32, device="cuda")
    dn = torch.empty_like(up)
    seeds = reco.alloc_seeds(dfr)
    tracks = reco.alloc_tracks(seeds)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev:
            ev[0].record(stream)
        reco.neighbours(dfr, up, dn, ws)
        if ev:
            ev[1].record(stream)
        reco.seed(dfr, up, dn, seeds, ws)
        if ev:
            ev[2].record(stream)
        reco.fit(dfr, seeds, None, tracks, ws)
        if ev:
            ev[3].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    n_seeds = int(seeds.n_seeds.item())
    n_hits = int(seeds.n_hits.item())
    assert int(seeds.status.item()) == 0

    # whole-step timing
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = elapsed / args.steps * 1e3

    # per-stage timing with events on the launch stream (separate pass)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    st = np.array([[e[j].elapsed_time(e[j + 1]) for j in range(3)] for e in evs])  # ms
    stage_ms = st.mean(axis=0)
    N = dfr.n_clusters
    stage_bytes = [
        B_NB_PER_CLUSTER * N,
        B_SEED_PER_CLUSTER * N + B_SEED_PER_HIT * n_hits + B_SEED_PER_SEED * n_seeds,
        B_FIT_PER_HIT * n_hits + B_FIT_PER_TRACK * n_seeds,
    ]
    names = ["tpc_neighbours", "tpc_ca_seed", "tpc_kalman_fit"]
    dom = int(np.argmax(stage_ms))
    achieved = stage_bytes[dom] / (stage_ms[dom] * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None, "kernel": names[dom],
            "algorithmic_bytes": int(stage_bytes[dom]), "avg_ms": round(float(stage_ms[dom]), 5)}

    value = N / (ms * 1e-3) / 1e6
    out = {
        "metric": "M clusters/s through CA seed+Kalman fit (plain vs batched); adjoint grads/s",
        "value": round(value, 3), "unit": "M clusters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": fr.meta["name"], "clusters": N, "tracks_generated": fr.meta["n_tracks"],
                   "seeds": n_seeds, "seed_hits": n_hits, "sectors": fr.n_sectors, "rows": fr.n_rows,
                   "mode": "plain"},
        "tracks_per_s": round(n_seeds / (ms * 1e-3), 1),
        "stage_ms": {n: round(float(v), 5) for n, v in zip(names, stage_ms)},
        "roofline": roof,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(fr, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
