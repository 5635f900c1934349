"""Autotuner for the whole-path launch: picks the mode (staged kernels or one
persistent kernel), for the persistent kernel the grid size and the fit
order (longest seeds first or seed order), and the fit's launch shape
(workgroup size, seeds per thread: tracks per wavefront = 64 x that), by
timing each candidate on the caller's own frames.  Results are cached in a JSON file keyed by device and
workload shape (TPCRECO_TUNE_CACHE, default ~/.cache/tpcreco/tune.json).

Every candidate produces identical results; only the time differs.
"""
from __future__ import annotations

import json
import os
from typing import Optional

import torch

from .reco import DeviceFrames, Reco


def _cache_path() -> str:
    return os.environ.get("TPCRECO_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "tpcreco", "tune.json"))


def _key(reco: Reco, frames: DeviceFrames) -> str:
    name = torch.cuda.get_device_name(reco.device)
    return "%s|N=%d|F=%d|S=%d|R=%d" % (name, frames.n_clusters, frames.n_frames, reco.cfg.n_sectors,
                                        reco.cfg.n_rows)


def candidates(reco: Reco):
    """(mode, tune) pairs; tune = (grid, sort_fit, fit_block, fit_spt)."""
    cap = reco.persistent_grid()
    out = [("staged", None)]
    for fb in (64, 128, 256):
        for spt in (1, 2):
            if (fb, spt) != (256, 1):
                out.append(("staged", (0, 0, fb, spt)))
    for g in sorted({cap, max(1, cap // 2), max(1, cap // 4)}, reverse=True):
        for sf in (1, 0):
            out.append(("persistent", (g, sf, 0, 0)))
    out.append(("persistent", (cap, 1, 128, 1)))
    return out


def time_candidate(reco: Reco, frames: DeviceFrames, mode, tune, out, repeats=5) -> float:
    stream = torch.cuda.current_stream(reco.device)
    reco.reconstruct(frames, mode, tune, out)          # warm-up
    times = []
    for _ in range(repeats):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        reco.reconstruct(frames, mode, tune, out)
        b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2]


def autotune(reco: Reco, frames: DeviceFrames, use_cache: bool = True, repeats: int = 5) -> dict:
    """Returns {"mode": ..., "tune": (grid, sort_fit, fit_block, fit_spt) or None, "ms": ..., "table": [...]}."""
    path = _cache_path()
    key = _key(reco, frames)
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            e = cache[key]
            return {"mode": e["mode"], "tune": tuple(e["tune"]) if e["tune"] else None,
                    "ms": e["ms"], "table": e.get("table", []), "cached": True}
    out = None
    table = []
    best: Optional[dict] = None
    for mode, tune in candidates(reco):
        if out is None:
            out = reco.reconstruct(frames, mode, tune)
        ms = time_candidate(reco, frames, mode, tune, out, repeats)
        table.append({"mode": mode, "tune": list(tune) if tune else None, "ms": ms})
        if best is None or ms < best["ms"]:
            best = {"mode": mode, "tune": tune, "ms": ms}
    best["table"] = table
    best["cached"] = False
    if use_cache:
        cache[key] = {"mode": best["mode"], "tune": list(best["tune"]) if best["tune"] else None,
                      "ms": best["ms"], "table": table}
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return best
