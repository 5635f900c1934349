"""Seeded synthetic TPC time frames: helix crossings of pad-row planes.

This module only produces inputs (cluster positions per frame, sector and pad
row, plus the truth behind them).  It contains none of the reconstruction
arithmetic: no neighbour search, no chaining, no track fit.  Both the CPU
oracle and the GPU library consume what it returns.

Geometry (a proposal; the paper fixes no detector numbers beyond the drift
volume being read out continuously in time frames, Sec. 4):

* ``n_sectors`` trapezoidal sectors; sector ``s`` has centre angle
  ``alpha_s = (s mod 18 + 1/2) * 20 deg`` and reads the A side (z > 0) for
  ``s < 18`` and the C side (z < 0) otherwise.  A single-sector geometry has
  ``alpha = 0`` and accepts both z signs.
* ``R`` pad rows per sector are planes at sector-local ``x = row_x[r]``,
  ``row_x[r] = fl32(85 + r * 160 / (R - 1))`` cm; a row is ``x * tan 10 deg``
  wide on either side of the centre line; the drift length is 250 cm.
* A track is a helix from the origin in a solenoidal field ``B_z``; its
  signed curvature (counter-clockwise positive) is ``-c * B_z * q / pT``.
  Crossings are exact circle/plane intersections in global coordinates, in
  float64, ordered by path length.

Randomness: one ``numpy.random.Generator(PCG64(seed))`` per call, drawn in a
fixed order, so a (config, seed) pair always yields the same frames.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

C_LIGHT = 0.00299792458          # cm^-1 GeV T^-1
TAN10 = math.tan(math.radians(10.0))
DRIFT_LENGTH = 250.0             # cm
R_OUTER = 250.0                  # cm, transverse radius at which a track leaves the gas volume
V_DRIFT = 2.5                    # cm / us (apparent z shift per us of collision time offset)


def make_row_x(n_rows: int = 152, x_first: float = 85.0, x_last: float = 245.0) -> np.ndarray:
    """Pad-row plane positions (float32), uniform pitch."""
    r = np.arange(n_rows, dtype=np.float64)
    return (x_first + r * (x_last - x_first) / (n_rows - 1)).astype(np.float32)


def sector_alpha(n_sectors: int) -> np.ndarray:
    if n_sectors == 1:
        return np.zeros(1)
    s = np.arange(n_sectors)
    return np.radians((s % 18 + 0.5) * 20.0)


def sector_side(n_sectors: int) -> np.ndarray:
    """+1 for A side (z>0), -1 for C side, 0 for a single sector reading both."""
    if n_sectors == 1:
        return np.zeros(1, dtype=np.int8)
    s = np.arange(n_sectors)
    return np.where(s < 18, 1, -1).astype(np.int8)


@dataclasses.dataclass
class Frames:
    """Clusters grouped per (frame, sector, row), global id order = storage order."""
    n_frames: int
    n_sectors: int
    n_rows: int
    row_x: np.ndarray            # float32 [R]
    row_offsets: np.ndarray      # int32 [F*S*R + 1]
    y: np.ndarray                # float32 [N]
    z: np.ndarray                # float32 [N]
    bz: float = 0.5
    sigma_y: float = 0.05
    sigma_z: float = 0.06
    # truth (optional)
    track_of: Optional[np.ndarray] = None     # int32 [N], -1 for noise
    y_true: Optional[np.ndarray] = None       # float64 [N] (local y before smearing, after shift/distortion)
    z_true: Optional[np.ndarray] = None
    s_true: Optional[np.ndarray] = None       # sin(phi) in the +x orientation
    t_true: Optional[np.ndarray] = None       # tan(lambda) in the +x orientation
    w_true: Optional[np.ndarray] = None       # q/pT in the +x orientation
    distortion: Optional[np.ndarray] = None   # float32 [S, R, 2] (dy, dz) added to the clusters
    meta: dict = dataclasses.field(default_factory=dict)
    err: Optional[np.ndarray] = None          # float32 [N, 2] per-cluster (sigma_y, sigma_z), if drawn

    @property
    def n_clusters(self) -> int:
        return int(self.y.shape[0])

    def row_slice(self, f: int, s: int, r: int) -> slice:
        i = (f * self.n_sectors + s) * self.n_rows + r
        return slice(int(self.row_offsets[i]), int(self.row_offsets[i + 1]))

    def frame_view(self, f: int) -> "Frames":
        """Frame ``f`` alone, with ids rebased to 0 (truth arrays sliced alike)."""
        SR = self.n_sectors * self.n_rows
        off = self.row_offsets[f * SR:(f + 1) * SR + 1]
        a, b = int(off[0]), int(off[-1])
        sl = slice(a, b)
        def cut(v):
            return None if v is None else v[sl]
        return Frames(1, self.n_sectors, self.n_rows, self.row_x, (off - a).astype(np.int32),
                      self.y[sl], self.z[sl], self.bz, self.sigma_y, self.sigma_z,
                      cut(self.track_of), cut(self.y_true), cut(self.z_true), cut(self.s_true),
                      cut(self.t_true), cut(self.w_true), self.distortion, dict(self.meta),
                      cut(self.err))


    def sector_view(self, f: int, s: int) -> "Frames":
        """Sector ``s`` of frame ``f`` alone, as a one-sector frame with ids
        rebased to 0 (its first cluster is global id ``first_id(f, s)``).
        Reconstruction within a sector never reads another sector, so a
        sector's links and seeds are those of the whole frame, rebased."""
        R = self.n_rows
        i0 = (f * self.n_sectors + s) * R
        off = self.row_offsets[i0:i0 + R + 1]
        a, b = int(off[0]), int(off[-1])
        sl = slice(a, b)

        def cut(v):
            return None if v is None else v[sl]
        return Frames(1, 1, R, self.row_x, (off - a).astype(np.int32), self.y[sl], self.z[sl], self.bz,
                      self.sigma_y, self.sigma_z, cut(self.track_of), cut(self.y_true), cut(self.z_true),
                      cut(self.s_true), cut(self.t_true), cut(self.w_true), None,
                      dict(self.meta, sector_of=(f, s), first_id=a), cut(self.err))

    def first_id(self, f: int, s: int) -> int:
        return int(self.row_offsets[(f * self.n_sectors + s) * self.n_rows])


# ----------------------------------------------------------------------------
# helix crossings

@dataclasses.dataclass
class Tracks:
    q: np.ndarray        # +-1
    inv_pt: np.ndarray   # 1/pT [GeV^-1] > 0
    phi0: np.ndarray     # direction at the origin (global)
    tgl: np.ndarray      # tan(lambda)
    nmax: np.ndarray     # crossings kept (truncation), large = all
    frame: np.ndarray    # frame index
    t0: np.ndarray       # collision time offset [us]

    def __len__(self):
        return int(self.q.shape[0])


def _crossings(tr: Tracks, row_x: np.ndarray, n_sectors: int, bz: float, max_turns: int,
               chunk: int = 4096):
    """All kept crossings of every track with every row plane, as flat arrays.

    Returns dict of arrays: track, sector, row, arc, y, z, s, t, w (truth in the
    +x orientation) ordered by (track, arc).
    """
    R = row_x.shape[0]
    xr = row_x.astype(np.float64)
    alpha = sector_alpha(n_sectors)
    side = sector_side(n_sectors)
    out = {k: [] for k in ("track", "sector", "row", "arc", "y", "z", "s", "t", "w")}
    for c0 in range(0, len(tr), chunk):
        c1 = min(len(tr), c0 + chunk)
        idx = np.arange(c0, c1)
        q = tr.q[idx].astype(np.float64)
        kap = -C_LIGHT * bz * q * tr.inv_pt[idx]          # signed curvature, ccw > 0
        Rc = 1.0 / np.abs(kap)
        ph0 = tr.phi0[idx]
        tgl = tr.tgl[idx]
        wtr = q * tr.inv_pt[idx]                           # q/pT
        cx = -np.sin(ph0) / kap                            # centre = origin + n / kappa, n = left normal
        cy = np.cos(ph0) / kap
        th0 = np.arctan2(-cy, -cx)
        looper = 2.0 * Rc < R_OUTER
        s_exit = np.where(looper, np.inf,
                          2.0 * np.arcsin(np.minimum(1.0, R_OUTER * np.abs(kap) / 2.0)) / np.abs(kap))
        zside = np.sign(tgl)
        # candidate sectors: global polar angle of the track at the radii each row plane spans
        if n_sectors == 1:
            pair_t = np.arange(len(idx))
            pair_s = np.zeros(len(idx), dtype=np.int64)
        else:
            # the polar angle of a branch is monotone in radius, so the sectors a
            # plane segment [x, x / cos 10deg] can be crossed in are those of its ends
            c10 = math.cos(math.radians(10.0))
            ak = np.abs(kap)[:, None]
            ua = ak * xr[None, :] / 2.0                                          # [n, R]
            ub = np.minimum(ak * xr[None, :] / (2.0 * c10), 1.0)
            ok = ua <= 1.0
            sg = np.sign(kap)[:, None]
            mask = np.zeros((len(idx), 18), dtype=bool)
            for uu in (ua, ub):
                a1 = np.arcsin(np.minimum(uu, 1.0))
                for psi, okb in ((ph0[:, None] + sg * a1, ok),
                                 (ph0[:, None] + sg * (math.pi - a1), ok & looper[:, None])):
                    sec18 = (np.floor(np.mod(psi, 2 * math.pi) / math.radians(20.0)).astype(np.int64)) % 18
                    rows_i, cols_i = np.nonzero(okb)
                    mask[rows_i, sec18[rows_i, cols_i]] = True
            pair_t, s18 = np.nonzero(mask)
            pair_s = np.where(zside[pair_t] >= 0, s18, s18 + 18)
        if pair_t.size == 0:
            continue
        al = alpha[pair_s]
        ux, uy = np.cos(al), np.sin(al)
        vx, vy = -uy, ux
        pcx, pcy = cx[pair_t], cy[pair_t]
        d = (ux * pcx + uy * pcy)[:, None] - xr[None, :]                  # [P, R]
        h2 = Rc[pair_t][:, None] ** 2 - d ** 2
        hval = np.sqrt(np.maximum(h2, 0.0))
        yc = (vx * pcx + vy * pcy)[:, None]
        for sgn in (1.0, -1.0):
            yl = yc + sgn * hval
            keep = (h2 >= 0.0) & (np.abs(yl) <= xr[None, :] * TAN10)
            if sgn < 0:
                keep &= h2 > 0.0            # tangent point counted once
            pi_, ri_ = np.nonzero(keep)
            if pi_.size == 0:
                continue
            ti = pair_t[pi_]
            dk, hk = d[pi_, ri_], hval[pi_, ri_]
            px = -dk * ux[pi_] + sgn * hk * vx[pi_]          # point minus centre
            py = -dk * uy[pi_] + sgn * hk * vy[pi_]
            th = np.arctan2(py, px)
            kk = kap[ti]
            dth = np.where(kk > 0, th - th0[ti], th0[ti] - th)
            arc0 = Rc[ti] * np.mod(dth, 2 * math.pi)
            ylv = yl[pi_, ri_]
            for turn in range(max_turns):
                arc = arc0 + turn * 2 * math.pi * Rc[ti]
                zz = tgl[ti] * arc
                sec = pair_s[pi_]
                ok = (arc <= s_exit[ti]) & (np.abs(zz) <= DRIFT_LENGTH)
                if n_sectors > 1:
                    ok &= np.where(side[sec] > 0, zz >= 0, zz < 0)
                if turn > 0:
                    ok &= looper[ti]
                if not ok.any():
                    break
                phi_loc = ph0[ti] + kk * arc - al[pi_]
                cphi = np.cos(phi_loc)
                fwd = cphi >= 0
                sfit = np.where(fwd, np.sin(phi_loc), -np.sin(phi_loc))
                tfit = np.where(fwd, tgl[ti], -tgl[ti])
                wfit = np.where(fwd, wtr[ti], -wtr[ti])
                sel = np.nonzero(ok)[0]
                out["track"].append(ti[sel] + c0)
                out["sector"].append(sec[sel])
                out["row"].append(ri_[sel])
                out["arc"].append(arc[sel])
                out["y"].append(ylv[sel])
                out["z"].append(zz[sel])
                out["s"].append(sfit[sel])
                out["t"].append(tfit[sel])
                out["w"].append(wfit[sel])
    res = {k: (np.concatenate(v) if v else np.zeros(0)) for k, v in out.items()}
    for k in ("track", "sector", "row"):
        res[k] = res[k].astype(np.int64)
    order = np.lexsort((res["arc"], res["track"]))
    res = {k: v[order] for k, v in res.items()}
    # truncation: keep the first nmax crossings of each track along its path
    if res["track"].size:
        t = res["track"]
        start = np.r_[0, np.nonzero(np.diff(t))[0] + 1]
        rank = np.arange(t.size) - np.repeat(start, np.diff(np.r_[start, t.size]))
        keep = rank < tr.nmax[t]
        res = {k: v[keep] for k, v in res.items()}
    return res


def _crossings_job(args):
    tr, row_x, n_sectors, bz, max_turns, base = args
    res = _crossings(tr, row_x, n_sectors, bz, max_turns)
    res["track"] = res["track"] + base
    return res


def _crossings_parallel(tr: Tracks, row_x, n_sectors, bz, max_turns, workers=None):
    """Same result as ``_crossings``; large track sets are split over threads
    (the work is numpy array code that runs without the interpreter lock).
    Threads, not forked processes: a fork of a process whose GPU runtime is
    already initialised (a profiler does that before the program starts)
    can deadlock in the child."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    n = len(tr)
    if workers is None:
        workers = min(16, len(os.sched_getaffinity(0)))
    if n < 20000 or workers <= 1:
        return _crossings(tr, row_x, n_sectors, bz, max_turns)
    bounds = np.linspace(0, n, workers * 4 + 1).astype(int)
    jobs = []
    for a, b in zip(bounds[:-1], bounds[1:]):
        sub = Tracks(*[getattr(tr, f.name)[a:b] for f in dataclasses.fields(Tracks)])
        jobs.append((sub, row_x, n_sectors, bz, max_turns, a))
    with ThreadPoolExecutor(workers) as pool:
        parts = list(pool.map(_crossings_job, jobs))
    return {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}


def _segment_order(key: np.ndarray, tieb: Optional[np.ndarray]) -> np.ndarray:
    """Permutation sorting by (key, tieb, original index): the order of
    ``np.lexsort((tieb, key))`` (``tieb`` None: by key, stable), computed as
    a sort by tieb followed by stable 16-bit radix passes over the key, which
    is several times faster on 10^7-10^8 clusters."""
    n = key.size
    if tieb is None:
        o1 = np.arange(n)
    else:
        o1 = np.argsort(tieb)
        t = tieb[o1]
        if np.any(t[1:] == t[:-1]):          # equal draws: keep their index order
            o1 = np.argsort(tieb, kind="stable")
    k = key[o1].astype(np.int64)
    if k.size and k.min() < 0:
        raise ValueError("negative segment key")
    shift = 0
    while shift == 0 or (k.size and (k.max() >> shift) > 0):
        part = ((k >> shift) & 0xFFFF).astype(np.uint16)
        p = np.argsort(part, kind="stable")
        o1 = o1[p]
        k = k[p]
        shift += 16
    return o1


def _draw_tracks(rng, n, phi_range, looper_frac, trunc_frac, n_rows, frame=0, t0=None):
    q = np.where(rng.random(n) < 0.5, -1, 1).astype(np.int8)
    inv_pt = rng.uniform(0.2, 5.0, n)
    if looper_frac > 0:
        lo = rng.random(n) < looper_frac
        inv_pt = np.where(lo, rng.uniform(1 / 0.3, 1 / 0.07, n), inv_pt)
    phi0 = rng.uniform(phi_range[0], phi_range[1], n)
    tgl = rng.uniform(-1.0, 1.0, n)
    nmax = np.full(n, 1 << 30, dtype=np.int64)
    if trunc_frac > 0:
        tr = rng.random(n) < trunc_frac
        nmax = np.where(tr, rng.integers(5, n_rows + 1, n), nmax)
    fr = np.full(n, frame, dtype=np.int32)
    tt = np.zeros(n) if t0 is None else t0
    return Tracks(q, inv_pt, phi0, tgl, nmax, fr, tt)


def _concat_tracks(parts: Sequence[Tracks]) -> Tracks:
    return Tracks(*[np.concatenate([getattr(p, f.name) for p in parts]) for f in dataclasses.fields(Tracks)])


def make_frames(*, n_sectors: int = 36, n_rows: int = 152, tracks_per_frame: Sequence[int] = (1000,),
                seed: int = 0, phi_range=(0.0, 2 * math.pi), looper_frac: float = 0.0,
                trunc_frac: float = 0.0, noise_frac: float = 0.0, n_collisions: int = 1,
                drift_window_us: float = 0.0, distortion_amp: float = 0.0, distortion_period: float = 38.0,
                bz: float = 0.5, sigma_y: float = 0.05, sigma_z: float = 0.06, smear: bool = True,
                shuffle: bool = True, max_turns: int = 3, keep_truth: bool = False,
                hit_eff: float = 1.0, tracks: Optional[Tracks] = None,
                err_scale: Optional[Sequence[float]] = None,
                noise_sectors: Optional[Sequence[int]] = None) -> Frames:
    """General generator; ``make_config`` fixes the parameters of the five workloads.

    ``err_scale=(lo, hi)`` gives every track cluster its own resolution: the
    nominal sigma_y and sigma_z times two independent factors drawn uniformly
    in [lo, hi], stored in ``err`` (noise clusters get the nominal values).
    ``noise_sectors`` puts the noise clusters only in the listed sectors
    (default: all), so that a frame whose tracks cover a few sectors keeps
    the noise density of a full frame there."""
    rng = np.random.Generator(np.random.PCG64(seed))
    row_x = make_row_x(n_rows)
    F = len(tracks_per_frame)
    if tracks is None:
        parts = []
        for f, nt in enumerate(tracks_per_frame):
            if n_collisions > 1:
                per = np.full(n_collisions, nt // n_collisions)
                per[: nt - per.sum()] += 1
                tcol = rng.uniform(0.0, drift_window_us, n_collisions)
                t0 = np.repeat(tcol, per)
            else:
                t0 = np.zeros(nt)
            parts.append(_draw_tracks(rng, nt, phi_range, looper_frac, trunc_frac, n_rows, f, t0))
        tracks = _concat_tracks(parts)
    cr = _crossings_parallel(tracks, row_x, n_sectors, bz, max_turns)
    if hit_eff < 1.0:
        # pad-row inefficiency: each crossing leaves a cluster with probability hit_eff
        keep = rng.random(cr["track"].size) < hit_eff
        cr = {k: v[keep] for k, v in cr.items()}
    n_sig = cr["track"].size
    y_true = cr["y"].copy()
    z_true = cr["z"].copy()
    frame = tracks.frame[cr["track"]].astype(np.int64)
    # drift shift: apparent z moves away from the membrane by v_drift * t0
    shift = V_DRIFT * tracks.t0[cr["track"]]
    zsgn = np.sign(z_true)
    zsgn[zsgn == 0] = 1.0
    z_true = z_true + zsgn * shift
    dist = None
    if distortion_amp > 0:
        amp = rng.uniform(0.0, distortion_amp, (n_sectors, 2))
        ph = rng.uniform(0.0, 2 * math.pi, (n_sectors, 2))
        r = np.arange(n_rows)
        dist = (amp[:, None, :] * np.sin(2 * math.pi * r[None, :, None] / distortion_period + ph[:, None, :]))
        dist = dist.astype(np.float32)
        y_true = y_true + dist[cr["sector"], cr["row"], 0].astype(np.float64)
        z_true = z_true + dist[cr["sector"], cr["row"], 1].astype(np.float64)
    fac = rng.uniform(err_scale[0], err_scale[1], (n_sig, 2)) if err_scale is not None else np.ones((n_sig, 2))
    if smear:
        ym = y_true + rng.normal(0.0, sigma_y * fac[:, 0], n_sig)
        zm = z_true + rng.normal(0.0, sigma_z * fac[:, 1], n_sig)
    else:
        ym, zm = y_true.copy(), z_true.copy()
    sec = cr["sector"]
    row = cr["row"]
    tid = cr["track"].astype(np.int64)
    # noise: a fraction of the total cluster count, uniform over rows and row area
    n_noise = int(round(noise_frac / (1.0 - noise_frac) * n_sig)) if noise_frac > 0 else 0
    if n_noise:
        nf = rng.integers(0, F, n_noise)
        if noise_sectors is None:
            ns = rng.integers(0, n_sectors, n_noise)
        else:
            ns = np.asarray(noise_sectors, dtype=np.int64)[rng.integers(0, len(noise_sectors), n_noise)]
        nr = rng.integers(0, n_rows, n_noise)
        half = row_x[nr].astype(np.float64) * TAN10
        ny = rng.uniform(-1.0, 1.0, n_noise) * half
        zmax = DRIFT_LENGTH + (V_DRIFT * drift_window_us if n_collisions > 1 else 0.0)
        sd = sector_side(n_sectors)[ns]
        zr = rng.uniform(0.0, zmax, n_noise)
        nz = np.where(sd > 0, zr, np.where(sd < 0, -zr, rng.uniform(-zmax, zmax, n_noise)))
        frame = np.concatenate([frame, nf])
        sec = np.concatenate([sec, ns])
        row = np.concatenate([row, nr])
        tid = np.concatenate([tid, np.full(n_noise, -1)])
        ym = np.concatenate([ym, ny])
        zm = np.concatenate([zm, nz])
        fac = np.concatenate([fac, np.ones((n_noise, 2))])
        nanv = np.full(n_noise, np.nan)
        y_true = np.concatenate([y_true, nanv])
        z_true = np.concatenate([z_true, nanv])
        st, tt, wt = (np.concatenate([cr[k], nanv]) for k in ("s", "t", "w"))
    else:
        st, tt, wt = cr["s"], cr["t"], cr["w"]
    key = (frame * n_sectors + sec) * n_rows + row
    tieb = rng.random(key.size) if shuffle else None
    order = _segment_order(key, tieb)
    NR = F * n_sectors * n_rows
    counts = np.bincount(key, minlength=NR)
    offs = np.zeros(NR + 1, dtype=np.int64)
    np.cumsum(counts, out=offs[1:])
    if offs[-1] >= 2 ** 31:
        raise ValueError("too many clusters for int32 ids")
    fr = Frames(F, n_sectors, n_rows, row_x, offs.astype(np.int32),
                ym[order].astype(np.float32), zm[order].astype(np.float32), bz, sigma_y, sigma_z)
    fr.track_of = tid[order].astype(np.int32)
    if keep_truth:
        fr.y_true, fr.z_true = y_true[order], z_true[order]
        fr.s_true, fr.t_true, fr.w_true = st[order], tt[order], wt[order]
    fr.distortion = dist
    if err_scale is not None:
        sig = np.stack([sigma_y * fac[order, 0], sigma_z * fac[order, 1]], 1)
        fr.err = np.ascontiguousarray(sig, dtype=np.float32)
    fr.meta = dict(n_tracks=len(tracks), n_signal=n_sig, n_noise=n_noise, seed=seed)
    fr.meta["tracks"] = tracks
    return fr


def drop_clusters(fr: Frames, keep: np.ndarray) -> Frames:
    """The clusters of ``fr`` where ``keep`` is true, in the same order, ids
    renumbered; truth arrays follow.  Used to plant gaps in tracks."""
    keep = np.asarray(keep, dtype=bool)
    seg = np.repeat(np.arange(fr.row_offsets.size - 1), np.diff(fr.row_offsets))
    counts = np.bincount(seg[keep], minlength=fr.row_offsets.size - 1)
    offs = np.zeros(fr.row_offsets.size, dtype=np.int32)
    np.cumsum(counts, out=offs[1:])
    def cut(v):
        return None if v is None else v[keep]
    return Frames(fr.n_frames, fr.n_sectors, fr.n_rows, fr.row_x, offs, fr.y[keep], fr.z[keep],
                  fr.bz, fr.sigma_y, fr.sigma_z, cut(fr.track_of), cut(fr.y_true), cut(fr.z_true),
                  cut(fr.s_true), cut(fr.t_true), cut(fr.w_true), fr.distortion, dict(fr.meta),
                  cut(fr.err))


def add_clusters(fr: Frames, frame, sector, row, y, z, track_of=None) -> Frames:
    """``fr`` with extra clusters appended at the end of their (frame, sector,
    row); ids renumbered, truth of the new clusters unknown (NaN)."""
    seg_new = (np.asarray(frame) * fr.n_sectors + np.asarray(sector)) * fr.n_rows + np.asarray(row)
    seg_old = np.repeat(np.arange(fr.row_offsets.size - 1), np.diff(fr.row_offsets))
    seg = np.concatenate([seg_old, seg_new])
    order = np.argsort(seg, kind="stable")
    counts = np.bincount(seg, minlength=fr.row_offsets.size - 1)
    offs = np.zeros(fr.row_offsets.size, dtype=np.int32)
    np.cumsum(counts, out=offs[1:])
    k = seg_new.size
    tof = np.full(k, -1, np.int32) if track_of is None else np.asarray(track_of, np.int32)
    def cat(v, extra):
        return None if v is None else np.concatenate([v, extra])[order]
    nan = np.full(k, np.nan)
    return Frames(fr.n_frames, fr.n_sectors, fr.n_rows, fr.row_x, offs,
                  cat(fr.y, np.asarray(y, np.float32)), cat(fr.z, np.asarray(z, np.float32)),
                  fr.bz, fr.sigma_y, fr.sigma_z, cat(fr.track_of, tof), cat(fr.y_true, nan),
                  cat(fr.z_true, nan), cat(fr.s_true, nan), cat(fr.t_true, nan), cat(fr.w_true, nan),
                  fr.distortion, dict(fr.meta),
                  None if fr.err is None else np.concatenate(
                      [fr.err, np.tile(np.float32([fr.sigma_y, fr.sigma_z]), (k, 1))])[order])


CONFIG_NAMES = (
    "single-sector-200",
    "full-tpc-event-1e4",
    "continuous-tf-50x1e4",
    "batched-64-uneven",
    "differentiable-1e5",
)


def config_params(k: int, scale: float = 1.0) -> dict:
    """Generator parameters of the five workloads; ``scale`` shrinks track counts."""
    def n(v):
        return max(1, int(round(v * scale)))
    if k == 0:
        return dict(n_sectors=1, tracks_per_frame=(n(200),), seed=0,
                    phi_range=(-math.radians(10.0), math.radians(10.0)), noise_frac=0.05)
    if k == 1:
        return dict(n_sectors=36, tracks_per_frame=(n(10000),), seed=1, looper_frac=0.08,
                    trunc_frac=0.5, noise_frac=0.10)
    if k == 2:
        return dict(n_sectors=36, tracks_per_frame=(n(500000),), seed=2, looper_frac=0.08,
                    trunc_frac=0.5, noise_frac=0.10, n_collisions=50, drift_window_us=100.0)
    if k == 3:
        rng = np.random.Generator(np.random.PCG64(1003))
        counts = np.floor(np.exp(rng.uniform(math.log(100), math.log(20000), 64))).astype(int)
        return dict(n_sectors=36, tracks_per_frame=tuple(n(c) for c in counts), seed=3,
                    looper_frac=0.08, trunc_frac=0.5, noise_frac=0.10)
    if k == 4:
        return dict(n_sectors=36, tracks_per_frame=(n(100000),), seed=4, looper_frac=0.08,
                    trunc_frac=0.5, noise_frac=0.10, distortion_amp=0.5)
    raise ValueError(k)


def make_config(k: int, scale: float = 1.0, keep_truth: bool = False, **over) -> Frames:
    p = config_params(k, scale)
    p.update(over)
    fr = make_frames(keep_truth=keep_truth, **p)
    fr.meta["config"] = k
    fr.meta["name"] = CONFIG_NAMES[k]
    fr.meta["scale"] = scale
    return fr


HIGHLAND = 0.0136                 # GeV, multiple-scattering constant
PION_MASS = 0.13957               # GeV


def highland_theta0(p, beta, x_over_x0):
    """Width of the projected scattering angle (Highland): 13.6 MeV / (beta p) sqrt(x/X0) (1 + 0.038 ln(x/X0))."""
    return HIGHLAND / (beta * p) * np.sqrt(x_over_x0) * (1.0 + 0.038 * np.log(x_over_x0))


PROTON_MASS = 0.93827             # GeV
ELECTRON_MASS = 0.51099895e-3     # GeV
BETHE_K = 0.307075e-3             # GeV cm^2 / mol
# (density g/cm^3, Z/A mol/g, mean excitation energy GeV)
ARGON_GAS = (1.662e-3, 0.45059, 188.0e-9)
# Ne-CO2-N2 90-10-5 by volume at 20 C, from its components by mass
# fraction (Z/A averaged, ln I averaged with weights w Z/A)
TPC_GAS = (0.948e-3, 0.4966, 121.8e-9)


def mean_dedx(p, mass, rho, z_over_a, mean_exc):
    """Mean energy loss per cm, GeV/cm, of unit-charge particles of momentum p
    (GeV/c) in a material (Bethe formula, no density effect)."""
    e = np.hypot(p, mass)
    beta2 = (p / e) ** 2
    bg2 = (p / mass) ** 2
    ratio = ELECTRON_MASS / mass
    wmax = 2.0 * ELECTRON_MASS * bg2 / (1.0 + 2.0 * (e / mass) * ratio + ratio * ratio)
    arg = 2.0 * ELECTRON_MASS * bg2 * wmax / (mean_exc * mean_exc)
    return BETHE_K * z_over_a * rho / beta2 * (0.5 * np.log(arg) - beta2)


def make_scattering_frame(*, n_tracks: int = 200, seed: int = 0, x0_cm: float = 300.0,
                          mass: float = PION_MASS, inv_pt=(0.5, 3.0), phi_range=(-0.06, 0.06),
                          tgl_range=(-0.8, 0.8), n_rows: int = 152, bz: float = 0.5,
                          sigma_y: float = 0.05, sigma_z: float = 0.06, smear: bool = True,
                          gas=None) -> Frames:
    """One sector (alpha = 0) of tracks stepped plane by plane with multiple scattering.

    Each track starts at the origin; from one pad-row plane to the next its
    exact helix in global coordinates (circle in x-y, straight in z against
    the transverse path) is intersected with the plane; after every crossing
    but the first, the direction receives two independent Gaussian kicks of
    width theta0 (Highland, with the 3-D path of the segment just traversed
    and the momentum and velocity for the given mass): one in the bending
    plane (phi changes by theta1 / cos(lambda)) and one in lambda; the total
    momentum is kept, so pT and the curvature follow lambda -- unless a gas
    (density, Z/A, mean excitation energy) is given: then the particle also
    loses energy over the segment, the mean loss integrated in 8 sub-steps of
    the path with the Bethe formula (mean_dedx) and a Gaussian fluctuation of
    Bohr's width (relativistic), and stops when it has no kinetic energy
    left.  A track stops when it misses the next plane or leaves the row
    width.  Truth at every
    cluster: y, z and the direction (s, t, w) of the segment leaving it.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    row_x = make_row_x(n_rows).astype(np.float64)
    n = n_tracks
    q = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    ipt = rng.uniform(inv_pt[0], inv_pt[1], n)
    phi = rng.uniform(phi_range[0], phi_range[1], n)
    lam = np.arctan(rng.uniform(tgl_range[0], tgl_range[1], n))
    p = 1.0 / (ipt * np.cos(lam))                      # total momentum, kept
    X = np.zeros(n)
    Y = np.zeros(n)
    Z = np.zeros(n)
    alive = np.ones(n, bool)
    recs = []
    for k in range(n_rows):
        xk = row_x[k]
        pt = p * np.cos(lam)
        kap = -C_LIGHT * bz * q / pt                 # signed curvature, ccw > 0
        cx = X - np.sin(phi) / kap
        cy = Y + np.cos(phi) / kap
        R = 1.0 / np.abs(kap)
        h2 = R * R - (xk - cx) ** 2
        ok = alive & (h2 > 0)
        h = np.sqrt(np.where(ok, h2, 0.0))
        # the crossing reached first along the motion: smallest positive turn
        th0 = np.arctan2(Y - cy, X - cx)
        best_turn = np.full(n, np.inf)
        best_y = np.zeros(n)
        for sg in (1.0, -1.0):
            yc = cy + sg * h
            th = np.arctan2(yc - cy, xk - cx)
            turn = np.where(kap > 0, th - th0, th0 - th)
            turn = np.mod(turn, 2 * math.pi)
            better = ok & (turn > 1e-12) & (turn < best_turn)
            best_turn = np.where(better, turn, best_turn)
            best_y = np.where(better, yc, best_y)
        ok &= np.isfinite(best_turn) & (best_turn < math.pi / 2)
        sxy = np.where(ok, R * best_turn, 0.0)
        Xn, Yn = np.full(n, xk), best_y
        Zn = Z + np.tan(lam) * sxy
        phin = phi + kap * sxy
        ok &= np.abs(Yn) <= xk * TAN10
        ok &= np.abs(Zn) <= DRIFT_LENGTH
        alive = ok
        if not alive.any():
            break
        # direction leaving this plane: kicked after every crossing but the first
        lamn = lam.copy()
        if k > 0:
            path = sxy * np.sqrt(1.0 + np.tan(lam) ** 2)
            beta = p / np.sqrt(p * p + mass * mass)
            th0s = highland_theta0(p, beta, np.maximum(path, 1e-12) / x0_cm)
            k1 = rng.normal(0.0, 1.0, n) * th0s
            k2 = rng.normal(0.0, 1.0, n) * th0s
            phin = phin + np.where(alive, k1 / np.cos(lam), 0.0)
            lamn = lam + np.where(alive, k2, 0.0)
            if gas is not None:
                rho, zoa, exc = gas
                e = np.hypot(p, mass)
                e0 = e.copy()
                pc = p.copy()
                for _ in range(8):
                    e = e - mean_dedx(pc, mass, rho, zoa, exc) * path / 8.0
                    pc = np.sqrt(np.maximum(e * e - mass * mass, 1e-30))
                b2 = (p / e0) ** 2
                var_e = BETHE_K * zoa * rho * path * ELECTRON_MASS * (1.0 - 0.5 * b2) / (1.0 - b2)
                e = e + rng.normal(0.0, 1.0, n) * np.sqrt(var_e)
                alive &= e > mass * 1.001
                p = np.where(alive, np.sqrt(np.maximum(e * e - mass * mass, 1e-30)), p)
        idx = np.nonzero(alive)[0]
        recs.append((idx, np.full(idx.size, k), Yn[idx], Zn[idx], np.sin(phin[idx]), np.tan(lamn[idx]),
                     q[idx] / (p[idx] * np.cos(lamn[idx]))))
        X, Y, Z, phi, lam = Xn, np.where(alive, Yn, Y), np.where(alive, Zn, Z), phin, lamn
    tid = np.concatenate([r[0] for r in recs])
    row = np.concatenate([r[1] for r in recs])
    yt = np.concatenate([r[2] for r in recs])
    zt = np.concatenate([r[3] for r in recs])
    st_ = np.concatenate([r[4] for r in recs])
    tt_ = np.concatenate([r[5] for r in recs])
    wt_ = np.concatenate([r[6] for r in recs])
    ym = yt + (rng.normal(0.0, sigma_y, yt.size) if smear else 0.0)
    zm = zt + (rng.normal(0.0, sigma_z, zt.size) if smear else 0.0)
    order = np.lexsort((tid, row))
    counts = np.bincount(row, minlength=n_rows)
    offs = np.zeros(n_rows + 1, dtype=np.int32)
    np.cumsum(counts, out=offs[1:])
    fr = Frames(1, 1, n_rows, row_x.astype(np.float32), offs, ym[order].astype(np.float32),
                zm[order].astype(np.float32), bz, sigma_y, sigma_z)
    fr.track_of = tid[order].astype(np.int32)
    fr.y_true, fr.z_true = yt[order], zt[order]
    fr.s_true, fr.t_true, fr.w_true = st_[order], tt_[order], wt_[order]
    fr.meta = dict(n_tracks=n, seed=seed, x0_cm=x0_cm, mass=mass)
    return fr
