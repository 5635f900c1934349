"""Python face of libtpcreco: torch tensors in, torch tensors out.

Every computation runs in the library's HIP kernels; this module only
allocates device memory with torch, fills the C structs and passes the
current torch stream.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional

import numpy as np
import torch

from . import _capi as C


@dataclasses.dataclass
class RecoConfig:
    """Reconstruction constants (cm, GeV/c, T).  See include/tpcreco.h."""
    row_x: np.ndarray
    n_sectors: int = 36
    bz: float = 0.5
    sigma_y: float = 0.05
    sigma_z: float = 0.06
    win_y: float = 2.5
    win_z: float = 2.5
    cut_y: float = 0.6
    cut_z: float = 0.75
    min_hits: int = 5
    max_sin: float = 0.999
    var_sin0: float = 1.0
    var_tgl0: float = 1.0
    var_qpt0: float = 100.0
    ckpt_rows: int = 16

    @property
    def n_rows(self) -> int:
        return int(len(self.row_x))


class DeviceFrames:
    """Clusters of ``n_frames`` frames resident on the device."""

    def __init__(self, row_offsets: torch.Tensor, y: torch.Tensor, z: torch.Tensor, n_frames: int,
                 offsets_host: Optional[np.ndarray] = None):
        self.row_offsets, self.y, self.z = row_offsets, y, z
        self.offsets_host = offsets_host
        self.n_frames = int(n_frames)
        self.n_clusters = int(y.numel())
        self.c = C.FramesC(self.n_frames, self.n_clusters, row_offsets.data_ptr(),
                           y.data_ptr() if self.n_clusters else None,
                           z.data_ptr() if self.n_clusters else None)

    @staticmethod
    def from_numpy(row_offsets, y, z, n_frames, n_sectors, n_rows, device="cuda") -> "DeviceFrames":
        off = np.ascontiguousarray(row_offsets, dtype=np.int64)
        if off.ndim != 1 or off.size != n_frames * n_sectors * n_rows + 1:
            raise ValueError("row_offsets must have n_frames*n_sectors*n_rows+1 entries")
        if off[0] != 0 or np.any(np.diff(off) < 0) or off[-1] != len(y) or len(y) != len(z):
            raise ValueError("row_offsets must start at 0, not decrease and end at len(y)")
        if off[-1] + off.size >= 2 ** 31:
            raise ValueError("too many clusters for int32 ids")
        t_off = torch.from_numpy(off.astype(np.int32)).to(device)
        t_y = torch.from_numpy(np.ascontiguousarray(y, dtype=np.float32)).to(device)
        t_z = torch.from_numpy(np.ascontiguousarray(z, dtype=np.float32)).to(device)
        return DeviceFrames(t_off, t_y, t_z, n_frames, off)

    def frame_view(self, f: int, segments_per_frame: int) -> "DeviceFrames":
        """Frame ``f`` alone: cluster ids rebased to 0 (y, z are views)."""
        off = self.offsets_host[f * segments_per_frame:(f + 1) * segments_per_frame + 1]
        a, b = int(off[0]), int(off[-1])
        t_off = torch.from_numpy((off - a).astype(np.int32)).to(self.y.device)
        return DeviceFrames(t_off, self.y[a:b], self.z[a:b], 1, off - a)


@dataclasses.dataclass
class Seeds:
    n_seeds: torch.Tensor      # device int32 scalar
    n_hits: torch.Tensor
    offsets: torch.Tensor
    hits: torch.Tensor
    frame: torch.Tensor
    sector: torch.Tensor
    first_row: torch.Tensor
    status: torch.Tensor       # device int32 status word
    hit_yz: Optional[torch.Tensor] = None   # [cap_hits, 2] float32 seed-hit coordinates, or None

    def c(self) -> C.SeedsC:
        return C.SeedsC(self.frame.numel(), self.hits.numel(), self.n_seeds.data_ptr(),
                        self.n_hits.data_ptr(), self.offsets.data_ptr(), self.hits.data_ptr(),
                        self.frame.data_ptr(), self.sector.data_ptr(), self.first_row.data_ptr(),
                        self.hit_yz.data_ptr() if self.hit_yz is not None else None)

    def to_numpy(self) -> dict:
        ns = int(self.n_seeds.item())
        nh = int(self.n_hits.item())
        return dict(offsets=self.offsets[:ns + 1].cpu().numpy(), hits=self.hits[:nh].cpu().numpy(),
                    frame=self.frame[:ns].cpu().numpy(), sector=self.sector[:ns].cpu().numpy(),
                    first_row=self.first_row[:ns].cpu().numpy())


@dataclasses.dataclass
class Tracks:
    x: torch.Tensor
    par: torch.Tensor
    cov: torch.Tensor
    chi2: torch.Tensor
    ndf: torch.Tensor
    status: torch.Tensor

    def c(self) -> C.TracksC:
        return C.TracksC(self.x.data_ptr(), self.par.data_ptr(), self.cov.data_ptr(),
                         self.chi2.data_ptr(), self.ndf.data_ptr(), self.status.data_ptr())


def _stream_handle(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Reco:
    """One reconstruction context on one device."""

    def __init__(self, cfg: RecoConfig, device: str = "cuda:0"):
        self.cfg = cfg
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the reconstruction runs on a HIP device only")
        self._row_x = np.ascontiguousarray(cfg.row_x, dtype=np.float32)
        cc = C.Config(cfg.n_sectors, len(self._row_x), self._row_x.ctypes.data_as(ctypes.c_void_p),
                      cfg.bz, cfg.sigma_y, cfg.sigma_z, cfg.win_y, cfg.win_z, cfg.cut_y, cfg.cut_z,
                      cfg.min_hits, cfg.max_sin, cfg.var_sin0, cfg.var_tgl0, cfg.var_qpt0,
                      cfg.ckpt_rows)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            C.check(C.lib().tpc_create(ctypes.byref(cc), ctypes.byref(h)))
        self._ctx = h
        self._ws: Optional[torch.Tensor] = None

    def close(self):
        if getattr(self, "_ctx", None):
            C.lib().tpc_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------
    def workspace_bytes(self, frames: DeviceFrames, stages: int = C.TPC_STAGE_ALL) -> int:
        n = ctypes.c_size_t()
        C.check(C.lib().tpc_workspace_bytes(self._ctx, ctypes.byref(frames.c), stages, ctypes.byref(n)))
        return int(n.value)

    def workspace(self, frames: DeviceFrames, stages: int = C.TPC_STAGE_ALL) -> torch.Tensor:
        """A cached workspace (grown on demand) large enough for ``stages``."""
        need = max(256, self.workspace_bytes(frames, stages))
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._ws

    def upload(self, fr) -> DeviceFrames:
        """Frames object with numpy fields (row_offsets, y, z, n_frames) -> device."""
        return DeviceFrames.from_numpy(fr.row_offsets, fr.y, fr.z, fr.n_frames, self.cfg.n_sectors,
                                       self.cfg.n_rows, self.device)

    # ------------------------------------------------------------------
    def neighbours(self, frames: DeviceFrames, up=None, dn=None, ws=None):
        N = frames.n_clusters
        up = torch.empty(N, dtype=torch.int32, device=self.device) if up is None else up
        dn = torch.empty(N, dtype=torch.int32, device=self.device) if dn is None else dn
        ws = self.workspace(frames) if ws is None else ws
        C.check(C.lib().tpc_neighbours(self._ctx, ctypes.byref(frames.c), up.data_ptr(), dn.data_ptr(),
                                       ws.data_ptr(), ws.numel(), _stream_handle(self.device)))
        return up, dn

    def neighbours_skip(self, frames: DeviceFrames, up=None, dn=None, ws=None):
        """tpc_neighbours_skip: partners up to two rows away where the
        adjacent rows give none."""
        N = frames.n_clusters
        up = torch.empty(N, dtype=torch.int32, device=self.device) if up is None else up
        dn = torch.empty(N, dtype=torch.int32, device=self.device) if dn is None else dn
        ws = self.workspace(frames) if ws is None else ws
        C.check(C.lib().tpc_neighbours_skip(self._ctx, ctypes.byref(frames.c), up.data_ptr(), dn.data_ptr(),
                                            ws.data_ptr(), ws.numel(), _stream_handle(self.device)))
        return up, dn

    def alloc_seeds(self, frames: DeviceFrames, cap_seeds=None, cap_hits=None, hit_yz=True) -> Seeds:
        """Seed buffers; with hit_yz the seeding also stores the coordinates of
        every seed hit, which the fit and the adjoint then read directly."""
        N = frames.n_clusters
        # every seed holds >= min_hits distinct clusters: these bounds never overflow
        cs = N // self.cfg.min_hits + 1 if cap_seeds is None else int(cap_seeds)
        ch = max(N, 1) if cap_hits is None else int(cap_hits)
        d, i = self.device, torch.int32
        return Seeds(torch.zeros(1, dtype=i, device=d), torch.zeros(1, dtype=i, device=d),
                     torch.zeros(cs + 1, dtype=i, device=d), torch.empty(ch, dtype=i, device=d),
                     torch.empty(cs, dtype=i, device=d), torch.empty(cs, dtype=i, device=d),
                     torch.empty(cs, dtype=i, device=d), torch.zeros(1, dtype=i, device=d),
                     torch.empty(ch, 2, dtype=torch.float32, device=d) if hit_yz else None)

    def seed(self, frames: DeviceFrames, up, dn, seeds: Optional[Seeds] = None, ws=None) -> Seeds:
        seeds = self.alloc_seeds(frames) if seeds is None else seeds
        ws = self.workspace(frames) if ws is None else ws
        sc = seeds.c()
        C.check(C.lib().tpc_ca_seed(self._ctx, ctypes.byref(frames.c), up.data_ptr(), dn.data_ptr(),
                                    ctypes.byref(sc), seeds.status.data_ptr(), ws.data_ptr(),
                                    ws.numel(), _stream_handle(self.device)))
        return seeds

    def seed_noalloc(self, frames: DeviceFrames, up, dn, seeds: Seeds) -> Seeds:
        """tpc_ca_seed_noalloc: seeding into caller-allocated ``seeds`` with
        the library's built-in scratch (no allocation in the call)."""
        sc = seeds.c()
        C.check(C.lib().tpc_ca_seed_noalloc(self._ctx, ctypes.byref(frames.c), up.data_ptr(), dn.data_ptr(),
                                            ctypes.byref(sc), seeds.status.data_ptr(),
                                            _stream_handle(self.device)))
        return seeds

    def alloc_tracks(self, seeds: Seeds) -> Tracks:
        T = seeds.frame.numel()
        d = self.device
        return Tracks(torch.empty(T, device=d), torch.empty(T, 5, device=d), torch.empty(T, 15, device=d),
                      torch.empty(T, device=d), torch.empty(T, dtype=torch.int32, device=d),
                      torch.empty(T, dtype=torch.int32, device=d))

    def _check_map(self, map_):
        if map_ is not None:
            if map_.dtype != torch.float32 or not map_.is_contiguous() or map_.device != self.device or \
                    tuple(map_.shape) != (self.cfg.n_sectors, self.cfg.n_rows, 2):
                raise ValueError("map must be a contiguous float32 [n_sectors, n_rows, 2] device tensor")

    def ckpt_bytes(self, seeds: Seeds) -> int:
        n = ctypes.c_size_t()
        sc = seeds.c()
        C.check(C.lib().tpc_ckpt_bytes(self._ctx, ctypes.byref(sc), ctypes.byref(n)))
        return int(n.value)

    def alloc_ckpt(self, seeds: Seeds) -> torch.Tensor:
        return torch.empty(self.ckpt_bytes(seeds) // 8, dtype=torch.float64, device=self.device)

    def fit(self, frames: DeviceFrames, seeds: Seeds, map_: Optional[torch.Tensor] = None,
            tracks: Optional[Tracks] = None, ws=None, ckpt: Optional[torch.Tensor] = None) -> Tracks:
        tracks = self.alloc_tracks(seeds) if tracks is None else tracks
        ws = self.workspace(frames) if ws is None else ws
        self._check_map(map_)
        sc = seeds.c()
        tc = tracks.c()
        C.check(C.lib().tpc_kalman_fit(self._ctx, ctypes.byref(frames.c), ctypes.byref(sc),
                                       None if map_ is None else map_.data_ptr(), ctypes.byref(tc),
                                       None if ckpt is None else ckpt.data_ptr(),
                                       0 if ckpt is None else ckpt.numel() * ckpt.element_size(),
                                       ws.data_ptr(), ws.numel(), _stream_handle(self.device)))
        return tracks

    def fit_material(self, frames: DeviceFrames, seeds: Seeds, x0: float, mass: float, chi2_cut: float,
                     tracks: Optional[Tracks] = None, rejected: Optional[torch.Tensor] = None, ws=None,
                     gas: Optional[tuple] = None):
        """tpc_kalman_fit_material, with energy loss in ``gas`` = (rho g/cm^3,
        Z/A, mean excitation energy GeV) if given: returns (Tracks, rejected
        uint8 per seed hit)."""
        tracks = self.alloc_tracks(seeds) if tracks is None else tracks
        if rejected is None:
            rejected = torch.zeros(max(seeds.hits.numel(), 1), dtype=torch.uint8, device=self.device)
        ws = self.workspace(frames) if ws is None else ws
        mat = C.Material(float(x0), float(mass), float(chi2_cut), *(float(v) for v in (gas or ())))
        sc = seeds.c()
        tc = tracks.c()
        C.check(C.lib().tpc_kalman_fit_material(self._ctx, ctypes.byref(frames.c), ctypes.byref(sc),
                                                ctypes.byref(mat), ctypes.byref(tc), rejected.data_ptr(),
                                                ws.data_ptr(), ws.numel(), _stream_handle(self.device)))
        return tracks, rejected

    def fit_rows(self, frames: DeviceFrames, seeds: Seeds, cluster_err: Optional[torch.Tensor] = None,
                 material: Optional[tuple] = None, tracks: Optional[Tracks] = None,
                 rejected: Optional[torch.Tensor] = None, ws=None):
        """tpc_kalman_fit_rows: seeds whose hits may skip pad rows, optional
        per-cluster errors ([N, 2] float32 sigma_y, sigma_z on the device) and
        material (x0, mass, chi2_cut), optionally followed by the gas for
        energy loss (rho, Z/A, mean excitation energy).  Returns (Tracks,
        rejected)."""
        tracks = self.alloc_tracks(seeds) if tracks is None else tracks
        if rejected is None:
            rejected = torch.zeros(max(seeds.hits.numel(), 1), dtype=torch.uint8, device=self.device)
        ws = self.workspace(frames) if ws is None else ws
        err = 0
        if cluster_err is not None:
            if (cluster_err.dtype != torch.float32 or cluster_err.device.type != self.device.type
                    or tuple(cluster_err.shape) != (frames.n_clusters, 2) or not cluster_err.is_contiguous()):
                raise ValueError("cluster_err must be a contiguous float32 [n_clusters, 2] tensor on the device")
            err = cluster_err.data_ptr()
        mat = None if material is None else ctypes.byref(C.Material(*(float(v) for v in material)))
        sc = seeds.c()
        tc = tracks.c()
        C.check(C.lib().tpc_kalman_fit_rows(self._ctx, ctypes.byref(frames.c), ctypes.byref(sc), err, mat,
                                            ctypes.byref(tc), rejected.data_ptr(), ws.data_ptr(), ws.numel(),
                                            _stream_handle(self.device)))
        return tracks, rejected

    def smooth(self, frames: DeviceFrames, seeds: Seeds, cluster_err: Optional[torch.Tensor] = None,
               material: Optional[tuple] = None, tracks: Optional[Tracks] = None, ws=None):
        """tpc_kalman_smooth: the fit over rows, then the state at every seed
        hit's plane.  Returns (Tracks, rejected, hit_par [cap_hits, 5],
        hit_cov [cap_hits, 15])."""
        tracks = self.alloc_tracks(seeds) if tracks is None else tracks
        H = max(seeds.hits.numel(), 1)
        rejected = torch.zeros(H, dtype=torch.uint8, device=self.device)
        hit_par = torch.empty(H, 5, dtype=torch.float32, device=self.device)
        hit_cov = torch.empty(H, 15, dtype=torch.float32, device=self.device)
        ws = self.workspace(frames) if ws is None else ws
        err = 0
        if cluster_err is not None:
            if (cluster_err.dtype != torch.float32 or cluster_err.device.type != self.device.type
                    or tuple(cluster_err.shape) != (frames.n_clusters, 2) or not cluster_err.is_contiguous()):
                raise ValueError("cluster_err must be a contiguous float32 [n_clusters, 2] tensor on the device")
            err = cluster_err.data_ptr()
        mat = None if material is None else ctypes.byref(C.Material(*(float(v) for v in material)))
        sc = seeds.c()
        tc = tracks.c()
        C.check(C.lib().tpc_kalman_smooth(self._ctx, ctypes.byref(frames.c), ctypes.byref(sc), err, mat,
                                          ctypes.byref(tc), rejected.data_ptr(), hit_par.data_ptr(),
                                          hit_cov.data_ptr(), ws.data_ptr(), ws.numel(),
                                          _stream_handle(self.device)))
        return tracks, rejected, hit_par, hit_cov

    def follow(self, frames: DeviceFrames, seeds: Seeds, gate_chi2: float, max_miss: int,
               rows: Optional[torch.Tensor] = None, tracks: Optional[Tracks] = None, ws=None):
        """Track following of every seed and duplicate removal (tpc_track_follow).

        Returns (rows [cap_seeds, n_rows] int32, Tracks); rows and tracks are
        valid for the first n_seeds entries.
        """
        T = seeds.frame.numel()
        if rows is None:
            rows = torch.empty(T, self.cfg.n_rows, dtype=torch.int32, device=self.device)
        tracks = self.alloc_tracks(seeds) if tracks is None else tracks
        ws = self.workspace(frames) if ws is None else ws
        prm = C.FollowParams(float(gate_chi2), int(max_miss))
        sc = seeds.c()
        tc = tracks.c()
        C.check(C.lib().tpc_track_follow(self._ctx, ctypes.byref(frames.c), ctypes.byref(sc),
                                         ctypes.byref(prm), rows.data_ptr(), ctypes.byref(tc),
                                         ws.data_ptr(), ws.numel(), _stream_handle(self.device)))
        return rows, tracks

    def alloc_merge(self, seeds: Seeds, legs: bool = True) -> dict:
        """Output tensors of tpc_track_merge (merged states and, with legs,
        the looper pairing)."""
        T = max(seeds.frame.numel(), 1)
        d = self.device
        out = dict(next=torch.empty(T, dtype=torch.int32, device=d), prev=torch.empty(T, dtype=torch.int32, device=d),
                   chi2=torch.empty(T, device=d), merged_par=torch.empty(T, 5, device=d),
                   merged_cov=torch.empty(T, 15, device=d))
        if legs:
            out.update(leg=torch.empty(T, dtype=torch.int32, device=d), leg_chi2=torch.empty(T, device=d))
        return out

    def merge(self, seeds: Seeds, tracks: Tracks, chi2_cut: float, out: Optional[dict] = None, legs: bool = True):
        """tpc_track_merge: links between fitted segments of neighbouring
        sectors, and (legs=True) the pairing of the legs of loopers.  Returns
        (next, prev, chi2, merged_par [T, 5], merged_cov [T, 15], leg,
        leg_chi2) per seed (leg, leg_chi2 None without legs); `out` from
        alloc_merge is filled in place."""
        out = self.alloc_merge(seeds, legs) if out is None else out
        if legs and "leg" not in out:
            raise ValueError("legs requested but out has no leg buffers")
        leg, lchi = (out["leg"], out["leg_chi2"]) if legs else (None, None)
        sc = seeds.c()
        tc = tracks.c()
        C.check(C.lib().tpc_track_merge(self._ctx, ctypes.byref(sc), ctypes.byref(tc), ctypes.c_float(chi2_cut),
                                        out["next"].data_ptr(), out["prev"].data_ptr(), out["chi2"].data_ptr(),
                                        out["merged_par"].data_ptr(), out["merged_cov"].data_ptr(),
                                        None if leg is None else leg.data_ptr(),
                                        None if lchi is None else lchi.data_ptr(), _stream_handle(self.device)))
        return out["next"], out["prev"], out["chi2"], out["merged_par"], out["merged_cov"], leg, lchi

    def refit(self, frames: DeviceFrames, seeds: Seeds, segments: Tracks, nxt: torch.Tensor, prv: torch.Tensor,
              leg: Optional[torch.Tensor] = None, map_: Optional[torch.Tensor] = None, out: Optional[dict] = None):
        """tpc_track_refit: track ids over the merging links, the refit of
        every chain of linked segments over all its hits (at the chain's
        head) and, with leg links, the joint circle of each pair of looper
        legs.  Returns a dict: track_id, refit (Tracks), and with leg
        loop_par [T, 4], loop_cov [T, 10], loop_chi2 [T]."""
        self._check_map(map_)
        if out is None:
            T = max(seeds.frame.numel(), 1)
            d = self.device
            out = dict(track_id=torch.empty(T, dtype=torch.int32, device=d), refit=self.alloc_tracks(seeds))
            if leg is not None:
                out.update(loop_par=torch.empty(T, 4, device=d), loop_cov=torch.empty(T, 10, device=d),
                           loop_chi2=torch.empty(T, device=d))
        lp = out.get("loop_par") if leg is not None else None
        sc = seeds.c()
        gc = segments.c()
        rc = out["refit"].c()
        C.check(C.lib().tpc_track_refit(self._ctx, ctypes.byref(frames.c), ctypes.byref(sc), ctypes.byref(gc),
                                        nxt.data_ptr(), prv.data_ptr(), None if leg is None else leg.data_ptr(),
                                        None if map_ is None else map_.data_ptr(), out["track_id"].data_ptr(),
                                        ctypes.byref(rc), None if lp is None else lp.data_ptr(),
                                        None if lp is None else out["loop_cov"].data_ptr(),
                                        None if lp is None else out["loop_chi2"].data_ptr(),
                                        _stream_handle(self.device)))
        return out

    def alloc_ctf(self, frames: DeviceFrames, seeds: Seeds) -> dict:
        T, N = seeds.frame.numel(), max(frames.n_clusters, 1)
        NR = frames.n_frames * self.cfg.n_sectors * self.cfg.n_rows
        caps = [T] * 9 + [N] * 3 + [NR] + [N] * 4
        d = {k: torch.empty(c, dtype=torch.int32, device=self.device) for k, c in zip(C.CTF_ARRAYS, caps)}
        d["counts"] = torch.zeros(len(C.CTF_ARRAYS), dtype=torch.int64, device=self.device)
        return d

    def ctf_build(self, frames: DeviceFrames, seeds: Seeds, rows: torch.Tensor, tracks: Tracks,
                  q_y: float, q_z: float, out: Optional[dict] = None, ws=None) -> dict:
        """tpc_ctf_build: the frame's track-model residual arrays (device tensors,
        valid up to out["counts"][k] entries each)."""
        out = self.alloc_ctf(frames, seeds) if out is None else out
        ws = self.workspace(frames) if ws is None else ws
        oc = C.CtfArraysC(*[out[k].data_ptr() for k in C.CTF_ARRAYS], out["counts"].data_ptr())
        sc = seeds.c()
        tc = tracks.c()
        C.check(C.lib().tpc_ctf_build(self._ctx, ctypes.byref(frames.c), ctypes.byref(sc), rows.data_ptr(),
                                      ctypes.byref(tc), float(q_y), float(q_z), ctypes.byref(oc),
                                      ws.data_ptr(), ws.numel(), _stream_handle(self.device)))
        return out

    def chi2_sum(self, seeds: Seeds, tracks: Tracks, loss: Optional[torch.Tensor] = None, ws=None):
        """Sum of chi2 over successfully fitted tracks (device float scalar)."""
        loss = torch.empty((), dtype=torch.float32, device=self.device) if loss is None else loss
        if ws is None:
            ws = self._ws if self._ws is not None else torch.empty(
                max(256, 8 * (seeds.frame.numel() // 256 + 2)), dtype=torch.uint8, device=self.device)
        sc = seeds.c()
        tc = tracks.c()
        C.check(C.lib().tpc_chi2_sum(self._ctx, ctypes.byref(sc), ctypes.byref(tc), loss.data_ptr(),
                                     ws.data_ptr(), ws.numel(), _stream_handle(self.device)))
        return loss

    def fit_adjoint(self, frames: DeviceFrames, seeds: Seeds, map_: torch.Tensor, tracks: Tracks,
                    ckpt: torch.Tensor, dloss: Optional[torch.Tensor] = None,
                    grad: Optional[torch.Tensor] = None, ws=None) -> torch.Tensor:
        """dloss * d(sum chi2)/d(map), seeds fixed (needs the checkpoints of ``fit``)."""
        self._check_map(map_)
        grad = torch.empty(self.cfg.n_sectors, self.cfg.n_rows, 2, dtype=torch.float32,
                           device=self.device) if grad is None else grad
        ws = self.workspace(frames) if ws is None else ws
        if dloss is not None:
            dloss = dloss.to(device=self.device, dtype=torch.float32).contiguous()
        sc = seeds.c()
        tc = tracks.c()
        C.check(C.lib().tpc_fit_adjoint(self._ctx, ctypes.byref(frames.c), ctypes.byref(sc),
                                        None if map_ is None else map_.data_ptr(), ctypes.byref(tc),
                                        ckpt.data_ptr(), ckpt.numel() * ckpt.element_size(),
                                        None if dloss is None else dloss.data_ptr(), grad.data_ptr(),
                                        ws.data_ptr(), ws.numel(), _stream_handle(self.device)))
        return grad

    def persistent_grid(self) -> int:
        return int(C.lib().tpc_persistent_grid(self._ctx))

    def reconstruct(self, frames: DeviceFrames, mode: str = "staged", tune=None, out=None, ws=None):
        """neighbours -> seeds -> fit for all frames, on one stream, no host
        synchronisation.  mode "staged" runs the stage kernels, "persistent"
        one persistent kernel, "persistent_graph" the persistent sequence as a
        HIP graph held by the context (captured on the first call with these
        buffers, replayed afterwards).  ``out`` = (up, dn, seeds, tracks) to
        reuse buffers (e.g. for graph capture).  tune = (grid, sort_fit[,
        fit_block, fit_spt]) or None."""
        if out is None:
            N = frames.n_clusters
            up = torch.empty(N, dtype=torch.int32, device=self.device)
            dn = torch.empty(N, dtype=torch.int32, device=self.device)
            seeds = self.alloc_seeds(frames)
            tracks = self.alloc_tracks(seeds)
        else:
            up, dn, seeds, tracks = out
        m = {"staged": C.TPC_MODE_STAGED, "persistent": C.TPC_MODE_PERSISTENT,
             "persistent_graph": C.TPC_MODE_PERSISTENT_GRAPH}[mode]
        if ws is None:
            ws = self.workspace(frames, C.TPC_STAGE_PERSISTENT if m else C.TPC_STAGE_ALL)
        t = None if tune is None else C.Tune(*([int(v) for v in tune] + [0] * (4 - len(tune))))
        sc = seeds.c()
        tc = tracks.c()
        C.check(C.lib().tpc_reconstruct(self._ctx, ctypes.byref(frames.c), m,
                                        None if t is None else ctypes.byref(t), up.data_ptr(),
                                        dn.data_ptr(), ctypes.byref(sc), ctypes.byref(tc),
                                        seeds.status.data_ptr(), ws.data_ptr(), ws.numel(),
                                        _stream_handle(self.device)))
        return up, dn, seeds, tracks


class ReconstructGraph:
    """The whole path for fixed frames and buffers, captured once as a HIP
    graph (through torch's graph capture) and replayed with one launch."""

    def __init__(self, reco: Reco, frames: DeviceFrames, mode: str = "persistent", tune=None):
        self.reco, self.frames, self.mode, self.tune = reco, frames, mode, tune
        N = frames.n_clusters
        d = reco.device
        self.up = torch.empty(N, dtype=torch.int32, device=d)
        self.dn = torch.empty(N, dtype=torch.int32, device=d)
        self.seeds = reco.alloc_seeds(frames)
        self.tracks = reco.alloc_tracks(self.seeds)
        stages = C.TPC_STAGE_PERSISTENT if mode == "persistent" else C.TPC_STAGE_ALL
        self.ws = torch.empty(max(256, reco.workspace_bytes(frames, stages)), dtype=torch.uint8, device=d)
        out = (self.up, self.dn, self.seeds, self.tracks)
        # one eager run (also warms the code objects), then capture on a side stream
        reco.reconstruct(frames, mode, tune, out, self.ws)
        torch.cuda.synchronize(d)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            reco.reconstruct(frames, mode, tune, out, self.ws)
        torch.cuda.synchronize(d)

    def replay(self):
        self.graph.replay()
        return self.up, self.dn, self.seeds, self.tracks


def rans_workspace(n: int, scale_bits: int, block_symbols: int, device="cuda:0") -> torch.Tensor:
    prm = C.RansParams(int(scale_bits), int(block_symbols))
    b = ctypes.c_size_t()
    C.check(C.lib().tpc_rans_workspace_bytes(int(n), ctypes.byref(prm), ctypes.byref(b)))
    return torch.empty(max(int(b.value), 1), dtype=torch.uint8, device=device)


def rans_max_bytes(n: int, value_range: int, scale_bits: int, block_symbols: int) -> int:
    prm = C.RansParams(int(scale_bits), int(block_symbols))
    b = ctypes.c_size_t()
    C.check(C.lib().tpc_rans_max_bytes(int(n), int(value_range), ctypes.byref(prm), ctypes.byref(b)))
    return int(b.value)


def rans_encode(symbols: torch.Tensor, scale_bits: int, block_symbols: int, out=None, ws=None,
                out_size=None, status=None):
    """tpc_rans_encode of a contiguous int32 device tensor.  Returns (out,
    out_size, status): the uint8 stream buffer, the stream's size and the
    device status (device tensors; nothing is synchronised)."""
    if symbols.dtype != torch.int32 or not symbols.is_contiguous() or symbols.device.type != "cuda":
        raise ValueError("symbols must be a contiguous int32 device tensor")
    n = symbols.numel()
    d = symbols.device
    if out is None:
        out = torch.empty(rans_max_bytes(n, 1 << 20, scale_bits, block_symbols), dtype=torch.uint8, device=d)
    ws = rans_workspace(n, scale_bits, block_symbols, d) if ws is None else ws
    out_size = torch.zeros(1, dtype=torch.int64, device=d) if out_size is None else out_size
    status = torch.zeros(1, dtype=torch.int32, device=d) if status is None else status
    prm = C.RansParams(int(scale_bits), int(block_symbols))
    C.check(C.lib().tpc_rans_encode(symbols.data_ptr() if n else None, n, ctypes.byref(prm),
                                    out.data_ptr(), out.numel(), out_size.data_ptr(),
                                    status.data_ptr(), ws.data_ptr(), ws.numel(),
                                    _stream_handle(d)))
    return out, out_size, status


def rans_decode(stream: torch.Tensor, size: int, cap: int, out=None, ws=None):
    """tpc_rans_decode of the first `size` bytes of a uint8 device tensor.
    Returns (symbols int32 [cap], n int64 [1], status int32 [1]) device tensors."""
    if stream.dtype != torch.uint8 or stream.device.type != "cuda" or not stream.is_contiguous():
        raise ValueError("stream must be a contiguous uint8 device tensor")
    d = stream.device
    out = torch.empty(max(int(cap), 1), dtype=torch.int32, device=d) if out is None else out
    if ws is None:
        b = ctypes.c_size_t()
        C.check(C.lib().tpc_rans_decode_workspace_bytes(ctypes.byref(b)))
        ws = torch.empty(int(b.value), dtype=torch.uint8, device=d)
    n = torch.zeros(1, dtype=torch.int64, device=d)
    st = torch.zeros(1, dtype=torch.int32, device=d)
    C.check(C.lib().tpc_rans_decode(stream.data_ptr(), int(size), out.data_ptr(), int(cap), n.data_ptr(),
                                    st.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle(d)))
    return out, n, st


def _rans_jobs(jobs):
    arr = (C.RansJobC * len(jobs))()
    for k, j in enumerate(jobs):
        sym = j["symbols"]
        if sym.dtype != torch.int32 or not sym.is_contiguous() or sym.device.type != "cuda":
            raise ValueError("symbols must be contiguous int32 device tensors")
        nd = j.get("n_device")
        arr[k] = C.RansJobC(sym.data_ptr() if sym.numel() else None, sym.numel(),
                            None if nd is None else nd.data_ptr(),
                            None if j.get("out") is None else j["out"].data_ptr(),
                            0 if j.get("out") is None else j["out"].numel(),
                            None if j.get("out_size") is None else j["out_size"].data_ptr(),
                            None if j.get("status") is None else j["status"].data_ptr())
    return arr


def rans_batch_workspace(jobs, scale_bits: int, block_symbols: int, device="cuda:0") -> torch.Tensor:
    prm = C.RansParams(int(scale_bits), int(block_symbols))
    b = ctypes.c_size_t()
    arr = _rans_jobs(jobs)
    C.check(C.lib().tpc_rans_batch_workspace_bytes(len(jobs), arr, ctypes.byref(prm), ctypes.byref(b)))
    return torch.empty(max(int(b.value), 1), dtype=torch.uint8, device=device)


def rans_encode_batch(jobs, scale_bits: int, block_symbols: int, ws=None):
    """tpc_rans_encode_batch.  jobs: dicts with "symbols" (int32 device tensor,
    its length the capacity), optional "n_device" (int64 device element with
    the count), "out" (uint8), "out_size" (int64 element), "status" (int32
    element); missing outputs are allocated.  Returns the jobs."""
    for j in jobs:
        d = j["symbols"].device
        if j.get("out") is None:
            j["out"] = torch.empty(rans_max_bytes(j["symbols"].numel(), 1 << 20, scale_bits, block_symbols),
                                   dtype=torch.uint8, device=d)
        if j.get("out_size") is None:
            j["out_size"] = torch.zeros(1, dtype=torch.int64, device=d)
        if j.get("status") is None:
            j["status"] = torch.zeros(1, dtype=torch.int32, device=d)
    ws = rans_batch_workspace(jobs, scale_bits, block_symbols, jobs[0]["symbols"].device) if ws is None else ws
    prm = C.RansParams(int(scale_bits), int(block_symbols))
    C.check(C.lib().tpc_rans_encode_batch(len(jobs), _rans_jobs(jobs), ctypes.byref(prm), ws.data_ptr(),
                                          ws.numel(), _stream_handle(jobs[0]["symbols"].device)))
    return jobs


class KalmanChi2(torch.autograd.Function):
    """loss = sum of fit chi2 over the (fixed) seeds, as a function of the
    [n_sectors, n_rows, 2] cluster correction map; backward runs the
    library's hand-written adjoint."""

    @staticmethod
    def forward(ctx, map_: torch.Tensor, reco: "Reco", frames: DeviceFrames, seeds: Seeds):
        m = map_.detach().contiguous()
        ckpt = reco.alloc_ckpt(seeds)
        tracks = reco.fit(frames, seeds, m, ckpt=ckpt)
        loss = reco.chi2_sum(seeds, tracks)
        ctx.reco, ctx.frames, ctx.seeds = reco, frames, seeds
        ctx.tracks, ctx.ckpt, ctx.map = tracks, ckpt, m
        return loss

    @staticmethod
    def backward(ctx, grad_out):
        g = ctx.reco.fit_adjoint(ctx.frames, ctx.seeds, ctx.map, ctx.tracks, ctx.ckpt,
                                 dloss=grad_out.reshape(()))
        return g, None, None, None
