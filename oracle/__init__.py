"""CPU oracle for the TPC tracking path -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it and the
two share no code.  The arithmetic lives in ``tpc_oracle.c`` (plain C,
single-precision neighbour search with every operation rounded, double
precision fit); this module builds it with gcc and wraps it with ctypes.

Every function takes its parameters explicitly; none has a built-in default
for a physics or algorithm constant.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tpc_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "rans_oracle.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

GCC_FLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
             "-shared", "-fPIC"]


# TPC_SANITIZE=1 builds and loads liboracle_san.so instead, instrumented
# with AddressSanitizer and UndefinedBehaviorSanitizer (run the interpreter
# with gcc's libasan and libubsan preloaded).
SANITIZE = os.environ.get("TPC_SANITIZE", "") == "1"
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]
if SANITIZE:
    _LIB = _LIB.replace("liboracle.so", "liboracle_san.so")


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (no fused multiply-add contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *GCC_FLAGS, *(SAN_FLAGS if SANITIZE else []), *_SRCS, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class FitParams(ctypes.Structure):
    _fields_ = [("bz", ctypes.c_double), ("sigma_y", ctypes.c_double),
                ("sigma_z", ctypes.c_double), ("max_sin", ctypes.c_double),
                ("var_sin0", ctypes.c_double), ("var_tgl0", ctypes.c_double),
                ("var_qpt0", ctypes.c_double)]


class Material(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("mass", ctypes.c_double), ("chi2_cut", ctypes.c_double),
                ("rho", ctypes.c_double), ("z_over_a", ctypes.c_double), ("mean_exc", ctypes.c_double)]


def _material(x0, mass, chi2_cut, gas):
    rho, zoa, exc = (0.0, 0.5, 1e-7) if gas is None else gas
    return Material(float(x0), float(mass), float(chi2_cut), float(rho), float(zoa), float(exc))


def transfer(p, x, da, xt, bz, max_sin):
    """State p at plane x rotated into the frame turned by da and carried to
    plane xt of that frame: (status, state, Jacobian)."""
    out = np.zeros(5)
    J = np.zeros((5, 5))
    st = lib().oracle_transfer(_p(np.ascontiguousarray(p, dtype=np.float64)), float(x), float(da), float(xt),
                               float(bz), float(max_sin), _p(out), _p(J))
    return int(st), out, J


def merge(tracks: dict, frame, sector, n_sectors, *, bz, max_sin, cut):
    """Mutual-best links between fitted segments of neighbouring sectors:
    (next, prev, chi2, merged_par [T, 5], merged_cov [T, 15]) per track (the
    linked pair combined at the outer segment's plane; zeros if unlinked)."""
    x = np.ascontiguousarray(tracks["x"], dtype=np.float64)
    par = np.ascontiguousarray(tracks["par"], dtype=np.float64)
    cov = np.ascontiguousarray(tracks["cov"], dtype=np.float64)
    st = np.ascontiguousarray(tracks["status"], dtype=np.int32)
    fr = np.ascontiguousarray(frame, dtype=np.int32)
    sc = np.ascontiguousarray(sector, dtype=np.int32)
    T = x.size
    nxt, prv, chi = np.empty(T, np.int32), np.empty(T, np.int32), np.empty(T)
    mp, mc = np.zeros((max(T, 1), 5)), np.zeros((max(T, 1), 15))
    lib().oracle_merge(T, _p(x), _p(par), _p(cov), _p(st), _p(fr), _p(sc), int(n_sectors), float(bz),
                       float(max_sin), float(cut), _p(nxt), _p(prv), _p(chi), _p(mp), _p(mc))
    return nxt, prv, chi, mp[:T], mc[:T]


def leg_circle(p, x, alpha, bz):
    """(status, m = (X_c, Y_c, kappa, tan lambda), 4x5 Jacobian) of a segment's circle."""
    m = np.zeros(4)
    J = np.zeros((4, 5))
    st = lib().oracle_leg_circle(_p(np.ascontiguousarray(p, dtype=np.float64)), float(x), float(alpha), float(bz),
                                 _p(m), _p(J))
    return int(st), m, J


def legs(tracks: dict, frame, sector, n_sectors, *, bz, cut):
    """Mutual-best pairing of the legs of loopers: (leg, leg_chi2) per track."""
    x = np.ascontiguousarray(tracks["x"], dtype=np.float64)
    par = np.ascontiguousarray(tracks["par"], dtype=np.float64)
    cov = np.ascontiguousarray(tracks["cov"], dtype=np.float64)
    st = np.ascontiguousarray(tracks["status"], dtype=np.int32)
    fr = np.ascontiguousarray(frame, dtype=np.int32)
    sc = np.ascontiguousarray(sector, dtype=np.int32)
    T = x.size
    leg, chi = np.empty(T, np.int32), np.empty(T)
    lib().oracle_legs(T, _p(x), _p(par), _p(cov), _p(st), _p(fr), _p(sc), int(n_sectors), float(bz), float(cut),
                      _p(leg), _p(chi))
    return leg, chi


def refit(seeds: dict, tracks: dict, nxt, prv, leg, y, z, row_x, n_rows, n_sectors, *, bz, sigma_y,
          sigma_z, max_sin, var_sin0, var_tgl0, var_qpt0, map_: Optional[np.ndarray] = None):
    """Tracks assembled from linked segments and refitted over all their hits.

    ``tracks`` holds the segments' fit status; ``nxt``, ``prv`` the
    sector-edge links, ``leg`` the looper-leg pairing (or None).  Returns a
    dict: track_id [T]; the chain refits x, par, cov, chi2, ndf, status at
    each chain's head (status 5 elsewhere); loop_par [T, 4], loop_cov [T, 10],
    loop_chi2 [T] (the joint circle of each leg pair at its smaller index,
    chi2 -1 elsewhere; absent when ``leg`` is None)."""
    offsets = np.ascontiguousarray(seeds["offsets"], dtype=np.int32)
    hits = np.ascontiguousarray(seeds["hits"], dtype=np.int32)
    sec = np.ascontiguousarray(seeds["sector"], dtype=np.int32)
    fr = np.ascontiguousarray(seeds["first_row"], dtype=np.int32)
    st = np.ascontiguousarray(tracks["status"], dtype=np.int32)
    nx = np.ascontiguousarray(nxt, dtype=np.int32)
    pv = np.ascontiguousarray(prv, dtype=np.int32)
    lg = None if leg is None else np.ascontiguousarray(leg, dtype=np.int32)
    y = np.ascontiguousarray(y, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    rx = np.ascontiguousarray(row_x, dtype=np.float64)
    T = len(offsets) - 1
    assert st.size == T and nx.size == T and pv.size == T and (lg is None or lg.size == T)
    assert hits.size == 0 or (hits.min() >= 0 and hits.max() < y.size), "seed hit ids outside the clusters"
    prm = FitParams(bz, sigma_y, sigma_z, max_sin, var_sin0, var_tgl0, var_qpt0)
    mp = None if map_ is None else np.ascontiguousarray(map_, dtype=np.float64)
    n1 = max(T, 1)
    out = dict(track_id=np.empty(n1, np.int32), x=np.empty(n1), par=np.empty((n1, 5)), cov=np.empty((n1, 15)),
               chi2=np.empty(n1), ndf=np.empty(n1, np.int32), status=np.empty(n1, np.int32))
    if lg is not None:
        out.update(loop_par=np.empty((n1, 4)), loop_cov=np.empty((n1, 10)), loop_chi2=np.empty(n1))
    q = lambda k: None if k not in out else _p(out[k])
    lib().oracle_refit(T, _p(offsets), _p(hits), _p(sec), _p(fr), _p(st), _p(nx), _p(pv),
                       None if lg is None else _p(lg), _p(y), _p(z), _p(rx), int(n_rows), int(n_sectors),
                       None if mp is None else _p(mp), ctypes.byref(prm), _p(out["track_id"]), _p(out["x"]),
                       _p(out["par"]), _p(out["cov"]), _p(out["chi2"]), _p(out["ndf"]), _p(out["status"]),
                       q("loop_par"), q("loop_cov"), q("loop_chi2"))
    return {k: v[:T] for k, v in out.items()}


def eloss(p, dx, mass, gas, direction=1.0):
    """Energy-loss map of the fit for one segment: (status, w', dw'/dt,
    dw'/dw, straggling variance of w)."""
    st = np.ascontiguousarray(p, dtype=np.float64)
    out = np.zeros(4)
    r = lib().oracle_eloss(_p(st), float(dx), ctypes.byref(_material(np.inf, mass, np.inf, gas)),
                           float(direction), _p(out))
    return (int(r),) + tuple(float(v) for v in out)


def bethe(beta_gamma, mass, z_over_a, mean_exc):
    """Mean energy loss per density, GeV cm^2/g (Bethe, unit charge, no
    density effect), as the fit with energy loss takes it."""
    return lib().oracle_bethe(float(beta_gamma), float(mass), float(z_over_a), float(mean_exc))


class FollowParams(ctypes.Structure):
    _fields_ = [("gate", ctypes.c_double), ("max_miss", ctypes.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(f) for f in _SRCS):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32 = ctypes.c_int32
        f32 = ctypes.c_float
        L.oracle_neighbours.argtypes = [i32, i32, P, P, P, f32, f32, f32, f32, P, P]
        L.oracle_neighbours.restype = None
        L.oracle_ca_seed.argtypes = [i32, i32, i32, P, P, P, i32, i32, i32, P, P, P, P, P, P, P]
        L.oracle_ca_seed.restype = i32
        L.oracle_propagate.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double, P, P]
        L.oracle_propagate.restype = i32
        L.oracle_fit.argtypes = [i32, P, P, P, P, P, P, P, i32, P, ctypes.POINTER(FitParams),
                                 P, P, P, P, P, P, P]
        L.oracle_fit.restype = None
        L.oracle_follow.argtypes = [i32, P, P, P, P, P, P, i32, i32, i32, P, P, P,
                                    ctypes.POINTER(FitParams), ctypes.POINTER(FollowParams),
                                    P, P, P, P, P, P, P, P]
        L.oracle_follow.restype = None
        u32, i64, sz = ctypes.c_uint32, ctypes.c_int64, ctypes.c_size_t
        L.oracle_rans_freqs.argtypes = [P, u32, ctypes.c_uint64, u32, P]
        L.oracle_rans_freqs.restype = i64
        L.oracle_rans_bound.argtypes = [i64, u32, u32]
        L.oracle_rans_bound.restype = sz
        L.oracle_rans_encode.argtypes = [P, i64, u32, u32, u32, P, sz, ctypes.POINTER(sz)]
        L.oracle_rans_encode.restype = i32
        L.oracle_rans_decode.argtypes = [P, sz, P, i64, ctypes.POINTER(i64)]
        L.oracle_rans_decode.restype = i32
        L.oracle_ctf_build.argtypes = [i32, i32, i32, i32, P, P, P, P, P, P, P, ctypes.c_float,
                                       ctypes.c_float, P, P]
        L.oracle_ctf_build.restype = None
        L.oracle_fit_material.argtypes = [i32, P, P, P, P, P, P, ctypes.POINTER(FitParams),
                                           ctypes.POINTER(Material), P, P, P, P, P, P, P, P]
        L.oracle_fit_material.restype = None
        d_ = ctypes.c_double
        L.oracle_transfer.argtypes = [P, d_, d_, d_, d_, d_, P, P]
        L.oracle_transfer.restype = i32
        L.oracle_merge.argtypes = [i32, P, P, P, P, P, P, i32, d_, d_, d_, P, P, P, P, P]
        L.oracle_merge.restype = None
        L.oracle_leg_circle.argtypes = [P, d_, d_, d_, P, P]
        L.oracle_leg_circle.restype = i32
        L.oracle_legs.argtypes = [i32, P, P, P, P, P, P, i32, d_, d_, P, P]
        L.oracle_legs.restype = None
        L.oracle_refit.argtypes = [i32, P, P, P, P, P, P, P, P, P, P, P, i32, i32, P,
                                   ctypes.POINTER(FitParams), P, P, P, P, P, P, P, P, P, P]
        L.oracle_refit.restype = None
        L.oracle_bethe.argtypes = [ctypes.c_double] * 4
        L.oracle_bethe.restype = ctypes.c_double
        L.oracle_eloss.argtypes = [P, ctypes.c_double, ctypes.POINTER(Material), ctypes.c_double, P]
        L.oracle_eloss.restype = i32
        L.oracle_neighbours_skip.argtypes = [i32, i32, P, P, P, f32, f32, f32, f32, P, P]
        L.oracle_neighbours_skip.restype = None
        L.oracle_fit_rows.argtypes = [i32, P, P, P, P, P, i32, i32, i32, P, P, P, P,
                                      ctypes.POINTER(FitParams), ctypes.POINTER(Material),
                                      P, P, P, P, P, P, P, P, P, P]
        L.oracle_fit_rows.restype = None
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def _check_layout(off, n_rows, n):
    """Row offsets must describe whole sectors of n_rows rows and n clusters."""
    if off.ndim != 1 or off.size < 1 or (off.size - 1) % n_rows != 0:
        raise ValueError("row_offsets must hold a whole number of sectors of %d rows plus one" % n_rows)
    if off[0] != 0 or np.any(np.diff(off) < 0) or int(off[-1]) != n:
        raise ValueError("row_offsets must start at 0, not decrease and end at the cluster count")


def neighbours(row_offsets, y, z, n_rows, win_y, win_z, cut_y, cut_z):
    """Returns (up, dn) int32 arrays: best triplet partners per cluster."""
    off = np.ascontiguousarray(row_offsets, dtype=np.int32)
    _check_layout(off, n_rows, len(y))
    y = np.ascontiguousarray(y, dtype=np.float32)
    z = np.ascontiguousarray(z, dtype=np.float32)
    n = int(off[-1])
    up = np.empty(n, np.int32)
    dn = np.empty(n, np.int32)
    lib().oracle_neighbours(len(off) - 1, n_rows, _p(off), _p(y), _p(z), win_y, win_z,
                            cut_y, cut_z, _p(up), _p(dn))
    return up, dn


def neighbours_skip(row_offsets, y, z, n_rows, win_y, win_z, cut_y, cut_z):
    """Returns (up, dn): best triplet partners per cluster, one or two rows
    away (a triplet spanning fewer rows always wins)."""
    off = np.ascontiguousarray(row_offsets, dtype=np.int32)
    _check_layout(off, n_rows, len(y))
    y = np.ascontiguousarray(y, dtype=np.float32)
    z = np.ascontiguousarray(z, dtype=np.float32)
    n = int(off[-1])
    up = np.empty(n, np.int32)
    dn = np.empty(n, np.int32)
    lib().oracle_neighbours_skip(len(off) - 1, n_rows, _p(off), _p(y), _p(z), win_y, win_z,
                                 cut_y, cut_z, _p(up), _p(dn))
    return up, dn


def ca_seed(row_offsets, up, dn, n_sectors, n_rows, min_hits):
    """Returns dict(offsets, hits, frame, sector, first_row) of the seeds."""
    off = np.ascontiguousarray(row_offsets, dtype=np.int32)
    up = np.ascontiguousarray(up, dtype=np.int32)
    dn = np.ascontiguousarray(dn, dtype=np.int32)
    n = int(off[-1])
    cap_s, cap_h = max(1, n // 2), max(1, n)
    offsets = np.empty(cap_s + 1, np.int32)
    hits = np.empty(cap_h, np.int32)
    fr = np.empty(cap_s, np.int32)
    se = np.empty(cap_s, np.int32)
    rw = np.empty(cap_s, np.int32)
    ns = ctypes.c_int32()
    nh = ctypes.c_int32()
    st = lib().oracle_ca_seed(len(off) - 1, n_sectors, n_rows, _p(off), _p(up), _p(dn), min_hits,
                              cap_s, cap_h, ctypes.byref(ns), ctypes.byref(nh), _p(offsets),
                              _p(hits), _p(fr), _p(se), _p(rw))
    if st != 0:
        raise RuntimeError("oracle seed capacity exceeded")
    k, h = ns.value, nh.value
    return dict(offsets=offsets[:k + 1].copy(), hits=hits[:h].copy(), frame=fr[:k].copy(),
                sector=se[:k].copy(), first_row=rw[:k].copy())


def propagate(p, dx, bz, max_sin):
    """Exact helix step of the oracle: returns (status, p_out[5], F[5,5])."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    po = np.empty(5)
    F = np.empty(25)
    st = lib().oracle_propagate(_p(p), float(dx), float(bz), float(max_sin), _p(po), _p(F))
    return st, po, F.reshape(5, 5)


def fit(seeds: dict, y, z, row_x, n_rows, *, bz, sigma_y, sigma_z, max_sin, var_sin0,
        var_tgl0, var_qpt0, map_: Optional[np.ndarray] = None):
    """Double-precision Kalman fit of every seed.

    Besides the fit, ``sin_margin`` reports each fit's closest approach to
    its direction thresholds: min(max_sin - |sin phi|, cos phi) at the start,
    then max_sin - max(|s|, |s'|) over the helix steps taken (negative at a
    step that failed; -inf for degenerate start points).

    ``y``, ``z`` are promoted to float64 (pass float64 truth to avoid the
    float32 rounding of stored clusters).  ``map_`` is [S, R, 2] (dy, dz)
    subtracted from the clusters of each (sector, row).
    """
    offsets = np.ascontiguousarray(seeds["offsets"], dtype=np.int32)
    hits = np.ascontiguousarray(seeds["hits"], dtype=np.int32)
    sec = np.ascontiguousarray(seeds["sector"], dtype=np.int32)
    fr = np.ascontiguousarray(seeds["first_row"], dtype=np.int32)
    y = np.ascontiguousarray(y, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    rx = np.ascontiguousarray(row_x, dtype=np.float64)
    T = len(offsets) - 1
    prm = FitParams(bz, sigma_y, sigma_z, max_sin, var_sin0, var_tgl0, var_qpt0)
    mp = None if map_ is None else np.ascontiguousarray(map_, dtype=np.float64)
    out = dict(x=np.empty(T), par=np.empty((T, 5)), cov=np.empty((T, 15)), chi2=np.empty(T),
               ndf=np.empty(T, np.int32), status=np.empty(T, np.int32), sin_margin=np.empty(T))
    lib().oracle_fit(T, _p(offsets), _p(hits), _p(sec), _p(fr), _p(y), _p(z), _p(rx), n_rows,
                     None if mp is None else _p(mp), ctypes.byref(prm), _p(out["x"]),
                     _p(out["par"]), _p(out["cov"]), _p(out["chi2"]), _p(out["ndf"]),
                     _p(out["status"]), _p(out["sin_margin"]))
    return out


def fit_material(seeds: dict, y, z, row_x, *, x0, mass, chi2_cut, bz, sigma_y, sigma_z, max_sin,
                 var_sin0, var_tgl0, var_qpt0, gas=None):
    """Fit with multiple scattering (radiation length x0 cm, mass GeV),
    energy loss in a gas (rho g/cm^3, Z/A, mean excitation GeV; None: none)
    and rejection of hits above chi2_cut.  Returns the fit's dict plus
    rejected (uint8 per seed hit) and margin per track."""
    offsets = np.ascontiguousarray(seeds["offsets"], dtype=np.int32)
    hits = np.ascontiguousarray(seeds["hits"], dtype=np.int32)
    fr = np.ascontiguousarray(seeds["first_row"], dtype=np.int32)
    y = np.ascontiguousarray(y, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    rx = np.ascontiguousarray(row_x, dtype=np.float64)
    T = len(offsets) - 1
    prm = FitParams(bz, sigma_y, sigma_z, max_sin, var_sin0, var_tgl0, var_qpt0)
    mat = _material(x0, mass, chi2_cut, gas)
    out = dict(x=np.empty(T), par=np.empty((T, 5)), cov=np.empty((T, 15)), chi2=np.empty(T),
               ndf=np.empty(T, np.int32), status=np.empty(T, np.int32),
               rejected=np.zeros(max(hits.size, 1), np.uint8), margin=np.empty(T))
    lib().oracle_fit_material(T, _p(offsets), _p(hits), _p(fr), _p(y), _p(z), _p(rx), ctypes.byref(prm),
                              ctypes.byref(mat), _p(out["x"]), _p(out["par"]), _p(out["cov"]),
                              _p(out["chi2"]), _p(out["ndf"]), _p(out["status"]), _p(out["rejected"]),
                              _p(out["margin"]))
    out["rejected"] = out["rejected"][:hits.size]
    return out


def fit_rows(seeds: dict, row_offsets, y, z, row_x, n_sectors, n_rows, *, err, x0, mass, chi2_cut,
             bz, sigma_y, sigma_z, max_sin, var_sin0, var_tgl0, var_qpt0, gas=None, smooth=False):
    """Fit of seeds whose hits may skip pad rows (each hit's row is looked up
    in ``row_offsets``), with per-cluster errors ``err`` ([N, 2] float32
    sigma_y, sigma_z; None: the constants) and material as in fit_material
    (x0=inf, chi2_cut=inf: none).  Returns fit_material's dict; with
    ``smooth`` also hit_par [H, 5] and hit_cov [H, 15] (packed), the
    smoothed state at every seed hit's plane."""
    offsets = np.ascontiguousarray(seeds["offsets"], dtype=np.int32)
    hits = np.ascontiguousarray(seeds["hits"], dtype=np.int32)
    frm = np.ascontiguousarray(seeds["frame"], dtype=np.int32)
    sec = np.ascontiguousarray(seeds["sector"], dtype=np.int32)
    off = np.ascontiguousarray(row_offsets, dtype=np.int32)
    y = np.ascontiguousarray(y, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    rx = np.ascontiguousarray(row_x, dtype=np.float64)
    ev = None
    if err is not None:
        ev = np.ascontiguousarray(err, dtype=np.float32)
        if ev.shape != (y.size, 2):
            raise ValueError("err must be [n_clusters, 2]")
    T = len(offsets) - 1
    n_frames = (off.size - 1) // (n_sectors * n_rows)
    prm = FitParams(bz, sigma_y, sigma_z, max_sin, var_sin0, var_tgl0, var_qpt0)
    mat = _material(x0, mass, chi2_cut, gas)
    out = dict(x=np.empty(T), par=np.empty((T, 5)), cov=np.empty((T, 15)), chi2=np.empty(T),
               ndf=np.empty(T, np.int32), status=np.empty(T, np.int32),
               rejected=np.zeros(max(hits.size, 1), np.uint8), margin=np.empty(T))
    hp = hc = None
    if smooth:
        out["hit_par"] = hp = np.zeros((max(hits.size, 1), 5))
        out["hit_cov"] = hc = np.zeros((max(hits.size, 1), 15))
    lib().oracle_fit_rows(T, _p(offsets), _p(hits), _p(frm), _p(sec), _p(off), n_frames, n_sectors, n_rows,
                          _p(y), _p(z), _p(rx), None if ev is None else _p(ev), ctypes.byref(prm),
                          ctypes.byref(mat), _p(out["x"]), _p(out["par"]), _p(out["cov"]), _p(out["chi2"]),
                          _p(out["ndf"]), _p(out["status"]), _p(out["rejected"]), _p(out["margin"]),
                          None if hp is None else _p(hp), None if hc is None else _p(hc))
    out["rejected"] = out["rejected"][:hits.size]
    if smooth:
        out["hit_par"] = hp[:hits.size]
        out["hit_cov"] = hc[:hits.size]
    return out


def follow(seeds: dict, row_offsets, y, z, row_x, n_sectors, n_rows, *, gate, max_miss, bz,
           sigma_y, sigma_z, max_sin, var_sin0, var_tgl0, var_qpt0):
    """Track following of every seed, then duplicate removal.

    Returns dict(rows [T, R] int32 cluster id per pad row or -1, x, par, cov,
    chi2, ndf, status (0 ok, 1-3 fit failure, 4 duplicate), margin).
    """
    offsets = np.ascontiguousarray(seeds["offsets"], dtype=np.int32)
    hits = np.ascontiguousarray(seeds["hits"], dtype=np.int32)
    frm = np.ascontiguousarray(seeds["frame"], dtype=np.int32)
    sec = np.ascontiguousarray(seeds["sector"], dtype=np.int32)
    fr = np.ascontiguousarray(seeds["first_row"], dtype=np.int32)
    off = np.ascontiguousarray(row_offsets, dtype=np.int32)
    y = np.ascontiguousarray(y, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    rx = np.ascontiguousarray(row_x, dtype=np.float64)
    T = len(offsets) - 1
    prm = FitParams(bz, sigma_y, sigma_z, max_sin, var_sin0, var_tgl0, var_qpt0)
    fp = FollowParams(float(gate), int(max_miss))
    out = dict(rows=np.empty((T, n_rows), np.int32), x=np.empty(T), par=np.empty((T, 5)),
               cov=np.empty((T, 15)), chi2=np.empty(T), ndf=np.empty(T, np.int32),
               status=np.empty(T, np.int32), margin=np.empty(T))
    n_frames = (off.size - 1) // (n_sectors * n_rows)
    lib().oracle_follow(T, _p(offsets), _p(hits), _p(frm), _p(sec), _p(fr), _p(off), n_frames, n_sectors, n_rows,
                        _p(y), _p(z), _p(rx), ctypes.byref(prm), ctypes.byref(fp), _p(out["rows"]),
                        _p(out["x"]), _p(out["par"]), _p(out["cov"]), _p(out["chi2"]),
                        _p(out["ndf"]), _p(out["status"]), _p(out["margin"]))
    return out


RANS_MAX_RANGE = 1 << 20


def rans_freqs(counts, n, L):
    """Scaled frequencies (sum 2^L) of a symbol histogram; None if more than 2^L symbols occur."""
    c = np.ascontiguousarray(counts, dtype=np.uint32)
    f = np.empty_like(c)
    d = lib().oracle_rans_freqs(_p(c), c.size, int(n), int(L), _p(f))
    return None if d < 0 else f


def rans_encode(sym, L, B, max_range=RANS_MAX_RANGE) -> bytes:
    """rANS stream of an int32 array (64 interleaved coders per block of B symbols)."""
    s = np.ascontiguousarray(sym, dtype=np.int32)
    lo, hi = (int(s.min()), int(s.max())) if s.size else (0, -1)
    R = hi - lo + 1 if s.size else 0
    cap = int(lib().oracle_rans_bound(s.size, min(max(R, 0), max_range), int(B))) if R <= max_range else 64
    out = np.empty(max(cap, 64), np.uint8)
    size = ctypes.c_size_t()
    st = lib().oracle_rans_encode(_p(s), s.size, int(L), int(B), int(max_range), _p(out), out.size,
                                  ctypes.byref(size))
    if st != 0:
        raise ValueError("oracle rANS encode failed (%d)" % st)
    return out[:size.value].tobytes()


def rans_decode(stream: bytes) -> np.ndarray:
    buf = np.frombuffer(stream, dtype=np.uint8)
    n = ctypes.c_int64()
    lib().oracle_rans_decode(_p(np.ascontiguousarray(buf)), buf.size, None, 0, ctypes.byref(n))
    out = np.empty(max(n.value, 1), np.int32)
    st = lib().oracle_rans_decode(_p(np.ascontiguousarray(buf)), buf.size, _p(out), out.size, ctypes.byref(n))
    if st != 0:
        raise ValueError("oracle rANS decode failed")
    return out[:n.value].copy()


CTF_ARRAYS = ("trk_seg", "trk_n", "trk_row0", "trk_y0h", "trk_y0l", "trk_z0h", "trk_z0l", "trk_dy1",
              "trk_dz1", "hit_drow", "hit_ry", "hit_rz", "seg_nfree", "free_yh", "free_yl", "free_zh",
              "free_zl")


def ctf_build(row_offsets, y, z, n_sectors, n_rows, rows, status, frame, sector, qy, qz) -> dict:
    """Track-model residual arrays of a frame (see rans_oracle.c), name -> int32 array."""
    off = np.ascontiguousarray(row_offsets, dtype=np.int32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    z = np.ascontiguousarray(z, dtype=np.float32)
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    st = np.ascontiguousarray(status, dtype=np.int32)
    fr = np.ascontiguousarray(frame, dtype=np.int32)
    se = np.ascontiguousarray(sector, dtype=np.int32)
    T = st.size
    N = int(off[-1])
    NR = off.size - 1
    caps = [max(T, 1)] * 9 + [max(N, 1)] * 3 + [max(NR, 1)] + [max(N, 1)] * 4
    bufs = [np.zeros(c, np.int32) for c in caps]
    ptrs = (ctypes.c_void_p * 17)(*[b.ctypes.data for b in bufs])
    cnt = np.zeros(17, np.int64)
    lib().oracle_ctf_build(T, n_rows, n_sectors, NR, _p(off), _p(y), _p(z), _p(rows), _p(st), _p(fr),
                           _p(se), float(qy), float(qz), ptrs, _p(cnt))
    return {k: bufs[i][:cnt[i]].copy() for i, k in enumerate(CTF_ARRAYS)}


def unpack_cov(c15: np.ndarray) -> np.ndarray:
    """Packed lower triangle (row by row) -> symmetric [.., 5, 5]."""
    c15 = np.asarray(c15)
    out = np.zeros(c15.shape[:-1] + (5, 5), dtype=c15.dtype)
    q = 0
    for i in range(5):
        for j in range(i + 1):
            out[..., i, j] = c15[..., q]
            out[..., j, i] = c15[..., q]
            q += 1
    return out


def chi2_sum(seeds, y, z, row_x, n_rows, map_, **prm) -> float:
    """Loss of the differentiable workload: sum of chi2 over tracks whose fit succeeds."""
    r = fit(seeds, y, z, row_x, n_rows, map_=map_, **prm)
    ok = r["status"] == 0
    return float(r["chi2"][ok].sum())


def fd_map_gradient(seeds, y, z, row_x, n_rows, map_, entries, h=1e-3, **prm):
    """Central finite differences (five-point) of ``chi2_sum`` w.r.t. map entries.

    ``entries`` is a list of (sector, row, axis).  Only the tracks of that
    sector that include that row are refitted (the others do not depend on it).
    """
    offsets = np.asarray(seeds["offsets"])
    n = np.diff(offsets)
    fr = np.asarray(seeds["first_row"])
    sec = np.asarray(seeds["sector"])
    out = np.empty(len(entries))
    for i, (s, r, a) in enumerate(entries):
        sel = np.nonzero((sec == s) & (fr <= r) & (fr + n > r))[0]
        if sel.size == 0:
            out[i] = 0.0
            continue
        sub = subset_seeds(seeds, sel)
        mp = np.array(map_, dtype=np.float64, copy=True)
        v0 = mp[s, r, a]
        vals = []
        for m in (2, 1, -1, -2):          # five-point central stencil, error O(h^4)
            mp[s, r, a] = v0 + m * h
            vals.append(chi2_sum(sub, y, z, row_x, n_rows, mp, **prm))
        out[i] = (-vals[0] + 8 * vals[1] - 8 * vals[2] + vals[3]) / (12 * h)
    return out


def subset_seeds(seeds, sel):
    offsets = np.asarray(seeds["offsets"])
    hits = np.asarray(seeds["hits"])
    n = np.diff(offsets)[sel]
    no = np.zeros(len(sel) + 1, np.int32)
    np.cumsum(n, out=no[1:])
    nh = np.concatenate([hits[offsets[i]:offsets[i + 1]] for i in sel]) if len(sel) else np.zeros(0, np.int32)
    return dict(offsets=no, hits=nh.astype(np.int32),
                frame=np.asarray(seeds["frame"])[sel], sector=np.asarray(seeds["sector"])[sel],
                first_row=np.asarray(seeds["first_row"])[sel])
