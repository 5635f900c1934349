"""ctypes declarations of libtpcreco's C-ABI (include/tpcreco.h).

Argument marshalling only.  The library is loaded after torch so that both
use the one HIP runtime torch brings; there is no fallback: a missing library
raises.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime the library binds to)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtpcreco_san.so" if os.environ.get("TPC_SANITIZE", "") == "1"
                        else "libtpcreco.so")

TPC_OK = 0
TPC_ERR_ARG = -1
TPC_ERR_CAPACITY = -2
TPC_ERR_HIP = -3
TPC_ERR_UNSUPPORTED = -4
TPC_ERR_WORKSPACE = -5

TPC_FIT_OK, TPC_FIT_INIT_FAIL, TPC_FIT_SIN_FAIL, TPC_FIT_NUM_FAIL = 0, 1, 2, 3
TPC_FOLLOW_DUPLICATE = 4
TPC_REFIT_NOT_HEAD = 5
TPC_REFIT_LONG_CHAIN = 6

TPC_STAGE_NEIGHBOURS = 1
TPC_STAGE_SEED = 2
TPC_STAGE_FIT = 4
TPC_STAGE_ADJOINT = 8
TPC_STAGE_FOLLOW = 32
TPC_STAGE_CTF = 64
TPC_STAGE_SKIP = 128
TPC_STAGE_SMOOTH = 256
TPC_STAGE_ALL = 511

P = ctypes.c_void_p
i32 = ctypes.c_int32
f32 = ctypes.c_float


class Config(ctypes.Structure):
    _fields_ = [("n_sectors", i32), ("n_rows", i32), ("row_x", P), ("bz", f32),
                ("sigma_y", f32), ("sigma_z", f32), ("win_y", f32), ("win_z", f32),
                ("cut_y", f32), ("cut_z", f32), ("min_hits", i32), ("max_sin", f32),
                ("var_sin0", f32), ("var_tgl0", f32), ("var_qpt0", f32), ("ckpt_rows", i32)]


class FramesC(ctypes.Structure):
    _fields_ = [("n_frames", i32), ("n_clusters", i32), ("row_offsets", P), ("y", P), ("z", P)]


class SeedsC(ctypes.Structure):
    _fields_ = [("cap_seeds", i32), ("cap_hits", i32), ("n_seeds", P), ("n_hits", P),
                ("offsets", P), ("hits", P), ("frame", P), ("sector", P), ("first_row", P),
                ("hit_yz", P)]


class TracksC(ctypes.Structure):
    _fields_ = [("x", P), ("par", P), ("cov", P), ("chi2", P), ("ndf", P), ("status", P)]


class Tune(ctypes.Structure):
    _fields_ = [("grid", i32), ("sort_fit", i32), ("fit_block", i32), ("fit_spt", i32)]


class Material(ctypes.Structure):
    _fields_ = [("x0", f32), ("mass", f32), ("chi2_cut", f32), ("rho", f32), ("z_over_a", f32),
                ("mean_exc", f32)]


class FollowParams(ctypes.Structure):
    _fields_ = [("gate_chi2", f32), ("max_miss", i32)]


class RansParams(ctypes.Structure):
    _fields_ = [("scale_bits", i32), ("block_symbols", i32)]


CTF_ARRAYS = ("trk_seg", "trk_n", "trk_row0", "trk_y0h", "trk_y0l", "trk_z0h", "trk_z0l", "trk_dy1",
              "trk_dz1", "hit_drow", "hit_ry", "hit_rz", "seg_nfree", "free_yh", "free_yl", "free_zh",
              "free_zl")


class CtfArraysC(ctypes.Structure):
    _fields_ = [(k, P) for k in CTF_ARRAYS] + [("counts", P)]


class RansJobC(ctypes.Structure):
    _fields_ = [("symbols", P), ("n", ctypes.c_int64), ("n_device", P), ("out", P), ("out_cap", ctypes.c_size_t),
                ("out_size", P), ("dev_status", P)]


TPC_RANS_BATCH_MAX = 24
TPC_MODE_STAGED = 0
TPC_MODE_PERSISTENT = 1
TPC_MODE_PERSISTENT_GRAPH = 2
TPC_STAGE_PERSISTENT = 16


class TpcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (status_string(code), code, msg))
        self.code = code


_lib = None

# name -> (restype, argtypes)
SIGNATURES = {
    "tpc_create": (i32, [ctypes.POINTER(Config), ctypes.POINTER(P)]),
    "tpc_destroy": (None, [P]),
    "tpc_workspace_bytes": (i32, [P, ctypes.POINTER(FramesC), i32, ctypes.POINTER(ctypes.c_size_t)]),
    "tpc_neighbours": (i32, [P, ctypes.POINTER(FramesC), P, P, P, ctypes.c_size_t, P]),
    "tpc_neighbours_skip": (i32, [P, ctypes.POINTER(FramesC), P, P, P, ctypes.c_size_t, P]),
    "tpc_ca_seed": (i32, [P, ctypes.POINTER(FramesC), P, P, ctypes.POINTER(SeedsC), P, P,
                          ctypes.c_size_t, P]),
    "tpc_ca_seed_noalloc": (i32, [P, ctypes.POINTER(FramesC), P, P, ctypes.POINTER(SeedsC), P, P]),
    "tpc_kalman_fit": (i32, [P, ctypes.POINTER(FramesC), ctypes.POINTER(SeedsC), P,
                             ctypes.POINTER(TracksC), P, ctypes.c_size_t, P, ctypes.c_size_t, P]),
    "tpc_ckpt_bytes": (i32, [P, ctypes.POINTER(SeedsC), ctypes.POINTER(ctypes.c_size_t)]),
    "tpc_chi2_sum": (i32, [P, ctypes.POINTER(SeedsC), ctypes.POINTER(TracksC), P, P, ctypes.c_size_t,
                           P]),
    "tpc_fit_adjoint": (i32, [P, ctypes.POINTER(FramesC), ctypes.POINTER(SeedsC), P,
                              ctypes.POINTER(TracksC), P, ctypes.c_size_t, P, P, P, ctypes.c_size_t,
                              P]),
    "tpc_reconstruct": (i32, [P, ctypes.POINTER(FramesC), i32, ctypes.POINTER(Tune), P, P,
                              ctypes.POINTER(SeedsC), ctypes.POINTER(TracksC), P, P, ctypes.c_size_t,
                              P]),
    "tpc_track_merge": (i32, [P, ctypes.POINTER(SeedsC), ctypes.POINTER(TracksC), ctypes.c_float, P, P, P, P, P,
                              P, P, P]),
    "tpc_track_refit": (i32, [P, ctypes.POINTER(FramesC), ctypes.POINTER(SeedsC), ctypes.POINTER(TracksC), P, P,
                              P, P, P, ctypes.POINTER(TracksC), P, P, P, P]),
    "tpc_track_follow": (i32, [P, ctypes.POINTER(FramesC), ctypes.POINTER(SeedsC),
                               ctypes.POINTER(FollowParams), P, ctypes.POINTER(TracksC), P,
                               ctypes.c_size_t, P]),
    "tpc_rans_workspace_bytes": (i32, [ctypes.c_int64, ctypes.POINTER(RansParams),
                                       ctypes.POINTER(ctypes.c_size_t)]),
    "tpc_rans_max_bytes": (i32, [ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(RansParams),
                                 ctypes.POINTER(ctypes.c_size_t)]),
    "tpc_rans_encode": (i32, [P, ctypes.c_int64, ctypes.POINTER(RansParams), P, ctypes.c_size_t, P, P, P,
                              ctypes.c_size_t, P]),
    "tpc_ctf_build": (i32, [P, ctypes.POINTER(FramesC), ctypes.POINTER(SeedsC), P, ctypes.POINTER(TracksC),
                            f32, f32, ctypes.POINTER(CtfArraysC), P, ctypes.c_size_t, P]),
    "tpc_rans_batch_workspace_bytes": (i32, [i32, P, ctypes.POINTER(RansParams), ctypes.POINTER(ctypes.c_size_t)]),
    "tpc_rans_encode_batch": (i32, [i32, P, ctypes.POINTER(RansParams), P, ctypes.c_size_t, P]),
    "tpc_kalman_fit_material": (i32, [P, ctypes.POINTER(FramesC), ctypes.POINTER(SeedsC),
                                      ctypes.POINTER(Material), ctypes.POINTER(TracksC), P, P,
                                      ctypes.c_size_t, P]),
    "tpc_kalman_fit_rows": (i32, [P, ctypes.POINTER(FramesC), ctypes.POINTER(SeedsC), P,
                                  ctypes.POINTER(Material), ctypes.POINTER(TracksC), P, P,
                                  ctypes.c_size_t, P]),
    "tpc_kalman_smooth": (i32, [P, ctypes.POINTER(FramesC), ctypes.POINTER(SeedsC), P,
                                ctypes.POINTER(Material), ctypes.POINTER(TracksC), P, P, P, P,
                                ctypes.c_size_t, P]),
    "tpc_rans_decode_workspace_bytes": (i32, [ctypes.POINTER(ctypes.c_size_t)]),
    "tpc_rans_decode": (i32, [P, ctypes.c_size_t, P, ctypes.c_int64, P, P, P, ctypes.c_size_t, P]),
    "tpc_persistent_grid": (i32, [P]),
    "tpc_status_string": (ctypes.c_char_p, [i32]),
    "tpc_last_error": (ctypes.c_char_p, []),
}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libtpcreco.so is not built (%s); run "
                              "`python -m paper_2412_13755_amd.build`" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(code: int) -> str:
    return lib().tpc_status_string(code).decode()


def last_error() -> str:
    return lib().tpc_last_error().decode()


def check(code: int) -> None:
    if code != TPC_OK:
        raise TpcError(code, last_error())
