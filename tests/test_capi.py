"""Host-side checks of the C-ABI (no GPU needed): the library loads, exports
every function include/tpcreco.h declares, and rejects bad arguments before
touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tpcreco.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tpc_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def capi():
    from paper_2412_13755_amd import _capi
    return _capi


def test_header_declares_the_path():
    names = declared_functions()
    for n in ("tpc_create", "tpc_destroy", "tpc_workspace_bytes", "tpc_neighbours", "tpc_ca_seed",
              "tpc_kalman_fit", "tpc_ckpt_bytes", "tpc_chi2_sum", "tpc_fit_adjoint",
              "tpc_track_follow", "tpc_track_merge", "tpc_rans_encode", "tpc_rans_workspace_bytes",
              "tpc_rans_max_bytes", "tpc_ctf_build", "tpc_rans_encode_batch",
              "tpc_rans_batch_workspace_bytes", "tpc_kalman_fit_material", "tpc_rans_decode",
              "tpc_rans_decode_workspace_bytes", "tpc_neighbours_skip", "tpc_kalman_fit_rows",
              "tpc_kalman_smooth", "tpc_status_string", "tpc_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(capi):
    L = capi.lib()
    for n in declared_functions():
        assert hasattr(L, n), n
    # and the binding declares a signature for each
    assert set(declared_functions()) <= set(capi.SIGNATURES)


def test_library_is_gfx950_only():
    """The shared object carries device code for gfx950 and no other target."""
    from paper_2412_13755_amd import _capi
    data = open(_capi.LIB_PATH, "rb").read()
    assert b"gfx950" in data
    for other in (b"gfx90a", b"gfx942", b"gfx1100", b"gfx908"):
        assert other not in data


def _cfg(capi, **over):
    row_x = np.linspace(85, 245, 152).astype(np.float32)
    d = dict(n_sectors=36, n_rows=152, row_x=row_x.ctypes.data_as(ctypes.c_void_p), bz=0.5,
             sigma_y=0.05, sigma_z=0.06, win_y=2.5, win_z=2.5, cut_y=0.6, cut_z=0.75, min_hits=5,
             max_sin=0.999, var_sin0=1.0, var_tgl0=1.0, var_qpt0=100.0, ckpt_rows=16)
    d.update(over)
    return capi.Config(**d), row_x


@pytest.mark.parametrize("bad", [dict(n_rows=2), dict(n_rows=300), dict(n_sectors=0), dict(bz=0.0),
                                 dict(sigma_y=0.0), dict(win_z=-1.0), dict(min_hits=2),
                                 dict(max_sin=1.0), dict(var_qpt0=0.0), dict(ckpt_rows=0),
                                 dict(row_x=None)])
def test_create_rejects_bad_config(capi, bad):
    cfg, _keep = _cfg(capi, **bad)
    h = ctypes.c_void_p()
    rc = capi.lib().tpc_create(ctypes.byref(cfg), ctypes.byref(h))
    assert rc == capi.TPC_ERR_ARG, capi.last_error()
    assert h.value is None
    assert capi.last_error()


def test_create_rejects_decreasing_rows(capi):
    row_x = np.linspace(245, 85, 152).astype(np.float32)
    cfg, _ = _cfg(capi, row_x=row_x.ctypes.data_as(ctypes.c_void_p))
    h = ctypes.c_void_p()
    assert capi.lib().tpc_create(ctypes.byref(cfg), ctypes.byref(h)) == capi.TPC_ERR_ARG


def test_calls_reject_null_context_and_frames(capi):
    L = capi.lib()
    fr = capi.FramesC(1, 0, None, None, None)
    assert L.tpc_neighbours(None, ctypes.byref(fr), None, None, None, 0, None) == capi.TPC_ERR_ARG
    sd = capi.SeedsC()
    assert L.tpc_ca_seed(None, ctypes.byref(fr), None, None, ctypes.byref(sd), None, None, 0,
                         None) == capi.TPC_ERR_ARG
    tr = capi.TracksC()
    assert L.tpc_kalman_fit(None, ctypes.byref(fr), ctypes.byref(sd), None, ctypes.byref(tr), None,
                            0, None, 0, None) == capi.TPC_ERR_ARG
    assert L.tpc_fit_adjoint(None, ctypes.byref(fr), ctypes.byref(sd), None, ctypes.byref(tr), None,
                             0, None, None, None, 0, None) == capi.TPC_ERR_ARG
    assert L.tpc_chi2_sum(None, ctypes.byref(sd), ctypes.byref(tr), None, None, 0,
                          None) == capi.TPC_ERR_ARG
    fp = capi.FollowParams(25.0, 3)
    assert L.tpc_track_follow(None, ctypes.byref(fr), ctypes.byref(sd), ctypes.byref(fp), None,
                              ctypes.byref(tr), None, 0, None) == capi.TPC_ERR_ARG
    assert L.tpc_neighbours_skip(None, ctypes.byref(fr), None, None, None, 0, None) == capi.TPC_ERR_ARG
    assert L.tpc_kalman_fit_rows(None, ctypes.byref(fr), ctypes.byref(sd), None, None, ctypes.byref(tr),
                                 None, None, 0, None) == capi.TPC_ERR_ARG
    assert L.tpc_kalman_smooth(None, ctypes.byref(fr), ctypes.byref(sd), None, None, ctypes.byref(tr),
                               None, None, None, None, 0, None) == capi.TPC_ERR_ARG
    assert "context" in L.tpc_last_error().decode()
    n = ctypes.c_size_t()
    assert L.tpc_ckpt_bytes(None, ctypes.byref(sd), ctypes.byref(n)) == capi.TPC_ERR_ARG
    n = ctypes.c_size_t()
    assert L.tpc_workspace_bytes(None, ctypes.byref(fr), 1, ctypes.byref(n)) == capi.TPC_ERR_ARG


def test_rans_host_checks(capi):
    L = capi.lib()
    n = ctypes.c_size_t()
    for bits, blk in ((0, 64), (17, 64), (12, 100), (12, 0)):
        p = capi.RansParams(bits, blk)
        assert L.tpc_rans_workspace_bytes(1000, ctypes.byref(p), ctypes.byref(n)) == capi.TPC_ERR_ARG
    p = capi.RansParams(12, 4096)
    assert L.tpc_rans_workspace_bytes(-1, ctypes.byref(p), ctypes.byref(n)) == capi.TPC_ERR_ARG
    assert L.tpc_rans_max_bytes(1000, 50, ctypes.byref(p), ctypes.byref(n)) == capi.TPC_OK
    assert n.value == 40 + 6 * 50 + 4 * 2 + 256 + 2 * 1000     # table: at most 6 bytes per present symbol
    assert L.tpc_rans_max_bytes(1000, (1 << 20) + 1, ctypes.byref(p), ctypes.byref(n)) == capi.TPC_ERR_ARG
    assert L.tpc_rans_encode(None, 10, ctypes.byref(p), None, 0, None, None, None, 0,
                             None) == capi.TPC_ERR_ARG
    jobs = (capi.RansJobC * 2)()
    jobs[0].n, jobs[1].n = 100, 1 << 31
    assert L.tpc_rans_batch_workspace_bytes(2, jobs, ctypes.byref(p), ctypes.byref(n)) == capi.TPC_ERR_ARG
    assert L.tpc_rans_batch_workspace_bytes(0, jobs, ctypes.byref(p), ctypes.byref(n)) == capi.TPC_ERR_ARG
    assert L.tpc_rans_batch_workspace_bytes(25, jobs, ctypes.byref(p), ctypes.byref(n)) == capi.TPC_ERR_ARG
    jobs[1].n = 50
    assert L.tpc_rans_batch_workspace_bytes(2, jobs, ctypes.byref(p), ctypes.byref(n)) == capi.TPC_OK
    assert L.tpc_rans_encode_batch(2, jobs, ctypes.byref(p), None, 0, None) == capi.TPC_ERR_ARG


def test_status_strings(capi):
    assert capi.status_string(0) == "TPC_OK"
    assert capi.status_string(-2) == "TPC_ERR_CAPACITY"
    assert capi.status_string(-5) == "TPC_ERR_WORKSPACE"
    assert capi.status_string(-99) == "TPC_ERR_UNKNOWN"


def test_binding_refuses_non_hip_device():
    from paper_2412_13755_amd.reco import Reco, RecoConfig
    with pytest.raises(ValueError):
        Reco(RecoConfig(row_x=np.linspace(85, 245, 152).astype(np.float32)), device="cpu")


def test_upload_validates_offsets():
    from paper_2412_13755_amd.reco import DeviceFrames
    y = np.zeros(4, np.float32)
    with pytest.raises(ValueError):
        DeviceFrames.from_numpy(np.array([0, 3, 2, 4]), y, y, 1, 1, 3, device="cpu")
    with pytest.raises(ValueError):
        DeviceFrames.from_numpy(np.array([0, 1, 2, 3]), y, y, 1, 1, 3, device="cpu")


def test_merge_host_checks(capi):
    # every check runs on the host before any launch; a zero-capacity call
    # returns TPC_OK without touching the device (the context is only read
    # by the launch)
    L = capi.lib()
    ctx = ctypes.create_string_buffer(8192)
    word = ctypes.c_int32(0)
    w = ctypes.addressof(word)
    sd = capi.SeedsC(0, 0, w, w, w, None, None, None, None, None)
    tr = capi.TracksC()
    buf = ctypes.create_string_buffer(64)
    b = ctypes.addressof(buf)
    assert L.tpc_track_merge(None, ctypes.byref(sd), ctypes.byref(tr), ctypes.c_float(30.0), b, b, b, None, None,
                             None, None, None) == capi.TPC_ERR_ARG
    assert "context" in L.tpc_last_error().decode()
    assert L.tpc_track_merge(ctx, None, ctypes.byref(tr), ctypes.c_float(30.0), b, b, b, None, None,
                             None, None, None) == capi.TPC_ERR_ARG
    for cut in (0.0, -1.0, float("nan"), float("inf")):
        assert L.tpc_track_merge(ctx, ctypes.byref(sd), ctypes.byref(tr), ctypes.c_float(cut), b, b, b, None, None,
                                 None, None, None) == capi.TPC_ERR_ARG
        assert "chi2_cut" in L.tpc_last_error().decode()
    assert L.tpc_track_merge(ctx, ctypes.byref(sd), ctypes.byref(tr), ctypes.c_float(30.0), b, b, b, b, None,
                             None, None, None) == capi.TPC_ERR_ARG
    assert "merged" in L.tpc_last_error().decode()
    assert L.tpc_track_merge(ctx, ctypes.byref(sd), ctypes.byref(tr), ctypes.c_float(30.0), b, b, b, None, None,
                             b, None, None) == capi.TPC_ERR_ARG
    assert "leg" in L.tpc_last_error().decode()
    assert L.tpc_track_merge(ctx, ctypes.byref(sd), ctypes.byref(tr), ctypes.c_float(30.0), b, b, b, None, None,
                             None, None, None) == capi.TPC_OK
