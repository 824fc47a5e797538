"""The C ABI library: it loads without a GPU, exports every entry point that
include/vfs.h declares, and rejects bad arguments before any device work
(these calls return before the first HIP runtime call, so they run on the
CPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vfs.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*(vfs_[a-z0-9_]+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def vfs():
    from paper_1909_07545_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libvfs.so not built (run __graft_entry__.build())")
    return _lib


def test_exports_every_declared_symbol(vfs):
    names = _declared()
    assert len(names) >= 14
    L = ctypes.CDLL(vfs.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n


def test_params_default_are_the_paper_values(vfs):
    import json
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_parameters.json")))
    d = vfs.default_params()
    assert (d["alpha0"], d["alpha1"], d["beta"], d["eta"], d["du_max"]) == \
        (g["alpha0"], g["alpha1"], g["beta"], g["eta"], g["du_max_px"])
    assert d["reg"] == "tgv" and d["theta_gamma"] == 0.0 and d["pass_iters"] == 0


CAM = dict(model="kb", width=64, height=48, fx=20.0, fy=20.0, cx=31.5, cy=23.5, k=(0.01, -0.005, 0.0, 0.0),
           fov_deg=180.0)


def _create(vfs, cam0=CAM, cam1=CAM, R=np.eye(3), t=(0.1, 0, 0), levels=3):
    L = vfs.lib()
    c0, c1 = vfs._camera(cam0), vfs._camera(cam1)
    Rr = (ctypes.c_double * 9)(*np.asarray(R, float).reshape(9))
    tt = (ctypes.c_double * 3)(*np.asarray(t, float))
    h = ctypes.c_void_p()
    st = L.vfs_rig_create(ctypes.byref(c0), ctypes.byref(c1), Rr, tt, levels, None, ctypes.byref(h))
    return st, L.vfs_last_error().decode()


def test_rig_create_rejects_bad_arguments(vfs):
    assert _create(vfs, t=(0.0, 0.0, 0.0))[0] == -5                                 # zero baseline
    assert _create(vfs, cam0=dict(CAM, k=(0, 0, 0, -0.05), fov_deg=200))[0] == -4   # non-monotone r_d
    assert _create(vfs, cam0=dict(CAM, model="pinhole", fov_deg=180))[0] == -4
    assert _create(vfs, cam1=dict(CAM, width=32))[0] == -1                          # size mismatch
    assert _create(vfs, levels=6)[0] == -1                                          # 48 not divisible by 32
    assert _create(vfs, levels=0)[0] == -1
    assert _create(vfs, cam0=dict(CAM, fx=0.0))[0] == -1
    st, msg = _create(vfs, t=(0.0, 0.0, 0.0))
    assert "baseline" in msg
    wide = dict(CAM, width=(1 << 20) + 32, cx=float(1 << 19))                       # above the row limit
    st, msg = _create(vfs, cam0=wide, cam1=wide)
    assert st == -1 and "width above" in msg
    L = vfs.lib()
    assert L.vfs_rig_create(None, None, None, None, 3, None, None) == -1


def test_solve_and_steps_reject_bad_arguments(vfs):
    L = vfs.lib()
    p = vfs._params(dict(vfs.default_params(), levels=3))
    one = (ctypes.c_void_p * 1)(1)
    assert L.vfs_solve_batch(None, 1, one, one, 256, one, one, one, None, None, ctypes.byref(p), None, None,
                             None) == -1
    assert L.vfs_solve_probe(None, 1, one, one, 256, ctypes.byref(p), None, None, None, None) == -1
    assert L.vfs_step_tensor(0, 4, 4, one, one, 9.0, 0.85, one, None) == -1
    assert L.vfs_step_tensor(8, 4, 4, one, one, 9.0, 0.85, one, None) == -1           # pitch < width
    bad = vfs._params(dict(vfs.default_params(), alpha1=0.0))
    assert L.vfs_step_pd(8, 8, 8, one, one, one, one, one, one, one, one, one, one, one, ctypes.byref(bad), 3,
                         None) == -1
    for npass in (1, 5, -2):
        badp = vfs._params(dict(vfs.default_params(), pass_iters=npass))
        assert L.vfs_step_pd(8, 8, 8, one, one, one, one, one, one, one, one, one, one, one, ctypes.byref(badp),
                             3, None) == -1
        assert "pass_iters" in L.vfs_last_error().decode()
    assert L.vfs_step_upsample(4, 4, 2, one, one, one, 8, one, one, None) == -1
    big = (1 << 20) + 1                                                               # rows above 2^20 elements
    assert L.vfs_step_pd(big, 1, big, one, one, one, one, one, one, one, one, one, one, one, ctypes.byref(p), 3,
                         None) == -1
    assert L.vfs_step_pd(0, 1, 1, one, one, one, one, one, one, one, one, one, one, one, ctypes.byref(p), 3,
                         None) == -1                                                  # empty image
    assert L.vfs_profile_enable(None, 1) == -1


def test_server_rejects_bad_configuration(vfs):
    L = vfs.lib()
    cfg = vfs.ServerConfig()
    assert L.vfs_server_config_default(ctypes.byref(cfg)) == 0
    assert (cfg.mode, cfg.hbm_budget_bytes, cfg.max_slots, cfg.use_graphs) == (0, 1 << 30, 16, 1)
    p = vfs._params(dict(vfs.default_params(), warps=10, iters=50))
    h = ctypes.c_void_p()
    for field, value in (("max_slots", 0), ("max_slots", 33), ("mode", 2), ("hbm_budget_bytes", 0)):
        bad = vfs.ServerConfig(cfg.mode, cfg.hbm_budget_bytes, cfg.max_slots, cfg.use_graphs)
        setattr(bad, field, value)
        assert L.vfs_server_create(ctypes.byref(bad), ctypes.byref(p), ctypes.byref(h)) == -1, field
    no_warps = vfs._params(dict(vfs.default_params(), warps=0))
    assert L.vfs_server_create(ctypes.byref(cfg), ctypes.byref(no_warps), ctypes.byref(h)) == -1
    assert "warps" in L.vfs_last_error().decode()
    assert L.vfs_server_create(ctypes.byref(cfg), ctypes.byref(p), None) == -1
    tk = ctypes.c_ulonglong()
    assert L.vfs_server_submit(None, None, None, None, 0, None, None, None, None, None, 9.0, 0.85,
                               ctypes.byref(tk)) == -1
    done = ctypes.c_int()
    assert L.vfs_server_poll(None, 1, ctypes.byref(done), None) == -1
    assert L.vfs_server_wait_all(None, 1.0) == -1


def test_binding_checks_buffers_before_the_library(vfs):
    """The binding passes bare pointers, so it checks every tensor's device,
    dtype and shape, and a batch's per-pair lengths, before calling into the
    library: mismatches raise here, on the CPU, and nothing is launched."""
    import types

    import torch
    rig = types.SimpleNamespace(height=4, width=6, handle=None, levels=1)
    cpu = torch.zeros((4, 6))
    with pytest.raises(TypeError, match="CUDA"):
        vfs.step_rank(cpu, cpu, cpu, cpu)
    with pytest.raises(ValueError, match="2-D"):
        vfs.step_gradient(torch.zeros(4), cpu, cpu, cpu)
    with pytest.raises(ValueError, match="I1s: 0 images for 1 pairs"):
        vfs.solve_batch(rig, [cpu], [], {})
    with pytest.raises(ValueError, match="betas: 2 values for 1 pairs"):
        vfs.solve_batch(rig, [cpu], [cpu], {}, betas=[9.0, 9.0])
    with pytest.raises(ValueError, match="out: 0 entries for 1 pairs"):
        vfs.solve_batch_noalloc(rig, [cpu], [cpu], {}, out=[])
    with pytest.raises(TypeError, match=r"I0s\[0\]: expected a contiguous CUDA tensor"):
        vfs.solve_probe(rig, [cpu], [cpu], {}, 0, 0)
