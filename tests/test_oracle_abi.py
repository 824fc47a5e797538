"""The oracle's C entry points named after the library's calls
(vfso_params_default, vfso_rig_create / destroy, vfso_rig_field,
vfso_solve / vfso_solve_batch, vfso_energy; host pointers): they load and
export every name, reject bad arguments, and give exactly what the oracle's
step functions give on the same inputs (they are plumbing over them)."""
import ctypes
import json
import os

import numpy as np
import pytest

import oracle
from synth import configs, scene

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NAMES = ["vfso_params_default", "vfso_rig_create", "vfso_rig_destroy", "vfso_rig_field", "vfso_solve",
         "vfso_solve_batch", "vfso_energy"]


@pytest.fixture(scope="module")
def L():
    lib = oracle.lib()
    for n in NAMES:
        assert hasattr(lib, n), n
    lib.vfso_rig_destroy.restype = None
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _rig(L, d):
    rig = d["rig"]
    c0, c1 = oracle._cam(rig["cam0"]), oracle._cam(rig["cam1"])
    R, t = oracle._R(rig["R"]), oracle._t(rig["t"])
    h = ctypes.c_void_p()
    st = L.vfso_rig_create(ctypes.byref(c0), ctypes.byref(c1), _p(R), _p(t), d["cfg"]["levels"], ctypes.byref(h))
    assert st == 0
    return h


def test_params_default_are_the_paper_values(L):
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_parameters.json")))
    p = oracle._Params()
    assert L.vfso_params_default(ctypes.byref(p)) == 0
    assert (p.alpha0, p.alpha1, p.beta, p.eta, p.du_max) == (g["alpha0"], g["alpha1"], g["beta"], g["eta"],
                                                             g["du_max_px"])
    assert (p.reg, p.theta_gamma, p.data_term) == (0, 0.0, 0)


def test_rig_create_rejects_bad_arguments(L):
    cfg = configs.get("c1")
    rig = scene.make_rig(cfg)
    c0 = oracle._cam(rig["cam0"])
    R = oracle._R(rig["R"])
    h = ctypes.c_void_p()
    zero = np.zeros(3)
    assert L.vfso_rig_create(ctypes.byref(c0), ctypes.byref(c0), _p(R), _p(zero), 3, ctypes.byref(h)) == -5
    t = oracle._t(rig["t"])
    assert L.vfso_rig_create(ctypes.byref(c0), ctypes.byref(c0), _p(R), _p(t), 9, ctypes.byref(h)) == -1
    assert L.vfso_rig_create(None, None, None, None, 3, ctypes.byref(h)) == -1


def test_solve_field_and_energy_equal_the_oracle_steps(L):
    d = scene.make_inputs("c1", 1)
    rig, cfg = d["rig"], d["cfg"]
    params = configs.solver_params(cfg, warps=2)
    h = _rig(L, d)
    try:
        H, W = cfg["height"], cfg["width"]
        I0, I1 = d["I0"][0].astype(np.float64), d["I1"][0].astype(np.float64)
        u, w = np.zeros((H, W)), np.zeros((H, W, 2))
        depth, z, valid = np.zeros((H, W)), np.zeros((H, W)), np.zeros((H, W), np.uint8)
        pp = oracle._par(params)
        assert L.vfso_solve(h, _p(I0), _p(I1), _p(u), _p(w), _p(depth), _p(z), _p(valid), ctypes.byref(pp)) == 0
        ref = oracle.solve(rig["cam0"], rig["cam1"], rig["R"], rig["t"], params, I0, I1)
        assert np.array_equal(u, ref["u"]) and np.array_equal(w, ref["w"])
        assert np.array_equal(depth, ref["depth"]) and np.array_equal(valid.astype(bool), ref["valid"])
        # a mismatched level count is refused
        bad = oracle._par(dict(params, levels=2))
        assert L.vfso_solve(h, _p(I0), _p(I1), _p(u), _p(w), _p(depth), None, None, ctypes.byref(bad)) == -1
        for level in range(cfg["levels"]):
            Hl, Wl = H >> level, W >> level
            g = np.zeros((Hl, Wl, 2))
            assert L.vfso_rig_field(h, level, 0, _p(g)) == 0
            assert np.array_equal(g, oracle.trajectory_field(rig["cam0"], rig["R"], rig["t"], level)[0])
            m = np.zeros((Hl, Wl))
            assert L.vfso_rig_field(h, level, 2, _p(m)) == 0
            assert np.array_equal(m.astype(np.uint8), oracle.level_mask(oracle.mask0(rig["cam0"]), level))
        assert L.vfso_rig_field(h, 1, 1, _p(np.zeros((H, W, 2)))) == -1
        rng = np.random.default_rng(3)
        msk = oracle.mask0(rig["cam0"]).astype(np.uint8)
        T = oracle.tensor(I0, msk, 9.0, 0.85)
        Iu, rho, v = rng.normal(size=(H, W)), rng.normal(size=(H, W)), rng.normal(size=(H, W, 2))
        e = ctypes.c_double()
        assert L.vfso_energy(W, H, ctypes.byref(pp), _p(T), _p(msk), _p(Iu), _p(rho), _p(u), _p(v),
                             ctypes.byref(e)) == 0
        assert e.value == oracle.energy(params, T, msk, Iu, rho, u, v)
    finally:
        L.vfso_rig_destroy(h)
