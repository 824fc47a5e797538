"""Warp-by-warp parity of the full solve schedules against the FP64 oracle
(teacher forcing).

The whole method is an iteration of warps: each warp linearises the data
term at the current warping vectors (Eqs. (3), (5)), runs K primal-dual
iterations of Eq. (11) with the resolvent of Eq. (13), and clips and
accumulates the increment (Sec. III-C, Algorithm 1).  A whole solve of a full
configuration chains 15 to 105 warps, and the L1 data term makes that chain
ill-conditioned: a rounding-sized change of the input moves the FP64 result
by far more than the FP32 bar.  Here the library runs its full solve (the
same kernels, grids and batch as the timed solve, through vfs_solve_probe)
and hands over its float32 state at the start of a warp; the oracle then
runs that one warp in FP64 from exactly that state, and the two results are
compared at the FP32 bar of the configurations: mean |u - u_oracle| <=
1e-4 px and max <= 1e-3 px over the level's mask, the same for |w - w_o|.
This separates the arithmetic of each warp (what a kernel bug would change)
from the amplification of the method.

Which warps, fixed before any run: every warp of every level on the 128x128
plane (3 x 5) and on the 640x480 room (5 x 10); the first, a middle and the
last warp of every level on the 1280x1024 190-degree room (warps 0, 5, 9 of
6 levels) and on pairs 0 and 7 of the 8-pair 2048x2048 200-degree batch
(warps 0, 7, 14 of 7 levels), the batch being the launch the benchmark
times.  The oracle uses its own trajectory field and flags; the state it
starts from (pyramid images, u, w, v, p, q) is the GPU's.  The linearisation
and the tensor of the GPU at the same warp are held to the bars of the step
tests (I_u 5e-6, tensor 2e-6, rho_c 5e-5 + 5e-6 |u_w|: rho_c = I1(y) - J0(x)
- u_w I_u carries u_w times the rounding of I_u, and u_w reaches 150 px on
the 2048x2048 pairs), and the pyramid images to the oracle's pre-rotation and
box filter (1e-5).

With 16-bit storage of the duals and the tensor pack (FP32 arithmetic) the
same comparison is held to the storage bar of 0.05 px mean (first and last
warp of every level on the 1280x1024 room and on pairs 0 and 7 of the batch
in FP16; pair 0 in BF16); its maximum is reported.
"""
import functools

import numpy as np
import pytest

import oracle
from synth import configs, scene

pytestmark = pytest.mark.gpu

FP32_MEAN, FP32_MAX = 1e-4, 1e-3
STORAGE_MEAN = 0.05


@pytest.fixture(scope="module")
def vfs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1909_07545_amd as v
    return v


@functools.lru_cache(maxsize=None)
def _workload(cid):
    """Rig, solver parameters and the batch the library solves: every pair of
    the configuration (the 2048x2048 batch: its 8 pairs)."""
    cfg = configs.get(cid)
    rig = scene.make_rig(cfg)
    pairs = [scene.render_pair(rig, cfg, b, with_gt=False)[:2] for b in range(cfg["batch"])]
    tens = [scene.pair_tensor_params(cfg, b) for b in range(cfg["batch"])]
    return cfg, rig, pairs, tens


@functools.lru_cache(maxsize=None)
def _level_fields(cid, level):
    cfg, rig, _, _ = _workload(cid)
    cam0, cam1, R, t = rig["cam0"], rig["cam1"], rig["R"], rig["t"]
    m = oracle.level_mask(oracle.mask0(cam0), level).astype(np.uint8)
    dv = oracle.data_valid(cam0, cam1, R, t, level)
    gam, _ = oracle.trajectory_field(cam0, R, t, level)
    return m, dv, gam


@functools.lru_cache(maxsize=None)
def _pyramid(cid, pair, level):
    """The oracle's pre-rotated pyramids of a pair at a level (FP64 from the
    float32 images the GPU receives)."""
    cfg, rig, pairs, _ = _workload(cid)
    I0, I1 = (np.asarray(a, np.float64) for a in pairs[pair])
    cf, _ = oracle.calibration_field(rig["cam0"], rig["cam1"], rig["R"])
    J0, J1 = I0, oracle.prerotate(I1, cf)
    for _ in range(level):
        J0, J1 = oracle.downsample(J0), oracle.downsample(J1)
    return J0, J1


_RIGS = {}


def _gpu_rig(vfs, cid):
    if cid not in _RIGS:
        cfg, rig, _, _ = _workload(cid)
        _RIGS[cid] = vfs.Rig(rig["cam0"], rig["cam1"], rig["R"], rig["t"], cfg["levels"])
    return _RIGS[cid]


_DEV = {}


def _device_pairs(cid):
    import torch
    if cid not in _DEV:
        _, _, pairs, _ = _workload(cid)
        _DEV[cid] = ([torch.from_numpy(p[0]).cuda() for p in pairs], [torch.from_numpy(p[1]).cuda() for p in pairs])
    return _DEV[cid]


def _f64(t):
    return t.detach().float().cpu().numpy().astype(np.float64)


def _oracle_warp(cid, params, level, beta, eta, st):
    """One warp of Algorithm 1 in FP64 from the GPU's state at its start."""
    m, dv, gam = _level_fields(cid, level)
    J0, J1 = _f64(st["J0"]), _f64(st["J1"])
    u, w, p = _f64(st["u"]), _f64(st["w"]), _f64(st["p"])
    tgv = params.get("reg", "tgv") == "tgv"
    v = _f64(st["v"]) if tgv else None
    q = _f64(st["q"]) if tgv else None
    T = oracle.tensor(J0, m, beta, eta)
    uw, gw, Iu, rho = oracle.linearise(J0, J1, gam, dv, u, w)
    sp, su, sv = oracle.steps(T, m, params["alpha0"], params["alpha1"], params.get("reg", "tgv"))
    res = oracle.pd_iterations(params, T, m, sp, su, sv, Iu, rho, u, v, p, q, int(params["iters"]))
    u1, w1 = oracle.clip_accumulate(params["du_max"], uw, gw, res["u"], w)
    return dict(T=T, Iu=Iu, rho=rho, gw=gw, u_pd=res["u"], u=u1, w=w1)


def _probe_and_compare(vfs, cid, pair, level, warp, storage=0):
    cfg, rig, pairs, tens = _workload(cid)
    params = configs.solver_params(cfg, storage=storage)
    I0s, I1s = _device_pairs(cid)
    R = _gpu_rig(vfs, cid)
    betas = [b for b, _ in tens]
    etas = [e for _, e in tens]
    st = vfs.solve_probe(R, I0s, I1s, params, level, warp, pair, betas=betas, etas=etas)
    beta, eta = tens[pair]
    o = _oracle_warp(cid, params, level, beta, eta, st)
    m = _level_fields(cid, level)[0].astype(bool)
    du = np.abs(_f64(st["u_next"]) - o["u"])[m]
    dw = np.linalg.norm(_f64(st["w_next"]) - o["w"], axis=-1)[m]
    dpd = np.abs(_f64(st["u_pd"]) - o["u_pd"])[m]
    tp = _f64(st["tpack"])
    res = dict(cid=cid, pair=pair, level=level, warp=warp, storage=storage,
               u_mean=float(du.mean()), u_max=float(du.max()), w_mean=float(dw.mean()), w_max=float(dw.max()),
               u_pd_max=float(dpd.max()),
               Iu_max=float(np.max(np.abs(tp[..., 3] - o["Iu"]))),
               rho_max=float(np.max(np.abs(_f64(st["rho"]) - o["rho"]))),
               # rho_c = I1(y) - J0(x) - u_w I_u carries u_w times the rounding of I_u
               rho_rel=float(np.max(np.abs(_f64(st["rho"]) - o["rho"]) / (5e-5 + 5e-6 * np.abs(_f64(st["u"]))))),
               T_max=float(np.max(np.abs(tp[..., :3] - o["T"]))))
    if warp == 0 and storage == 0:
        J0o, J1o = _pyramid(cid, pair, level)
        res["J0_max"] = float(np.max(np.abs(_f64(st["J0"]) - J0o)))
        res["J1_max"] = float(np.max(np.abs(_f64(st["J1"]) - J1o)))
    print("warp parity", res, flush=True)
    return res


def _assert_fp32(r):
    assert r["u_mean"] <= FP32_MEAN and r["u_max"] <= FP32_MAX, r
    assert r["w_mean"] <= FP32_MEAN and r["w_max"] <= FP32_MAX, r
    assert r["T_max"] <= 2e-6 and r["Iu_max"] <= 5e-6 and r["rho_rel"] <= 1.0, r
    if "J0_max" in r:
        assert r["J0_max"] <= 1e-6 and r["J1_max"] <= 1e-5, r


def _cases(cid, warps_of_level, pairs=(0,)):
    cfg = configs.get(cid)
    return [(cid, b, l, w) for b in pairs for l in range(cfg["levels"])[::-1] for w in warps_of_level(cfg)]


FP32_CASES = (_cases("c1", lambda c: range(c["warps"])) + _cases("c2", lambda c: range(c["warps"]))
              + _cases("c3", lambda c: (0, 5, 9)) + _cases("c5", lambda c: (0, 7, 14), pairs=(0, 7)))


@pytest.mark.parametrize("cid,pair,level,warp", FP32_CASES,
                         ids=[f"{c}-pair{b}-L{l}-w{w}" for c, b, l, w in FP32_CASES])
def test_fp32_warp_meets_the_bar(vfs, cid, pair, level, warp):
    _assert_fp32(_probe_and_compare(vfs, cid, pair, level, warp))


STORAGE_CASES = ([(c, b, l, w, 1) for c, b, l, w in _cases("c3", lambda c: (0, 9))]
                 + [(c, b, l, w, 1) for c, b, l, w in _cases("c5", lambda c: (0, 14), pairs=(0, 7))]
                 + [(c, b, l, w, 2) for c, b, l, w in _cases("c3", lambda c: (0, 9))]
                 + [(c, b, l, w, 2) for c, b, l, w in _cases("c5", lambda c: (0, 14))])


@pytest.mark.parametrize("cid,pair,level,warp,storage", STORAGE_CASES,
                         ids=[f"{c}-pair{b}-L{l}-w{w}-{'f16' if s == 1 else 'bf16'}"
                              for c, b, l, w, s in STORAGE_CASES])
def test_16bit_storage_warp_within_the_storage_bar(vfs, cid, pair, level, warp, storage):
    r = _probe_and_compare(vfs, cid, pair, level, warp, storage)
    assert r["u_mean"] <= STORAGE_MEAN and r["w_mean"] <= STORAGE_MEAN, r


def test_probe_rejects_bad_requests(vfs):
    cfg, rig, pairs, tens = _workload("c1")
    params = configs.solver_params(cfg)
    I0s, I1s = _device_pairs("c1")
    R = _gpu_rig(vfs, "c1")
    for lvl, wp, pr in ((cfg["levels"], 0, 0), (-1, 0, 0), (0, cfg["warps"], 0), (0, 0, 1)):
        with pytest.raises(vfs.VfsError, match="probe"):
            vfs.solve_probe(R, I0s, I1s, params, lvl, wp, pr)
