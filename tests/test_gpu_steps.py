"""GPU parity of each step of the method against the FP64 oracle, on the
same seeded inputs (the oracle receives the float32 values the GPU gets).

Sizes: C1 (128x128), a ragged 200x136 rig (neither dimension a multiple of
the primal-dual tile of 62 columns x 64 rows), and the full 2048x2048 level 0
of the batched 200-degree configuration.  Tolerances are the FP32 rounding of
each step (stated per test).
"""
import numpy as np
import pytest

import oracle
from synth import configs, scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vfs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1909_07545_amd as v
    return v


def _t(a, dtype=None):
    import torch
    a = np.ascontiguousarray(a)
    t = torch.from_numpy(a if dtype is None else a.astype(dtype))
    return t.cuda()


def _np(t):
    return t.detach().cpu().numpy()


def f32(a):
    """The float32 value the GPU receives, as float64 for the oracle."""
    return np.asarray(a, np.float32).astype(np.float64)


_FLAGS = {}


def oracle_flags(rig, level):
    key = (id(rig), level)
    if key not in _FLAGS:
        _FLAGS[key] = _oracle_flags(rig, level)
    return _FLAGS[key]


def _oracle_flags(rig, level):
    cam0, cam1, R, t = rig["cam0"], rig["cam1"], rig["R"], rig["t"]
    m = oracle.level_mask(oracle.mask0(cam0), level).astype(np.uint8)
    mx = np.zeros_like(m)
    my = np.zeros_like(m)
    mx[:, :-1] = m[:, :-1] & m[:, 1:]
    my[:-1, :] = m[:-1, :] & m[1:, :]
    dv = oracle.data_valid(cam0, cam1, R, t, level)
    _, epi = oracle.trajectory_field(cam0, R, t, level)
    return (m | (mx << 1) | (my << 2) | (dv << 3) | (epi << 4)).astype(np.uint8)


RIGS = ["c1", "r200", "c2", "c5", "ucm", "eucm"]


_RIGS = {}


def _rig(cid):
    if cid not in _RIGS:
        _RIGS[cid] = scene.make_rig(configs.get(cid))
    return _RIGS[cid]


@pytest.mark.parametrize("cid", RIGS)
def test_rig_fields(vfs, cid):
    """Flags bit-exact; trajectory field and calibration field within float32
    rounding of the FP64 values."""
    rig = _rig(cid)
    cfg = configs.get(cid)
    R = vfs.Rig(rig["cam0"], rig["cam1"], rig["R"], rig["t"], cfg["levels"])
    for l in range(cfg["levels"]):
        fl = _np(R.field(l, vfs.FIELD_FLAGS))
        assert np.array_equal(fl, oracle_flags(rig, l)), f"level {l}"
        g = _np(R.field(l, vfs.FIELD_TRAJECTORY))
        go, _ = oracle.trajectory_field(rig["cam0"], rig["R"], rig["t"], l)
        assert np.max(np.abs(g - go)) < 1e-6, f"level {l}"
    c = _np(R.field(0, vfs.FIELD_CALIBRATION))
    co, _ = oracle.calibration_field(rig["cam0"], rig["cam1"], rig["R"])
    assert np.max(np.abs(c - co)) < 2e-5


def _smooth_image(H, W, seed, lo=0.1, hi=0.9):
    rng = np.random.default_rng(seed)
    jj, ii = np.meshgrid(np.arange(W), np.arange(H))
    s = np.zeros((H, W))
    for _ in range(12):
        k = rng.uniform(0.01, 0.3, 2) * rng.choice([-1, 1], 2)
        s += np.cos(k[0] * jj + k[1] * ii + rng.uniform(0, 6.3)) / np.linalg.norm(k)
    s = (s - s.min()) / (s.max() - s.min())
    return (lo + (hi - lo) * s + 0.01 * rng.normal(size=(H, W))).astype(np.float32)


def _level_inputs(cid, level, seed=0):
    rig = _rig(cid)
    H, W = rig["cam0"]["height"] >> level, rig["cam0"]["width"] >> level
    flags = oracle_flags(rig, level)
    J0 = _smooth_image(H, W, seed)
    J1 = _smooth_image(H, W, seed + 1)
    gam, _ = oracle.trajectory_field(rig["cam0"], rig["R"], rig["t"], level)
    return rig, flags, J0, J1, gam.astype(np.float32)


@pytest.mark.parametrize("cid,level", [("c1", 0), ("r200", 0), ("c2", 1), ("c5", 0)])
def test_tensor(vfs, cid, level):
    """Eq. (12) on the level image: float32 vs FP64 within 2e-6."""
    import torch
    rig, flags, J0, _, _ = _level_inputs(cid, level)
    H, W = J0.shape
    tp = torch.zeros((H, W, 4), device="cuda")
    for beta, eta in ((9.0, 0.85), (11.3, 0.72)):
        vfs.step_tensor(_t(J0), _t(flags), beta, eta, tp)
        To = oracle.tensor(f32(J0), flags & 1, beta, eta)
        assert np.max(np.abs(_np(tp)[..., :3] - To)) < 2e-6


@pytest.mark.parametrize("cid,level", [("c1", 0), ("r200", 0), ("c2", 1), ("c5", 0)])
def test_linearise_and_clip(vfs, cid, level):
    """Eqs. (3), (5) at the warped point, with the clip and accumulation of
    the previous warp: u, u_w, w, gamma_w, I_u, rho_c within 5e-6."""
    import torch
    rig, flags, J0, J1, gam = _level_inputs(cid, level, seed=3)
    H, W = J0.shape
    rng = np.random.default_rng(4)
    jj, ii = np.meshgrid(np.arange(W), np.arange(H))
    u_w = (2.0 + np.sin(0.05 * jj) * np.cos(0.04 * ii)).astype(np.float32)
    u = (u_w + rng.uniform(-0.5, 0.5, (H, W))).astype(np.float32)
    w = (u_w[..., None] * gam + rng.uniform(-0.3, 0.3, (H, W, 2))).astype(np.float32)
    gw = gam.copy()
    tu, tuw, tw, tgw = _t(u), _t(u_w), _t(w), _t(gw)
    tp = torch.zeros((H, W, 4), device="cuda")
    rho = torch.zeros((H, W), device="cuda")
    vfs.step_linearise(_t(J0), _t(J1), _t(gam), _t(flags), tu, tuw, tw, tgw, tp, rho, True, False, 0.2)
    uo, wo = oracle.clip_accumulate(0.2, f32(u_w), f32(gw), f32(u), f32(w))
    uwo, gwo, Iuo, rhoo = oracle.linearise(f32(J0), f32(J1), f32(gam), (flags >> 3) & 1, uo, wo)
    assert np.max(np.abs(_np(tu) - uo)) < 5e-6
    assert np.max(np.abs(_np(tw) - wo)) < 5e-6
    assert np.max(np.abs(_np(tuw) - uwo)) < 5e-6
    # renormalising a short bicubic sample (next to an epipole guard) scales its rounding
    assert np.max(np.abs(_np(tgw) - gwo)) < 5e-5
    assert np.max(np.abs(_np(tp)[..., 3] - Iuo)) < 5e-6
    assert np.max(np.abs(_np(rho) - rhoo)) < 5e-5


@pytest.mark.parametrize("H,W", [(128, 128), (136, 200), (1, 7), (3, 2), (2048, 2048)])
def test_rank(vfs, H, W):
    """The rank transform (5x5, share of strictly darker neighbours, edges
    clamped): the neighbour counts are integers decided by float32
    comparisons on both sides, so they must match exactly; random values
    and a quantised image full of ties."""
    import torch
    rng = np.random.default_rng(H * 7 + W)
    I0 = _smooth_image(H, W, 11) if min(H, W) > 8 else rng.random((H, W)).astype(np.float32)
    I1 = (np.round(rng.random((H, W)) * 5) / 5).astype(np.float32)
    R0 = torch.full((H, W), float("nan"), device="cuda")
    R1 = torch.full((H, W), float("nan"), device="cuda")
    vfs.step_rank(_t(I0), _t(I1), R0, R1)
    for got, I in ((R0, I0), (R1, I1)):
        g = _np(got).astype(np.float64) * 24.0
        assert np.array_equal(np.rint(g), np.rint(oracle.rank_transform(f32(I), 2) * 24.0))
        assert np.max(np.abs(g - np.rint(g))) < 1e-5


@pytest.mark.parametrize("H,W", [(128, 128), (136, 200), (1, 7), (3, 2), (2048, 2048)])
def test_gradient(vfs, H, W):
    """Gradient magnitude (central differences, edges clamped): float32 vs
    FP64 on the same float32 inputs within 1e-6 (values up to about 1)."""
    import torch
    rng = np.random.default_rng(H * 5 + W)
    I0 = _smooth_image(H, W, 13) if min(H, W) > 8 else rng.random((H, W)).astype(np.float32)
    I1 = rng.random((H, W)).astype(np.float32)
    G0 = torch.full((H, W), float("nan"), device="cuda")
    G1 = torch.full((H, W), float("nan"), device="cuda")
    vfs.step_gradient(_t(I0), _t(I1), G0, G1)
    for got, I in ((G0, I0), (G1, I1)):
        assert np.max(np.abs(_np(got).astype(np.float64) - oracle.gradient_magnitude(f32(I)))) < 1e-6


def _pd_state(cid, level, tgv=True, seed=5):
    rig, flags, J0, _, _ = _level_inputs(cid, level, seed=seed)
    H, W = J0.shape
    m = flags & 1
    T = oracle.tensor(f32(J0), m, 9.0, 0.85).astype(np.float32)
    rng = np.random.default_rng(seed)
    Iu = (rng.normal(0, 0.05, (H, W)) * ((flags >> 3) & 1)).astype(np.float32)
    rho = (rng.normal(0, 0.05, (H, W)) * ((flags >> 3) & 1)).astype(np.float32)
    u = (1.5 + 0.3 * rng.random((H, W))).astype(np.float32)
    v = (0.05 * rng.normal(size=(H, W, 2)) * m[..., None]).astype(np.float32)
    p = oracle.project_balls(0.7 * rng.normal(size=(H, W, 2)), 2).reshape(H, W, 2) * m[..., None]
    q = oracle.project_balls(0.7 * rng.normal(size=(H, W, 4)), 4).reshape(H, W, 4) * m[..., None]
    return flags, T, Iu, rho, u, v, p.astype(np.float32), q.astype(np.float32)


@pytest.mark.parametrize("cid,level,K,reg,tg,npass", [
    ("c1", 0, 1, "tgv", 0.0, 0), ("c1", 0, 2, "tgv", 0.0, 0), ("c1", 0, 3, "tgv", 0.0, 0),
    ("r200", 0, 4, "tv", 0.0, 0), ("c1", 0, 50, "tgv", 0.0, 0), ("c5", 0, 5, "tgv", 0.0, 0),
    ("r200", 1, 6, "tgv", 0.4, 0), ("r200", 0, 7, "tgv", 0.0, 0), ("r200", 0, 50, "tv", 0.0, 0),
    ("c1", 1, 30, "tgv", 0.3, 0), ("c2", 0, 20, "tgv", 0.0, 0), ("c5", 0, 3, "tgv", 0.0, 0),
    ("c1", 0, 50, "tgv", 0.0, 3), ("r200", 0, 8, "tv", 0.0, 3), ("r200", 1, 11, "tgv", 0.4, 3),
    ("c5", 0, 8, "tgv", 0.0, 3), ("c1", 0, 50, "tgv", 0.0, 4), ("r200", 0, 9, "tgv", 0.0, 4),
    ("r200", 0, 6, "tv", 0.0, 4), ("c2", 0, 14, "tgv", 0.0, 4), ("c5", 0, 6, "tgv", 0.0, 2),
    ("c5", 0, 4, "tgv", 0.0, 0), ("r200", 0, 3, "tgv", 0.3, 3), ("r200", 0, 2, "tgv", 0.0, 2)])
def test_primal_dual(vfs, cid, level, K, reg, tg, npass):
    """K iterations of Eq. (11) from a warp start: u, v, p, q within 2e-5 of
    the FP64 oracle (float32 accumulates ~1e-7 per iteration).  npass: the
    iterations per pass of the multi-iteration launches (0: the library's
    choice, 4 on the 2048x2048 level, 3 on smaller pairs), so that the 2-, 3-
    and 4-iteration kernels all run, with the first pass of a warp (K >= N,
    its first iteration the dual half alone) and without it (K < N starts with
    a dual-only launch), and with the remainders of K - N that need one- and
    two-iteration launches."""
    import torch
    tgv = reg == "tgv"
    flags, T, Iu, rho, u, v, p, q = _pd_state(cid, level, tgv)
    H, W = u.shape
    params = dict(configs.PAPER_PARAMS, levels=1, warps=1, iters=K, reg=reg, theta_gamma=tg, pass_iters=npass)
    tpack = np.concatenate([T, Iu[..., None]], -1).astype(np.float32)
    tu, tp = _t(u), _t(p)
    tv, tq = (_t(v), _t(q)) if tgv else (None, None)
    vfs.step_pd(_t(tpack), _t(rho), _t(flags), tu, tv, tp, tq, params, K)
    torch.cuda.synchronize()
    m = flags & 1
    sp, su, sv = oracle.steps(f32(T), m, params["alpha0"], params["alpha1"], reg)
    st = oracle.pd_iterations(params, f32(T), m, sp, su, sv, f32(Iu), f32(rho), f32(u), f32(v), f32(p), f32(q), K)
    tol = 2e-5
    assert np.max(np.abs(_np(tu) - st["u"])) < tol
    assert np.max(np.abs(_np(tp) - st["p"])) < tol
    if tgv:
        assert np.max(np.abs(_np(tv) - st["v"])) < tol
        assert np.max(np.abs(_np(tq) - st["q"])) < tol


# Half an ulp at magnitude 1 of the 16-bit formats (FP16: 10 fraction bits,
# BF16: 7): the most a stored dual component (|p|, |q| <= 1 after the
# projections) moves when it is rounded.
HALF_ULP = {1: 2.0 ** -12, 2: 2.0 ** -9}


@pytest.mark.parametrize("cid,level,K,reg,storage,npass", [
    ("c5", 0, 8, "tgv", 1, 3), ("c5", 0, 8, "tgv", 2, 3), ("c5", 0, 7, "tgv", 1, 2), ("c5", 0, 6, "tgv", 2, 2),
    ("c5", 0, 10, "tv", 1, 3), ("c1", 0, 50, "tgv", 1, 3), ("c1", 0, 50, "tgv", 1, 2), ("c1", 0, 11, "tgv", 2, 3),
    ("r200", 0, 9, "tgv", 1, 4), ("r200", 1, 11, "tgv", 2, 3), ("r200", 0, 8, "tv", 2, 3), ("c2", 0, 20, "tgv", 1, 2)])
def test_primal_dual_16bit_storage(vfs, cid, level, K, reg, storage, npass):
    """K iterations of Eq. (11) with the duals and the tensor pack stored as
    FP16 / BF16 (FP32 arithmetic, u and v FP32), by the 2-, 3- and
    4-iteration pass kernels, against the FP64 oracle started from the same
    16-bit values of p, q, T and I_u.  The GPU rounds p and q each time a
    launch stores them (at most once per iteration), the oracle never.  One
    rounding moves a dual component by at most h (half an ulp at magnitude
    1), and moves the next primal step by at most h too (the preconditioned
    primal step tau sums the dual changes with weights whose abs-sum is 1);
    the iteration is nonexpansive in its preconditioned metric, so K
    roundings add up to at most K h there.  Bars: max |d| <= 2 K h (a factor
    2 for propagation measured pixel by pixel rather than in that metric),
    mean |d| <= sqrt(K) h (independent, unbiased roundings), each plus the
    FP32 bar of the 32-bit test, for u, v, p and q."""
    import torch
    tgv = reg == "tgv"
    flags, T, Iu, rho, u, v, p, q = _pd_state(cid, level, tgv)
    H, W = u.shape
    dt = torch.float16 if storage == 1 else torch.bfloat16
    params = dict(configs.PAPER_PARAMS, levels=1, warps=1, iters=K, reg=reg, storage=storage, pass_iters=npass)
    tp16 = torch.from_numpy(np.concatenate([T, Iu[..., None]], -1).astype(np.float32)).to(dt).cuda()
    p16 = torch.from_numpy(p).to(dt).cuda()
    q16 = torch.from_numpy(q).to(dt).cuda() if tgv else None
    tu = _t(u)
    tv = _t(v) if tgv else None
    back = lambda t: t.float().cpu().numpy().astype(np.float64)  # noqa: E731
    T0, Iu0, p0 = back(tp16)[..., :3], back(tp16)[..., 3], back(p16)
    q0 = back(q16) if tgv else None
    vfs.step_pd(tp16, _t(rho), _t(flags), tu, tv, p16, q16, params, K)
    torch.cuda.synchronize()
    m = flags & 1
    sp, su, sv = oracle.steps(T0, m, params["alpha0"], params["alpha1"], reg)
    st = oracle.pd_iterations(params, T0, m, sp, su, sv, Iu0, f32(rho), f32(u), f32(v), p0, q0, K)
    h = HALF_ULP[storage]
    max_bar, mean_bar = 2 * K * h + 2e-5, np.sqrt(K) * h + 2e-5
    inside = m.astype(bool)
    got = dict(u=_np(tu), p=back(p16))
    if tgv:
        got.update(v=_np(tv), q=back(q16))
    for k, g in got.items():
        d = np.abs(g - st[k])[inside]
        print(cid, level, K, reg, storage, npass, k, float(d.mean()), float(d.max()), mean_bar, max_bar, flush=True)
        assert d.max() <= max_bar and d.mean() <= mean_bar, (k, float(d.mean()), float(d.max()))


@pytest.mark.parametrize("storage,npass,K", [(0, 2, 7), (0, 3, 8), (0, 4, 9), (0, 4, 3), (1, 3, 8), (2, 4, 6)])
def test_primal_dual_reads_nothing_outside_the_image(vfs, storage, npass, K):
    """The pass kernels address a row through a buffer resource whose record
    count is the image width, and give rows outside the image a count of 0.
    A ragged 201 x 150 image in planes of 256-element rows with 6 rows below
    it: with NaN in every float (and every flag bit set) outside the image,
    each output inside the image is bitwise what it is with zeros there, and
    finite -- the kernels read nothing outside the image.  Pass depths 2, 3,
    4, with and without the first pass of a warp, FP32 and 16-bit storage."""
    import torch
    H, W, P, extra = 150, 201, 256, 6
    rng = np.random.default_rng(11)
    yy, xx = np.mgrid[0:H, 0:W]
    m = ((xx - 100.0) ** 2 + (yy - 74.5) ** 2 <= 72.0 ** 2).astype(np.uint8)
    mx = np.zeros_like(m)
    mx[:, :-1] = m[:, :-1] & m[:, 1:]
    my = np.zeros_like(m)
    my[:-1] = m[:-1] & m[1:]
    data = m & (rng.random((H, W)) < 0.9)
    flags = (m | (mx << 1) | (my << 2) | (data << 3)).astype(np.uint8)
    J0 = _smooth_image(H, W, 3)
    T = oracle.tensor(f32(J0), m, 9.0, 0.85).astype(np.float32)
    Iu = (rng.normal(0, 0.05, (H, W)) * data).astype(np.float32)
    rho = (rng.normal(0, 0.05, (H, W)) * data).astype(np.float32)
    u = (1.5 + 0.3 * rng.random((H, W))).astype(np.float32)
    v = (0.05 * rng.normal(size=(H, W, 2)) * m[..., None]).astype(np.float32)
    p = (oracle.project_balls(0.7 * rng.normal(size=(H, W, 2)), 2).reshape(H, W, 2) * m[..., None]).astype(np.float32)
    q = (oracle.project_balls(0.7 * rng.normal(size=(H, W, 4)), 4).reshape(H, W, 4) * m[..., None]).astype(np.float32)
    tpack = np.concatenate([T, Iu[..., None]], -1).astype(np.float32)
    dt = {0: torch.float32, 1: torch.float16, 2: torch.bfloat16}[storage]
    params = dict(configs.PAPER_PARAMS, levels=1, warps=1, iters=K, reg="tgv", storage=storage, pass_iters=npass)

    def run(fill):
        def plane(a, dtype, fill_value):
            shape = (H + extra, P) + a.shape[2:]
            t = torch.full(shape, fill_value, dtype=dtype, device="cuda")
            t[:H, :W] = torch.from_numpy(a).to(dtype).cuda()
            return t
        f = plane(flags, torch.uint8, 255 if fill else 0)
        nan = float("nan") if fill else 0.0
        st = dict(tpack=plane(tpack, dt, nan), rho=plane(rho, torch.float32, nan), u=plane(u, torch.float32, nan),
                  v=plane(v, torch.float32, nan), p=plane(p, dt, nan), q=plane(q, dt, nan))
        vfs.step_pd(st["tpack"], st["rho"], f, st["u"], st["v"], st["p"], st["q"], params, K, width=W, height=H)
        torch.cuda.synchronize()
        return {k: st[k][:H, :W].float().cpu() for k in ("u", "v", "p", "q")}

    clean, dirty = run(False), run(True)
    for k in clean:
        assert torch.isfinite(clean[k]).all() and torch.equal(clean[k], dirty[k]), k


@pytest.mark.parametrize("cid,level", [("c1", 1), ("r200", 1), ("c5", 1)])
def test_upsample(vfs, cid, level):
    """Mask-aware x2 transfer of (u, w) (Sec. IV-B): within 2e-6."""
    import torch
    rig = _rig(cid)
    flags_c = oracle_flags(rig, level)
    Hc, Wc = flags_c.shape
    rng = np.random.default_rng(6)
    uc = rng.uniform(0, 4, (Hc, Wc)).astype(np.float32)
    wc = rng.uniform(-4, 4, (Hc, Wc, 2)).astype(np.float32)
    uf = torch.zeros((2 * Hc, 2 * Wc), device="cuda")
    wf = torch.zeros((2 * Hc, 2 * Wc, 2), device="cuda")
    vfs.step_upsample(_t(flags_c), _t(uc), _t(wc), uf, wf)
    uo, wo = oracle.upsample(flags_c & 1, f32(uc), f32(wc))
    assert np.max(np.abs(_np(uf) - uo)) < 2e-6
    assert np.max(np.abs(_np(wf) - wo)) < 2e-6


@pytest.mark.parametrize("cid", ["c1", "c2", "c5", "ucm", "eucm"])
def test_triangulate(vfs, cid):
    """Closest-approach depth in single precision (rays from the rig's
    radial table, built in double precision at set-up) against the FP64
    oracle on the same float32 warp vectors.  A float32 ray is off by about
    1e-7 rad (the rounding of the table, of the polar angle and of the pixel
    position x + w).  When the two rays turn by such an angle, a point seen
    at ranges d0 and d1 under the parallax angle |a x b| moves by about
    (d0 + d1) 1e-7 / |a x b|, so the relative error of d0 is about
    (1 + d1 / d0) 1e-7 / |a x b|: the bar is 1e-5 + 5e-7 (1 + d1 / d0) /
    |a x b|, with d1 from the oracle's rays (d1 / d0 is large for points
    within a few baselines of camera 0).  Validity is decided by
    |a x b|^2 > 1e-12 and the signs of the two ranges; it must be identical
    wherever the oracle's |a x b|^2 is at least 4e-12 (outside the band where
    float32 rounding reaches the threshold: |w| below about 1e-3 px); inside
    the band both answers are correct."""
    import torch
    rig = _rig(cid)
    cfg = configs.get(cid)
    cam = rig["cam0"]
    H, W = cam["height"], cam["width"]
    R = vfs.Rig(rig["cam0"], rig["cam1"], rig["R"], rig["t"], cfg["levels"])
    gam, _ = oracle.trajectory_field(cam, rig["R"], rig["t"], 0)
    rng = np.random.default_rng(7)
    w = (gam * rng.uniform(-0.5, 6.0, (H, W, 1))).astype(np.float32)
    depth = torch.zeros((H, W), device="cuda")
    z = torch.zeros((H, W), device="cuda")
    valid = torch.zeros((H, W), dtype=torch.uint8, device="cuda")
    vfs.step_triangulate(R, _t(w), depth, z, valid)
    dv = oracle.data_valid(cam, rig["cam1"], rig["R"], rig["t"], 0)
    do, zo, vo = oracle.triangulate(cam, rig["R"], rig["t"], f32(w), dv)
    vg = _np(valid).astype(bool)
    jj, ii = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    x0 = np.stack([jj.ravel(), ii.ravel()], -1)
    ra = oracle.unproject(cam, x0)
    rb = oracle.unproject(cam, x0 + f32(w).reshape(-1, 2))
    n = np.cross(ra, rb)
    nn = np.linalg.norm(n, axis=-1).reshape(H, W)
    # range along b of the closest approach, from the oracle's rays (for the bar)
    C = -(np.asarray(rig["R"]).T @ np.asarray(rig["t"]))
    d1 = (np.sum(np.cross(np.broadcast_to(C, ra.shape), ra) * n, -1) /
          np.maximum(np.sum(n * n, -1), 1e-300)).reshape(H, W)
    band = nn ** 2 < 4e-12
    flips = vg != vo
    print(cid, "validity flips", int(flips.sum()), "of them in the rounding band", int((flips & band).sum()),
          "band pixels", int(band.sum()), flush=True)
    assert not (flips & ~band).any()
    ok = vo & vg
    assert ok.sum() > 0.5 * vo.sum()
    bar = 1e-5 + 5e-7 * (1.0 + np.abs(d1[ok]) / do[ok]) / nn[ok]
    rel = np.abs(_np(depth)[ok] - do[ok]) / do[ok]
    print(cid, "depth rel. error max", float(rel.max()), "share of bar", float((rel / bar).max()), flush=True)
    assert np.all(rel <= bar), (rel.max(), (rel / bar).max())
    assert np.all(np.abs(_np(z)[ok] - zo[ok]) / do[ok] <= bar)
    assert np.all(np.isinf(_np(depth)[~vg]))


@pytest.mark.parametrize("W,H", [(1, 1), (5, 3), (2, 70), (63, 2), (57, 9)])
@pytest.mark.parametrize("npass", [2, 3, 4])
def test_primal_dual_degenerate_sizes(vfs, W, H, npass):
    """K = 9 iterations of Eq. (11) on images smaller than one wavefront's
    strip or one march's halo (a single pixel, a few rows or columns, one
    strip with its halo lanes past the image): every pass kernel against the
    FP64 oracle at the step bar, with the first pass of a warp and a
    remainder launch (9 = N + a multiple of N + a remainder for N = 2, 4)."""
    import torch
    K = 9
    rng = np.random.default_rng(100 * W + H)
    m = (rng.random((H, W)) < 0.85).astype(np.uint8)
    m[0, 0] = 1
    mx = np.zeros_like(m)
    mx[:, :-1] = m[:, :-1] & m[:, 1:]
    my = np.zeros_like(m)
    my[:-1] = m[:-1] & m[1:]
    data = m & (rng.random((H, W)) < 0.9).astype(np.uint8)
    flags = (m | (mx << 1) | (my << 2) | (data << 3)).astype(np.uint8)
    J0 = rng.uniform(0.1, 0.9, (H, W)).astype(np.float32)
    T = oracle.tensor(f32(J0), m, 9.0, 0.85).astype(np.float32)
    Iu = (rng.normal(0, 0.05, (H, W)) * data).astype(np.float32)
    rho = (rng.normal(0, 0.05, (H, W)) * data).astype(np.float32)
    u = (1.5 + 0.3 * rng.random((H, W))).astype(np.float32)
    v = (0.05 * rng.normal(size=(H, W, 2)) * m[..., None]).astype(np.float32)
    p = (oracle.project_balls(0.7 * rng.normal(size=(H, W, 2)), 2).reshape(H, W, 2) * m[..., None]).astype(np.float32)
    q = (oracle.project_balls(0.7 * rng.normal(size=(H, W, 4)), 4).reshape(H, W, 4) * m[..., None]).astype(np.float32)
    params = dict(configs.PAPER_PARAMS, levels=1, warps=1, iters=K, reg="tgv", pass_iters=npass)
    tpack = np.concatenate([T, Iu[..., None]], -1).astype(np.float32)
    tu, tv, tp, tq = _t(u), _t(v), _t(p), _t(q)
    print("degenerate", W, H, npass, flush=True)
    vfs.step_pd(_t(tpack), _t(rho), _t(flags), tu, tv, tp, tq, params, K)
    torch.cuda.synchronize()
    sp, su, sv = oracle.steps(f32(T), m, params["alpha0"], params["alpha1"], "tgv")
    st = oracle.pd_iterations(params, f32(T), m, sp, su, sv, f32(Iu), f32(rho), f32(u), f32(v), f32(p), f32(q), K)
    for k, g in (("u", tu), ("v", tv), ("p", tp), ("q", tq)):
        assert np.max(np.abs(_np(g) - st[k])) < 2e-5, k
