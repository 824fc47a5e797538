"""Pins of the oracle's solver: the primal-dual iteration (Eq. (11)) against
the optimality conditions of the energy (Eq. (10)), its energy behaviour,
the whole loop (Algorithm 1 in the pyramid of Sec. IV-B) against an
independent rectified solver, and recovered depth against rendered ground
truth.
"""
import numpy as np
import pytest

import oracle
from synth import configs, scene
from tests import rectified


PAPER = configs.PAPER_PARAMS


def _small_problem(seed, H=10, W=12, tgv=True):
    rng = np.random.default_rng(seed)
    m = np.ones((H, W), np.uint8)
    m[rng.random((H, W)) < 0.12] = 0
    J = 0.5 + 0.3 * np.sin(0.7 * np.arange(W)[None, :] + 0.4 * np.arange(H)[:, None]) + 0.05 * rng.random((H, W))
    T = oracle.tensor(J, m, 9.0, 0.85)
    Iu = rng.normal(0, 0.08, (H, W)) * m
    rho = rng.normal(0, 0.1, (H, W)) * m
    params = dict(PAPER, levels=1, warps=1, iters=0, reg="tgv" if tgv else "tv")
    return params, T, m, Iu, rho


def _np_grad(u, m):
    H, W = m.shape
    mx = np.zeros((H, W), bool)
    my = np.zeros((H, W), bool)
    mx[:, :-1] = (m[:, :-1] > 0) & (m[:, 1:] > 0)
    my[:-1, :] = (m[:-1, :] > 0) & (m[1:, :] > 0)
    gx = np.zeros_like(u)
    gy = np.zeros_like(u)
    gx[:, :-1] = u[:, 1:] - u[:, :-1]
    gy[:-1, :] = u[1:, :] - u[:-1, :]
    return gx * mx, gy * my, mx, my


def _np_div(px, py, mx, my):
    ax, ay = px * mx, py * my
    d = ax + ay
    d[:, 1:] -= ax[:, :-1]
    d[1:, :] -= ay[:-1, :]
    return d


@pytest.mark.parametrize("tgv", [True, False], ids=["tgv", "tv"])
def test_pd_converges_to_a_minimiser_of_the_energy(tgv):
    """After many iterations the iterates satisfy the optimality conditions of
    the linearised energy lambda|rho_c + u I_u| + alpha1|T grad u - v| +
    alpha0|grad v| (subdifferential calculus on Eq. (10), written here from
    the energy, independently of the iteration):
      p in d|.|(T grad u - v), q in d|.|(grad v), alpha1 p + alpha0 div q = 0,
      alpha1 div(T p) in lambda I_u sign(rho_c + u I_u)."""
    params, T, m, Iu, rho = _small_problem(11, tgv=tgv)
    H, W = m.shape
    z = np.zeros((H, W))
    sp, tu, tv = oracle.steps(T, m, params["alpha0"], params["alpha1"], params["reg"])
    st = oracle.pd_iterations(params, T, m, sp, tu, tv, Iu, rho, z, np.zeros((H, W, 2)),
                              np.zeros((H, W, 2)), np.zeros((H, W, 4)), 60000)
    u, p = st["u"], st["p"]
    v = st["v"] if tgv else np.zeros((H, W, 2))
    a0, a1, lam = params["alpha0"], params["alpha1"], params["lambda"]
    gx, gy, mx, my = _np_grad(u, m)
    inm = m > 0
    # p in the subdifferential of the Euclidean norm at T grad u - v
    r1 = T[..., 0] * gx + T[..., 1] * gy - v[..., 0]
    r2 = T[..., 1] * gx + T[..., 2] * gy - v[..., 1]
    rn = np.hypot(r1, r2)
    assert np.all(np.hypot(p[..., 0], p[..., 1])[inm] <= 1 + 1e-12)
    act = inm & (rn > 1e-3)
    assert act.sum() > 10
    assert np.max(np.abs(p[..., 0] - r1 / np.where(rn > 0, rn, 1))[act]) < 1e-3
    assert np.max(np.abs(p[..., 1] - r2 / np.where(rn > 0, rn, 1))[act]) < 1e-3
    # u: alpha1 div(T p) in lambda I_u d|.|(rho_bar)
    dtp = _np_div(T[..., 0] * p[..., 0] + T[..., 1] * p[..., 1],
                  T[..., 1] * p[..., 0] + T[..., 2] * p[..., 1], mx, my)
    rb = rho + u * Iu
    act = inm & (np.abs(rb) > 1e-4)
    assert act.sum() > 5
    assert np.max(np.abs(a1 * dtp - lam * Iu * np.sign(rb))[act]) < 1e-3
    tie = inm & ~act
    assert np.all(np.abs(a1 * dtp)[tie] <= lam * np.abs(Iu)[tie] + 1e-3)
    if tgv:
        q = st["q"]
        d11, d12, _, _ = _np_grad(v[..., 0], m)
        d21, d22, _, _ = _np_grad(v[..., 1], m)
        gn = np.sqrt(d11 ** 2 + d12 ** 2 + d21 ** 2 + d22 ** 2)
        assert np.all(np.linalg.norm(q, axis=-1)[inm] <= 1 + 1e-12)
        act = inm & (gn > 1e-3)
        for c, d in enumerate((d11, d12, d21, d22)):
            assert np.max(np.abs(q[..., c] - d / np.where(gn > 0, gn, 1))[act], initial=0) < 1e-3
        # v: alpha1 p + alpha0 div q = 0
        r = a1 * p[..., 0] + a0 * _np_div(q[..., 0], q[..., 1], mx, my)
        s = a1 * p[..., 1] + a0 * _np_div(q[..., 2], q[..., 3], mx, my)
        assert np.max(np.abs(r[inm])) < 1e-3 and np.max(np.abs(s[inm])) < 1e-3


def test_pd_energy_decreases_over_inner_loops(c1_inputs):
    """Reading of "non-increasing energy" for a primal-dual method (which is
    not a descent method: after each warp the energy rises for the first few
    iterations while the duals adapt): over every inner loop of the C1 solve
    the linearised energy ends below where it starts."""
    d = c1_inputs
    rig, cfg = d["rig"], d["cfg"]
    cam0, R, t = rig["cam0"], rig["R"], rig["t"]
    params = configs.solver_params(cfg)
    I0 = d["I0"][0].astype(np.float64)
    I1 = d["I1"][0].astype(np.float64)
    cf, vc = oracle.calibration_field(cam0, rig["cam1"], R)
    J0, J1 = [I0], [oracle.prerotate(I1, cf)]
    for _ in range(1, params["levels"]):
        J0.append(oracle.downsample(J0[-1]))
        J1.append(oracle.downsample(J1[-1]))
    m0 = oracle.mask0(cam0)
    for l in range(params["levels"]):
        ml = oracle.level_mask(m0, l)
        dl = oracle.data_valid(cam0, rig["cam1"], R, t, l)
        gam, _ = oracle.trajectory_field(cam0, R, t, l)
        T = oracle.tensor(J0[l], ml, params["beta"], params["eta"])
        sp, tu, tv = oracle.steps(T, ml, params["alpha0"], params["alpha1"])
        H, W = ml.shape
        u, w = np.zeros((H, W)), np.zeros((H, W, 2))
        v, p, q = np.zeros((H, W, 2)), np.zeros((H, W, 2)), np.zeros((H, W, 4))
        for _ in range(3):
            uw, gw, Iu, rho = oracle.linearise(J0[l], J1[l], gam, dl, u, w)
            st = oracle.pd_iterations(params, T, ml, sp, tu, tv, Iu, rho, u, v, p, q, params["iters"], trace=True)
            E = st["energy"]
            assert E[-1] < E[0]
            u, v, p, q = st["u"], st["v"], st["p"], st["q"]
            u, w = oracle.clip_accumulate(params["du_max"], uw, gw, u, w)


@pytest.mark.parametrize("tgv", [True, False], ids=["tgv", "tv"])
def test_pd_energy_converges_to_its_minimum(tgv):
    """Long run on a small problem: the energy settles (relative change below
    1e-6 over the second half of 2e4 iterations; the rate is sublinear, so
    the tail keeps moving at the 1e-8 level) and no earlier iterate has a
    lower energy than the limit (the limit is a minimiser, so its energy is
    the minimum)."""
    params, T, m, Iu, rho = _small_problem(14, H=16, W=16, tgv=tgv)
    z = np.zeros(m.shape)
    sp, tu, tv = oracle.steps(T, m, params["alpha0"], params["alpha1"], params["reg"])
    st = oracle.pd_iterations(params, T, m, sp, tu, tv, Iu, rho, z, np.zeros(m.shape + (2,)),
                              np.zeros(m.shape + (2,)), np.zeros(m.shape + (4,)), 20000, trace=True)
    E = st["energy"]
    half = E[len(E) // 2:]
    assert (half.max() - half.min()) / E[-1] < 1e-6
    assert np.all(E >= E[-1] * (1 - 1e-9))


def test_clip_special_case():
    """du_max = inf and one warp on one level: u is the primal-dual output and
    w = u gamma'(x) (Eq. (9) with a single piece)."""
    cam = dict(model="equidistant", width=48, height=40, fx=14.0, fy=14.0, cx=23.5, cy=19.5,
               k=(0.0,) * 4, fov_deg=170.0)
    R, t = np.eye(3), np.array([0.1, 0.0, 0.0])
    rng = np.random.default_rng(12)
    I0 = rng.random((40, 48))
    I1 = np.roll(I0, 1, axis=1)
    params = dict(PAPER, levels=1, warps=1, iters=40, du_max=np.inf)
    out = oracle.solve(cam, cam, R, t, params, I0, I1)
    gam, _ = oracle.trajectory_field(cam, R, t, 0)
    assert np.max(np.abs(out["w"] - out["u"][..., None] * gam)) < 1e-15
    # and it is the inner loop's result
    ml = oracle.mask0(cam)
    dl = oracle.data_valid(cam, cam, R, t, 0)
    T = oracle.tensor(I0, ml, params["beta"], params["eta"])
    sp, tu, tv = oracle.steps(T, ml, params["alpha0"], params["alpha1"])
    uw, gw, Iu, rho = oracle.linearise(I0, I1, gam, dl, np.zeros((40, 48)), np.zeros((40, 48, 2)))
    st = oracle.pd_iterations(params, T, ml, sp, tu, tv, Iu, rho, np.zeros((40, 48)), np.zeros((40, 48, 2)),
                              np.zeros((40, 48, 2)), np.zeros((40, 48, 4)), 40)
    assert np.array_equal(st["u"], out["u"])


def test_warped_tangent_is_continuous_at_an_epipole():
    """Around an epipole the trajectory field turns through every direction
    (Sec. III-B), and its sample there is a short sum of opposed vectors.  The
    warped tangent is that sample over max(|sample|, 1/2): unit length where
    the bicubic taps stay away from the epipole, 0 at the epipole itself, and
    tending to 0 as the warped point approaches it (a unit renormalisation
    would jump there)."""
    H, W, e = 20, 24, (11.0, 8.0)
    jj, ii = np.meshgrid(np.arange(W, dtype=float), np.arange(H, dtype=float))
    r = np.stack([jj - e[0], ii - e[1]], -1)
    n = np.linalg.norm(r, axis=-1, keepdims=True)
    gam = np.where(n > 0, r / np.where(n > 0, n, 1.0), 0.0)
    Z = np.zeros((H, W))

    def tangent(points):
        w = np.zeros((H, W, 2))
        w[..., 0] = points[..., 0] - jj
        w[..., 1] = points[..., 1] - ii
        _, gw, _, _ = oracle.linearise(Z, Z, gam, np.zeros((H, W), np.uint8), Z, w)
        return gw

    # far from the epipole: unit length, and within the interpolation error of the radial direction
    far = (np.abs(jj - e[0]) >= 4) | (np.abs(ii - e[1]) >= 4)
    pts = np.stack([jj + 0.37, ii + 0.61], -1)
    g = tangent(pts)
    assert np.max(np.abs(np.linalg.norm(g, axis=-1)[far] - 1.0)) < 1e-12
    rad = (pts - np.array(e)) / np.linalg.norm(pts - np.array(e), axis=-1, keepdims=True)
    assert np.min(np.sum(g * rad, axis=-1)[far]) > 0.99
    # at the epipole and approaching it along several directions
    for d in ((1.0, 0.0), (0.6, -0.8), (-0.28, 0.96)):
        prev = None
        for delta in (1e-2, 1e-4, 1e-6, 1e-9, 0.0):
            p = np.broadcast_to(np.array([e[0] + delta * d[0], e[1] + delta * d[1]]), (H, W, 2)).copy()
            length = float(np.linalg.norm(tangent(p)[0, 0]))
            assert length <= 40.0 * delta + 1e-15, (d, delta, length)
            prev = length
        assert prev == 0.0
    # Lipschitz in the warped point on a fine grid across the epipole
    xs = e[0] + np.linspace(-2.5, 2.5, W)
    ys = e[1] + np.linspace(-2.5, 2.5, H)
    gx, gy = np.meshgrid(xs, ys)
    g = tangent(np.stack([gx, gy], -1))
    h = xs[1] - xs[0]
    assert np.max(np.linalg.norm(np.diff(g, axis=1), axis=-1)) / h < 6.0
    assert np.max(np.linalg.norm(np.diff(g, axis=0), axis=-1)) / (ys[1] - ys[0]) < 6.0


def test_pinhole_x_translation_equals_rectified_solver():
    """Pinhole with pure x-translation reduces to the conventional (1, 0)
    rectified search: the oracle's whole loop equals an independently written
    rectified TGV-L1 solver."""
    W, H = 96, 64
    cam = dict(model="pinhole", width=W, height=H, fx=40.0, fy=40.0, cx=(W - 1) / 2, cy=(H - 1) / 2,
               k=(0.0,) * 4, fov_deg=120.0)
    rng = np.random.default_rng(13)
    jj, ii = np.meshgrid(np.arange(W), np.arange(H))
    tex = 0.5 + 0.25 * np.sin(0.35 * jj + 0.2 * ii) + 0.15 * np.cos(0.13 * jj - 0.31 * ii)
    disp = 1.5 + 0.5 * np.sin(0.05 * jj)
    I0 = tex + 0.01 * rng.normal(size=(H, W))
    I1 = 0.5 + 0.25 * np.sin(0.35 * (jj - disp) + 0.2 * ii) + 0.15 * np.cos(0.13 * (jj - disp) - 0.31 * ii)
    params = dict(PAPER, levels=3, warps=3, iters=25)
    out = oracle.solve(cam, cam, np.eye(3), [0.1, 0.0, 0.0], params, I0, I1)
    m0 = oracle.mask0(cam)
    ref = rectified.solve(I0, I1, m0, 3, 3, 25, params["lambda"], params["alpha0"], params["alpha1"],
                          params["beta"], params["eta"], params["du_max"])
    assert np.max(np.abs(out["u"] - ref)) < 1e-10
    assert np.array_equal(out["w"][..., 1], np.zeros((H, W)))
    assert np.max(np.abs(out["w"][..., 0] - out["u"])) == 0.0
    # and the pinhole triangulation gives Z = f b / disparity where valid
    ok = out["valid"] & (out["u"] > 0.2)
    assert np.max(np.abs(out["Z"][ok] - 40.0 * 0.1 / out["u"][ok]) / out["Z"][ok]) < 1e-9


def _eval_pixels(cam, R, t, gt, erode=3):
    m0 = oracle.mask0(cam).astype(bool)
    H, W = m0.shape
    e = m0.copy()
    for _ in range(erode):
        n = e.copy()
        n[1:, :] &= e[:-1, :]
        n[:-1, :] &= e[1:, :]
        n[:, 1:] &= e[:, :-1]
        n[:, :-1] &= e[:, 1:]
        e = n
    _, epi = oracle.trajectory_field(cam, R, t, 0)
    flow = gt["flow"]
    disp = np.linalg.norm(np.where(np.isfinite(flow), flow, 0.0), axis=-1)
    return e & gt["visible"] & (disp >= 0.5) & (epi == 0) & np.isfinite(gt["range"])


def _c1_solution(d):
    rig, gt = d["rig"], d["gt"][0]
    params = configs.solver_params(d["cfg"])
    out = oracle.solve(rig["cam0"], rig["cam1"], rig["R"], rig["t"], params, d["I0"][0], d["I1"][0])
    ev = _eval_pixels(rig["cam0"], rig["R"], rig["t"], gt)
    return out, gt, ev


def test_c1_plane_correspondences_are_unbiased(c1_inputs):
    """The recovered warp vectors lie on the true epipolar curves and are not
    biased along them: over the evaluation pixels of the C1 plane, the mean
    signed error along the true flow is within +-0.02 px and the median
    distance across it within 0.01 px (a wrong trajectory field, level
    intrinsics or pre-rotation shows up here)."""
    out, gt, ev = _c1_solution(c1_inputs)
    assert ev.sum() > 2000
    err = (out["w"] - gt["flow"])[ev]
    fl = gt["flow"][ev]
    fn = fl / np.linalg.norm(fl, axis=1, keepdims=True)
    along = np.sum(err * fn, 1)
    across = err[:, 0] * fn[:, 1] - err[:, 1] * fn[:, 0]
    assert abs(np.mean(along)) <= 0.02
    assert np.median(np.abs(across)) <= 0.01


@pytest.mark.xfail(strict=True, reason="proposed accuracy bar not met by the method at lambda = 50: "
                   "measured median EPE 0.096 px and median relative range error 10.5 % on the C1 "
                   "plane (unbiased, noise-limited; lambda is not given in the paper)")
def test_c1_plane_depth_matches_ground_truth(c1_inputs):
    """Method check on a known scene with the bars proposed before any GPU
    run: median end-point error <= 0.05 px and median relative range error
    <= 3 %."""
    out, gt, ev = _c1_solution(c1_inputs)
    epe = np.linalg.norm(out["w"] - gt["flow"], axis=-1)[ev]
    rel = (np.abs(out["depth"] - gt["range"]) / gt["range"])[ev & out["valid"]]
    assert np.median(epe) <= 0.05, np.median(epe)
    assert np.median(rel) <= 0.03, np.median(rel)


@pytest.mark.slow
@pytest.mark.xfail(strict=True, reason="proposed bar not met by the method as printed: measured 13.8 % "
                   "tau > 1 px outliers on the C2 room.  The error is an upward disparity bias that "
                   "grows with noise and with the number of warps (the one-sided difference of Eq. (5) "
                   "shares the noise sample of I1(y) between the residual and I_u; a central "
                   "difference removes most of it), plus the 7 px reach of 5 levels x 10 warps x 0.2 px")
def test_c2_room_outliers(c2_inputs):
    """Method check on the box-and-sphere room: KITTI-style tau > 1 px outliers
    <= 10 % of evaluation pixels."""
    d = c2_inputs
    rig, gt = d["rig"], d["gt"][0]
    params = configs.solver_params(d["cfg"])
    out = oracle.solve(rig["cam0"], rig["cam1"], rig["R"], rig["t"], params, d["I0"][0], d["I1"][0])
    ev = _eval_pixels(rig["cam0"], rig["R"], rig["t"], gt)
    assert ev.sum() > 50000
    epe = np.linalg.norm(out["w"] - gt["flow"], axis=-1)[ev]
    frac = np.mean(epe > 1.0)
    assert frac <= 0.10, frac


@pytest.mark.parametrize("reg", ["tgv", "tv"])
def test_identical_or_textureless_pairs_give_zero_displacement(reg, c1_inputs):
    """Degenerate inputs with a closed-form answer.  On the unrotated 128x128
    rig (pre-rotation is the identity), a pair of identical images has zero
    residual at zero displacement, and a textureless pair has no data term at
    all; from the zero start the duals stay zero, so every warp of every
    level keeps u = 0 (Eqs. (8)-(13)), w = 0, and with zero displacement the
    two rays of a translating rig are parallel: no depth anywhere."""
    d = c1_inputs
    rig, cfg = d["rig"], d["cfg"]
    assert np.array_equal(np.asarray(rig["R"]), np.eye(3))
    params = configs.solver_params(cfg, reg=reg)
    I0 = d["I0"][0].astype(np.float64)
    for A, B in ((I0, I0), (np.full_like(I0, 0.4), np.full_like(I0, 0.4))):
        o = oracle.solve(rig["cam0"], rig["cam1"], rig["R"], rig["t"], params, A, B)
        assert not o["u"].any() and not o["w"].any()
        assert not o["valid"].any()


def test_clip_and_accumulate_worked_values():
    """Sec. III-C / Algorithm 1: a warp's increment du = u - u_w is clipped to
    [-0.2, 0.2] px element by element, u becomes u_w + du and w moves by du
    along the warped tangent.  Hand-computed values: an increment above,
    below and inside the clip, and exactly at its edge."""
    u_w = np.array([[1.0, 1.0, 1.0, -2.0]])
    u = np.array([[1.5, 0.7, 1.1, -1.8]])
    gw = np.array([[[0.6, 0.8], [1.0, 0.0], [0.0, -1.0], [-0.8, 0.6]]])
    w = np.array([[[10.0, 20.0], [-3.0, 4.0], [0.5, 0.5], [0.0, 0.0]]])
    u2, w2 = oracle.clip_accumulate(0.2, u_w, gw, u, w)
    np.testing.assert_allclose(u2, [[1.2, 0.8, 1.1, -1.8]], rtol=0, atol=1e-15)
    np.testing.assert_allclose(w2, [[[10.12, 20.16], [-3.2, 4.0], [0.5, 0.4], [-0.16, 0.12]]], rtol=0, atol=1e-14)


def test_linearisation_closed_form_on_linear_images():
    """Eqs. (3), (5) at y = x + w, pinned where every sample is exact:
    bilinear sampling reproduces a linear image and Keys' bicubic kernel
    reproduces a constant field, so with I1 = a x + b y + c, I0 = d x + e y
    + f and the unit tangent (cos p, sin p) everywhere, the one-sided
    difference along the tangent is I_u = a cos p + b sin p, and
    rho_c = I1(x + w) - I0(x) - u I_u, at every pixel whose samples stay
    inside the image; where the data term is off both are 0; u_w = u."""
    H, W = 24, 30
    i, j = np.mgrid[0:H, 0:W].astype(np.float64)
    a, b, c, d, e, f = 0.013, -0.021, 0.4, -0.007, 0.011, 0.3
    I1 = a * j + b * i + c
    I0 = d * j + e * i + f
    p = 0.7
    gam = np.broadcast_to(np.array([np.cos(p), np.sin(p)]), (H, W, 2)).copy()
    wv = np.array([1.3, -0.6])
    w = np.broadcast_to(wv, (H, W, 2)).copy()
    rng = np.random.default_rng(8)
    u = rng.uniform(-2, 2, (H, W))
    dvalid = (rng.random((H, W)) < 0.8).astype(np.uint8)
    uw, gw, Iu, rho = oracle.linearise(I0, I1, gam, dvalid, u, w)
    inner = np.zeros((H, W), bool)
    inner[3:-3, 3:-3] = True
    on = inner & (dvalid == 1)
    Iu_want = a * np.cos(p) + b * np.sin(p)
    rho_want = (a * (j + wv[0]) + b * (i + wv[1]) + c) - I0 - u * Iu_want
    assert np.abs(gw - gam)[inner].max() < 1e-12
    assert np.abs(Iu - Iu_want)[on].max() < 1e-12
    assert np.abs(rho - rho_want)[on].max() < 1e-12
    assert not Iu[dvalid == 0].any() and not rho[dvalid == 0].any()
    assert np.array_equal(uw, u)
