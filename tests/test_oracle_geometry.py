"""Pins of the oracle's geometry: camera models, trajectory field (Sec. III-B),
calibration field and pre-rotation (Sec. IV-A), triangulation (Sec. III-D).

Each check is against a closed form, a brute-force construction or the
renderer's independent camera model and ground truth.
"""
import numpy as np
import pytest
import torch

import oracle
from synth import configs, scene

KB = dict(model="kb", width=320, height=240, fx=80.0, fy=80.0, cx=159.5, cy=119.5,
          k=(0.02, -0.01, 0.002, -0.0003), fov_deg=190.0)
EQ = dict(KB, model="equidistant", k=(0.0, 0.0, 0.0, 0.0))
PH = dict(model="pinhole", width=96, height=72, fx=50.0, fy=50.0, cx=47.5, cy=35.5,
          k=(0.0, 0.0, 0.0, 0.0), fov_deg=120.0)


def _rot(axis, deg):
    return scene._rotation(axis, deg)


def _angle(a, b):
    a = a / np.linalg.norm(a, axis=-1, keepdims=True)
    b = b / np.linalg.norm(b, axis=-1, keepdims=True)
    cross = a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]
    dot = np.sum(a * b, -1)
    return np.abs(np.arctan2(cross, dot))


def _pixels(cam, n, rng, margin=2.0):
    x = rng.uniform(margin, cam["width"] - 1 - margin, n)
    y = rng.uniform(margin, cam["height"] - 1 - margin, n)
    return np.stack([x, y], -1)


# ----------------------------------------------------------------- camera model

@pytest.mark.parametrize("cam", [KB, EQ, PH], ids=["kb", "equidistant", "pinhole"])
def test_projection_round_trip(cam):
    rng = np.random.default_rng(0)
    x = _pixels(cam, 4000, rng)
    r = oracle.unproject(cam, x)
    assert np.allclose(np.linalg.norm(r, axis=1), 1.0, atol=1e-14)
    # only points inside the field of view where the model is invertible
    th = np.arctan2(np.linalg.norm(r[:, :2], axis=1), r[:, 2])
    keep = th < np.deg2rad(cam["fov_deg"]) / 2
    xb, ok = oracle.project(cam, r[keep] * rng.uniform(0.1, 50.0, (keep.sum(), 1)))
    assert ok.all()
    assert np.max(np.abs(xb - x[keep])) < 1e-9


def test_equidistant_closed_form():
    rng = np.random.default_rng(1)
    x = _pixels(EQ, 2000, rng)
    r = oracle.unproject(EQ, x)
    rd = np.hypot(x[:, 0] - EQ["cx"], x[:, 1] - EQ["cy"]) / EQ["fx"]
    th = np.arctan2(np.linalg.norm(r[:, :2], axis=1), r[:, 2])
    assert np.max(np.abs(th - rd)) < 1e-12
    # Kannala-Brandt with k = 0 is the equidistant model
    kb0 = dict(KB, k=(0.0, 0.0, 0.0, 0.0))
    assert np.max(np.abs(oracle.unproject(kb0, x) - r)) < 1e-12


def test_kb_against_renderer_camera():
    """The renderer's independent camera model gives the same rays."""
    rng = np.random.default_rng(2)
    x = _pixels(KB, 2000, rng)
    r = oracle.unproject(KB, x)
    rr, th = scene.cam_rays(KB, torch.from_numpy(x[:, 0]), torch.from_numpy(x[:, 1]))
    # compare where the radial map is invertible: r_d <= r_d(FOV/2)
    t95 = np.deg2rad(95.0)
    rmax = t95 + 0.02 * t95 ** 3 - 0.01 * t95 ** 5 + 0.002 * t95 ** 7 - 0.0003 * t95 ** 9
    inside = np.hypot(x[:, 0] - KB["cx"], x[:, 1] - KB["cy"]) / KB["fx"] <= rmax
    assert inside.sum() > 1000
    assert np.max(np.abs(rr.numpy()[inside] - r[inside])) < 1e-11


def test_pinhole_closed_form():
    x = np.array([[10.0, 20.0], [47.5, 35.5], [90.0, 3.0]])
    r = oracle.unproject(PH, x)
    m = np.stack([(x[:, 0] - PH["cx"]) / PH["fx"], (x[:, 1] - PH["cy"]) / PH["fy"], np.ones(3)], -1)
    m /= np.linalg.norm(m, axis=1, keepdims=True)
    assert np.max(np.abs(r - m)) < 1e-15


def test_non_monotone_kb_rejected():
    bad = dict(KB, k=(0.0, 0.0, 0.0, -0.05), fov_deg=200.0)   # r_d' < 0 before 100 deg
    assert oracle.camera_check(bad) == -4
    assert oracle.camera_check(KB) == 0
    assert oracle.camera_check(dict(PH, fov_deg=180.0)) == -4


# ----------------------------------------------------------------- masks

def test_level_mask_nearest_neighbour():
    m0 = oracle.mask0(KB)
    rd = np.hypot((np.arange(320)[None, :] - 159.5) / 80.0, (np.arange(240)[:, None] - 119.5) / 80.0)
    th = np.deg2rad(95.0)
    rmax = th + 0.02 * th ** 3 - 0.01 * th ** 5 + 0.002 * th ** 7 - 0.0003 * th ** 9
    assert np.array_equal(m0.astype(bool), rd <= rmax)
    for l in (1, 2, 3):
        ml = oracle.level_mask(m0, l)
        o = 1 << (l - 1)
        assert np.array_equal(ml, m0[o::1 << l, o::1 << l])


# ----------------------------------------------------------------- trajectory field

def _brute_force_tangent(cam, R, t, x, depths):
    """Epipolar curve of pixel x traced by projecting points d r0(x) + t' at
    many depths d along its back-projected ray into the pre-rotated second
    camera (renderer's camera model).  The tangent at each point is a small
    symmetric chord in inverse depth, oriented toward increasing disparity.
    Also returns the polar angle of each projected point (the curve is only
    traced where the model is invertible)."""
    rays, _ = scene.cam_rays(cam, torch.tensor([x[0]]), torch.tensor([x[1]]))
    r0 = rays.numpy()[0]
    tp = np.asarray(R).T @ np.asarray(t)
    inv = 1.0 / np.asarray(depths)
    h = 1e-5

    def P(s):
        X = r0[None, :] / s[:, None] + tp[None, :]
        return scene.cam_project(cam, torch.from_numpy(X)).numpy(), X

    pts, X = P(inv)
    tans = P(inv + h)[0] - P(inv - h)[0]
    th = np.arctan2(np.linalg.norm(X[:, :2], axis=1), X[:, 2])
    return pts, tans, th


@pytest.mark.parametrize("which", ["kb190", "c2"])
def test_trajectory_tangent_to_brute_force_epipolar_curve(which):
    if which == "c2":
        rig = scene.make_rig(configs.get("c2"))
        cam, R, t = rig["cam0"], rig["R"], rig["t"]
    else:
        cam, R, t = KB, _rot([0.3, -0.5, 0.8], 4.0), np.array([0.1, 0.02, -0.03])
    rng = np.random.default_rng(3)
    depths = np.logspace(-1, 4, 400)
    tp = R.T @ t
    tpn = tp / np.linalg.norm(tp)
    gam_field, _ = oracle.trajectory_field(cam, R, t, 0)
    m0 = oracle.mask0(cam)
    worst_exact, worst_interp, n = 0.0, 0.0, 0
    for x in _pixels(cam, 40, rng, margin=4.0):
        pts, tans, thp = _brute_force_tangent(cam, R, t, x, depths)
        inside = (pts[:, 0] > 3) & (pts[:, 0] < cam["width"] - 4) & (pts[:, 1] > 3) & (pts[:, 1] < cam["height"] - 4)
        inside &= thp < np.deg2rad(cam["fov_deg"]) / 2
        rays = oracle.unproject(cam, pts)
        away = np.abs(rays @ tpn) < np.cos(np.deg2rad(3.0))
        ij = np.clip(np.rint(pts[:, ::-1]).astype(int), 0, [cam["height"] - 1, cam["width"] - 1])
        inmask = m0[ij[:, 0], ij[:, 1]].astype(bool)
        big = np.linalg.norm(tans, axis=1) > 1e-9
        keep = inside & away & inmask & big
        if not keep.any():
            continue
        g, epi = oracle.trajectory_at(cam, R, t, pts[keep])
        assert not epi.any()
        worst_exact = max(worst_exact, _angle(g, tans[keep]).max())
        gi = oracle.sample_trajectory(gam_field, pts[keep])
        worst_interp = max(worst_interp, _angle(gi, tans[keep]).max())
        n += keep.sum()
    assert n > 1000
    assert worst_exact < 1e-5
    assert worst_interp < 2e-3


def test_pinhole_x_translation_is_exactly_horizontal():
    g, epi = oracle.trajectory_field(PH, np.eye(3), [0.12, 0.0, 0.0], 0)
    assert not epi.any()
    assert np.array_equal(g[..., 0], np.ones(g.shape[:2]))
    assert np.array_equal(g[..., 1], np.zeros(g.shape[:2]))


def test_pinhole_lateral_translation_is_constant():
    t = np.array([0.05, -0.03, 0.0])
    g, _ = oracle.trajectory_field(PH, np.eye(3), t, 0)
    assert np.max(_angle(g.reshape(-1, 2), np.broadcast_to(t[:2], (g.size // 2, 2)))) < 1e-6


@pytest.mark.parametrize("cam", [PH, EQ], ids=["pinhole", "equidistant"])
def test_forward_translation_is_radial(cam):
    g, epi = oracle.trajectory_field(cam, np.eye(3), [0.0, 0.0, 0.2], 0)
    jj, ii = np.meshgrid(np.arange(cam["width"]), np.arange(cam["height"]))
    rad = np.stack([jj - cam["cx"], ii - cam["cy"]], -1)
    keep = (~epi.astype(bool)) & (np.linalg.norm(rad, axis=-1) > 1.0)
    if cam["model"] == "equidistant":
        keep &= oracle.mask0(cam).astype(bool)
    # camera 1's centre is at -t, behind camera 0: image points move toward the centre
    dots = np.sum(g * rad, -1)
    assert np.all(dots[keep] < 0)
    assert np.max(_angle(g[keep], -rad[keep])) < 1e-6


def test_independent_of_baseline_length():
    R = _rot([1.0, 2.0, 0.5], 3.0)
    t = np.array([0.07, 0.01, 0.02])
    g1, e1 = oracle.trajectory_field(KB, R, t, 1)
    g2, e2 = oracle.trajectory_field(KB, R, 10 * t, 1)
    assert np.array_equal(e1, e2)
    assert np.max(np.abs(g1 - g2)) < 1e-9


def test_analytic_jacobian_direction():
    """gamma'(x) is the direction of D pi(r0(x)) t' (Eq. (7), the |t| -> 0 limit)."""
    R = _rot([0.1, 1.0, 0.2], 2.0)
    t = np.array([0.06, 0.0, 0.0])
    tp = R.T @ t
    rng = np.random.default_rng(4)
    x = _pixels(KB, 500, rng, margin=5)
    r = oracle.unproject(KB, x)
    k = KB["k"]
    X, Y, Z = r[:, 0], r[:, 1], r[:, 2]
    rho = np.hypot(X, Y)
    th = np.arctan2(rho, Z)
    rd = th + k[0] * th ** 3 + k[1] * th ** 5 + k[2] * th ** 7 + k[3] * th ** 9
    drd = 1 + 3 * k[0] * th ** 2 + 5 * k[1] * th ** 4 + 7 * k[2] * th ** 6 + 9 * k[3] * th ** 8
    # d theta / dX = (Z X / rho, Z Y / rho, -rho) / |X|^2 ; d(X/rho)/dX etc.
    n2 = X * X + Y * Y + Z * Z
    dth = np.stack([Z * X / rho, Z * Y / rho, -rho], -1) / n2[:, None]
    cx, sy = X / rho, Y / rho
    dcx = np.stack([Y * Y, -X * Y, np.zeros_like(X)], -1) / rho[:, None] ** 3
    dsy = np.stack([-X * Y, X * X, np.zeros_like(X)], -1) / rho[:, None] ** 3
    Jx = KB["fx"] * (drd[:, None] * dth * cx[:, None] + rd[:, None] * dcx)
    Jy = KB["fy"] * (drd[:, None] * dth * sy[:, None] + rd[:, None] * dsy)
    ana = np.stack([Jx @ tp, Jy @ tp], -1)
    g, epi = oracle.trajectory_at(KB, R, t, x)
    keep = ~epi
    assert np.max(_angle(g[keep], ana[keep])) < 1e-5


# ----------------------------------------------------------------- calibration / pre-rotation

def test_calibration_field_zero_for_identity():
    cf, valid = oracle.calibration_field(KB, KB, np.eye(3))
    assert np.array_equal(cf, np.zeros_like(cf))
    m0 = oracle.mask0(KB)
    assert np.array_equal(valid[m0.astype(bool)], np.ones(m0.sum(), np.uint8))


def test_prerotation_undoes_a_pure_rotation():
    """Render the same room from a camera rotated by R (t = 0); pre-rotating
    that image with the calibration field reproduces the unrotated render."""
    cfg = configs.get("c2")
    cfg.update(width=160, height=120, f=55.0, supersample=2, noise=0.0)
    cam = scene.make_camera("kb", 160, 120, 55.0, 180.0, (0.02, -0.01, 0.004, -0.001))
    R = _rot([0.4, 1.0, -0.3], 5.0)
    rng = np.random.default_rng(5)
    room = scene.Room(rng, cfg, [np.zeros(3)])
    I0 = scene._render(cam, room, np.zeros(3), np.eye(3), 2)
    I1 = scene._render(cam, room, np.zeros(3), R.T, 2)
    cf, valid = oracle.calibration_field(cam, cam, R)
    I1p = oracle.prerotate(I1, cf)
    m = oracle.mask0(cam).astype(bool) & valid.astype(bool)
    # stay away from the rim of the field of view (black outside)
    jj, ii = np.meshgrid(np.arange(160), np.arange(120))
    core = np.hypot(jj - 79.5, ii - 59.5) < 50
    d = (I1p - I0)[m & core]
    assert np.sqrt(np.mean(d ** 2)) < 0.01


# ----------------------------------------------------------------- triangulation

def test_triangulation_recovers_rendered_range(c2_inputs):
    rig, gt = c2_inputs["rig"], c2_inputs["gt"][0]
    cam = rig["cam0"]
    dvalid = np.ones((cam["height"], cam["width"]), np.uint8)
    flow = np.where(np.isfinite(gt["flow"]), gt["flow"], 0.0)
    depth, Z, valid = oracle.triangulate(cam, rig["R"], rig["t"], flow, dvalid)
    _, epi = oracle.trajectory_field(cam, rig["R"], rig["t"], 0)
    keep = gt["inside"] & np.isfinite(gt["range"]) & (np.linalg.norm(flow, axis=-1) > 0.05) & (epi == 0)
    assert keep.sum() > 100000
    assert valid[keep].all()
    rel = np.abs(depth[keep] - gt["range"][keep]) / gt["range"][keep]
    assert np.max(rel) < 1e-9
    assert np.max(np.abs(Z[keep] - gt["Z"][keep]) / gt["range"][keep]) < 1e-9


def test_triangulation_pinhole_rectified_depth():
    b = 0.1
    disp = np.random.default_rng(6).uniform(0.5, 8.0, (PH["height"], PH["width"]))
    w = np.stack([disp, np.zeros_like(disp)], -1)
    depth, Z, valid = oracle.triangulate(PH, np.eye(3), [b, 0.0, 0.0], w, np.ones(disp.shape, np.uint8))
    assert valid.all()
    assert np.max(np.abs(Z - PH["fx"] * b / disp) / Z) < 1e-9


@pytest.mark.parametrize("t", [(0.2, 0.0, 0.0), (0.0, 0.0, -0.15), (0.1, -0.1, 0.05)])
def test_epipole_guard_is_the_2_degree_cone_around_the_baseline(t):
    """The trajectory field is undefined at the epipoles (Sec. III-B): the
    pixels flagged are exactly those whose ray, by the equidistant closed
    form theta = r / f, lies within 2 degrees of +t or -t (R = I), and those
    pixels carry a zero tangent; all others carry a unit one.  Pixels within
    1e-9 of the cone's boundary are not judged."""
    g, epi = oracle.trajectory_field(EQ, np.eye(3), list(t), 0)
    H, W = EQ["height"], EQ["width"]
    i, j = np.mgrid[0:H, 0:W].astype(np.float64)
    dx, dy = j - EQ["cx"], i - EQ["cy"]
    th = np.hypot(dx, dy) / EQ["fx"]
    ph = np.arctan2(dy, dx)
    ray = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], -1)
    tu = np.asarray(t, np.float64) / np.linalg.norm(t)
    ct = np.abs(ray @ tu)
    lim = np.cos(np.deg2rad(2.0))
    judged = (np.abs(ct - lim) > 1e-9) & (th < np.deg2rad(EQ["fov_deg"]) / 2)
    want = ct > lim
    assert want[judged].any(), "the cone must reach the image for this check"
    assert np.array_equal(epi.astype(bool)[judged], want[judged])
    n = np.linalg.norm(g, axis=-1)
    assert np.all(n[epi.astype(bool)] == 0.0)
    assert np.allclose(n[judged & ~want], 1.0, atol=1e-12)


@pytest.mark.parametrize("cam", [KB, EQ, PH], ids=["kb", "equidistant", "pinhole"])
def test_image_circle_mask_closed_form(cam):
    """The level-0 mask (Sec. IV-B) is the set of pixels whose normalised
    radius is at most the radial map at half the field of view: theta for the
    equidistant model, tan(theta) for the pinhole, the Kannala-Brandt
    polynomial theta (1 + k1 theta^2 + ... + k4 theta^8); pixels within 1e-9
    of the boundary are not judged."""
    m = oracle.mask0(cam).astype(bool)
    H, W = cam["height"], cam["width"]
    i, j = np.mgrid[0:H, 0:W].astype(np.float64)
    rn = np.hypot((j - cam["cx"]) / cam["fx"], (i - cam["cy"]) / cam["fy"])
    th = np.deg2rad(cam["fov_deg"]) / 2
    if cam["model"] == "pinhole":
        rmax = np.tan(th)
    else:
        k1, k2, k3, k4 = cam["k"]
        rmax = th * (1 + k1 * th ** 2 + k2 * th ** 4 + k3 * th ** 6 + k4 * th ** 8)
    judged = np.abs(rn - rmax) > 1e-9
    assert np.array_equal(m[judged], (rn <= rmax)[judged])
    assert m.any()
    if cam["model"] != "pinhole":
        assert not m[0, 0] and not m[-1, -1]     # the image circle leaves the corners out
