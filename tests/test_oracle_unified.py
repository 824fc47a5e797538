"""Pins of the oracle's unified (UCM) and enhanced unified (EUCM) camera
models (Sec. III-B: any model with a defined projection; Sec. III-D: these
two have a closed-form unprojection).

Each check is against something other than the oracle's own formulas: the
textbook models they reduce to (xi = 0 or alpha = 0: pinhole; EUCM with
beta = 1: UCM with xi = alpha / (1 - alpha) and focal length f / (1 - alpha)),
the round trip between the radial projection and the closed-form inverse
(two different formulas), the renderer's camera (Newton on the radial map
with a finite-difference slope), the angle limits where the maps stop being
invertible, and the brute-force epipolar curve.
"""
import numpy as np
import pytest
import torch

import oracle
from synth import configs, scene
from tests.test_oracle_geometry import _angle, _brute_force_tangent, _pixels

BASE = dict(width=320, height=240, fx=90.0, fy=90.0, cx=159.5, cy=119.5, fov_deg=180.0)
UCMS = [dict(BASE, model="unified", k=(xi, 0.0, 0.0, 0.0)) for xi in (0.4, 1.0, 1.6)]
EUCMS = [dict(BASE, model="eucm", k=(a, b, 0.0, 0.0)) for a, b in ((0.55, 0.9), (0.62, 1.1), (0.7, 1.5))]
PH = dict(BASE, model="pinhole", k=(0.0, 0.0, 0.0, 0.0), fov_deg=120.0)


def _points(n, rng, max_deg):
    th = np.deg2rad(rng.uniform(0.0, max_deg, n))
    ph = rng.uniform(-np.pi, np.pi, n)
    d = rng.uniform(0.2, 30.0, n)
    return d[:, None] * np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], -1)


def test_zero_parameters_are_the_pinhole():
    rng = np.random.default_rng(0)
    X = _points(3000, rng, 55.0)
    x_ph, _ = oracle.project(PH, X)
    for cam in (dict(PH, model="unified"), dict(PH, model="eucm", k=(0.0, 1.3, 0.0, 0.0))):
        x, ok = oracle.project(cam, X)
        assert ok.all()
        assert np.max(np.abs(x - x_ph)) < 1e-10
        px = _pixels(PH, 2000, rng)
        assert np.max(np.abs(oracle.unproject(cam, px) - oracle.unproject(PH, px))) < 1e-13


@pytest.mark.parametrize("alpha", [0.3, 0.5, 0.62])
def test_eucm_with_unit_beta_is_the_unified_model(alpha):
    rng = np.random.default_rng(1)
    eu = dict(BASE, model="eucm", k=(alpha, 1.0, 0.0, 0.0), fov_deg=170.0)
    uc = dict(eu, model="unified", k=(alpha / (1 - alpha), 0.0, 0.0, 0.0), fx=BASE["fx"] / (1 - alpha),
              fy=BASE["fy"] / (1 - alpha))
    X = _points(3000, rng, 85.0)
    a, _ = oracle.project(eu, X)
    b, _ = oracle.project(uc, X)
    assert np.max(np.abs(a - b)) < 1e-9
    px = _pixels(eu, 2000, rng)
    ra, rb = oracle.unproject(eu, px), oracle.unproject(uc, px)
    assert np.max(np.abs(ra - rb)) < 1e-12


@pytest.mark.parametrize("cam", UCMS + EUCMS, ids=[f"ucm{c['k'][0]}" for c in UCMS] +
                         [f"eucm{c['k'][0]}-{c['k'][1]}" for c in EUCMS])
def test_closed_form_inverse_round_trip(cam):
    """project(unproject(x)) = x and unproject(project(X)) = X / |X| inside
    the invertible range: the radial projection and the closed-form inverse
    are independent formulas."""
    rng = np.random.default_rng(2)
    tmax = np.rad2deg(scene._uth_max(cam))
    X = _points(4000, rng, min(0.95 * tmax, 120.0))
    x, ok = oracle.project(cam, X)
    assert ok.all()
    r = oracle.unproject(cam, x)
    assert np.max(np.abs(r - X / np.linalg.norm(X, axis=1, keepdims=True))) < 1e-12
    xb, _ = oracle.project(cam, r * 3.0)
    assert np.max(np.abs(xb - x)) < 1e-9


@pytest.mark.parametrize("cam", UCMS + EUCMS, ids=[f"ucm{c['k'][0]}" for c in UCMS] +
                         [f"eucm{c['k'][0]}-{c['k'][1]}" for c in EUCMS])
def test_against_renderer_camera(cam):
    rng = np.random.default_rng(3)
    x = _pixels(cam, 3000, rng)
    r = oracle.unproject(cam, x)
    rr, th = scene.cam_rays(cam, torch.from_numpy(x[:, 0]), torch.from_numpy(x[:, 1]))
    rmax = float(scene._urd(cam, np.float64(min(0.98 * scene._uth_max(cam), np.deg2rad(150.0)))))
    inside = np.hypot(x[:, 0] - cam["cx"], x[:, 1] - cam["cy"]) / cam["fx"] <= rmax
    assert inside.sum() > 400
    assert np.max(np.abs(rr.numpy()[inside] - r[inside])) < 1e-9


def test_angle_limits():
    """The unified map is invertible up to acos(-1/xi) for xi > 1 (largest
    radius) and up to acos(-xi) for xi < 1 (the radius diverges); the model
    check rejects fields of view beyond."""
    step = np.pi / 4096
    for xi in (1.6, 2.5):
        lim = np.arccos(-1.0 / xi)
        cam = dict(BASE, model="unified", k=(xi, 0.0, 0.0, 0.0), fov_deg=2 * np.rad2deg(lim) - 1.0)
        rays = oracle.unproject(cam, np.array([[cam["cx"] + 1e6, cam["cy"]]]))
        th = np.arctan2(np.hypot(rays[0, 0], rays[0, 1]), rays[0, 2])
        assert lim - step <= th <= lim + 1e-12
        assert oracle.camera_check(cam) == 0
        assert oracle.camera_check(dict(cam, fov_deg=2 * np.rad2deg(lim) + 1.0)) == -4
    xi = 0.4
    lim = np.arccos(-xi)
    cam = dict(BASE, model="unified", k=(xi, 0.0, 0.0, 0.0))
    rays = oracle.unproject(cam, np.array([[cam["cx"] + 1e9, cam["cy"]]]))
    th = np.arctan2(np.hypot(rays[0, 0], rays[0, 1]), rays[0, 2])
    assert lim - 2 * step <= th <= lim + 1e-12
    assert oracle.camera_check(dict(cam, k=(-0.1, 0.0, 0.0, 0.0))) == -1
    assert oracle.camera_check(dict(cam, model="eucm", k=(1.2, 1.0, 0.0, 0.0))) == -1


@pytest.mark.parametrize("which", ["ucm", "eucm"])
def test_trajectory_tangent_to_brute_force_epipolar_curve(which):
    rig = scene.make_rig(configs.get(which))
    cam, R, t = rig["cam0"], rig["R"], rig["t"]
    rng = np.random.default_rng(4)
    depths = np.logspace(-1, 4, 400)
    tpn = (R.T @ t) / np.linalg.norm(R.T @ t)
    m0 = oracle.mask0(cam)
    worst, n = 0.0, 0
    for x in _pixels(cam, 40, rng, margin=4.0):
        pts, tans, thp = _brute_force_tangent(cam, R, t, x, depths)
        inside = (pts[:, 0] > 3) & (pts[:, 0] < cam["width"] - 4) & (pts[:, 1] > 3) & (pts[:, 1] < cam["height"] - 4)
        inside &= thp < np.deg2rad(cam["fov_deg"]) / 2
        rays = oracle.unproject(cam, pts)
        away = np.abs(rays @ tpn) < np.cos(np.deg2rad(3.0))
        ij = np.clip(np.rint(pts[:, ::-1]).astype(int), 0, [cam["height"] - 1, cam["width"] - 1])
        keep = inside & away & m0[ij[:, 0], ij[:, 1]].astype(bool) & (np.linalg.norm(tans, axis=1) > 1e-9)
        if not keep.any():
            continue
        g, epi = oracle.trajectory_at(cam, R, t, pts[keep])
        assert not epi.any()
        worst = max(worst, _angle(g, tans[keep]).max())
        n += keep.sum()
    assert n > 1000
    assert worst < 1e-5
