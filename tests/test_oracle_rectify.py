"""Pins of the oracle's rectification to a virtual pinhole view and back (the
comparison with a rectified pipeline, Sec. V-A).

- The rotations: orthonormal, right-handed, the two virtual cameras differ by
  a pure translation (|t|, 0, 0) along virtual x for random rigs, y is
  perpendicular to the mean optical axis, identity for a rig that already is
  rectified; the library's host routine gives the same rotations.
- Against the renderer: rectifying a rendered fisheye pair reproduces the
  renderer's own pinhole images of the same scene seen from both camera
  centres in the virtual orientation (which pins the camera-1 rotation too),
  and a wrong orientation does not.
- The way back: unrectify(rectify(image)) returns a smooth image within the
  bilinear interpolation error, only where the view covers the pixel.
- A camera that already is the pinhole view maps onto itself exactly.
"""
import numpy as np
import pytest

import oracle
from synth import configs, scene


def _random_rig(rng):
    a = rng.normal(size=3)
    R = scene._rotation(a, rng.uniform(0.0, 25.0))
    t = rng.normal(size=3) * 0.1
    t[0] = abs(t[0]) + 0.05
    return R, t


def test_rotations_make_a_pure_x_translation():
    rng = np.random.default_rng(0)
    for _ in range(20):
        R, t = _random_rig(rng)
        Rv0, Rv1, b = oracle.rectify_rotations(R, t)
        for M in (Rv0, Rv1):
            assert np.max(np.abs(M @ M.T - np.eye(3))) < 1e-14
            assert abs(np.linalg.det(M) - 1.0) < 1e-14
        assert abs(b - np.linalg.norm(t)) < 1e-15
        X0 = rng.normal(size=(50, 3)) + [0.0, 0.0, 4.0]
        X1 = X0 @ R.T + t
        d = X1 @ Rv1.T - X0 @ Rv0.T
        assert np.max(np.abs(d - [b, 0.0, 0.0])) < 1e-13
        axis = 0.5 * (np.array([0.0, 0.0, 1.0]) + R.T @ [0.0, 0.0, 1.0])
        assert abs(Rv0[1] @ axis) < 1e-14
        assert Rv0[2] @ axis > 0.0
    Rv0, Rv1, b = oracle.rectify_rotations(np.eye(3), [0.2, 0.0, 0.0])
    assert np.array_equal(Rv0, np.eye(3)) and np.array_equal(Rv1, np.eye(3)) and b == 0.2
    with pytest.raises(ValueError):
        oracle.rectify_rotations(np.eye(3), [0.0, 0.0, 0.0])
    with pytest.raises(ValueError):
        oracle.rectify_rotations(np.eye(3), [0.0, 0.0, 0.3])


def test_library_rotations_match():
    """The library's host routine (no device work) against the oracle."""
    import paper_1909_07545_amd as vfs
    rng = np.random.default_rng(1)
    for _ in range(10):
        R, t = _random_rig(rng)
        a = oracle.rectify_rotations(R, t)
        b = vfs.rectify_rotations(R, t)
        assert np.max(np.abs(a[0] - b[0])) < 1e-15 and np.max(np.abs(a[1] - b[1])) < 1e-15
        assert a[2] == b[2]


def _room_cfg():
    cfg = configs.get("c2")
    cfg.update(width=256, height=192, f=None, supersample=3, noise=0.0, tex_k=(0.3, 2.0))
    return cfg


@pytest.mark.parametrize("fov", [90.0, 150.0])
def test_rectified_fisheye_matches_pinhole_render(fov):
    """A rig rotated by 20 degrees with an oblique baseline, so that the
    virtual orientation is far from both cameras'."""
    cfg = _room_cfg()
    rig = scene.make_rig(cfg)
    rig["R"] = scene._rotation([0.4, 1.0, -0.3], 20.0)
    rig["t"] = np.array([0.06, 0.02, -0.015])
    I0, I1, _ = scene.render_pair(rig, cfg, 0, with_gt=False)
    sc = scene.make_scene(rig, cfg, 0)
    Rv0, Rv1, b = oracle.rectify_rotations(rig["R"], rig["t"])
    pin = scene.pinhole_view(96, fov)
    c1 = -rig["R"].T @ rig["t"]
    for I, Rv, origin in ((I0, Rv0, np.zeros(3)), (I1, Rv1, c1)):
        cam = rig["cam0"]
        got, valid = oracle.rectify(cam, Rv, pin, I)
        ref = scene.render_view(pin, sc, origin, Rv0.T, 3).astype(np.float64)
        v = valid.astype(bool)
        assert v.mean() > 0.9
        rms = np.sqrt(np.mean((got - ref)[v] ** 2))
        # plausible mistakes: the transposed rotation; the other camera's rotation
        for wrong in (Rv.T, Rv1 if Rv is Rv0 else Rv0):
            bad, vb = oracle.rectify(cam, wrong, pin, I)
            both = v & vb.astype(bool)
            rms_bad = np.sqrt(np.mean((bad - ref)[both] ** 2))
            print(fov, rms, rms_bad)
            assert rms < 0.03 and rms_bad > 3 * rms


def test_round_trip_on_a_smooth_image():
    cam = scene.make_camera("kb", 200, 160, None, 180.0, (0.02, -0.01, 0.0, 0.0))
    jj, ii = np.meshgrid(np.arange(200), np.arange(160))
    img = 0.5 + 0.3 * np.sin(0.05 * jj + 0.02 * ii) * np.cos(0.03 * ii)
    R, t = scene._rotation([0.3, -1.0, 0.2], 10.0), np.array([0.1, 0.01, 0.0])
    Rv0, _, _ = oracle.rectify_rotations(R, t)
    for fov, size in ((90.0, 200), (165.0, 400)):
        pin = scene.pinhole_view(size, fov)
        view, vv = oracle.rectify(cam, Rv0, pin, img)
        back, vb = oracle.unrectify(cam, Rv0, pin, view, vv)
        m = vb.astype(bool)
        assert m.sum() > 3000
        assert np.max(np.abs(back - img)[m]) < 2e-3
        # covered pixels are exactly those whose ray lands inside the view in front of it
        r = oracle.unproject(cam, np.stack([jj.ravel(), ii.ravel()], -1).astype(float)).reshape(160, 200, 3)
        V = r @ Rv0.T
        z = np.where(V[..., 2] > 0, V[..., 2], np.nan)
        px = pin["cx"] + pin["fx"] * V[..., 0] / z
        py = pin["cy"] + pin["fy"] * V[..., 1] / z
        inside = (px >= 1) & (px <= size - 2) & (py >= 1) & (py <= size - 2) & oracle.mask0(cam).astype(bool)
        assert not (inside & ~m).any()
        assert not (m & ~oracle.mask0(cam).astype(bool)).any()


def test_a_pinhole_camera_is_its_own_view():
    pin = scene.pinhole_view(64, 100.0)
    img = np.random.default_rng(3).random((64, 64))
    got, valid = oracle.rectify(pin, np.eye(3), pin, img)
    v = valid.astype(bool)
    assert v.all()
    assert np.max(np.abs(got - img)) < 1e-12
    back, vb = oracle.unrectify(pin, np.eye(3), pin, img)
    assert vb.all() and np.max(np.abs(back - img)) < 1e-12
