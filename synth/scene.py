"""Seeded synthetic fisheye stereo inputs with rendered ground truth.

Input generation only: it holds none of the method's arithmetic (no
trajectory field, warping, tensor or primal-dual step).  It carries its own
camera model for ray casting, written independently of both the oracle and
the GPU library, so that the ground truth it renders is an independent check
of either.

Recipe (stands in for the paper's synthetic and real datasets, which are not
available):

* Seeds: ``numpy.random.SeedSequence(config seed)`` spawned into
  {rig, scene, texture, noise}; per pair of a batch, the scene / texture /
  noise streams are spawned again.
* Rig: camera 0 at the origin; camera 1 sees X1 = R X0 + t with
  t = (baseline, 0, 0) and R a rotation by ``rot_deg`` about a seeded axis.
  Kannala-Brandt coefficients k ~ U[-r, r] are rejection-sampled until
  d r_d / d theta >= 0.2 on [0, FOV/2] (10^4-point grid); f inscribes the
  image circle, f = (min(W, H)/2) / r_d(FOV/2), when the configuration does
  not give it.  Both cameras share the intrinsics.
* Scenes: ``plane`` -- fronto-parallel plane Z = z0 with a 2-D texture in
  metric (X, Y); ``room`` -- an axis-aligned room around both cameras with
  ~6 spheres and ~6 boxes at the configured depth range and a 3-D solid
  texture per object.
* Texture: 64 random cosines, |k| ~ U[kmin, kmax] cycles/m, random direction
  and phase, amplitude 1/|k|, mapped to [0, 1] as 0.5 + 0.5 s / sum|a|
  (objects of the room shift the mean by up to +-0.25).
* Rendering: FP64 ray casting with ss x ss stratified samples per pixel;
  pixels outside the camera's FOV are 0; additive Gaussian noise
  (sigma = 0.01 by default, not clamped); stored as float32.
* Ground truth at each camera-0 pixel centre: the hit point X, range |X|,
  Z, the correspondence x1 = pi0(X + R^T t) in the pre-rotated image, and
  visibility from camera 1.
"""
from __future__ import annotations

import numpy as np
import torch

from . import configs as _configs

# ----------------------------------------------------------------- camera model
# Arrays here are torch float64 CPU tensors (multi-threaded elementwise work);
# parameters are plain floats.


def _rd(k, th):
    t2 = th * th
    return th * (1.0 + t2 * (k[0] + t2 * (k[1] + t2 * (k[2] + t2 * k[3]))))


def _drd(k, th):
    t2 = th * th
    return 1.0 + t2 * (3 * k[0] + t2 * (5 * k[1] + t2 * (7 * k[2] + t2 * 9 * k[3])))


def _kcoef(cam):
    return tuple(cam.get("k", (0.0,) * 4)) if cam["model"] == "kb" else (0.0, 0.0, 0.0, 0.0)


UNIFIED = ("unified", "eucm")


def _urd(cam, th):
    """Radial map of the unified (xi) and enhanced unified (alpha, beta)
    models from their projections: m = (x, y) / (xi |X| + z) and
    m = (x, y) / (alpha sqrt(beta (x^2 + y^2) + z^2) + (1 - alpha) z),
    evaluated for the unit ray at angle th (torch or numpy)."""
    lib = torch if isinstance(th, torch.Tensor) else np
    s, c = lib.sin(th), lib.cos(th)
    k = cam["k"]
    if cam["model"] == "unified":
        return s / (k[0] + c)
    return s / (k[0] * lib.sqrt(k[1] * s * s + c * c) + (1.0 - k[0]) * c)


def _uth_max(cam):
    """Largest angle (on a fine grid) up to which the unified radial map is
    defined and increasing."""
    th = np.linspace(0.0, np.pi, 200_001)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = _urd(cam, th)
    ok = np.isfinite(r) & (r >= 0) & np.concatenate([[True], np.diff(r) > 0])
    bad = np.nonzero(~ok)[0]
    return th[bad[0] - 1] if len(bad) else np.pi


def cam_rays(cam, px, py):
    """Unit rays (..., 3) and polar angles of pixel coordinates (Newton on the radial map)."""
    mx = (px - cam["cx"]) / cam["fx"]
    my = (py - cam["cy"]) / cam["fy"]
    rd = torch.sqrt(mx * mx + my * my)
    if cam["model"] == "pinhole":
        n = torch.sqrt(mx * mx + my * my + 1.0)
        return torch.stack([mx / n, my / n, 1.0 / n], -1), torch.atan(rd)
    if cam["model"] in UNIFIED:
        # Newton with a central-difference slope, on [0, the invertible range]
        tmax = _uth_max(cam)
        th = torch.clamp(torch.atan(rd), max=tmax)
        h = 1e-7
        for _ in range(80):
            d = (_urd(cam, th + h) - _urd(cam, th - h)) / (2 * h)
            d = torch.where(d.abs() > 1e-9, d, torch.full_like(d, 1e-9))
            nt = torch.clamp(th - (_urd(cam, th) - rd) / d, 0.0, tmax)
            done = float((nt - th).abs().max()) < 1e-15
            th = nt
            if done:
                break
        s = torch.where(rd > 0, torch.sin(th) / torch.where(rd > 0, rd, torch.ones_like(rd)), torch.ones_like(rd))
        return torch.stack([s * mx, s * my, torch.cos(th)], -1), th
    k = _kcoef(cam)
    th = torch.clamp(rd, max=np.pi)
    if any(k):
        for _ in range(60):
            d = _drd(k, th)
            d = torch.where(d.abs() > 1e-6, d, torch.full_like(d, 1e-6))
            nt = torch.clamp(th - (_rd(k, th) - rd) / d, 0.0, np.pi)
            done = float((nt - th).abs().max()) < 1e-14
            th = nt
            if done:
                break
    s = torch.where(rd > 0, torch.sin(th) / torch.where(rd > 0, rd, torch.ones_like(rd)), torch.ones_like(rd))
    return torch.stack([s * mx, s * my, torch.cos(th)], -1), th


def cam_project(cam, X):
    """Pixel coordinates (..., 2) of points X (..., 3) in the camera frame."""
    rho = torch.sqrt(X[..., 0] ** 2 + X[..., 1] ** 2)
    if cam["model"] == "pinhole":
        return torch.stack([cam["cx"] + cam["fx"] * X[..., 0] / X[..., 2],
                            cam["cy"] + cam["fy"] * X[..., 1] / X[..., 2]], -1)
    th = torch.atan2(rho, X[..., 2])
    rd = _urd(cam, th) if cam["model"] in UNIFIED else _rd(_kcoef(cam), th)
    sr = torch.where(rho > 0, rd / torch.where(rho > 0, rho, torch.ones_like(rho)), torch.zeros_like(rho))
    return torch.stack([cam["cx"] + cam["fx"] * sr * X[..., 0], cam["cy"] + cam["fy"] * sr * X[..., 1]], -1)


def _np_rd(k, th):
    t2 = th * th
    return th * (1.0 + t2 * (k[0] + t2 * (k[1] + t2 * (k[2] + t2 * k[3]))))


def _np_drd(k, th):
    t2 = th * th
    return 1.0 + t2 * (3 * k[0] + t2 * (5 * k[1] + t2 * (7 * k[2] + t2 * 9 * k[3])))


def _rotation(axis, deg):
    a = np.asarray(axis, np.float64)
    a = a / np.linalg.norm(a)
    th = np.deg2rad(deg)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * K @ K


def sample_kb(rng, kr, fov_deg, min_slope=0.2):
    """k ~ U[-kr, kr]^4, redrawn until the radial map is monotone on [0, FOV/2]."""
    th = np.linspace(0.0, np.deg2rad(fov_deg) / 2, 10_000)
    for _ in range(100_000):
        k = rng.uniform(-kr, kr, 4)
        if np.all(_np_drd(k, th) >= min_slope):
            return k
    raise RuntimeError("no monotone Kannala-Brandt draw")


def make_camera(model, W, H, f, fov_deg, k=(0.0, 0.0, 0.0, 0.0)):
    if f is None:
        if model in UNIFIED:
            rd = float(_urd(dict(model=model, k=k), np.deg2rad(fov_deg) / 2))
        else:
            rd = _np_rd(k if model == "kb" else (0.0, 0.0, 0.0, 0.0), np.deg2rad(fov_deg) / 2)
        f = (min(W, H) / 2.0) / rd
    return dict(model=model, width=int(W), height=int(H), fx=float(f), fy=float(f),
                cx=(W - 1) / 2.0, cy=(H - 1) / 2.0, k=tuple(float(x) for x in k),
                fov_deg=float(fov_deg))


def make_rig(cfg, rng=None):
    """Camera pair and relative pose (X1 = R X0 + t) of a configuration."""
    if rng is None:
        rng = np.random.default_rng(np.random.SeedSequence(cfg["seed"]).spawn(4)[0])
    if cfg["model"] == "kb":
        k = sample_kb(rng, cfg["kb_range"], cfg["fov_deg"])
    elif cfg["model"] in UNIFIED:
        k = np.asarray(cfg["model_params"], np.float64)
    else:
        k = np.zeros(4)
    cam = make_camera(cfg["model"], cfg["width"], cfg["height"], cfg.get("f"), cfg["fov_deg"], k)
    axis = rng.normal(size=3)
    R = _rotation(axis, cfg["rot_deg"]) if cfg["rot_deg"] else np.eye(3)
    t = np.array([cfg["baseline"], 0.0, 0.0])
    return dict(cam0=cam, cam1=dict(cam), R=R, t=t)


# ----------------------------------------------------------------- scenes


class Texture:
    def __init__(self, rng, dim, kmin, kmax, n=64):
        kk = rng.uniform(kmin, kmax, n)
        d = rng.normal(size=(n, dim))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        self.k = torch.from_numpy(2 * np.pi * kk[:, None] * d)
        self.a = torch.from_numpy(1.0 / kk)
        self.asum = float(np.sum(1.0 / kk))
        self.ph = torch.from_numpy(rng.uniform(0, 2 * np.pi, n))

    def __call__(self, P):
        Pt = P.reshape(-1, P.shape[-1])
        ph = Pt[:, 0:1] * self.k[:, 0] + self.ph
        for d in range(1, P.shape[-1]):
            ph = ph + Pt[:, d:d + 1] * self.k[:, d]
        return ((torch.cos(ph) * self.a).sum(-1) / self.asum).reshape(P.shape[:-1])


class Plane:
    def __init__(self, rng, cfg):
        self.z = cfg["plane_z"]
        self.tex = Texture(rng, 2, *cfg["tex_k"])

    def cast(self, o, d):
        dz = d[..., 2]
        ok = dz > 1e-12
        tz = torch.where(ok, (self.z - float(o[2])) / torch.where(ok, dz, torch.ones_like(dz)),
                         torch.full_like(dz, float("inf")))
        return tz, torch.where(ok, 0, -1)

    def shade(self, P, obj):
        v = 0.5 + 0.5 * self.tex(P[..., :2])
        return torch.where(obj >= 0, v, torch.full_like(v, 0.5))


class Room:
    def __init__(self, rng, cfg, centres):
        dmin, dmax = cfg["depth_range"]
        lo = -rng.uniform(0.5 * dmax, dmax, 3)
        hi = rng.uniform(0.5 * dmax, dmax, 3)
        lo[1] = -rng.uniform(max(1.2, 0.15 * dmax), max(1.5, 0.3 * dmax))   # floor
        self.lo, self.hi = torch.from_numpy(lo), torch.from_numpy(hi)
        self.spheres, self.boxes = [], []
        tries = 0
        while (len(self.spheres) < 6 or len(self.boxes) < 6) and tries < 10_000:
            tries += 1
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            if d[2] < -0.3:
                continue
            dist = rng.uniform(dmin + 1.0, 0.7 * dmax)
            c = d * dist
            if np.any(c < lo + 0.5) or np.any(c > hi - 0.5):
                continue
            if len(self.spheres) < 6:
                r = rng.uniform(0.3, 1.5)
                if all(np.linalg.norm(c - o) - r > dmin for o in centres):
                    self.spheres.append((torch.from_numpy(c), float(r)))
                    continue
            if len(self.boxes) < 6:
                h = rng.uniform(0.15, 0.75, 3)
                if all(np.max(np.abs(c - o) - h) > dmin for o in centres):
                    self.boxes.append((torch.from_numpy(c - h), torch.from_numpy(c + h)))
        n_obj = 1 + len(self.spheres) + len(self.boxes)
        self.tex = [Texture(rng, 3, *cfg["tex_k"]) for _ in range(n_obj)]
        self.mean = rng.uniform(-0.25, 0.25, n_obj)

    def cast(self, o, d):
        o = torch.as_tensor(o, dtype=torch.float64)
        inv = 1.0 / d
        t1 = (self.lo - o) * inv
        t2 = (self.hi - o) * inv
        best = torch.amin(torch.maximum(t1, t2), dim=-1)      # exit of the room interior
        obj = torch.zeros(best.shape, dtype=torch.int32)
        for i, (c, r) in enumerate(self.spheres):
            oc = o - c
            b = d @ oc
            disc = b * b - (float(oc @ oc) - r * r)
            ok = disc > 0
            th = -b - torch.sqrt(torch.clamp(disc, min=0.0))
            hit = ok & (th > 1e-9) & (th < best)
            best = torch.where(hit, th, best)
            obj = torch.where(hit, 1 + i, obj)
        for i, (blo, bhi) in enumerate(self.boxes):
            a1 = (blo - o) * inv
            a2 = (bhi - o) * inv
            tn = torch.amax(torch.minimum(a1, a2), dim=-1)
            tf = torch.amin(torch.maximum(a1, a2), dim=-1)
            hit = (tn <= tf) & (tn > 1e-9) & (tn < best)
            best = torch.where(hit, tn, best)
            obj = torch.where(hit, 1 + len(self.spheres) + i, obj)
        return best, obj

    def shade(self, P, obj):
        v = torch.zeros(P.shape[:-1], dtype=torch.float64)
        for i in range(len(self.tex)):
            sel = obj == i
            if bool(sel.any()):
                m = float(self.mean[i])
                v[sel] = 0.5 + 0.5 * (m + (1 - abs(m)) * self.tex[i](P[sel]))
        return v


# ----------------------------------------------------------------- rendering


def _grid(W, r0, r1):
    ii, jj = torch.meshgrid(torch.arange(r0, r1, dtype=torch.float64),
                            torch.arange(W, dtype=torch.float64), indexing="ij")
    return jj, ii


def _render(cam, scene, origin, Rcw, ss, rows=128):
    """Image of a camera at ``origin`` whose rays in the world frame are Rcw @ r."""
    H, W = cam["height"], cam["width"]
    img = torch.zeros((H, W), dtype=torch.float64)
    half = np.deg2rad(cam["fov_deg"]) / 2
    offs = (np.arange(ss) + 0.5) / ss - 0.5
    Rt = torch.from_numpy(np.ascontiguousarray(np.asarray(Rcw, np.float64).T))
    o = torch.from_numpy(np.asarray(origin, np.float64))
    for r0 in range(0, H, rows):
        r1 = min(H, r0 + rows)
        jj, ii = _grid(W, r0, r1)
        acc = torch.zeros(ii.shape, dtype=torch.float64)
        for oy in offs:
            for ox in offs:
                rays, _ = cam_rays(cam, jj + float(ox), ii + float(oy))
                d = rays @ Rt
                tt, obj = scene.cast(o, d)
                fin = torch.isfinite(tt)
                P = torch.where(fin[..., None], o + torch.where(fin, tt, 0.0)[..., None] * d, 0.0)
                v = scene.shade(P, obj)
                acc += torch.where(fin, v, torch.full_like(v, 0.5))
        _, thc = cam_rays(cam, jj, ii)
        img[r0:r1] = torch.where(thc <= half, acc / (ss * ss), torch.zeros_like(acc))
    return img.numpy()


def make_scene(rig, cfg, pair=0):
    """The scene of pair ``pair`` of a configuration (in camera 0's frame)."""
    ss_scene = np.random.SeedSequence(cfg["seed"]).spawn(4)[1]
    s_rng = np.random.default_rng(ss_scene.spawn(pair + 1)[pair])
    R, t = np.asarray(rig["R"]), np.asarray(rig["t"])
    if cfg["scene"] == "plane":
        return Plane(s_rng, cfg)
    return Room(s_rng, cfg, [np.zeros(3), -R.T @ t])


def pinhole_view(size, fov_deg):
    """Square pinhole camera whose horizontal field of view is ``fov_deg``;
    its circular mask (``fov_deg`` of the dict) reaches the image corners."""
    half = np.deg2rad(fov_deg) / 2
    f = (size / 2.0) / np.tan(half)
    diag = 2.0 * np.rad2deg(np.arctan(np.sqrt(2.0) * np.tan(half) * (1.0 + 1.0 / size)))
    return make_camera("pinhole", size, size, f, min(diag, 179.9))


def render_view(cam, scene, origin, Rcw, ss):
    """Image of any camera at ``origin`` whose rays in camera 0's frame are Rcw @ r."""
    return _render(cam, scene, origin, Rcw, ss).astype(np.float32)


def render_pair(rig, cfg, pair=0, with_gt=True):
    """(I0, I1, gt) for pair ``pair`` of a configuration's batch."""
    ss_noise = np.random.SeedSequence(cfg["seed"]).spawn(4)[3]
    n_rng = np.random.default_rng(ss_noise.spawn(pair + 1)[pair])
    R, t = np.asarray(rig["R"]), np.asarray(rig["t"])
    c1_centre = -R.T @ t
    scene = make_scene(rig, cfg, pair)
    ss = int(cfg.get("supersample", 1))
    I0 = _render(rig["cam0"], scene, np.zeros(3), np.eye(3), ss)
    I1 = _render(rig["cam1"], scene, c1_centre, R.T, ss)
    sig = cfg.get("noise", 0.0)
    if sig:
        I0 = I0 + n_rng.normal(0, sig, I0.shape)
        I1 = I1 + n_rng.normal(0, sig, I1.shape)
    gt = ground_truth(rig, scene) if with_gt else None
    return I0.astype(np.float32), I1.astype(np.float32), gt


def ground_truth(rig, scene):
    cam0, cam1 = rig["cam0"], rig["cam1"]
    R, t = np.asarray(rig["R"], np.float64), np.asarray(rig["t"], np.float64)
    H, W = cam0["height"], cam0["width"]
    jj, ii = _grid(W, 0, H)
    rays, th = cam_rays(cam0, jj, ii)
    tt, obj = scene.cast(np.zeros(3), rays)
    fin = torch.isfinite(tt)
    X = torch.where(fin, tt, 0.0)[..., None] * rays
    tp = torch.from_numpy(R.T @ t)
    x1 = cam_project(cam0, X + tp)
    c1 = torch.from_numpy(-R.T @ t)
    d = X - c1
    dist = torch.linalg.norm(d, dim=-1)
    dn = d / torch.where(dist > 0, dist, torch.ones_like(dist))[..., None]
    tt1, _ = scene.cast(c1, dn)
    X1 = X @ torch.from_numpy(np.ascontiguousarray(R.T)) + torch.from_numpy(t)
    th1 = torch.atan2(torch.linalg.norm(X1[..., :2], dim=-1), X1[..., 2])
    vis = fin & (tt1 > dist - 1e-6 * torch.clamp(dist, min=1.0)) & (th1 <= np.deg2rad(cam1["fov_deg"]) / 2)
    inside = th <= np.deg2rad(cam0["fov_deg"]) / 2
    rng_ = torch.where(fin, tt, torch.full_like(tt, float("inf")))
    flow = x1 - torch.stack([jj, ii], -1)
    return dict(X=X.numpy(), range=rng_.numpy(), Z=X[..., 2].numpy(), x1=x1.numpy(), flow=flow.numpy(),
                visible=(vis & inside).numpy(), inside=inside.numpy())


def pair_tensor_params(cfg, pair):
    """Per-pair (beta, eta) of configurations with image-driven tensor draws."""
    if not cfg.get("per_pair_tensor"):
        p = _configs.PAPER_PARAMS
        return p["beta"], p["eta"]
    ss = np.random.SeedSequence(cfg["seed"]).spawn(5)[4]
    rng = np.random.default_rng(ss.spawn(pair + 1)[pair])
    return float(rng.uniform(*cfg["beta_range"])), float(rng.uniform(*cfg["eta_range"]))


def make_inputs(cid, pairs=None):
    """Rig and rendered pairs of a configuration: dict(cfg, rig, I0[], I1[], gt[])."""
    cfg = _configs.get(cid)
    rig = make_rig(cfg)
    n = cfg["batch"] if pairs is None else pairs
    out = dict(cfg=cfg, rig=rig, I0=[], I1=[], gt=[], tensor=[])
    for b in range(n):
        I0, I1, gt = render_pair(rig, cfg, b)
        out["I0"].append(I0)
        out["I1"].append(I1)
        out["gt"].append(gt)
        out["tensor"].append(pair_tensor_params(cfg, b))
    return out
