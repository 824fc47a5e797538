"""Serving workload: seeded rigs at three image sizes, a pool of rendered
pairs per (rig, size), and a Poisson arrival trace.

Rigs: Kannala-Brandt k ~ U[-0.05, 0.05]^4 (monotone draws), baseline
|t| ~ U[0.05, 0.12] m along x, rotation of U[0, 3] degrees about a random
axis; per size f = 0.34375 W, centred principal point, 180 degree field of
view.  Scenes: box-and-sphere rooms at 1-10 m, noise sigma 0.01.  Requests:
exactly 256 / 171 / 85 of 320x240 / 640x480 / 1024x768 (3:2:1), shuffled,
rig uniform over the rigs, exponential inter-arrival times at a given rate.
The solver cost does not depend on the image content, so requests reuse a
small pool of rendered pairs.
"""
from __future__ import annotations

import numpy as np

from . import configs as _configs
from . import scene as _scene


def spec() -> dict:
    return dict(_configs.SERVING)


def serving_rigs(sp: dict | None = None) -> list[list[dict]]:
    """rigs[r][s]: camera pair, pose and level count of rig r at size s."""
    sp = sp or spec()
    rng = np.random.default_rng(np.random.SeedSequence(sp["seed"]).spawn(3)[0])
    out = []
    for _ in range(sp["rigs"]):
        k = _scene.sample_kb(rng, 0.05, sp["fov_deg"])
        base = rng.uniform(*sp["baseline_range"])
        axis = rng.normal(size=3)
        deg = rng.uniform(0.0, sp["rot_max_deg"])
        R = _scene._rotation(axis, deg) if deg > 0 else np.eye(3)
        t = np.array([base, 0.0, 0.0])
        per = []
        for (W, H), L in zip(sp["sizes"], sp["levels"]):
            cam = _scene.make_camera("kb", W, H, sp["f_over_w"] * W, sp["fov_deg"], k)
            per.append(dict(cam0=cam, cam1=dict(cam), R=R, t=t, levels=int(L)))
        out.append(per)
    return out


def scene_cfg(sp: dict, r: int, s: int) -> dict:
    W, H = sp["sizes"][s]
    return dict(id=f"serve_r{r}_s{s}", seed=sp["seed"] + 1000 + 10 * r + s, width=W, height=H,
                scene="room", depth_range=(1.0, 10.0), tex_k=(0.5, 8.0), noise=0.01, supersample=1)


def render_pool(rigs: list[list[dict]], per: int = 1, sp: dict | None = None, sizes=None) -> dict:
    """{(r, s): [(I0, I1), ...]} rendered pairs (float32 numpy)."""
    sp = sp or spec()
    pool = {}
    for r, per_rig in enumerate(rigs):
        for s, rig in enumerate(per_rig):
            if sizes is not None and s not in sizes:
                continue
            cfg = scene_cfg(sp, r, s)
            pool[(r, s)] = [_scene.render_pair(rig, cfg, p, with_gt=False)[:2] for p in range(per)]
    return pool


def make_trace(rate: float, n: int | None = None, sp: dict | None = None, seed_offset: int = 0) -> list[dict]:
    """Requests in arrival order: dict(t=arrival seconds, size=s, rig=r, pair=p)."""
    sp = sp or spec()
    n = n or sp["requests"]
    ratio = np.asarray(sp["ratio"], np.float64)
    counts = np.floor(n * ratio / ratio.sum()).astype(int)
    counts[np.argsort(-(n * ratio / ratio.sum() - counts))[: n - counts.sum()]] += 1
    rng = np.random.default_rng(np.random.SeedSequence(sp["seed"] + seed_offset).spawn(3)[1])
    sizes = np.concatenate([np.full(c, s) for s, c in enumerate(counts)])
    rng.shuffle(sizes)
    rigs = rng.integers(0, sp["rigs"], n)
    gaps = rng.exponential(1.0 / rate, n)
    gaps[0] = 0.0
    t = np.cumsum(gaps)
    return [dict(t=float(t[i]), size=int(sizes[i]), rig=int(rigs[i])) for i in range(n)]
