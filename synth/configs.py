"""Workload definitions: the five evaluation configurations and the solver
parameters of the paper (Sec. IV-C).  Plain data only: nothing here computes
any step of the method.

Configurations (sizes, camera models, levels / warps / iterations):

* ``c1`` plane128  -- 128x128 equidistant f = 40 px, 180 deg, R = I,
  t = (0.1, 0, 0) m, fronto-parallel textured plane at 3 m; 3 levels,
  5 warps, 50 iterations, lambda = 50.
* ``c2`` room640   -- 640x480 Kannala-Brandt f = 220 px, k ~ U[-0.05, 0.05]
  (rejection-sampled to a monotone radial map), 180 deg mask, |t| = 0.06 m
  along x, rotation 2 deg about a seeded axis, box-and-sphere room at
  1-10 m; 5 levels, 10 warps, 100 iterations.
* ``c3`` room1280  -- 1280x1024 Kannala-Brandt 190 deg, f inscribing the image
  circle, rig as c2, room at 0.5-20 m; 6 levels, 10 warps, 150 iterations.
* ``c5`` batch2048 -- 8 pairs of 2048x2048 Kannala-Brandt 200 deg, one rig as
  c3, 8 independent rooms at 0.5-20 m, per-pair beta ~ U[6, 12] and
  eta ~ U[0.7, 1.0]; 7 levels, 15 warps, 200 iterations.
* ``r200``  ragged -- 200x136 Kannala-Brandt 185 deg (not a multiple of the
  GPU tile in either direction), 3 levels, used only by parity tests.

The serving mix (requests of 320x240 / 640x480 / 1024x768) is described by
``SERVING``.
"""
from __future__ import annotations

import copy

# Parameters printed in Sec. IV-C (alpha0, alpha1, beta, eta; 0.2 px clip of
# the incremental disparity).  lambda is not given in the paper: 50 is taken
# for every configuration.  theta_gamma = 0 selects theta = 1.
PAPER_PARAMS = {
    "alpha0": 17.0,
    "alpha1": 1.2,
    "beta": 9.0,
    "eta": 0.85,
    "du_max": 0.2,
    "lambda": 50.0,
    "theta_gamma": 0.0,
    "reg": "tgv",
}

SEED_BASE = 1909_07545


def _cfg(cid, **kw):
    base = dict(id=cid, seed=SEED_BASE + kw.pop("seed_offset"), batch=1, supersample=4,
                noise=0.01, per_pair_tensor=False)
    base.update(kw)
    return base


CONFIGS = {
    "c1": _cfg("c1", seed_offset=1, name="plane128", width=128, height=128, model="equidistant",
               f=40.0, fov_deg=180.0, kb_range=0.0, baseline=0.1, rot_deg=0.0, scene="plane",
               plane_z=3.0, tex_k=(0.3, 3.0), levels=3, warps=5, iters=50),
    "c2": _cfg("c2", seed_offset=2, name="room640", width=640, height=480, model="kb", f=220.0,
               fov_deg=180.0, kb_range=0.05, baseline=0.06, rot_deg=2.0, scene="room",
               depth_range=(1.0, 10.0), tex_k=(0.5, 8.0), levels=5, warps=10, iters=100),
    "c3": _cfg("c3", seed_offset=3, name="room1280", width=1280, height=1024, model="kb", f=None,
               fov_deg=190.0, kb_range=0.05, baseline=0.06, rot_deg=2.0, scene="room",
               depth_range=(0.5, 20.0), tex_k=(0.5, 8.0), levels=6, warps=10, iters=150,
               supersample=2),
    "c5": _cfg("c5", seed_offset=5, name="batch2048", width=2048, height=2048, model="kb", f=None,
               fov_deg=200.0, kb_range=0.05, baseline=0.06, rot_deg=2.0, scene="room",
               depth_range=(0.5, 20.0), tex_k=(0.5, 8.0), levels=7, warps=15, iters=200,
               batch=8, supersample=1, per_pair_tensor=True, beta_range=(6.0, 12.0),
               eta_range=(0.7, 1.0)),
    # unified (xi = 1.2, from the paper's list of models with a closed-form
    # inverse) and enhanced unified (alpha 0.62, beta 1.1) rigs, 200 degrees
    "ucm": _cfg("ucm", seed_offset=12, name="unified320", width=320, height=240, model="unified",
                model_params=(1.2, 0.0, 0.0, 0.0), f=None, fov_deg=200.0, kb_range=0.0, baseline=0.08,
                rot_deg=2.5, scene="room", depth_range=(1.0, 10.0), tex_k=(0.5, 8.0), levels=3, warps=4,
                iters=30, supersample=2),
    "eucm": _cfg("eucm", seed_offset=13, name="eunified320", width=320, height=240, model="eucm",
                 model_params=(0.62, 1.1, 0.0, 0.0), f=None, fov_deg=200.0, kb_range=0.0, baseline=0.08,
                 rot_deg=2.5, scene="room", depth_range=(1.0, 10.0), tex_k=(0.5, 8.0), levels=3, warps=4,
                 iters=30, supersample=2),
    "r200": _cfg("r200", seed_offset=11, name="ragged200", width=200, height=136, model="kb",
                 f=None, fov_deg=185.0, kb_range=0.05, baseline=0.08, rot_deg=3.0, scene="room",
                 depth_range=(1.0, 10.0), tex_k=(0.5, 8.0), levels=3, warps=4, iters=30),
    # comparison with rectified pinhole views (the paper's comparison: 800x800,
    # 180-degree fisheye, the same schedule for both)
    "rect800": _cfg("rect800", seed_offset=14, name="rect800", width=800, height=800, model="equidistant",
                    f=None, fov_deg=180.0, kb_range=0.0, baseline=0.12, rot_deg=2.0, scene="room",
                    depth_range=(1.0, 10.0), tex_k=(0.5, 8.0), levels=5, warps=10, iters=100, supersample=2),
}

# Serving mix: 512 requests, sizes 320x240 / 640x480 / 1024x768 in the ratio
# 3:2:1, 4 seeded Kannala-Brandt rigs (|t| ~ U[0.05, 0.12] m along x, rotation
# up to 3 deg), f = 0.34375 W, 180 deg; levels 4/5/5, 10 warps, 50 iterations.
SERVING = dict(seed=SEED_BASE + 4, requests=512, sizes=((320, 240), (640, 480), (1024, 768)),
               ratio=(3, 2, 1), rigs=4, baseline_range=(0.05, 0.12), rot_max_deg=3.0,
               f_over_w=0.34375, fov_deg=180.0, levels=(4, 5, 5), warps=10, iters=50)


def solver_params(cfg: dict, **override) -> dict:
    """Solver parameters of a configuration (paper values + its L / N / K)."""
    p = copy.deepcopy(PAPER_PARAMS)
    p.update(levels=cfg["levels"], warps=cfg["warps"], iters=cfg["iters"])
    p.update(override)
    return p


def get(cid: str) -> dict:
    return copy.deepcopy(CONFIGS[cid])


def pix_iters(cfg: dict, batch: int | None = None) -> int:
    """Primal-dual pixel-iterations of one solve: sum_l H_l W_l * N * K * pairs."""
    b = cfg["batch"] if batch is None else batch
    tot = sum((cfg["width"] >> l) * (cfg["height"] >> l) for l in range(cfg["levels"]))
    return tot * cfg["warps"] * cfg["iters"] * b
