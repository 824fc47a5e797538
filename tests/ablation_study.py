"""Ablation of the warping schedule on rendered scenes with ground truth (a
script, not collected by pytest; it needs a GPU).

  python -m tests.ablation_study OUT.json [--pairs P] [--noise SIGMA]

Reproduces the shape of the paper's timing / accuracy trade-off (Sec. IV-C:
error against the number of warps N at a 0.2 px clip, time against N; error
against the clip delta-u_max for several N) on the 640x480 Kannala-Brandt
room configuration (5 levels, 100 primal-dual iterations per warp, FP32):
for every pixel inside the level-0 mask whose data term is on and whose
scene point camera 1 sees, the endpoint error of the recovered
correspondence x + w against the rendered one (in the pre-rotated frame),
and the share of pixels whose error exceeds 1 px and 3 px (the paper's
thresholds; 5 px is reported beside).  Time is the GPU time of one whole
solve (median of 3).  --noise sets the Gaussian noise of the renders
(default: the configuration's 0.01).  tests/test_gpu_ablation.py runs the
same measurement on a reduced grid.
"""
from __future__ import annotations

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def prepare(vfs, cfg, pairs):
    """Rig and rendered scenes: (I0, I1, rendered flow, evaluated pixels) per pair."""
    import torch

    from synth import scene

    rig = scene.make_rig(cfg)
    R = vfs.Rig(rig["cam0"], rig["cam1"], rig["R"], rig["t"], cfg["levels"])
    flags = R.field(0, vfs.FIELD_FLAGS).cpu().numpy()
    data_on = (flags & vfs.F_DATA) != 0
    scenes = []
    t0 = time.time()
    for b in range(pairs):
        I0, I1, gt = scene.render_pair(rig, cfg, b, with_gt=True)
        keep = data_on & gt["visible"]
        scenes.append((torch.from_numpy(I0).cuda(), torch.from_numpy(I1).cuda(), gt["flow"], keep))
    log(f"ablation: {pairs} pairs rendered in {time.time() - t0:.1f} s")
    return R, scenes


def run(vfs, cfg, R, scenes, warps, du_max):
    """Outlier shares (error > 1, 3, 5 px), median endpoint error and GPU
    time per solve of one schedule over the scenes."""
    import numpy as np
    import torch

    from synth import configs

    params = configs.solver_params(cfg, warps=warps, du_max=du_max)
    errs, times = [], []
    for I0, I1, flow, keep in scenes:
        ts = []
        for _ in range(3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            o = vfs.solve(R, I0, I1, params)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        times.append(float(np.median(ts)))
        w = o["w"].cpu().numpy()
        errs.append(np.linalg.norm(w - flow, axis=-1)[keep])
    e = np.concatenate(errs)
    return {"warps": warps, "du_max": du_max, "tau1_pct": round(100 * float(np.mean(e > 1.0)), 2),
            "tau3_pct": round(100 * float(np.mean(e > 3.0)), 2), "tau5_pct": round(100 * float(np.mean(e > 5.0)), 2),
            "epe_median": round(float(np.median(e)), 4), "ms_per_solve": round(1e3 * float(np.mean(times)), 2),
            "pixels": int(e.size)}


def main():
    import paper_1909_07545_amd as vfs
    from synth import configs

    out_path = sys.argv[1]
    pairs = int(sys.argv[sys.argv.index("--pairs") + 1]) if "--pairs" in sys.argv else 4
    cfg = configs.get("c2")
    if "--noise" in sys.argv:
        cfg["noise"] = float(sys.argv[sys.argv.index("--noise") + 1])
    R, scenes = prepare(vfs, cfg, pairs)
    res = {"workload": f"c2: {pairs} rendered 640x480 KB rooms (noise sigma {cfg['noise']}), {cfg['levels']} levels, "
                       f"{cfg['iters']} iterations per warp, FP32 TGV-L1, lambda {configs.PAPER_PARAMS['lambda']}",
           "by_warps": [], "by_clip": []}
    for n in range(1, 21):
        r = run(vfs, cfg, R, scenes, n, 0.2)
        res["by_warps"].append(r)
        log(f"ablation: {r}")
    for n in (1, 2, 5, 10, 20):
        for du in (0.1, 0.2, 0.3, 0.5, 0.7, 1.0):
            r = run(vfs, cfg, R, scenes, n, du)
            res["by_clip"].append(r)
            log(f"ablation: {r}")
    with open(out_path, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
