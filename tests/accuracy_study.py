"""Accuracy studies against full FP64 oracle solves (a script, not collected
by pytest; it needs a GPU and a few minutes of host CPU).

  python -m tests.accuracy_study precision OUT.json [c3,c5]
      FP32 / FP16 / BF16 storage of one 1280x1024 190-degree pair (6 levels x
      10 warps x 150 iterations) and of pair 0 of the 2048x2048 200-degree
      batch (7 x 15 x 200): displacement and depth error against the oracle,
      next to the conditioning floor (the oracle's own solve of the input
      perturbed by 1e-6 relative, against its unperturbed solve).

  python -m tests.accuracy_study serving OUT.json
      The serving workload's solver settings (10 warps x 50 iterations,
      levels 4 / 5 / 5): one pair per (size, rig 0 / 1) served by the FP16
      continuous-batching server and by the plain FP32 server, against the
      oracle.

  python -m tests.accuracy_study data_term OUT.json
      Brightness-constancy against the rank-transform and gradient-magnitude
      data terms on rendered scenes with ground truth (the 128x128 plane, 4
      pairs of the 640x480 Kannala-Brandt room): unchanged images, I1 through
      a strictly increasing intensity curve, I1 under a radial gain
      (vignetting of camera 1 only), and I1 plus a constant.  Error of x + w against the rendered correspondence
      over pixels whose data term is on and that camera 1 sees.

  python -m tests.accuracy_study rectified OUT.json
      The comparison with a rectified pipeline (Sec. V-A, Table I, Fig. 7) on
      4 rendered 800x800 180-degree equidistant rooms: the same energy and
      schedule on pinhole views of 90, 120 and 165 degrees (vfs_rectify,
      pinhole rig R = I, t = (b, 0, 0)), the result taken back to the fisheye
      image (vfs_unrectify) as a 3-D point on each pixel's ray and projected
      into camera 1, so that both methods' correspondences are compared with
      the rendered ones in fisheye pixels.  Pixels a view does not cover count
      as erroneous for it.
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


def _errors(out, o, m):
    import numpy as np
    u = out["u"].cpu().numpy()
    w = out["w"].cpu().numpy()
    du = np.abs(u - o["u"])[m]
    dw = np.linalg.norm(w - o["w"], axis=-1)[m]
    vg = out["valid"].cpu().numpy().astype(bool)
    both = vg & o["valid"].astype(bool)
    rel = np.abs(out["depth"].cpu().numpy()[both] - o["depth"][both]) / o["depth"][both]
    return {"u_mean": float(du.mean()), "u_p99": float(np.percentile(du, 99)), "u_max": float(du.max()),
            "w_mean": float(dw.mean()), "depth_rel_median": float(np.median(rel)),
            "depth_rel_p90": float(np.percentile(rel, 90)), "validity_flips": int(np.sum(vg != o["valid"]))}


def precision():
    import numpy as np
    import torch

    import oracle
    import paper_1909_07545_amd as vfs
    from synth import configs, scene

    table = {}
    for cid in (sys.argv[3].split(",") if len(sys.argv) > 3 else ("c3", "c5")):
        cfg = configs.get(cid)
        params = configs.solver_params(cfg)
        rig = scene.make_rig(cfg)
        log(f"precision: rendering {cid} pair 0")
        I0, I1 = scene.render_pair(rig, cfg, 0, with_gt=False)[:2]
        beta, eta = scene.pair_tensor_params(cfg, 0)
        params = dict(params, beta=beta, eta=eta)
        R = vfs.Rig(rig["cam0"], rig["cam1"], rig["R"], rig["t"], params["levels"])
        t0, t1 = torch.from_numpy(I0).cuda(), torch.from_numpy(I1).cuda()
        outs = {name: vfs.solve(R, t0, t1, dict(params, storage=st))
                for name, st in (("f32", 0), ("f16", 1), ("bf16", 2))}
        torch.cuda.synchronize()
        t = time.perf_counter()
        o = oracle.solve(rig["cam0"], rig["cam1"], rig["R"], rig["t"], params, I0.astype(np.float64),
                         I1.astype(np.float64))
        log(f"precision: {cid} oracle solve took {time.perf_counter() - t:.1f} s")
        m = oracle.mask0(rig["cam0"]).astype(bool)
        row = {name: _errors(out, o, m) for name, out in outs.items()}
        # conditioning floor, from the oracle alone: its own solve of I0 perturbed by 1e-6 relative
        # (the size of float32's per-step differences) against its unperturbed solve
        rng = np.random.default_rng(0)
        I0p = I0.astype(np.float64) * (1 + 1e-6 * rng.standard_normal(I0.shape))
        op = oracle.solve(rig["cam0"], rig["cam1"], rig["R"], rig["t"], params, I0p, I1.astype(np.float64))
        d = np.abs(op["u"] - o["u"])[m]
        row["floor_oracle_input_1e-6"] = {"u_mean": float(d.mean()), "u_p99": float(np.percentile(d, 99)),
                                          "u_max": float(d.max())}
        table[cid] = row
        log(f"precision: {cid} {json.dumps(row)}")
    return {"precision": table}


def serving():
    import numpy as np
    import torch

    import oracle
    import paper_1909_07545_amd as vfs
    from synth import configs, serving as sv

    sp = sv.spec()
    rigs = sv.serving_rigs(sp)
    pool = sv.render_pool(rigs, 1, sp)
    base = configs.solver_params(dict(levels=1, warps=sp["warps"], iters=sp["iters"]))
    rows = []
    for s in range(len(sp["sizes"])):
        for r in (0, 1):
            rg = rigs[r][s]
            h = vfs.Rig(rg["cam0"], rg["cam1"], rg["R"], rg["t"], rg["levels"])
            I0, I1 = pool[(r, s)][0]
            i0, i1 = torch.from_numpy(I0).cuda(), torch.from_numpy(I1).cuda()
            got = {}
            for name, st, mode in (("fp16_batched", 1, "batched"), ("fp32_plain", 0, "plain")):
                params = dict(base, storage=st)
                o = dict(u=torch.empty((h.height, h.width), device="cuda"),
                         depth=torch.empty((h.height, h.width), device="cuda"))
                with vfs.Server(params, mode=mode) as srv:
                    srv.submit(h, i0, i1, o, params["beta"], params["eta"])
                    srv.wait_all(600.0)
                got[name] = o["u"].cpu().numpy()
            t0 = time.perf_counter()
            ref = oracle.solve(rg["cam0"], rg["cam1"], rg["R"], rg["t"], dict(base, levels=rg["levels"]),
                               I0.astype(np.float64), I1.astype(np.float64))
            m = oracle.mask0(rg["cam0"]).astype(bool)
            row = {"size": f"{h.width}x{h.height}", "rig": r, "oracle_s": round(time.perf_counter() - t0, 1)}
            for name, u in got.items():
                d = np.abs(u - ref["u"])[m]
                row[name] = {"u_mean": float(d.mean()), "u_p99": float(np.percentile(d, 99)),
                             "u_max": float(d.max())}
            rows.append(row)
            log(f"serving accuracy: {json.dumps(row)}")
    return {"serving_accuracy": rows}


def data_term():
    import numpy as np
    import torch

    import paper_1909_07545_amd as vfs
    from synth import configs, scene

    def curve(I, cam):
        return 1.25 * I + 0.03 + 0.1 * np.tanh(3.0 * I)

    def vignette(I, cam):
        H, W = I.shape
        jj, ii = np.meshgrid(np.arange(W), np.arange(H))
        r2 = ((jj - cam["cx"]) ** 2 + (ii - cam["cy"]) ** 2) / (0.25 * (W * W + H * H))
        return I * (1.0 - 0.45 * r2)

    def offset(I, cam):
        return I + 0.15

    changes = {"none": None, "curve": curve, "vignette": vignette, "offset": offset}
    terms = ([("brightness", configs.PAPER_PARAMS["lambda"])] + [("rank", lam) for lam in (2.0, 5.0, 15.0, 30.0)] +
             [("gradient", lam) for lam in (15.0, 50.0)])
    rows = []
    for cid, pairs in (("c1", 1), ("c2", 4)):
        cfg = configs.get(cid)
        rig = scene.make_rig(cfg)
        R = vfs.Rig(rig["cam0"], rig["cam1"], rig["R"], rig["t"], cfg["levels"])
        flags = R.field(0, vfs.FIELD_FLAGS).cpu().numpy()
        data_on = (flags & vfs.F_DATA) != 0
        scenes = []
        for b in range(pairs):
            I0, I1, gt = scene.render_pair(rig, cfg, b, with_gt=True)
            scenes.append((I0, I1, gt["flow"], data_on & gt["visible"]))
        log(f"data term: {cid} {pairs} pairs rendered")
        for cname, ch in changes.items():
            for term, lam in terms:
                params = configs.solver_params(cfg, data_term=term, **{"lambda": lam})
                errs = []
                for I0, I1, flow, keep in scenes:
                    I1c = I1 if ch is None else ch(I1.astype(np.float64), rig["cam1"]).astype(np.float32)
                    o = vfs.solve(R, torch.from_numpy(I0).cuda(), torch.from_numpy(np.ascontiguousarray(I1c)).cuda(),
                                  params)
                    errs.append(np.linalg.norm(o["w"].cpu().numpy() - flow, axis=-1)[keep])
                e = np.concatenate(errs)
                row = {"config": cid, "change": cname, "data_term": term, "lambda": lam,
                       "tau1_pct": round(100 * float(np.mean(e > 1.0)), 2),
                       "tau5_pct": round(100 * float(np.mean(e > 5.0)), 2),
                       "epe_median": round(float(np.median(e)), 4)}
                rows.append(row)
                log(f"data term: {json.dumps(row)}")
    return {"workload": "c1: 128x128 equidistant plane, 1 pair; c2: 640x480 KB room, 4 pairs; schedules of the "
                        "configurations, FP32 TGV-L1", "rows": rows}


def rectified():
    import numpy as np
    import torch

    import paper_1909_07545_amd as vfs
    from synth import configs, scene

    cfg = configs.get("rect800")
    pairs = 4
    rig = scene.make_rig(cfg)
    cam, R, t = rig["cam0"], np.asarray(rig["R"]), np.asarray(rig["t"])
    params = configs.solver_params(cfg)
    F = vfs.Rig(cam, rig["cam1"], R, t, cfg["levels"])
    flags = F.field(0, vfs.FIELD_FLAGS).cpu().numpy()
    Rv0, Rv1, b = vfs.rectify_rotations(R, t)
    H, W = cam["height"], cam["width"]
    jj, ii = torch.meshgrid(torch.arange(W, dtype=torch.float64), torch.arange(H, dtype=torch.float64),
                            indexing="xy")
    rays, _ = scene.cam_rays(cam, jj, ii)
    rays = rays.numpy()
    tp = torch.from_numpy(R.T @ t)
    scenes = []
    for k in range(pairs):
        I0, I1, gt = scene.render_pair(rig, cfg, k, with_gt=True)
        keep = ((flags & vfs.F_DATA) != 0) & gt["visible"]
        scenes.append((torch.from_numpy(I0).cuda(), torch.from_numpy(I1).cuda(), gt, keep))
    log(f"rectified: {pairs} pairs rendered")

    def timed(fn):
        ts, out = [], None
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return out, 1e3 * float(np.median(ts))

    def summary(errs, rel, covered, ms):
        e = np.concatenate(errs)
        c = np.concatenate(covered)
        r = np.concatenate(rel)
        return {"coverage_pct": round(100 * float(c.mean()), 2),
                "tau1_pct": round(100 * float(np.mean(~(e <= 1.0))), 2),
                "tau3_pct": round(100 * float(np.mean(~(e <= 3.0))), 2),
                "tau3_pct_covered": round(100 * float(np.mean(~(e[c] <= 3.0))), 2),
                "accurate_px": int(np.sum(e <= 3.0)),
                "range_rel_err_median_covered": round(float(np.median(r)), 4),
                "ms_per_solve": round(ms, 2)}

    res = {"workload": f"{pairs} rendered 800x800 equidistant rooms, 180 degrees, baseline {cfg['baseline']} m, "
                       f"{cfg['levels']} levels x {cfg['warps']} warps x {cfg['iters']} iterations, FP32 TGV-L1, "
                       f"lambda {params['lambda']}; error of the correspondence in camera 1 (fisheye pixels, "
                       f"pre-rotated frame) against the rendered one; accurate = error <= 3 px",
           "methods": {}}
    errs, rel, cov, ms_all = [], [], [], []
    for I0, I1, gt, keep in scenes:
        out, ms = timed(lambda: vfs.solve(F, I0, I1, params))
        w = out["w"].cpu().numpy()
        errs.append(np.linalg.norm(w - gt["flow"], axis=-1)[keep])
        d = out["depth"].cpu().numpy()
        ok = out["valid"].cpu().numpy().astype(bool) & keep
        rel.append(np.abs(d[ok] - gt["range"][ok]) / gt["range"][ok])
        cov.append(np.ones(int(keep.sum()), bool))
        ms_all.append(ms)
    res["methods"]["fisheye_180"] = summary(errs, rel, cov, float(np.mean(ms_all)))
    log(f"rectified: fisheye {res['methods']['fisheye_180']}")

    for fov in (90.0, 120.0, 165.0):
        pin = scene.pinhole_view(W, fov)
        P = vfs.Rig(pin, pin, np.eye(3), np.array([b, 0.0, 0.0]), cfg["levels"])
        errs, rel, cov, ms_all, ms_rect = [], [], [], [], []
        for I0, I1, gt, keep in scenes:
            J0 = torch.empty((W, W), device="cuda")
            J1 = torch.empty((W, W), device="cuda")
            v0 = torch.empty((W, W), dtype=torch.uint8, device="cuda")
            v1 = torch.empty((W, W), dtype=torch.uint8, device="cuda")

            def rect():
                vfs.rectify(cam, Rv0, pin, I0, J0, v0)
                vfs.rectify(rig["cam1"], Rv1, pin, I1, J1, v1)
            _, mr = timed(rect)
            ms_rect.append(mr)
            out, ms = timed(lambda: vfs.solve(P, J0, J1, params))
            ms_all.append(ms)
            vv = (v0 & v1).contiguous()           # both views have image data
            uf = torch.empty((H, W), device="cuda")
            uv = torch.empty((H, W), dtype=torch.uint8, device="cuda")
            vfs.unrectify(cam, Rv0, pin, out["u"], uf, vv, uv)
            u = uf.cpu().numpy().astype(np.float64)
            c = uv.cpu().numpy().astype(bool)
            # 3-D point on the pixel's ray at the virtual depth f b / u, projected into camera 1
            V = rays @ Rv0.T
            z = pin["fx"] * b / np.where(u > 1e-3, u, np.nan)
            rng_est = z / V[..., 2]
            X = torch.from_numpy(rng_est[..., None] * rays)
            x1 = scene.cam_project(cam, X + tp).numpy()
            x0 = np.stack([jj.numpy(), ii.numpy()], -1)
            wr = np.where(np.isfinite(x1), x1 - x0, 0.0)      # a point at infinity: no displacement
            e = np.linalg.norm(wr - gt["flow"], axis=-1)
            e = np.where(c, e, np.inf)
            errs.append(e[keep])
            cov.append(c[keep])
            okr = c & keep & np.isfinite(rng_est)
            rel.append(np.abs(rng_est[okr] - gt["range"][okr]) / gt["range"][okr])
        name = f"rectified_{int(fov)}"
        res["methods"][name] = summary(errs, rel, cov, float(np.mean(ms_all)))
        res["methods"][name]["ms_rectify_pair"] = round(float(np.mean(ms_rect)), 3)
        log(f"rectified: {name} {res['methods'][name]}")
    ours = res["methods"]["fisheye_180"]["accurate_px"]
    res["additional_accurate_pct"] = {k: round(100.0 * (ours - v["accurate_px"]) / max(v["accurate_px"], 1), 2)
                                      for k, v in res["methods"].items() if k != "fisheye_180"}
    return res


def main():
    what, out = sys.argv[1], sys.argv[2]
    res = {"precision": precision, "serving": serving, "data_term": data_term, "rectified": rectified}[what]()
    with open(out, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
