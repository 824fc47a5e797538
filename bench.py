"""Benchmark: primal-dual Mpixel-iterations per second of the whole method on
one MI355X, with the level-0 primal-dual kernel against the HBM roofline and
the FP64 CPU oracle timed beside it.

A step is one whole batched solve (pre-rotation, pyramids, every level x
warp x primal-dual iteration, triangulation) of the workload's pairs, inputs
already resident in HBM.  Default workload: 8 pairs of 2048x2048
Kannala-Brandt 200-degree fisheye images (seeded box-and-sphere rooms),
7 levels x 15 warps x 200 iterations, FP32 TGV-L1.

Then the serving study: 512 requests of three sizes and four rigs arrive as
a Poisson stream; the same trace is served by the plain FP32 server (one pair
at a time) and by the FP16 continuous-batching server, and the line reports
p50 / p99 latency and pairs/s of both.

Prints one JSON line.  Usage: python bench.py [--steps K] [--warmup W]
[--config c5|c3|c2|c1] [--gpus 1] [--no-cpu-baseline] [--no-serving]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic (compulsory) HBM bytes per pixel of one launch of the level-0
# primal-dual pass, which carries several iterations of Eq. (11) (the
# library reports how many) in one pass over memory: reads u 4, v 8, p 8,
# q 16, tensor pack 16, rho_c 4, flags 1 (57 B); writes u 4, v 8, p 8, q 16
# (36 B).  The textbook state (with ubar, vbar in memory) would move 117 B per
# pixel-iteration.
BYTES_PER_PIX_LAUNCH = 93
# The same kernel with p, q and the tensor pack stored as 16-bit values:
# reads u 4, v 8, p 4, q 8, tensor pack 8, rho_c 4, flags 1; writes u 4, v 8, p 4, q 8.
BYTES_PER_PIX_LAUNCH_16 = 61
TEXTBOOK_BYTES_PER_PIX_ITER = 117
HBM_PEAK_GBS = 8000.0
# the best streaming copy measured on this MI355X (one float per thread,
# 4 GiB buffers): what an access pattern like the pass's can reach
BEST_COPY_GBS = 6240.0
VALU_PEAK_LANE_INSTR_S = 256 * 4 * 16 * 2.4e9


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # 3 warm-up and 20 timed solves of the headline workload (about 16 s of
    # timed GPU work); the FP16 and graph-replay legs beside it time at most 5
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c5")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-fp16", action="store_true", help="skip the FP16-storage measurement")
    ap.add_argument("--input-cache", default=None,
                    help="npz file to reuse rendered inputs across runs (written if missing)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy a 1 GiB device buffer (a plain copy kernel of known size, "
                         "for scaling hardware traffic counters)")
    ap.add_argument("--pass-iters", type=int, default=0,
                    help="primal-dual iterations per pass (0: the library's choice by pair size)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving study")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the graph-replay timing (for counter-collection runs of the profiler)")
    ap.add_argument("--serving-only", action="store_true", help="run only the serving study (prints its JSON)")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-rates", type=lambda v: [float(x) for x in v.split(",")], default=[0.5, 0.8, 1.0, 1.5],
                    help="arrival rates as fractions of the plain server's closed-loop pairs/s")
    ap.add_argument("--serve-budget-gib", type=float, default=1.0)
    ap.add_argument("--serve-slots", type=int, default=16)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); the path shards "
              "by image pair across GPUs but no multi-GPU run is part of it", file=sys.stderr)
        sys.exit(2)
    if args.serving_only:
        print(json.dumps({"serving": serving_study(args)}), flush=True)
        return

    import numpy as np
    import torch

    import paper_1909_07545_amd as vfs
    from synth import configs, scene

    cfg = configs.get(args.config)
    params = configs.solver_params(cfg, pass_iters=args.pass_iters)
    rig = scene.make_rig(cfg)
    n = cfg["batch"]
    t0 = time.time()
    if args.input_cache and os.path.exists(args.input_cache):
        z = np.load(args.input_cache)
        pairs = [(z[f"I0_{b}"], z[f"I1_{b}"]) for b in range(n)]
    else:
        log(f"bench: rendering {n} pair(s) of {cfg['width']}x{cfg['height']} ({cfg['name']})")
        pairs = [scene.render_pair(rig, cfg, b, with_gt=False)[:2] for b in range(n)]
        if args.input_cache:
            np.savez(args.input_cache, **{f"I{k}_{b}": pairs[b][k] for b in range(n) for k in (0, 1)})
    tens = [scene.pair_tensor_params(cfg, b) for b in range(n)]
    log(f"bench: inputs ready in {time.time() - t0:.1f} s")

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    I0s = [torch.from_numpy(p[0]).to(dev) for p in pairs]
    I1s = [torch.from_numpy(p[1]).to(dev) for p in pairs]
    R = vfs.Rig(rig["cam0"], rig["cam1"], rig["R"], rig["t"], params["levels"])
    betas = [b for b, _ in tens]
    etas = [e for _, e in tens]
    outs = None
    for i in range(args.warmup):
        outs = vfs.solve_batch(R, I0s, I1s, params, betas=betas, etas=etas, out=outs)
        torch.cuda.synchronize()
        log(f"bench: warmup step {i} done")
    vfs.profile_enable(R, True)
    vfs.profile_read(R, reset=True)
    torch.cuda.synchronize()
    # events between the steps on the stream the solves run on (no
    # synchronisation inside the timed region): the spread of single steps
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    marks[0].record()
    for i in range(args.steps):
        outs = vfs.solve_batch(R, I0s, I1s, params, betas=betas, etas=etas, out=outs)
        marks[i + 1].record()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    step_ms = sorted(marks[i].elapsed_time(marks[i + 1]) for i in range(args.steps))
    pd_ms, pd_launches, iters_per_launch = vfs.profile_read(R, reset=True)
    vfs.profile_enable(R, False)
    log(f"bench: {args.steps} timed steps in {dt:.3f} s")

    pix_iter = configs.pix_iters(cfg)
    side_steps = min(args.steps, 5)
    ms_per_step = 1e3 * dt / args.steps
    value = pix_iter / (dt / args.steps) / 1e6

    # the same steps replayed from the graph the library captures at the first
    # solve of this configuration (no timing events inside)
    graph = None
    if not args.no_graph:
        graph = graph_replay(vfs, torch, R, I0s, I1s, params, betas, etas, outs, pix_iter, side_steps)

    W, H = cfg["width"], cfg["height"]
    avg_launch_s = (pd_ms / pd_launches) / 1e3 if pd_launches else float("nan")
    # algorithmic bytes of one launch: 117 B per pixel-iteration (the textbook
    # state of Eq. (11) read and written once per iteration) x the pixel-
    # iterations one launch carries; the pass keeps the intermediate
    # iterations in registers, so this rate is an effective one and exceeds
    # the HBM peak
    textbook_bytes = TEXTBOOK_BYTES_PER_PIX_ITER * iters_per_launch * W * H * n
    achieved = textbook_bytes / avg_launch_s / 1e9
    # bytes the pass must move at least: every state plane read and written once per launch
    bytes_per_launch = BYTES_PER_PIX_LAUNCH * W * H * n
    compulsory = bytes_per_launch / avg_launch_s / 1e9
    traffic = measured_traffic(args.config, iters_per_launch)
    counters = traffic / avg_launch_s / 1e9 if traffic else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "frac_kind": "effective: 117 B per pixel-iteration x pixel-iterations per launch",
                "kernel": f"level-0 primal-dual pass ({iters_per_launch} iterations of Eq. (11) per launch, "
                          f"pdn_kernel<TGV>)",
                "iters_per_launch": iters_per_launch,
                "avg_launch_us": round(avg_launch_s * 1e6, 2), "launches": pd_launches,
                "textbook_bytes_per_launch": textbook_bytes,
                "compulsory_bytes_per_launch": bytes_per_launch,
                "compulsory_GBs": round(compulsory, 1),
                "frac_compulsory": round(compulsory / HBM_PEAK_GBS, 4),
                "counters_GBs": round(counters, 1) if counters else None,
                "frac_counters": round(counters / HBM_PEAK_GBS, 4) if counters else None,
                "level0_Mpix_iter_s": round(iters_per_launch * W * H * n / avg_launch_s / 1e6, 1)}

    # The same launch against the vector-issue peak: a wave64 vector
    # instruction occupies one of 256 CUs x 4 SIMDs of 16 lanes for 4 cycles at
    # 2.4 GHz (packed FP32 instructions are not used), i.e. 39.3 T lane-instructions/s.
    valu = measured_valu(args.config, iters_per_launch)
    alu = None
    if valu is not None and pd_launches:
        peak_li = VALU_PEAK_LANE_INSTR_S / 1e12
        achieved_li = valu * 64 / avg_launch_s / 1e12
        alu = {"bound": "alu", "achieved": round(achieved_li, 2), "peak": round(peak_li, 2),
               "unit": "T lane-instructions/s", "frac": round(achieved_li / peak_li, 4),
               "model": "every wave64 vector instruction holds a 16-lane SIMD for 4 cycles; a fraction above 1 "
                        "means part of the mix issues in fewer cycles (the pass is then issue-bound)",
               "valu_wave64_per_launch": valu,
               "source": f"profiles/pdn{iters_per_launch}_kernel_batch2048_valu.json"}

    fp16 = None
    if not args.no_fp16:
        p16 = dict(params, storage=1)
        outs16 = vfs.solve_batch(R, I0s, I1s, p16, betas=betas, etas=etas)
        torch.cuda.synchronize()
        vfs.profile_enable(R, True)
        vfs.profile_read(R, reset=True)
        t0 = time.perf_counter()
        for i in range(side_steps):
            outs16 = vfs.solve_batch(R, I0s, I1s, p16, betas=betas, etas=etas, out=outs16)
        torch.cuda.synchronize()
        dt16 = time.perf_counter() - t0
        ms16, n16, _ = vfs.profile_read(R, reset=True)
        vfs.profile_enable(R, False)
        a16 = (ms16 / n16) / 1e3 if n16 else float("nan")
        du = torch.stack([(o16["u"] - o["u"]).abs().mean() for o16, o in zip(outs16, outs)]).mean().item()
        fp16 = {"value": round(pix_iter / (dt16 / side_steps) / 1e6, 1), "ms_per_step": round(1e3 * dt16 / side_steps, 2),
                "steps": side_steps,
                "avg_launch_us": round(a16 * 1e6, 2),
                "achieved_GBs": round(BYTES_PER_PIX_LAUNCH_16 * W * H * n / a16 / 1e9, 1),
                "mean_abs_u_diff_vs_fp32_px": round(du, 5)}
        log(f"bench: fp16 storage {side_steps} steps in {dt16:.3f} s")

    if alu is not None:
        # the roof that binds: HBM by the counters (against the best streaming
        # copy measured on this GPU) or vector issue, whichever is closer to its peak
        hbm_near = roofline["counters_GBs"] / BEST_COPY_GBS if roofline["counters_GBs"] else None
        roofline["binding"] = ("vector issue" if hbm_near is None or alu["frac"] > hbm_near else "hbm") + \
            f" (vector issue at {alu['frac']:.2f} of the 4-cycle model's peak" + \
            (f", HBM traffic at {hbm_near:.2f} of the best copy measured, {BEST_COPY_GBS:.0f} GB/s)" if hbm_near
             else ")")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cfg, rig, pairs[0], tens[0], params, args.cpu_seconds)

    serve = None
    if not args.no_serving:
        del outs, I0s, I1s
        torch.cuda.empty_cache()
        serve = serving_study(args)
        at = min(serve["sweep"], key=lambda r: abs(r["rate_factor"] - 0.8))
        serve["summary"] = {
            "rate_pairs_per_s": at["rate_pairs_per_s"], "rate_factor": at["rate_factor"],
            "fp32_plain": {k: at["plain_fp32"][k] for k in ("p50_ms", "p99_ms", "pairs_per_s")},
            "fp16_batched": {k: at["batched_fp16"][k] for k in ("p50_ms", "p99_ms", "pairs_per_s")},
            "closed_loop_pairs_per_s": {"fp32_plain": serve["closed_loop_plain_fp32"]["pairs_per_s"],
                                        "fp16_batched": serve["closed_loop_batched_fp16"]["pairs_per_s"]}}

    line = {
        "metric": "primal-dual Mpix-iter/s", "value": round(value, 1), "unit": "Mpix-iter/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 2),
        "step_ms": {"median": round(float(np.median(step_ms)), 2), "p10": round(float(np.percentile(step_ms, 10)), 2),
                    "p90": round(float(np.percentile(step_ms, 90)), 2)},
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded rendered fisheye rooms)",
        "config": {"workload": f"{args.config} {cfg['name']}: {n} x {W}x{H} {cfg['model']} {cfg['fov_deg']:.0f}deg, "
                               f"{cfg['levels']} levels x {cfg['warps']} warps x {cfg['iters']} iters, FP32 TGV-L1",
                   "pairs": n, "width": W, "height": H, "levels": cfg["levels"], "warps": cfg["warps"],
                   "iters": cfg["iters"], "pix_iter_per_step": pix_iter},
        "roofline": roofline,
        "alu": alu,
        "graph_replay": graph,
        "cpu_baseline": cpu,
        "fp16_storage": fp16,
        "serving": serve,
    }
    print(json.dumps(line), flush=True)


def graph_replay(vfs, torch, R, I0s, I1s, params, betas, etas, outs, pix_iter, steps):
    """Solves of the workload replayed from the HIP graph the library captures
    at the first solve of the configuration; outputs compared with the eager
    solve's."""
    outs_g = vfs.solve_batch(R, I0s, I1s, params, betas=betas, etas=etas)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        outs_g = vfs.solve_batch(R, I0s, I1s, params, betas=betas, etas=etas, out=outs_g)
    torch.cuda.synchronize()
    dtg = time.perf_counter() - t0
    same = all(torch.equal(a[k], b[k]) for a, b in zip(outs, outs_g) for k in ("u", "w", "depth"))
    log(f"bench: {steps} graph replays in {dtg:.3f} s (outputs equal to eager: {same})")
    return {"value": round(pix_iter / (dtg / steps) / 1e6, 1), "ms_per_step": round(1e3 * dtg / steps, 2), "steps": steps,
            "outputs_equal_eager": same}


def _pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, np.float64), q))


def serving_study(args, log_prefix="serving"):
    """Serving mix: 512 requests (320x240 / 640x480 / 1024x768 in the ratio
    3:2:1, 4 rigs), Poisson arrivals at a fraction of the plain server's
    closed-loop rate; the same trace replayed against the plain FP32 server
    (first come first served, one pair at a time, eager launches) and the
    FP16 continuous-batching server (size buckets, HBM budget, graph
    replays).  Latency = completion seen by the server - arrival."""
    import numpy as np
    import torch

    import paper_1909_07545_amd as vfs
    from synth import configs, serving

    sp = serving.spec()
    t0 = time.time()
    rigs = serving.serving_rigs(sp)
    pool = serving.render_pool(rigs, 1, sp)
    log(f"{log_prefix}: {len(pool)} pairs rendered in {time.time() - t0:.1f} s")
    handles = {(r, s): vfs.Rig(rg["cam0"], rg["cam1"], rg["R"], rg["t"], rg["levels"])
               for r, per in enumerate(rigs) for s, rg in enumerate(per)}
    imgs = {k: (torch.from_numpy(v[0][0]).cuda(), torch.from_numpy(v[0][1]).cuda()) for k, v in pool.items()}
    base = configs.solver_params(dict(levels=1, warps=sp["warps"], iters=sp["iters"]), pass_iters=args.pass_iters)
    p32, p16 = dict(base, storage=0), dict(base, storage=1)
    n = args.serve_requests
    trace0 = serving.make_trace(1.0, n, sp)
    outs = []
    for q in trace0:
        rg = handles[(q["rig"], q["size"])]
        outs.append(dict(depth=torch.empty((rg.height, rg.width), device="cuda"),
                         u=torch.empty((rg.height, rg.width), device="cuda"),
                         valid=torch.empty((rg.height, rg.width), dtype=torch.uint8, device="cuda")))
    torch.cuda.synchronize()
    beta, eta = base["beta"], base["eta"]

    def run(server_kw, params, trace, closed=False):
        with vfs.Server(params, **server_kw) as srv:
            # warm the buckets / workspaces (graph capture, first allocations)
            for s in range(len(sp["sizes"])):
                rg = handles[(0, s)]
                o = dict(depth=torch.empty((rg.height, rg.width), device="cuda"))
                srv.submit(rg, *imgs[(0, s)], o, beta, eta)
            srv.wait_all(600.0)
            tick0 = srv.stats()["ticks"]
            tickets, t_sub = [], []
            start = time.perf_counter()
            for i, q in enumerate(trace):
                if not closed:
                    due = start + q["t"]
                    while True:
                        now = time.perf_counter()
                        if now >= due:
                            break
                        if due - now > 2e-3:
                            time.sleep(due - now - 1e-3)
                rg = handles[(q["rig"], q["size"])]
                t_sub.append(time.perf_counter())
                tickets.append(srv.submit(rg, *imgs[(q["rig"], q["size"])], outs[i], beta, eta))
            srv.wait_all(600.0)
            lat = [srv.poll(t)[1] for t in tickets]
            adm = [srv.times(t)[0] for t in tickets]
            st = srv.stats()
        done = [t + l for t, l in zip(t_sub, lat)]
        span = max(done) - t_sub[0]
        by_size = {}
        for s, (W, H) in enumerate(sp["sizes"]):
            ls = [l for l, q in zip(lat, trace) if q["size"] == s]
            by_size[f"{W}x{H}"] = {"p50_ms": round(1e3 * _pct(ls, 50), 2), "p99_ms": round(1e3 * _pct(ls, 99), 2)}
        return {"pairs_per_s": round(len(trace) / span, 2), "p50_ms": round(1e3 * _pct(lat, 50), 2),
                "p99_ms": round(1e3 * _pct(lat, 99), 2), "mean_queue_ms": round(1e3 * float(np.mean(adm)), 2),
                "by_size": by_size, "ticks": st["ticks"] - tick0, "peak_active": st["peak_active"],
                "pool_peak_MiB": round(st["pool_peak_bytes"] / 2**20, 1)}

    plain_kw = dict(mode="plain")
    batched_kw = dict(mode="batched", hbm_budget_bytes=int(args.serve_budget_gib * 2**30),
                      max_slots=args.serve_slots, use_graphs=True)
    res = {}
    res["closed_loop_plain_fp32"] = run(plain_kw, p32, trace0, closed=True)
    rate0 = res["closed_loop_plain_fp32"]["pairs_per_s"]
    log(f"{log_prefix}: plain FP32 closed loop {rate0} pairs/s")
    res["closed_loop_batched_fp16"] = run(batched_kw, p16, trace0, closed=True)
    log(f"{log_prefix}: batched FP16 closed loop {res['closed_loop_batched_fp16']['pairs_per_s']} pairs/s")
    res["closed_loop_batched_fp16_16GiB"] = run(dict(batched_kw, hbm_budget_bytes=16 << 30), p16, trace0,
                                                closed=True)
    log(f"{log_prefix}: batched FP16 closed loop, 16 GiB budget: "
        f"{res['closed_loop_batched_fp16_16GiB']['pairs_per_s']} pairs/s")
    # served results of the last closed-loop run against solving each alone
    # (bitwise), for one request of every (rig, size)
    seen, checked, equal = set(), 0, 0
    for i, q in enumerate(trace0):
        key = (q["rig"], q["size"])
        if key in seen:
            continue
        seen.add(key)
        rg = handles[key]
        alone = vfs.solve_batch(rg, [imgs[key][0]], [imgs[key][1]], dict(p16, levels=rg.levels), betas=[beta],
                                etas=[eta])[0]
        checked += 1
        equal += int(torch.equal(alone["u"], outs[i]["u"]) and torch.equal(alone["depth"], outs[i]["depth"]))
    res["alone_vs_served_bitwise"] = {"checked": checked, "equal": equal}
    log(f"{log_prefix}: {equal} of {checked} served requests equal their alone solve bitwise")
    sweep = []
    for f in args.serve_rates:
        trace = serving.make_trace(f * rate0, n, sp)
        row = {"rate_factor": f, "rate_pairs_per_s": round(f * rate0, 2)}
        row["plain_fp32"] = run(plain_kw, p32, trace)
        row["batched_fp16"] = run(batched_kw, p16, trace)
        log(f"{log_prefix}: rate x{f}: plain p50/p99 {row['plain_fp32']['p50_ms']}/{row['plain_fp32']['p99_ms']} ms, "
            f"batched {row['batched_fp16']['p50_ms']}/{row['batched_fp16']['p99_ms']} ms")
        sweep.append(row)
    res["sweep"] = sweep
    res["workload"] = (f"{n} requests, sizes {sp['sizes']} ratio {sp['ratio']}, {sp['rigs']} KB rigs, "
                       f"levels {sp['levels']} x {sp['warps']} warps x {sp['iters']} iters")
    res["batched_config"] = {"hbm_budget_GiB": args.serve_budget_gib, "max_slots_per_size": args.serve_slots,
                             "graphs": True, "storage": "fp16"}
    return res


def measured_valu(config, n):
    """Wave64 vector instructions per launch of the dominant kernel (n
    iterations per pass) from the committed rocprofv3 counter summary
    (SQ_INSTS_VALU), or None if there is none for this workload or the
    kernel source has changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"pdn{n}_kernel_batch2048_valu.json")
    if config != "c5" or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, "paper_1909_07545_amd", "csrc", "pd.hip"), "rb").read()
    if hashlib.sha256(src).hexdigest()[:16] != rec["pd_hip_sha256_prefix"]:
        return None
    return rec["valu_wave64_instructions_per_launch"]


def measured_traffic(config, n):
    """HBM bytes per launch of the dominant kernel (the level-0 pass of n
    iterations) from the committed rocprofv3 counter summary (FETCH_SIZE +
    WRITE_SIZE, scaled by a plain copy), or None if there is none for this
    workload or the kernel source has changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"pdn{n}_kernel_batch2048_traffic.json")
    if config != "c5" or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, "paper_1909_07545_amd", "csrc", "pd.hip"), "rb").read()
    if hashlib.sha256(src).hexdigest()[:16] != rec["pd_hip_sha256_prefix"]:
        return None
    return rec["traffic_bytes_per_launch"]


def cpu_baseline(cfg, rig, pair, tens, params, seconds):
    """The FP64 oracle's primal-dual iterations (the hot loop) on pair 0's
    full-resolution level-0 problem, for a bounded number of iterations, on
    all host threads and on one; beside it the oracle's whole method
    (Algorithm 1 in the pyramid, triangulation) on the 128x128 plane and the
    640x480 room in full, all threads."""
    import ctypes

    import numpy as np

    import oracle
    from synth import configs, scene

    gomp = ctypes.CDLL("libgomp.so.1")
    all_threads = gomp.omp_get_max_threads()

    I0 = pair[0].astype(np.float64)
    I1 = pair[1].astype(np.float64)
    cam0, R, t = rig["cam0"], rig["R"], rig["t"]
    log("bench: cpu baseline set-up (oracle, level 0 of pair 0)")
    cf, _ = oracle.calibration_field(cam0, rig["cam1"], R)
    J1 = oracle.prerotate(I1, cf)
    m = oracle.mask0(cam0)
    dv = oracle.data_valid(cam0, rig["cam1"], R, t, 0)
    gam, _ = oracle.trajectory_field(cam0, R, t, 0)
    beta, eta = tens
    T = oracle.tensor(I0, m, beta, eta)
    sp, tu, tv = oracle.steps(T, m, params["alpha0"], params["alpha1"])
    H, W = m.shape
    u = np.zeros((H, W))
    w = np.zeros((H, W, 2))
    _, _, Iu, rho = oracle.linearise(I0, J1, gam, dv, u, w)
    z2, z4 = np.zeros((H, W, 2)), np.zeros((H, W, 4))
    t0 = time.perf_counter()
    st = oracle.pd_iterations(params, T, m, sp, tu, tv, Iu, rho, u, z2, z2, z4, 2)
    per_iter = (time.perf_counter() - t0) / 2
    k = int(max(2, min(200, seconds / max(per_iter, 1e-6))))
    t0 = time.perf_counter()
    oracle.pd_iterations(params, T, m, sp, tu, tv, Iu, rho, st["u"], st["v"], st["p"], st["q"], k,
                         ubar=st["ubar"], vbar=st["vbar"])
    dt = time.perf_counter() - t0
    val = W * H * k / dt / 1e6
    log(f"bench: cpu baseline {k} iterations in {dt:.1f} s on {all_threads} threads")
    # one thread: a tenth of the iterations
    k1 = max(2, k // 10)
    gomp.omp_set_num_threads(1)
    t0 = time.perf_counter()
    oracle.pd_iterations(params, T, m, sp, tu, tv, Iu, rho, st["u"], st["v"], st["p"], st["q"], k1,
                         ubar=st["ubar"], vbar=st["vbar"])
    dt1 = time.perf_counter() - t0
    gomp.omp_set_num_threads(all_threads)
    log(f"bench: cpu baseline {k1} iterations in {dt1:.1f} s on 1 thread")
    whole = {}
    for cid in ("c1", "c2"):
        c = configs.get(cid)
        d = scene.make_inputs(cid, 1)
        rg = d["rig"]
        t0 = time.perf_counter()
        oracle.solve(rg["cam0"], rg["cam1"], rg["R"], rg["t"], configs.solver_params(c),
                     d["I0"][0].astype(np.float64), d["I1"][0].astype(np.float64))
        dtw = time.perf_counter() - t0
        whole[cid] = {"Mpix_iter_s": round(configs.pix_iters(c) / dtw / 1e6, 2), "seconds": round(dtw, 2),
                      "workload": f"{c['name']}: {c['width']}x{c['height']}, {c['levels']} levels x "
                                  f"{c['warps']} warps x {c['iters']} iters, whole method"}
        log(f"bench: cpu baseline whole method {cid} in {dtw:.1f} s")
    return {"value": round(val, 2), "unit": "Mpix-iter/s", "cores": all_threads, "kind": "oracle",
            "sample": f"{k} primal-dual iterations of Eq. (11) on pair 0's full {W}x{H} level-0 problem "
                      f"(FP64 C oracle, OpenMP over rows), {dt:.1f} s",
            "nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)),
            "one_core": {"value": round(W * H * k1 / dt1 / 1e6, 2), "iterations": k1, "seconds": round(dt1, 1)},
            "whole_method_all_cores": whole}


if __name__ == "__main__":
    main()
