"""Benchmark of the batched HJCD-IK solve on one MI355X.

One step = one hjcd_solve over the whole batch (seed init, PO-CCD, PJ-IK,
collision filter, top-k selection) with every input resident in HBM.
Workload: Panda-like 7-DoF chain, 1,000 targets x 1,024 seeds, 60 link
spheres, 32 obstacle spheres, top-8 (the batched configuration).

Prints one JSON line.  `value` = collision-free solves per second at 1 mm /
1 deg (targets with a returned collision-free seed within tolerance, per
second of wall time).  `roofline` prices the dominant kernel, PJ-IK
(k_polish), by its algorithmic FP32 flops (per-unit counts x executed units,
counted live by the kernel) against the MI355X FP32 vector peak, with the
PO-CCD kernel's figures beside it; `cpu_baseline` times the FP64 oracle on a
bounded sample of the same workload on the host cores.  Further sections:
the uneven multi-robot batch (eager vs graph plan), the serving streams
(served vs plain) and, with --large, the 100,000 x 256 20-joint workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector peak (AMD public spec)
PEAK_HBM_GBS = 8000.0


# ---------------------------------------------------------------------------
# Algorithmic FP32 flops of the per-seed solve kernels per executed unit.
# Counted from the kernel's arithmetic (add/mul = 1, fma = 2, each
# transcendental sin / cos / atan2 / sqrt / log / div = 1); see the design doc.
# ---------------------------------------------------------------------------
def fk_flops(n, modified=True, tool_rot=False):
    return (57 if modified else 51) * n + 18 + (45 if tool_rot else 0)


RESIDUAL = 64 + 3  # residual + cost


def unit_flops(n, modified=True, tool_rot=False):
    fk = fk_flops(n, modified, tool_rot)
    return dict(
        cd_iter=fk + RESIDUAL + 6 + 116 * n + 178,
        pol_iter=fk + RESIDUAL + 669 + 110 * n,
        pol_trial=fk + RESIDUAL + 2 * n + 1,
        pol_dogleg=94 * n + 200,
        pol_single=36 * n + 2,
        perturb=9 * n,
        seed=5 * n + 2 * (fk + RESIDUAL + 1),  # seed init + final FK of both stages
    )


def stage_flops(n, st, modified=True, tool_rot=False):
    """(PO-CCD kernel, PJ-IK kernel) algorithmic flops of one solve."""
    u = unit_flops(n, modified, tool_rot)
    final = fk_flops(n, modified, tool_rot) + RESIDUAL + 1
    cd = st["cd_iters"] * u["cd_iter"] + st["cd_perturb"] * u["perturb"] + st["seeds"] * (5 * n + final)
    pol = (st["pol_iters"] * u["pol_iter"] + st["pol_trials"] * u["pol_trial"] + st["pol_dogleg"] * u["pol_dogleg"]
           + st["pol_single"] * u["pol_single"] + st["pol_perturb"] * u["perturb"] + st["seeds"] * final)
    return cd, pol


def algorithmic_flops(n, st, modified=True, tool_rot=False):
    u = unit_flops(n, modified, tool_rot)
    return (st["cd_iters"] * u["cd_iter"] + st["pol_iters"] * u["pol_iter"]
            + st["pol_trials"] * u["pol_trial"] + st["pol_dogleg"] * u["pol_dogleg"]
            + st["pol_single"] * u["pol_single"]
            + (st["cd_perturb"] + st["pol_perturb"]) * u["perturb"] + st["seeds"] * u["seed"])


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_polish_batched_panda_1000x1024_traffic.txt")
KERNEL_SOURCES = ("hjcd_device.hpp", "hjcd_launch.hpp", "hjcd_solve_inst.hip")


def kernel_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2510_07514_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per k_polish launch from the committed FETCH_SIZE / WRITE_SIZE
    counter runs (scaled by the plain-copy calibration), or None when the
    kernel's sources changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.startswith("#"):
            k, v = line.strip().split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("sources_sha256") != kernel_sources_sha():
        return None
    return int(float(kv["traffic_bytes_per_launch"]))


def cpu_baseline(batch, n_targets):
    """FP64 oracle on the first n_targets targets of the batch (all their
    seeds, uniform Philox seeds like the GPU run), all host cores."""
    import oracle as O
    rob = batch.robots[0]
    sub_q = batch.q_star[:n_targets]
    tg = O.targets_from_qstar(rob, sub_q).astype(np.float64)
    M = int(batch.seed_offsets[1] - batch.seed_offsets[0])
    offs = np.arange(n_targets + 1, dtype=np.int64) * M
    cores = os.cpu_count() or 1
    t0 = time.perf_counter()
    out = O.solve(rob, batch.scene, tg, offs, batch.params, seeds=None, nthreads=cores)
    dt = time.perf_counter() - t0
    solved = int(out["solved"].sum())
    return {"value": solved / dt, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": f"first {n_targets} of {batch.T} targets x {M} seeds, FP64, {dt:.1f} s wall",
            "solved": solved, "seconds": dt}


def measure(H, ctx, torch, batch, steps, warmup):
    """Time `steps` whole hjcd_solve calls on one single-robot batch with
    inputs resident in HBM; the k_solve time comes from the library's HIP
    events on the launch stream."""
    rob = batch.robots[0]
    n, T, k = rob.dof, batch.T, batch.params["top_k"]
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    rb = H.hjcd_load_robot(ctx, rob)
    sc = H.hjcd_load_scene(ctx, batch.scene.spheres, batch.scene.boxes)
    with torch.cuda.stream(stream):
        # targets = FK(q*) by the library's own FK kernel
        qs = torch.as_tensor(np.ascontiguousarray(np.asarray(batch.q_star, np.float32).T)).to(dev)
        pose = torch.zeros(7, T, device=dev)
        H.hjcd_fk(ctx, rb, qs, pose, None, stream=stream)
        targets = pose.contiguous()
        del qs
        q_out = torch.zeros(T * k, n, device=dev)
        ep = torch.zeros(T * k, device=dev)
        eo = torch.zeros(T * k, device=dev)
        fl = torch.zeros(T * k, dtype=torch.uint8, device=dev)
        nf = torch.zeros(T, dtype=torch.int32, device=dev)
        sv = torch.zeros(T, dtype=torch.uint8, device=dev)
    p = H.params_from_dict(batch.params, collect_stats=True)

    def step():
        H.hjcd_solve(ctx, [rb], sc, targets, batch.seed_offsets, p, q_out, ep, eo, fl, nf, sv, stream=stream)

    for _ in range(warmup):
        step()
    stream.synchronize()
    torch.cuda.synchronize()
    kern_ms, step_ms = [], []
    agg = None
    t_start = time.perf_counter()
    for _ in range(steps):
        t0 = time.perf_counter()
        step()
        st = H.hjcd_get_stats(ctx)  # waits for this step's last event on `stream`
        step_ms.append((time.perf_counter() - t0) * 1e3)
        kern_ms.append(st["ms_polish"])
        if agg is None:
            agg = {kk: 0 for kk in st}
        for kk, v in st.items():
            agg[kk] += v
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    n_solved = int(sv.sum().item())
    ms_per_step = wall * 1e3 / steps
    per_step = {kk: v / steps for kk, v in agg.items()}
    f_cd, f_pol = stage_flops(n, per_step)
    kavg = float(np.mean(kern_ms))
    achieved = f_pol / (kavg * 1e-3) / 1e12
    cd_ms = per_step["ms_cd"]
    roof = {"bound": "alu", "kernel": f"k_polish (PJ-IK, {n} joints)", "achieved": round(achieved, 3),
            "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
            "traffic": None, "kernel_ms": round(kavg, 4), "algorithmic_gflop_per_launch": round(f_pol / 1e9, 3),
            "cd_kernel": {"kernel": "k_cd (PO-CCD)", "kernel_ms": round(cd_ms, 4),
                          "algorithmic_gflop_per_launch": round(f_cd / 1e9, 3),
                          "achieved": round(f_cd / (cd_ms * 1e-3) / 1e12, 3) if cd_ms > 0 else None},
            "both_stages_achieved": round((f_cd + f_pol) / ((kavg + cd_ms) * 1e-3) / 1e12, 3)}
    return {"value": round(n_solved / (ms_per_step / 1e3), 1), "ms_per_step": round(ms_per_step, 3),
            "solved_targets": n_solved, "success_rate": round(n_solved / T, 4),
            "latency_ms": {"p50": round(float(np.percentile(step_ms, 50)), 3),
                           "p99": round(float(np.percentile(step_ms, 99)), 3)},
            "stage_ms": {kk: round(per_step[kk], 4) for kk in
                         ("ms_cd", "ms_resample", "ms_polish", "ms_collide", "ms_select", "ms_total")},
            "work_per_step": {kk: int(per_step[kk]) for kk in
                              ("seeds", "cd_iters", "cd_perturb", "pol_iters", "pol_trials", "pol_dogleg",
                               "pol_single", "pol_perturb", "coll_coarse", "coll_fine")},
            "roofline": roof}


def uneven(H, ctx, torch, steps, log):
    """The uneven batch (4,096 targets over 6-, 7- and 12-joint chains, seeds
    log-uniform in [16, 2048]): eager hjcd_solve vs one autotuned plan (a
    hipGraph replay of the whole batch)."""
    from paper_2510_07514_amd import workload as W
    b = W.config_uneven()
    rbs = [H.hjcd_load_robot(ctx, r) for r in b.robots]
    sc = H.hjcd_load_scene(ctx, b.scene.spheres, b.scene.boxes)
    T, k, n_max = b.T, b.params["top_k"], b.n_max
    targets = torch.zeros(7, T, device="cuda")
    for ri, rob in enumerate(b.robots):
        idx = np.nonzero(b.robot_of_target == ri)[0]
        qs = np.ascontiguousarray(np.asarray([b.q_star[t] for t in idx], np.float32).T)
        pose = torch.zeros(7, len(idx), device="cuda")
        H.hjcd_fk(ctx, rbs[ri], torch.as_tensor(qs).cuda(), pose, None)
        targets[:, torch.as_tensor(idx).cuda()] = pose
    torch.cuda.synchronize()
    outs = [torch.zeros(T * k, n_max, device="cuda"), torch.zeros(T * k, device="cuda"),
            torch.zeros(T * k, device="cuda"), torch.zeros(T * k, dtype=torch.uint8, device="cuda"),
            torch.zeros(T, dtype=torch.int32, device="cuda"), torch.zeros(T, dtype=torch.uint8, device="cuda")]
    p = H.params_from_dict(b.params)
    stream = torch.cuda.Stream()

    def timed(fn):
        fn()
        stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        stream.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    ms_eager = timed(lambda: H.hjcd_solve(ctx, rbs, sc, targets, b.seed_offsets, p, *outs,
                                          robot_of_target=b.robot_of_target, stream=stream))
    solved_eager = int(outs[5].sum().item())
    t0 = time.perf_counter()
    plan = H.hjcd_plan_create(ctx, rbs, sc, targets, b.seed_offsets, p, *outs, robot_of_target=b.robot_of_target,
                              tune=True, stream=stream)
    ms_create = (time.perf_counter() - t0) * 1e3
    ms_plan = timed(lambda: H.hjcd_plan_execute(plan, stream=stream))
    solved_plan = int(outs[5].sum().item())
    choices = [H.hjcd_plan_choice(plan, r) for r in range(len(b.robots))]
    plan.close()
    row = {"workload": f"uneven_{T}_targets_{int(b.seed_offsets[-1])}_seeds",
           "robots": [f"{r.name}:{r.dof}dof" for r in b.robots],
           "eager": {"ms_per_solve": round(ms_eager, 3), "solves_per_s": round(solved_eager / ms_eager * 1e3, 1)},
           "plan": {"ms_per_solve": round(ms_plan, 3), "solves_per_s": round(solved_plan / ms_plan * 1e3, 1),
                    "create_ms_incl_autotune": round(ms_create, 1)},
           "solved_targets": solved_plan,
           "choices": [{"variant": c["variant"], "block_threads": c["block_threads"], "ms": round(c["ms"], 3),
                        "seeds": c["seeds"]} for c in choices]}
    log(f"uneven: {row}")
    return row


def serving(H, ctx, torch, rates, duration, slots, chunk, plain_cap, log):
    """Poisson request streams served by the continuous-batching server and
    by the plain one-request-per-launch server (same requests, same keys)."""
    from paper_2510_07514_amd import workload as W
    out = []
    for rate in rates:
        s = W.serving_stream(float(rate), duration)
        rob, scene = s["robot"], s["scene"]
        rb = H.hjcd_load_robot(ctx, rob)
        sc = H.hjcd_load_scene(ctx, scene.spheres, scene.boxes)
        n_req = len(s["arrival"])
        # target poses = FK(q*) by the library's FK kernel
        qs = np.concatenate(s["q_star"]).astype(np.float32)
        qd = torch.as_tensor(np.ascontiguousarray(qs.T)).cuda()
        pose = torch.zeros(7, qs.shape[0], device="cuda")
        H.hjcd_fk(ctx, rb, qd, pose, None)
        torch.cuda.synchronize()
        poses = pose.cpu().numpy().T.copy()
        offs = np.concatenate([[0], np.cumsum(s["n_targets"])])
        params = H.params_from_dict(s["params"])
        row = {"rate_req_s": rate, "requests": int(n_req), "targets": int(offs[-1]),
               "mean_seeds_per_target": round(float(np.mean(s["seeds_per_target"])), 1)}
        if rate == rates[0]:
            # warm-up: the first requests of the stream through both modes, so
            # that kernel loading and first-touch allocation stay out of the
            # measured windows
            for mode in (H.HJCD_SERVE_BATCHED, H.HJCD_SERVE_PLAIN):
                srv = H.hjcd_server_create(ctx, rb, sc, params, mode=mode, max_slots=slots, chunk_iters=chunk)
                for i in range(min(n_req, 32)):
                    H.hjcd_server_submit(srv, poses[offs[i]:offs[i + 1]], int(s["seeds_per_target"][i]), int(offs[i]),
                                         0.0)
                H.hjcd_server_start(srv)
                H.hjcd_server_wait(srv, 120.0)
                srv.close()
        for mode, name in ((H.HJCD_SERVE_BATCHED, "served"), (H.HJCD_SERVE_PLAIN, "plain")):
            m = n_req if mode == H.HJCD_SERVE_BATCHED else min(n_req, plain_cap)
            srv = H.hjcd_server_create(ctx, rb, sc, params, mode=mode, max_slots=slots, chunk_iters=chunk,
                                       max_queue=n_req + 1)
            for i in range(m):
                H.hjcd_server_submit(srv, poses[offs[i]:offs[i + 1]], int(s["seeds_per_target"][i]), int(offs[i]),
                                     float(s["arrival"][i]))
            t0 = time.perf_counter()
            H.hjcd_server_start(srv)
            H.hjcd_server_wait(srv, 600.0)
            wall = time.perf_counter() - t0
            st = H.hjcd_server_get_stats(srv)
            srv.close()
            row[name] = {"requests": m, "solves_per_s": round(st["solves_per_s"], 1),
                         "p50_latency_ms": round(st["p50_latency_ms"], 3),
                         "p99_latency_ms": round(st["p99_latency_ms"], 3),
                         "targets_solved": int(st["targets_solved"]), "targets_done": int(st["targets_done"]),
                         "chunks": int(st["chunks"]), "mean_resident_slots": round(st["mean_resident_slots"], 1),
                         "wall_s": round(wall, 3)}
            log(f"serving {name} at {rate} req/s: {row[name]}")
        row["speedup_solves_per_s"] = round(row["served"]["solves_per_s"] / max(row["plain"]["solves_per_s"], 1e-9), 2)
        out.append(row)
        rb.close()
        sc.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--targets", type=int, default=1000)
    ap.add_argument("--seeds", type=int, default=1024)
    ap.add_argument("--cpu-targets", type=int, default=512)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-uneven", action="store_true")
    ap.add_argument("--no-tiny", action="store_true", help="skip the 8 x 64 latency case (profiling runs)")
    ap.add_argument("--large", action="store_true", help="also time the 100,000 x 256 random 20-joint workload")
    ap.add_argument("--serve-rates", default="2000,10000,50000")
    ap.add_argument("--serve-duration", type=float, default=1.0, help="seconds of each request stream")
    ap.add_argument("--serve-slots", type=int, default=1 << 22, help="resident seed slots of the server")
    ap.add_argument("--serve-chunk", type=int, default=4, help="iterations per serving chunk")
    ap.add_argument("--plain-cap", type=int, default=4000, help="requests of each stream the plain server runs")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run plain device copies of MIB MiB (scales the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the solve has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(max(args.steps, 1)):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_mib": args.copy_calibration, "copies": max(args.steps, 1),
                          "bytes_read_per_copy": n * 4, "bytes_written_per_copy": n * 4}), flush=True)
        return

    from paper_2510_07514_amd import hjcd as H
    from paper_2510_07514_amd import workload as W

    batch = W.config_batched(T=args.targets, M=args.seeds, host_seeds=False)
    ctx = H.hjcd_ctx_create(0)
    m = measure(H, ctx, torch, batch, args.steps, args.warmup)
    rob = batch.robots[0]
    n, T, k = rob.dof, batch.T, batch.params["top_k"]
    steps = args.steps
    line = {
        "metric": "collision-free IK solves/s at 1mm/1deg",
        "value": m["value"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batched_panda_{T}x{args.seeds}", "targets": T,
                   "seeds_per_target": args.seeds, "dof": n, "link_spheres": int(rob.sphere_link.shape[0]),
                   "obstacle_spheres": int(batch.scene.spheres.shape[0]), "top_k": k,
                   "cd_sweeps": batch.params["cd_sweeps"], "polish_iters": batch.params["polish_iters"]},
        "solved_targets": m["solved_targets"],
        "success_rate": m["success_rate"],
        "latency_ms": m["latency_ms"],
        "stage_ms": m["stage_ms"],
        "work_per_step": m["work_per_step"],
        "roofline": dict(m["roofline"], traffic=measured_traffic()),
    }
    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    # the tiny configuration (8 targets x 64 seeds): the latency of one small solve
    if not args.no_tiny:
        tb = W.config_tiny(host_seeds=False)
        mt = measure(H, ctx, torch, tb, 50, 5)
        line["tiny"] = {"workload": "tiny_panda_8x64", "ms_per_solve": mt["ms_per_step"],
                        "latency_ms": mt["latency_ms"], "solved_targets": mt["solved_targets"],
                        "stage_ms": mt["stage_ms"]}
        log(f"tiny: {line['tiny']}")
    if not args.no_uneven:
        line["uneven"] = uneven(H, ctx, torch, 5, log)
    if args.large:
        lb = W.config_large()
        ml = measure(H, ctx, torch, lb, 3, 1)
        line["large"] = dict({"workload": f"large_random20_{lb.T}x{int(lb.seed_offsets[1])}", "top_k": lb.params["top_k"],
                              "cd_sweeps": lb.params["cd_sweeps"], "polish_iters": lb.params["polish_iters"]}, **ml)
        log(f"large: {line['large']}")
    if not args.no_serve:
        rates = [int(x) for x in args.serve_rates.split(",") if x]
        line["serving"] = {"workload": "poisson_panda_1-16_targets_32-1024_seeds", "chunk_iters": args.serve_chunk,
                           "max_slots": args.serve_slots, "duration_s": args.serve_duration,
                           "rates": serving(H, ctx, torch, rates, args.serve_duration, args.serve_slots,
                                            args.serve_chunk, args.plain_cap, log)}
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(batch, min(args.cpu_targets, T))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
