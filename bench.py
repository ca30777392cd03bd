"""Benchmark of batched and served HJCD-IK on one MI355X.

Prints one JSON line.  The headline is the serving workload: a Poisson
stream of IK requests (1-16 Panda-like targets each, 32-1,024 seeds per
target, the 32-sphere scene of the batched workload) at 10,000 requests/s,
served by the continuous-batching server; `value` = collision-free solves
per second at 1 mm / 1 deg over a 10 s window that follows a 1 s warm-up,
with p50 / p99 request latency beside it.  The plain form (one hjcd_solve
launch sequence per request) runs the same first requests of the stream, and
`speedup_vs_plain` compares both modes on that same request set.  The other
rates (2,000 and 50,000 requests/s) are reported the same way.

`steps` / `ms_per_step` time K whole hjcd_solve calls of the batched
workload (1,000 targets x 1,024 seeds, top-8, inputs resident in HBM), whose
PJ-IK kernel (`k_polish`) is priced in `roofline`: the oracle's FP64
operation counts per executed unit of work (measured in the CPU-baseline run
on the same workload) x the units the kernel counts in the timed launches,
over the kernel's HIP-event time on its stream, against the FP32 vector peak.
Further sections: the uneven three-robot batch (eager solve vs graph plan),
the large 20-joint workload (100,000 x 256), the DoF-scaling chains and the
8 x 64 tiny solve.  `cpu_baseline` times the FP64 oracle on a bounded sample
of the batched workload on the host cores (and single-threaded).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector peak (AMD public spec)
PEAK_HBM_GBS = 8000.0

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_polish_batched_panda_1000x1024_traffic.txt")
KERNEL_SOURCES = ("hjcd_device.hpp", "hjcd_launch.hpp", "hjcd_solve_inst.hip")

# executed units the PJ-IK kernel counts -> the oracle's operation category of
# the same unit (an iteration is one evaluation (FK, Jacobian inputs,
# residual) plus the LM linearisation and step; every seed is evaluated once
# more for its final state)
POLISH_UNITS = (("pol_iters", ("eval", "pj_iter")), ("pol_trials", ("pj_trial",)),
                ("pol_dogleg", ("pj_dogleg",)), ("pol_single", ("pj_single",)),
                ("pol_perturb", ("pj_perturb",)), ("seeds", ("eval",)))
CD_UNITS = (("cd_iters", ("eval", "cd_iter")), ("cd_perturb", ("cd_perturb",)), ("seeds", ("init", "eval")))


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


def cpu_model():
    """Host CPU as /proc/cpuinfo names it: the model string plus family, model
    and stepping numbers (a virtualised host may report only a brand name, and
    the numbers still identify the core generation) and the visible threads."""
    info = {}
    try:
        for line in open("/proc/cpuinfo"):
            key, _, val = line.partition(":")
            key = key.strip()
            if key in ("model name", "cpu family", "model", "stepping") and key not in info:
                info[key] = val.strip()
            if len(info) == 4:
                break
    except OSError:
        pass
    name = info.get("model name") or platform.processor() or "unknown"
    ids = ", ".join(f"{k} {info[k]}" for k in ("cpu family", "model", "stepping") if k in info)
    return f"{name} ({ids}; {os.cpu_count()} threads visible)" if ids else name


def cpu_baseline(batch, n_targets, n_single):
    """FP64 oracle on the first n_targets targets of the batch (all their
    seeds, uniform Philox seeds like the GPU run) on the host cores, and on
    the first n_single targets single-threaded.  Also returns the oracle's
    operation counts per executed unit of work (Alg. PO-CCD / PJ-IK units),
    counted in the multi-threaded run."""
    import oracle as O
    rob = batch.robots[0]
    M = int(batch.seed_offsets[1] - batch.seed_offsets[0])

    def run(nt, threads):
        tg = O.targets_from_qstar(rob, batch.q_star[:nt]).astype(np.float64)
        offs = np.arange(nt + 1, dtype=np.int64) * M
        t0 = time.perf_counter()
        out = O.solve(rob, batch.scene, tg, offs, batch.params, seeds=None, nthreads=threads)
        return int(out["solved"].sum()), time.perf_counter() - t0

    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = min(cores, 16)
    O.ops_reset()
    solved, dt = run(n_targets, cores)
    ops = O.ops_get()
    solved1, dt1 = run(n_single, 1)
    per_unit = {k: {"flops": v["flops"] / v["units"], "transcendental": v["trans"] / v["units"]}
                for k, v in ops.items() if v["units"] > 0}
    return {"value": round(solved / dt, 2), "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": f"first {n_targets} of {batch.T} targets x {M} seeds of {batch.name}, FP64, {dt:.1f} s wall",
            "cpu_model": cpu_model(), "solved": solved, "seconds": round(dt, 2),
            "single_thread": {"value": round(solved1 / dt1, 3), "unit": "solves/s", "cores": 1,
                              "sample": f"first {n_single} targets x {M} seeds, {dt1:.1f} s wall",
                              "targets_per_s": round(n_single / dt1, 3)}}, per_unit


def unit_flops(per_unit, units):
    """flops and transcendental calls per unit kind from the oracle's
    per-unit counts."""
    out = {}
    for name, cats in units:
        out[name] = (sum(per_unit.get(c, {}).get("flops", 0.0) for c in cats),
                     sum(per_unit.get(c, {}).get("transcendental", 0.0) for c in cats))
    return out


def algorithmic(per_unit, units, st):
    """(flops, transcendental calls) of one launch: executed units x the
    oracle's operation counts per unit."""
    f = t = 0.0
    for name, (uf, ut) in unit_flops(per_unit, units).items():
        f += st[name] * uf
        t += st[name] * ut
    return f, t


def measure(H, ctx, torch, batch, steps, warmup):
    """Time `steps` whole hjcd_solve calls on one single-robot batch with
    inputs resident in HBM; stage times come from the library's HIP events
    on the launch stream, executed units from the kernels' counters."""
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
    # timed steps: stage times only (the kernels a caller without statistics runs);
    # the executed-work counts come from one more solve with counters, whose
    # results are the same bit for bit
    p = H.params_from_dict(batch.params, collect_stats=2)
    p_count = H.params_from_dict(batch.params, collect_stats=1)

    def step(params=p):
        H.hjcd_solve(ctx, [rb], sc, targets, batch.seed_offsets, params, q_out, ep, eo, fl, nf, sv, stream=stream)

    for _ in range(warmup):
        step()
    stream.synchronize()
    torch.cuda.synchronize()
    step_ms, agg = [], None
    t_start = time.perf_counter()
    for _ in range(steps):
        t0 = time.perf_counter()
        step()
        st = H.hjcd_get_stats(ctx)  # waits for this step's last event on `stream`
        step_ms.append((time.perf_counter() - t0) * 1e3)
        if agg is None:
            agg = {kk: 0 for kk in st}
        for kk, v in st.items():
            agg[kk] += v
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    n_solved = int(sv.sum().item())
    best_ep = ep.view(T, k)[:, 0].cpu().numpy()
    best_eo = eo.view(T, k)[:, 0].cpu().numpy()
    ms_per_step = wall * 1e3 / steps
    per_step = {kk: v / steps for kk, v in agg.items()}
    q_timed = q_out.clone()
    step(p_count)
    counts = H.hjcd_get_stats(ctx)
    if not torch.equal(q_out, q_timed):
        raise RuntimeError("the solve with counters returned other configurations than the timed solves")
    rb.close()
    sc.close()
    return {"value": round(n_solved / (ms_per_step / 1e3), 1), "ms_per_step": round(ms_per_step, 3),
            "solved_targets": n_solved, "success_rate": round(n_solved / T, 4),
            "best_err_median": {"pos_m": float(np.median(best_ep)), "ori_rad": float(np.median(best_eo))},
            "latency_ms": {"p50": round(float(np.percentile(step_ms, 50)), 3),
                           "p99": round(float(np.percentile(step_ms, 99)), 3)},
            "stage_ms": {kk: round(per_step[kk], 4) for kk in
                         ("ms_cd", "ms_resample", "ms_polish", "ms_collide", "ms_select", "ms_total")},
            "work_per_step": {kk: int(counts[kk]) for kk in
                              ("seeds", "cd_iters", "cd_perturb", "pol_iters", "pol_trials", "pol_dogleg",
                               "pol_single", "pol_perturb", "coll_coarse", "coll_fine")}}


def roofline(m, per_unit, n):
    """The PJ-IK kernel's algorithmic FP32 rate (oracle operation counts per
    executed unit x the units of one launch / the kernel's event time)."""
    w = m["work_per_step"]
    roof = {"bound": "alu", "kernel": f"k_polish (PJ-IK, {n} joints)", "workload": m["workload"],
            "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "kernel_ms": m["stage_ms"]["ms_polish"],
            "traffic": measured_traffic()}
    if per_unit is None:
        roof.update(achieved=None, frac=None, note="no oracle operation counts (--no-cpu)")
        return roof
    f_pol, t_pol = algorithmic(per_unit, POLISH_UNITS, w)
    f_cd, t_cd = algorithmic(per_unit, CD_UNITS, w)
    kms = m["stage_ms"]["ms_polish"]
    cms = m["stage_ms"]["ms_cd"]
    ach = f_pol / (kms * 1e-3) / 1e12
    roof.update(achieved=round(ach, 3), frac=round(ach / PEAK_FP32_TFLOPS, 4),
                algorithmic_gflop_per_launch=round(f_pol / 1e9, 3),
                transcendental_g_per_launch=round(t_pol / 1e9, 4),
                flops_per_unit={kk: round(v[0], 1) for kk, v in unit_flops(per_unit, POLISH_UNITS).items()},
                frac_of_unpacked_fma_rate=round(ach / (PEAK_FP32_TFLOPS / 2), 4),
                cd_kernel={"kernel": "k_cd (PO-CCD)", "kernel_ms": cms,
                           "oracle_gflop_per_launch": round(f_cd / 1e9, 3),
                           "oracle_flops_per_unit": {kk: round(v[0], 1)
                                                     for kk, v in unit_flops(per_unit, CD_UNITS).items()},
                           "achieved": None,
                           "note": "the oracle scores every candidate with a full FK evaluation (two per "
                                   "joint), the kernel in closed form by a rigid rotation of the end "
                                   "effector: the oracle's counts overstate the kernel's arithmetic, so "
                                   "no rate is derived from them"})
    return roof


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


def dof_scaling(H, ctx, torch, log):
    """The chained Panda-like robots (7, 12, 18, 24 DoF, open world, B =
    1,000 seeds per target): throughput of a 1,000-target batch and the
    latency of a one-target solve."""
    from paper_2510_07514_amd import workload as W
    rows = []
    for dof in (7, 12, 18, 24):
        b = W.config_dof(dof)
        mb = measure(H, ctx, torch, b, 3, 1)
        one = W.config_dof(dof, T=1)
        m1 = measure(H, ctx, torch, one, 30, 3)
        row = {"dof": dof, "robot": b.robots[0].name, "seeds_per_target": 1000,
               "batch_1000_targets": {"ms_per_solve": mb["ms_per_step"], "solves_per_s": mb["value"],
                                      "success_rate": mb["success_rate"], "stage_ms": mb["stage_ms"]},
               "one_target": {"ms_p50": m1["latency_ms"]["p50"], "ms_p99": m1["latency_ms"]["p99"],
                              "solved": m1["solved_targets"]}}
        log(f"dof scaling: {row}")
        rows.append(row)
    return rows


def resampling(H, ctx, torch, batch, log):
    """Paper-mode resampling (Alg. HJCD-IK: PO-CCD on all M seeds, then
    floor(B/K) noisy copies of the K best polished) on the batched workload,
    against K = B = M (every CD seed polished): latency and accuracy."""
    rows = []
    M = int(batch.seed_offsets[1] - batch.seed_offsets[0])
    for K, B in [(0, 0)] + [(K, B) for K in (8, 32, 128) for B in (64, 256, 1000) if B >= K]:
        b = batch
        b.params = dict(batch.params, resample_K=K, resample_B=B)
        m = measure(H, ctx, torch, b, 5, 1)
        Bp = (B // K) * K if K else M
        rows.append({"K": K if K else M, "B": B if K else M, "polished_per_target": Bp,
                     "ms_per_solve": m["ms_per_step"], "solves_per_s": m["value"], "success_rate": m["success_rate"],
                     "best_err_median": m["best_err_median"],
                     "stage_ms": {kk: m["stage_ms"][kk] for kk in ("ms_cd", "ms_resample", "ms_polish", "ms_collide")}})
        log(f"resampling: {rows[-1]}")
    batch.params = dict(batch.params, resample_K=0, resample_B=0)
    return rows


def tracking(H, ctx, torch, log, tracks=256, steps=100, M=64, k=8, cold_M=1024):
    """Poses along paths (Sec. V demonstration): 256 Panda-like tracks (the
    batched workload's robot and scene), 100 poses each; every pose solved
    from the previous pose's 8 solutions (64 warm seeds) with the nearest-
    solution selection, against the cost selection on the same warm seeds and
    a cold start (1,024 uniform seeds) per pose."""
    from paper_2510_07514_amd import workload as W
    b = W.config_batched(T=1, M=1)
    rob = b.robots[0]
    n = rob.dof
    paths = W.tracking_paths(rob, tracks, steps)
    rb = H.hjcd_load_robot(ctx, rob)
    sc = H.hjcd_load_scene(ctx, b.scene.spheres, b.scene.boxes)
    qd = torch.as_tensor(np.ascontiguousarray(paths.reshape(-1, n).T)).cuda()
    pose = torch.zeros(7, steps * tracks, device="cuda")
    H.hjcd_fk(ctx, rb, qd, pose, None)
    torch.cuda.synchronize()
    targets = [pose[:, s * tracks:(s + 1) * tracks].contiguous() for s in range(steps)]
    stream = torch.cuda.Stream()
    out = {}
    for mode in ("near", "cost", "cold"):
        p = H.params_from_dict(dict(b.params, top_k=k, rng_seed=9))
        MM = cold_M if mode == "cold" else M
        offs = np.arange(tracks + 1, dtype=np.int64) * MM
        o = [torch.zeros(tracks * k, n, device="cuda"), torch.zeros(tracks * k, device="cuda"),
             torch.zeros(tracks * k, device="cuda"), torch.zeros(tracks * k, dtype=torch.uint8, device="cuda"),
             torch.zeros(tracks, dtype=torch.int32, device="cuda"), torch.zeros(tracks, dtype=torch.uint8, device="cuda")]
        prev = torch.as_tensor(np.repeat(paths[0], k, axis=0)).cuda()
        ref = torch.as_tensor(paths[0]).cuda()
        seeds = torch.zeros(n, tracks * MM, device="cuda")
        chosen, lat, solved = [paths[0]], [], 0
        for s in range(1, steps):
            keys = torch.as_tensor((np.arange(tracks) + s * tracks).astype(np.int32)).cuda()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if mode == "cold":
                H.hjcd_solve(ctx, [rb], sc, targets[s], offs, p, *o, target_keys=keys, stream=stream)
            else:
                H.hjcd_warm_seeds(ctx, rb, prev, k, MM, p, seeds, target_keys=keys, stream=stream)
                if mode == "near":
                    H.hjcd_solve_near(ctx, [rb], sc, targets[s], offs, p, ref, *o, seeds=seeds, target_keys=keys,
                                      stream=stream)
                else:
                    H.hjcd_solve(ctx, [rb], sc, targets[s], offs, p, *o, seeds=seeds, target_keys=keys, stream=stream)
            stream.synchronize()
            lat.append((time.perf_counter() - t0) * 1e3)
            solved += int(o[5].sum().item())
            prev = o[0].clone()
            ref = o[0].view(tracks, k, n)[:, 0].contiguous()
            chosen.append(ref.cpu().numpy())
        ch = np.asarray(chosen)
        move = np.abs(np.diff(ch, axis=0)).max(axis=2)
        out[mode] = {"seeds_per_pose": MM, "ms_per_pose_p50": round(float(np.percentile(lat, 50)), 3),
                     "ms_per_pose_p99": round(float(np.percentile(lat, 99)), 3),
                     "success_rate": round(solved / (tracks * (steps - 1)), 4),
                     "joint_move_per_step_rad": {"median": round(float(np.median(move)), 4),
                                                 "p99": round(float(np.percentile(move, 99)), 4),
                                                 "max": round(float(move.max()), 3)},
                     "steps_moving_over_0.5_rad": int((move > 0.5).sum())}
        log(f"tracking {mode}: {out[mode]}")
    rb.close()
    sc.close()
    return {"workload": f"tracking_panda_{tracks}_tracks_x_{steps}_poses", "top_k": k, "modes": out}


def _window_stats(info, mask, t0=None):
    """solves/s, p50 / p99 latency over the completed requests selected by
    `mask` (solves/s = targets solved / (last completion - start), start =
    t0 or the first arrival)."""
    sel = info[mask]
    if sel.shape[0] == 0:
        return {"requests": 0}
    lat = (sel["done_s"] - sel["arrival_s"]) * 1e3
    start = float(sel["arrival_s"].min()) if t0 is None else t0
    span = float(sel["done_s"].max()) - start
    solved = int(sel["n_solved"].sum())
    return {"requests": int(sel.shape[0]), "targets": int(sel["n_targets"].sum()), "targets_solved": solved,
            "solves_per_s": round(solved / span, 1) if span > 0 else None,
            "p50_latency_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_latency_ms": round(float(np.percentile(lat, 99)), 3), "span_s": round(span, 3)}


def serving(H, ctx, torch, rates, window, warm, prefix, slots, chunk, pipes, log):
    """Poisson request streams: the continuous-batching server on the whole
    stream (warm-up + window; statistics over the requests that arrive in the
    window) and both modes on the stream's first `prefix` requests (the same
    requests, same keys)."""
    from paper_2510_07514_amd import workload as W
    out = []
    for ri, rate in enumerate(rates):
        s = W.serving_stream(float(rate), warm + window)
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
        del qd, pose
        offs = np.concatenate([[0], np.cumsum(s["n_targets"])])
        params = H.params_from_dict(s["params"])
        n_pre = min(n_req, prefix)
        row = {"rate_req_s": rate, "requests": int(n_req), "targets": int(offs[-1]),
               "mean_targets_per_request": round(float(np.mean(s["n_targets"])), 2),
               "mean_seeds_per_target": round(float(np.mean(s["seeds_per_target"])), 1),
               "window_s": window, "warmup_s": warm, "same_prefix_requests": int(n_pre)}
        if ri == 0:
            # kernel loading and first-touch allocation outside every measurement
            for mode in (H.HJCD_SERVE_BATCHED, H.HJCD_SERVE_PLAIN):
                srv = H.hjcd_server_create(ctx, rb, sc, params, mode=mode, max_slots=slots, chunk_iters=chunk,
                                           pipelines=pipes)
                for i in range(min(n_req, 32)):
                    H.hjcd_server_submit(srv, poses[offs[i]:offs[i + 1]], int(s["seeds_per_target"][i]), int(offs[i]),
                                         0.0)
                H.hjcd_server_start(srv)
                H.hjcd_server_wait(srv, 120.0)
                srv.close()
        infos = {}
        for mode, name, m in ((H.HJCD_SERVE_BATCHED, "served", n_req), (H.HJCD_SERVE_PLAIN, "plain", n_pre)):
            srv = H.hjcd_server_create(ctx, rb, sc, params, mode=mode, max_slots=slots, chunk_iters=chunk,
                                       max_queue=m + 1, pipelines=pipes)
            for i in range(m):
                H.hjcd_server_submit(srv, poses[offs[i]:offs[i + 1]], int(s["seeds_per_target"][i]), int(offs[i]),
                                     float(s["arrival"][i]))
            t0 = time.perf_counter()
            H.hjcd_server_start(srv)
            H.hjcd_server_wait(srv, 900.0)
            wall = time.perf_counter() - t0
            st = H.hjcd_server_get_stats(srv)
            info = H.hjcd_server_poll_all(srv)
            srv.close()
            info = info[np.argsort(info["tag"], kind="stable")]  # tag = first target index: arrival order
            infos[name] = info
            log(f"serving {name} at {rate} req/s: {m} requests in {wall:.1f} s, {int(st['chunks'])} chunks")
            if name == "served":
                row["served_window"] = dict(_window_stats(info, info["arrival_s"] >= warm, t0=warm),
                                            chunks=int(st["chunks"]),
                                            mean_resident_slots=round(st["mean_resident_slots"], 1),
                                            resident_slots_peak=int(st["resident_slots_peak"]),
                                            overlapped_steps=int(st["overlapped_steps"]))
        pre = np.arange(n_req) < n_pre
        row["served_same_prefix"] = _window_stats(infos["served"], pre)
        row["plain_same_prefix"] = _window_stats(infos["plain"], np.ones(infos["plain"].shape[0], bool))
        a, b = row["served_same_prefix"]["solves_per_s"], row["plain_same_prefix"]["solves_per_s"]
        row["speedup_vs_plain"] = round(a / b, 2) if a and b else None
        log(f"serving at {rate} req/s: {json.dumps(row)}")
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
    ap.add_argument("--cpu-targets", type=int, default=1000)
    ap.add_argument("--cpu-single-targets", type=int, default=64)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-uneven", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the 100,000 x 256 random 20-joint workload")
    ap.add_argument("--no-dof", action="store_true", help="skip the DoF-scaling chains")
    ap.add_argument("--no-resample", action="store_true", help="skip the paper-mode resampling sweep")
    ap.add_argument("--no-tracking", action="store_true", help="skip the path-tracking runs")
    ap.add_argument("--no-tiny", action="store_true", help="skip the 8 x 64 latency case (profiling runs)")
    ap.add_argument("--serve-rates", default="2000,10000,50000")
    ap.add_argument("--headline-rate", type=int, default=10000)
    ap.add_argument("--serve-window", type=float, default=10.0, help="seconds of each measured request window")
    ap.add_argument("--serve-warmup", type=float, default=1.0, help="seconds of stream before the window")
    ap.add_argument("--serve-prefix", type=int, default=10000,
                    help="first requests of each stream run by both modes (the same-request comparison)")
    ap.add_argument("--serve-slots", type=int, default=1 << 22, help="resident seed slots of the server")
    ap.add_argument("--serve-chunk", type=int, default=20,
                    help="iterations per serving chunk (20 = a whole stage at the default iterations)")
    ap.add_argument("--serve-pipelines", type=int, default=2,
                    help="scheduler steps of the server in flight at once (1-4)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run plain device copies of MIB MiB (scales the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): this build has no multi-GPU path",
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

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    ctx = H.hjcd_ctx_create(0)
    batch = W.config_batched(T=args.targets, M=args.seeds, host_seeds=False)
    m = measure(H, ctx, torch, batch, args.steps, args.warmup)
    m["workload"] = f"batched_panda_{batch.T}x{args.seeds}"
    log(f"batched: {json.dumps(m)}")
    rob = batch.robots[0]
    line = {
        "metric": "collision-free IK solves/s at 1mm/1deg + p50/p99 latency, served vs plain",
        "value": None,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "step_workload": m["workload"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
    }
    scene_note = ("obstacle centres uniform in the stated cube, rejected within 0.3 m of the base and in the "
                  "column |c_xy| < 0.25 m, z < 0.55 m above it")
    if not args.no_serve:
        rates = [int(x) for x in args.serve_rates.split(",") if x]
        if args.headline_rate not in rates:
            rates.append(args.headline_rate)
        sv = serving(H, ctx, torch, rates, args.serve_window, args.serve_warmup, args.serve_prefix,
                     args.serve_slots, args.serve_chunk, args.serve_pipelines, log)
        head = next(r for r in sv if r["rate_req_s"] == args.headline_rate)
        line["value"] = head["served_window"]["solves_per_s"]
        line["p50_latency_ms"] = head["served_window"]["p50_latency_ms"]
        line["p99_latency_ms"] = head["served_window"]["p99_latency_ms"]
        line["plain"] = head["plain_same_prefix"]
        line["served_same_prefix"] = head["served_same_prefix"]
        line["speedup_vs_plain"] = head["speedup_vs_plain"]
        line["config"] = {"workload": f"serving_poisson_{args.headline_rate}_req_s_panda_1-16_targets_32-1024_seeds",
                          "rate_req_s": args.headline_rate, "window_s": args.serve_window,
                          "warmup_s": args.serve_warmup, "same_prefix_requests": head["same_prefix_requests"],
                          "dof": rob.dof, "link_spheres": int(rob.sphere_link.shape[0]),
                          "obstacle_spheres": int(batch.scene.spheres.shape[0]), "top_k": 1,
                          "chunk_iters": args.serve_chunk, "pipelines": args.serve_pipelines,
                          "max_slots": args.serve_slots,
                          "cd_sweeps": 20, "polish_iters": 20, "scene": scene_note}
        line["serving"] = sv
    else:
        line["value"] = m["value"]
        line["config"] = {"workload": m["workload"], "scene": scene_note}
    line["batched"] = dict(m, config={"targets": batch.T, "seeds_per_target": args.seeds, "dof": rob.dof,
                                      "link_spheres": int(rob.sphere_link.shape[0]),
                                      "obstacle_spheres": int(batch.scene.spheres.shape[0]),
                                      "top_k": batch.params["top_k"], "cd_sweeps": batch.params["cd_sweeps"],
                                      "polish_iters": batch.params["polish_iters"]})
    if not args.no_tiny:
        tb = W.config_tiny(host_seeds=False)
        mt = measure(H, ctx, torch, tb, 50, 5)
        line["tiny"] = {"workload": "tiny_panda_8x64", "ms_per_solve": mt["ms_per_step"],
                        "latency_ms": mt["latency_ms"], "solved_targets": mt["solved_targets"],
                        "stage_ms": mt["stage_ms"]}
        log(f"tiny: {line['tiny']}")
    if not args.no_uneven:
        line["uneven"] = uneven(H, ctx, torch, 5, log)
    if not args.no_large:
        lb = W.config_large()
        ml = measure(H, ctx, torch, lb, 3, 1)
        line["large"] = dict({"workload": f"large_random20_{lb.T}x{int(lb.seed_offsets[1])}",
                              "top_k": lb.params["top_k"], "cd_sweeps": lb.params["cd_sweeps"],
                              "polish_iters": lb.params["polish_iters"], "obstacle_spheres": 128,
                              "obstacle_boxes": 128, "scene": scene_note}, **ml)
        log(f"large: {line['large']}")
    if not args.no_dof:
        line["dof_scaling"] = dof_scaling(H, ctx, torch, log)
    if not args.no_tracking:
        line["tracking"] = tracking(H, ctx, torch, log)
    if not args.no_resample:
        line["resampling"] = {"workload": m["workload"], "rows": resampling(H, ctx, torch, batch, log)}
    per_unit = None
    if not args.no_cpu:
        cb, per_unit = cpu_baseline(batch, min(args.cpu_targets, batch.T), min(args.cpu_single_targets, batch.T))
        line["cpu_baseline"] = cb
        log(f"cpu baseline: {cb}")
    line["roofline"] = roofline(m, per_unit, rob.dof)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
