"""GPU tests of the serving loop (hjcd_server_*, through the C ABI):
continuous batching gives every request the result it gets alone, the
served decisions follow the serving rule applied to the FP64 oracle's
per-seed runs, and admission respects the slot pool."""
import numpy as np
import pytest

import oracle as O
from gpu_common import say
from paper_2510_07514_amd import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_07514_amd import hjcd
    return hjcd


@pytest.fixture(scope="module")
def ctx(H):
    c = H.hjcd_ctx_create(0)
    yield c
    c.close()


def _requests(rob, n_req, seed, max_targets=4, seeds=(32, 160)):
    rng = np.random.default_rng(seed)
    out, tag = [], 0
    for _ in range(n_req):
        k = int(rng.integers(1, max_targets + 1))
        m = int(rng.integers(seeds[0], seeds[1] + 1))
        tg = O.targets_from_qstar(rob, W.uniform_configs(rng, rob, k))
        out.append(dict(targets=tg, M=m, tag=tag))
        tag += k
    return out


def _serve(H, ctx, rb, sc, params, reqs, arrivals=None, one_by_one=False, timeout=60.0, **cfg):
    srv = H.hjcd_server_create(ctx, rb, sc, params, **cfg)
    H.hjcd_server_start(srv)
    ids, res = [], []
    for i, r in enumerate(reqs):
        t = 0.0 if arrivals is None else float(arrivals[i])
        ids.append(H.hjcd_server_submit(srv, r["targets"], r["M"], r["tag"], t))
        if one_by_one:
            H.hjcd_server_wait(srv, timeout)
    H.hjcd_server_wait(srv, timeout)
    infos = {}
    while True:
        got = H.hjcd_server_poll(srv, 256)
        if not got:
            break
        for g in got:
            infos[g["request_id"]] = g
    for i, r in zip(ids, reqs):
        res.append(H.hjcd_server_result(srv, i, len(r["targets"])))
    st = H.hjcd_server_get_stats(srv)
    srv.close()
    return res, [infos[i] for i in ids], st


def _load(H, ctx, rob, scene):
    rb = H.hjcd_load_robot(ctx, rob)
    sc = H.hjcd_load_scene(ctx, scene.spheres, scene.boxes)
    return rb, sc


def test_serve_alone_equals_mix(H, ctx):
    """Each request's served result is bit-identical whether it runs alone or
    batched with others (all arriving together, and under a slot pool small
    enough that requests wait for admission), and on one or four step
    pipelines with staggered arrivals."""
    say("case: serving alone vs mix")
    s = W.serving_stream(1000.0, 0.01)
    rob, scene = s["robot"], s["scene"]
    p = dict(s["params"], cd_sweeps=12, polish_iters=12)
    params = H.params_from_dict(p)
    rb, sc = _load(H, ctx, rob, scene)
    reqs = _requests(rob, 10, 7)
    alone, _, st_a = _serve(H, ctx, rb, sc, params, reqs, one_by_one=True, chunk_iters=3, max_slots=1 << 14)
    mix, info_m, st_m = _serve(H, ctx, rb, sc, params, reqs, chunk_iters=3, max_slots=1 << 14)
    small = max(((len(r["targets"]) * r["M"] + 63) // 64) * 64 for r in reqs)
    tight, info_t, st_t = _serve(H, ctx, rb, sc, params, reqs, chunk_iters=3, max_slots=small + 64)
    # arrivals spread over the steps, on one pipeline and on four (requests
    # admitted while other steps run start on the free pipelines)
    arr = np.arange(len(reqs)) * 2e-4
    one, _, st_1 = _serve(H, ctx, rb, sc, params, reqs, arrivals=arr, chunk_iters=3, max_slots=1 << 14, pipelines=1)
    four, _, st_4 = _serve(H, ctx, rb, sc, params, reqs, arrivals=arr, chunk_iters=3, max_slots=1 << 14, pipelines=4)
    # four pipelines sharing a pool that holds about two requests: admission waits for slots
    # that another pipeline's requests free
    four_t, _, st_4t = _serve(H, ctx, rb, sc, params, reqs, arrivals=arr, chunk_iters=3, max_slots=2 * small + 64,
                              pipelines=4)
    say(f"  chunks alone {st_a['chunks']} mix {st_m['chunks']} tight {st_t['chunks']} "
        f"staggered on 1 / 4 pipelines {st_1['chunks']} / {st_4['chunks']} "
        f"(overlapped {st_1['overlapped_steps']} / {st_4['overlapped_steps']}), tight on 4 {st_4t['chunks']} "
        f"(overlapped {st_4t['overlapped_steps']}); "
        f"peak slots mix {st_m['resident_slots_peak']} tight {st_t['resident_slots_peak']} (pool {st_t['max_slots']})")
    for i, r in enumerate(reqs):
        for other in (mix[i], tight[i], one[i], four[i], four_t[i]):
            for key in ("q", "err_p", "err_o", "flag"):
                assert np.array_equal(alone[i][key], other[key]), (i, key)
    assert all(st["completed"] == len(reqs) for st in (st_m, st_t, st_1, st_4, st_4t))
    assert st_t["resident_slots_peak"] <= st_t["max_slots"]
    assert st_4t["resident_slots_peak"] <= st_4t["max_slots"]
    # the mixed run really overlapped requests on the device
    assert st_m["resident_slots_peak"] > small
    assert st_m["chunks"] < st_a["chunks"]
    # one pipeline never overlaps steps; four did, and gave the same results
    assert st_1["overlapped_steps"] == 0 and st_4["overlapped_steps"] > 0


# Cost 0.5 (|r_p|^2 + phi^2) below which seeds have converged to single
# precision's floor: |r_p| and phi of about 1e-6 and less, where FP32 FK and
# residual rounding (~1e-7 m / rad) decides their order.
COST_FLOOR = 1e-12


def _served_reference(rob, scene, tg, M, tag, p, chunk):
    """The serving rule on oracle per-seed runs: uniform seed m of target k
    (key tag + k) through PO-CCD and PJ-IK.  A seed whose PJ-IK exit test
    first passes at iteration f is checked at the end of the first chunk
    ending at or after f; every seed is checked at the end.  The target is
    solved at the first chunk end with a checked collision-free seed within
    tolerance (its lowest (cost, index) such seed), else it returns its
    lowest (collision, cost, index) seed."""
    K = p["polish_iters"]
    out = []
    sh = O.SceneHandle(scene)
    ref = O.solve(rob, sh, np.asarray(tg, np.float64), np.arange(len(tg) + 1, dtype=np.int64) * M,
                  dict(p, top_k=1), seeds=None,
                  target_keys=np.arange(tag, tag + len(tg), dtype=np.uint32))
    bounds = list(range(chunk, K, chunk)) + [K]
    for k in range(len(tg)):
        key = tag + k
        fro = np.zeros(M, np.int64)
        for m in range(M):
            th0 = O.uniform_seed(rob, p["rng_seed"], m, key)
            r1 = O.cd(rob, tg[k], p, m, key, th0)
            r2 = O.polish(rob, tg[k], p, m, key, r1["theta"])
            assert np.allclose(r2["theta"], ref["q_seed"][k * M + m], atol=1e-12)
            f = r2["stats"]["frozen_at"]
            fro[m] = K + 1 if f < 0 else f
        sl = slice(k * M, (k + 1) * M)
        ep, eo = ref["errp_seed"][sl], ref["erro_seed"][sl]
        cost, flag = ref["cost_seed"][sl], ref["flag_seed"][sl]
        ok = (flag == 0) & (ep <= p["succ_pos"]) & (eo <= p["succ_ori"])
        pick, solved, cand = None, False, np.zeros(0, np.int64)
        for b in bounds:
            elig = ok & ((fro <= b) if b < K else True)
            if elig.any():
                idx = np.nonzero(elig)[0]
                pick = int(idx[np.lexsort((idx, cost[idx]))[0]])
                solved = True
                cand = idx
                break
        if pick is None:
            idx = np.arange(M)
            pick = int(np.lexsort((idx, cost, flag))[0])
        # seeds the rule could equally pick: eligible at the deciding chunk end
        # with a cost at the single-precision floor, like the pick's (their
        # order is decided by rounding, an order of equal keys)
        ties = cand[cost[cand] < COST_FLOOR] if cost[pick] < COST_FLOOR else np.array([pick])
        out.append(dict(seed=pick, solved=solved, q=ref["q_seed"][k * M + pick], flag=int(flag[pick]),
                        ep=ep[pick], eo=eo[pick], ties_q=ref["q_seed"][k * M + ties]))
    return out


@pytest.mark.parametrize("chunk", [3, 20])
def test_serve_matches_oracle_serving_rule(H, ctx, chunk):
    """Two requests of the tiny workload (8 targets x 64 seeds) served in
    chunks of 3 iterations (retirement at every third PJ-IK iteration) and of
    20 (one chunk per stage, the first PJ-IK chunk in the step that ends
    PO-CCD) against the serving rule on oracle runs."""
    say(f"case: serving vs oracle serving rule, chunks of {chunk}")
    b = W.config_tiny(host_seeds=False)
    rob = b.robots[0]
    p = dict(b.params)
    tg = O.targets_from_qstar(rob, b.q_star)
    M = 64
    reqs = [dict(targets=tg[:4], M=M, tag=0), dict(targets=tg[4:], M=M, tag=4)]
    rb, sc = _load(H, ctx, rob, b.scene)
    res, info, st = _serve(H, ctx, rb, sc, H.params_from_dict(p), reqs, chunk_iters=chunk, max_slots=4096)
    ref = _served_reference(rob, b.scene, tg[:4], M, 0, p, chunk) + \
        _served_reference(rob, b.scene, tg[4:], M, 4, p, chunk)
    q = np.concatenate([r["q"] for r in res])
    ep = np.concatenate([r["err_p"] for r in res])
    fl = np.concatenate([r["flag"] for r in res])
    agree = 0
    for t in range(8):
        same = np.max(np.abs(q[t] - ref[t]["q"])) < 1e-3 and int(fl[t]) == ref[t]["flag"]
        # or another of the seeds converged to the rounding floor that the
        # rule could equally pick
        tie = not same and int(fl[t]) == ref[t]["flag"] and bool(
            np.any(np.max(np.abs(ref[t]["ties_q"] - q[t][None, :]), axis=1) < 1e-3))
        say(f"  target {t}: ref seed {ref[t]['seed']} solved {ref[t]['solved']} ep {ref[t]['ep']:.2e}; "
            f"gpu ep {ep[t]:.2e} flag {fl[t]} same {same} floor tie {tie} ({len(ref[t]['ties_q'])} at the floor)")
        agree += same or tie
    assert agree >= 7
    n_solved = sum(i["n_solved"] for i in info)
    assert abs(n_solved - sum(r["solved"] for r in ref)) <= 1
    for t in range(8):
        f = O.fk(rob, q[t].astype(np.float64))
        r = O.residual(tg[t][:3].astype(np.float64), tg[t][3:].astype(np.float64), f["p_ee"], f["R_ee"])
        assert abs(np.linalg.norm(r["rp"]) - ep[t]) < 1e-5


def test_plain_mode_equals_solve(H, ctx):
    """The plain server runs each request as one hjcd_solve (top-1) with
    target keys tag + i: its results equal a direct call's."""
    import torch
    say("case: plain server vs hjcd_solve")
    s = W.serving_stream(1000.0, 0.01)
    rob, scene = s["robot"], s["scene"]
    p = dict(s["params"], cd_sweeps=8, polish_iters=8)
    params = H.params_from_dict(p)
    rb, sc = _load(H, ctx, rob, scene)
    reqs = _requests(rob, 4, 11)
    res, info, st = _serve(H, ctx, rb, sc, params, reqs, mode=H.HJCD_SERVE_PLAIN, max_slots=1 << 12)
    n = rob.dof
    for r, got in zip(reqs, res):
        T, M = len(r["targets"]), r["M"]
        targets = torch.as_tensor(np.ascontiguousarray(r["targets"].T)).cuda()
        keys = torch.as_tensor(np.arange(r["tag"], r["tag"] + T, dtype=np.uint32).view(np.int32)).cuda()
        q = torch.zeros(T, n, device="cuda")
        ep = torch.zeros(T, device="cuda")
        eo = torch.zeros(T, device="cuda")
        fl = torch.zeros(T, dtype=torch.uint8, device="cuda")
        nf = torch.zeros(T, dtype=torch.int32, device="cuda")
        sv = torch.zeros(T, dtype=torch.uint8, device="cuda")
        H.hjcd_solve(ctx, [rb], sc, targets, np.arange(T + 1, dtype=np.int64) * M, params, q, ep, eo, fl, nf, sv,
                     target_keys=keys)
        torch.cuda.synchronize()
        assert np.array_equal(q.cpu().numpy(), got["q"])
        assert np.array_equal(ep.cpu().numpy(), got["err_p"])
        assert np.array_equal(fl.cpu().numpy(), got["flag"])


def test_server_rejects_bad_requests(H, ctx):
    say("case: server argument checks")
    s = W.serving_stream(1000.0, 0.01)
    rob, scene = s["robot"], s["scene"]
    params = H.params_from_dict(s["params"])
    rb, sc = _load(H, ctx, rob, scene)
    srv = H.hjcd_server_create(ctx, rb, sc, params, max_slots=256, max_targets=8)
    tg = O.targets_from_qstar(rob, W.uniform_configs(np.random.default_rng(0), rob, 2))
    with pytest.raises(H.HJCDError) as e:
        H.hjcd_server_submit(srv, tg, 200, 0, 0.0)  # 400 seeds > 256 slots
    assert e.value.status == H.HJCD_E_NOMEM
    bad = tg.copy()
    bad[0, 3:] = 0
    with pytest.raises(H.HJCDError) as e:
        H.hjcd_server_submit(srv, bad, 8, 0, 0.0)
    assert e.value.status == H.HJCD_E_INVALID
    with pytest.raises(H.HJCDError):
        H.hjcd_server_result(srv, 12345, 1)
    srv.close()
    with pytest.raises(H.HJCDError):
        H.hjcd_server_create(ctx, rb, sc, H.params_from_dict(dict(s["params"], polish_iters=0)))
    with pytest.raises(H.HJCDError):
        H.hjcd_server_create(ctx, rb, sc, params, chunk_iters=0)
    # a memory budget is a cap: the pool is the whole 64-slot blocks within
    # it, and a budget below one block is refused
    per_slot = 4 * (rob.dof + 3) + 9
    with pytest.raises(H.HJCDError) as e:
        H.hjcd_server_create(ctx, rb, sc, params, hbm_budget=per_slot * 63)
    assert e.value.status == H.HJCD_E_NOMEM
    srv = H.hjcd_server_create(ctx, rb, sc, params, hbm_budget=per_slot * 200)
    assert H.hjcd_server_get_stats(srv)["max_slots"] == 192
    srv.close()


def test_serving_stream_latency_accounting(H, ctx):
    """A short Poisson stream: every request completes, latencies are
    done - arrival >= 0 with admission after arrival, and the pool never
    holds more than its slots."""
    say("case: serving stream accounting")
    s = W.serving_stream(2000.0, 0.05)
    rob, scene = s["robot"], s["scene"]
    params = H.params_from_dict(s["params"])
    rb, sc = _load(H, ctx, rob, scene)
    reqs = []
    tag = 0
    for i in range(len(s["arrival"])):
        tg = O.targets_from_qstar(rob, s["q_star"][i])
        reqs.append(dict(targets=tg, M=int(s["seeds_per_target"][i]), tag=tag))
        tag += len(tg)
    res, info, st = _serve(H, ctx, rb, sc, params, reqs, arrivals=s["arrival"], chunk_iters=4,
                           max_slots=1 << 16)
    say(f"  {len(reqs)} requests, p50 {st['p50_latency_ms']:.2f} ms p99 {st['p99_latency_ms']:.2f} ms, "
        f"solved {st['targets_solved']}/{st['targets_done']}, peak slots {st['resident_slots_peak']}")
    assert st["completed"] == len(reqs)
    assert st["targets_done"] == sum(len(r["targets"]) for r in reqs)
    assert st["resident_slots_peak"] <= st["max_slots"]
    for i in info:
        assert i["admitted_s"] >= i["arrival_s"] - 1e-9 and i["done_s"] >= i["admitted_s"]
    assert 0 < st["p50_latency_ms"] <= st["p99_latency_ms"]
    for r, got in zip(reqs, res):
        ok = (got["flag"] == 0) & (got["err_p"] <= 1e-3) & (got["err_o"] <= np.float32(np.pi / 180))
        assert ok.sum() == next(x["n_solved"] for x in info if x["tag"] == r["tag"])


def test_serve_long_chain(H, ctx):
    """A 24-joint chain through the serving loop (the bucket whose chunks keep
    the spread line search, single-coordinate trials and both stages'
    perturbations in LDS): alone equals mixed bit for bit, and the results
    follow the serving rule on the oracle's per-seed runs."""
    say("case: serving a 24-joint chain")
    rob = W.random_chain(np.random.default_rng(24), 24)
    scene = W.config_batched(T=1, M=1).scene
    p = dict(W.default_params(top_k=1), cd_sweeps=12, polish_iters=12)
    params = H.params_from_dict(p)
    rb, sc = _load(H, ctx, rob, scene)
    reqs = _requests(rob, 4, 21, max_targets=2, seeds=(32, 64))
    alone, _, _ = _serve(H, ctx, rb, sc, params, reqs, one_by_one=True, chunk_iters=3, max_slots=1 << 13)
    mix, info, st = _serve(H, ctx, rb, sc, params, reqs, chunk_iters=3, max_slots=1 << 13)
    for i in range(len(reqs)):
        for key in ("q", "err_p", "err_o", "flag"):
            assert np.array_equal(alone[i][key], mix[i][key]), (i, key)
    agree = total = 0
    for r, got in zip(reqs, mix):
        ref = _served_reference(rob, scene, r["targets"], r["M"], r["tag"], p, 3)
        for t in range(len(r["targets"])):
            same = np.max(np.abs(got["q"][t] - ref[t]["q"])) < 1e-3 and int(got["flag"][t]) == ref[t]["flag"]
            tie = not same and int(got["flag"][t]) == ref[t]["flag"] and bool(
                np.any(np.max(np.abs(ref[t]["ties_q"] - got["q"][t][None, :]), axis=1) < 1e-3))
            say(f"  target {r['tag'] + t}: ref solved {ref[t]['solved']} ep {ref[t]['ep']:.2e}; "
                f"gpu ep {got['err_p'][t]:.2e} same {same} floor tie {tie}")
            agree += same or tie
            total += 1
    assert agree >= total - 1
