"""Tracking (Sec. V demonstration: poses along a path, each solved from the
previous solution set, the solution nearest the current configuration
returned) through the C ABI: warm-start seeds and the nearest-solution
selection against the oracle, the whole tracking solve against its stages,
and continuity along paths."""
import numpy as np
import pytest

import oracle as O
from gpu_common import cuda, say, soa, targets_soa
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


def _sync():
    import torch
    torch.cuda.synchronize()


def test_warm_seeds_match_oracle(H, ctx):
    import torch
    say("case: warm-start seeds vs oracle")
    rob = W.panda_like()
    rb = H.hjcd_load_robot(ctx, rob)
    rng = np.random.default_rng(12)
    T, k, M, ns = 5, 8, 150, 9  # row stride beyond the dof (mixed-dof outputs)
    q_prev = np.zeros((T * k, ns), np.float32)
    q_prev[:, :7] = W.uniform_configs(rng, rob, T * k)
    q_prev[3, 1] = 5.0  # clipped
    keys = np.array([4, 99, 0, 17, 2 ** 31 + 1], np.uint32)
    pd = W.default_params(rng_seed=77, sigma=0.04, mu=0.001)
    out = torch.zeros(7, T * M, device="cuda")
    H.hjcd_warm_seeds(ctx, rb, cuda(q_prev), k, M, H.params_from_dict(pd), out, target_keys=cuda(keys.view(np.int32)))
    _sync()
    g = out.cpu().numpy().T
    ref = O.warm_seeds(rob, q_prev[:, :7].astype(np.float64), k, M, pd, target_keys=keys)
    d = np.abs(g - ref).max()
    say(f"  {T * M} seeds, max |gpu - oracle| {d:.2e}")
    assert d < 2e-6
    # seeds m < k are the previous solutions themselves (clipped), bit for bit
    for t in range(T):
        np.testing.assert_array_equal(g[t * M:t * M + k], np.clip(q_prev[t * k:(t + 1) * k, :7],
                                                                   rob.q_min.astype(np.float32),
                                                                   rob.q_max.astype(np.float32)))


def test_select_near_exact(H, ctx):
    import torch
    say("case: nearest-solution selection vs oracle")
    rng = np.random.default_rng(13)
    counts = np.array([0, 1, 5, 64, 65, 700, 7])
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    S, T, n, ns, k = int(offs[-1]), len(counts), 7, 8, 6
    cost = (rng.integers(0, 50, size=S) * 0.125).astype(np.float32)
    flag = rng.integers(0, 2, size=S).astype(np.uint8)
    ep = rng.uniform(0, 2e-3, size=S).astype(np.float32)
    eo = rng.uniform(0, 0.03, size=S).astype(np.float32)
    q = (rng.integers(-16, 16, size=(n, S)) / 8.0).astype(np.float32)  # exact squared distances, ties
    q_ref = np.zeros((T, ns), np.float32)
    q_ref[:, :n] = rng.integers(-16, 16, size=(T, n)) / 8.0
    p = H.hjcd_params_default(top_k=k)
    outs = dict(q=torch.zeros(T * k, ns, device="cuda"), ep=torch.zeros(T * k, device="cuda"),
                eo=torch.zeros(T * k, device="cuda"), fl=torch.zeros(T * k, dtype=torch.uint8, device="cuda"),
                nf=torch.zeros(T, dtype=torch.int32, device="cuda"), sv=torch.zeros(T, dtype=torch.uint8, device="cuda"))
    H.hjcd_select_near(ctx, offs, n, ns, p, cuda(q), cuda(cost), cuda(ep), cuda(eo), cuda(flag), cuda(q_ref),
                       outs["q"], outs["ep"], outs["eo"], outs["fl"], outs["nf"], outs["sv"])
    _sync()
    o = {kk: v.cpu().numpy() for kk, v in outs.items()}
    sp, so = float(np.float32(1e-3)), float(np.float32(np.pi / 180))
    for t in range(T):
        b0, M = int(offs[t]), int(counts[t])
        order = O.select_near(flag[b0:b0 + M].astype(np.int32), cost[b0:b0 + M].astype(np.float64),
                              ep[b0:b0 + M].astype(np.float64), eo[b0:b0 + M].astype(np.float64),
                              q[:, b0:b0 + M].T.astype(np.float64), q_ref[t, :n].astype(np.float64), k, sp, so)
        assert o["nf"][t] == int((flag[b0:b0 + M] == 0).sum())
        solved = 0
        for r in range(k):
            slot = t * k + r
            m = order[r]
            if m < 0:
                assert o["fl"][slot] == 255
                continue
            s = b0 + m
            assert np.array_equal(o["q"][slot, :n], q[:, s]) and np.all(o["q"][slot, n:] == 0), (t, r)
            assert o["ep"][slot] == ep[s] and o["fl"][slot] == flag[s]
            solved |= int(flag[s] == 0 and ep[s] <= sp and eo[s] <= so)
        assert o["sv"][t] == solved


def _fk_targets(rob, q):
    return O.targets_from_qstar(rob, q)


def test_solve_near_equals_its_stages(H, ctx):
    """hjcd_solve_near = PO-CCD, PJ-IK, collision and hjcd_select_near on
    the same warm seeds, bit for bit; and hjcd_solve on the same seeds
    returns the same per-target n_free and solved flags."""
    import torch
    say("case: tracking solve vs its stages")
    b = W.config_batched(T=1, M=1)
    rob = b.robots[0]
    n = rob.dof
    paths = W.tracking_paths(rob, 12, 2)
    T, k, M = 12, 8, 128
    rb = H.hjcd_load_robot(ctx, rob)
    sc = H.hjcd_load_scene(ctx, b.scene.spheres, b.scene.boxes)
    q_prev = np.repeat(paths[0], k, axis=0)  # the previous pose's configuration, k copies
    params = W.default_params(top_k=k, rng_seed=21)
    p = H.params_from_dict(params)
    seeds = torch.zeros(n, T * M, device="cuda")
    H.hjcd_warm_seeds(ctx, rb, cuda(q_prev), k, M, p, seeds)
    tg = targets_soa(_fk_targets(rob, paths[1]))
    q_ref = cuda(paths[0])
    offs = np.arange(T + 1, dtype=np.int64) * M

    def outs():
        return [torch.zeros(T * k, n, device="cuda"), torch.zeros(T * k, device="cuda"), torch.zeros(T * k, device="cuda"),
                torch.zeros(T * k, dtype=torch.uint8, device="cuda"), torch.zeros(T, dtype=torch.int32, device="cuda"),
                torch.zeros(T, dtype=torch.uint8, device="cuda")]

    whole = outs()
    H.hjcd_solve_near(ctx, [rb], sc, tg, offs, p, q_ref, *whole, seeds=seeds)
    plain = outs()
    H.hjcd_solve(ctx, [rb], sc, tg, offs, p, *plain, seeds=seeds)
    q = seeds.clone()
    ep, eo, cost = (torch.zeros(T * M, device="cuda") for _ in range(3))
    H.hjcd_cd(ctx, rb, tg, offs, p, q)
    H.hjcd_polish(ctx, rb, tg, offs, p, q, ep, eo, cost)
    fl = torch.zeros(T * M, dtype=torch.uint8, device="cuda")
    H.hjcd_collide(ctx, rb, sc, q, fl)
    chain = outs()
    H.hjcd_select_near(ctx, offs, n, n, p, q, cost, ep, eo, fl, q_ref, *chain)
    _sync()
    for nm, a, g in zip(("q", "err_p", "err_o", "flag", "n_free", "solved"), whole, chain):
        assert torch.equal(a, g), nm
    assert torch.equal(whole[4], plain[4]) and torch.equal(whole[5], plain[5])
    say(f"  solved {int(whole[5].sum())}/{T}")


def test_tracking_paths_continuous(H, ctx):
    """Sixteen Panda-like tracks, 40 poses each: every pose solved from the
    previous solution set (128 warm seeds), the returned solution nearest the
    previous one.  Along the path the nearest selection keeps the joint
    motion per step small; the cost selection on the same seeds jumps between
    solution branches more.  Sampled returned solutions reproduce their
    errors in the oracle's FK."""
    import torch
    say("case: tracking along paths")
    rob = W.panda_like()
    rob.min_link_gap = 0
    steps, T, k, M = 40, 16, 8, 128
    paths = W.tracking_paths(rob, T, steps, period=80)
    rb = H.hjcd_load_robot(ctx, rob)
    params = W.default_params(top_k=k, rng_seed=31)
    p = H.params_from_dict(params)
    offs = np.arange(T + 1, dtype=np.int64) * M
    jumps = {}
    for mode in ("near", "cost"):
        # the first pose from its own exact configuration (the robot starts there)
        cur = torch.as_tensor(np.repeat(paths[0], k, axis=0)).cuda()
        chosen = [paths[0]]
        solved = 0
        for s in range(1, steps):
            seeds = torch.zeros(rob.dof, T * M, device="cuda")
            H.hjcd_warm_seeds(ctx, rb, cur, k, M, p, seeds, target_keys=cuda((np.arange(T) + s * T).astype(np.int32)))
            tg = targets_soa(_fk_targets(rob, paths[s]))
            o = [torch.zeros(T * k, rob.dof, device="cuda"), torch.zeros(T * k, device="cuda"),
                 torch.zeros(T * k, device="cuda"), torch.zeros(T * k, dtype=torch.uint8, device="cuda"),
                 torch.zeros(T, dtype=torch.int32, device="cuda"), torch.zeros(T, dtype=torch.uint8, device="cuda")]
            if mode == "near":
                q_ref = cuda(chosen[-1])
                H.hjcd_solve_near(ctx, [rb], None, tg, offs, p, q_ref, *o, seeds=seeds)
            else:
                H.hjcd_solve(ctx, [rb], None, tg, offs, p, *o, seeds=seeds)
            _sync()
            qo = o[0].cpu().numpy().reshape(T, k, rob.dof)
            solved += int(o[5].sum().item())
            chosen.append(qo[:, 0].copy())
            cur = o[0]
            if s % 13 == 0:
                ep = o[1].cpu().numpy().reshape(T, k)
                for t in range(0, T, 5):
                    f = O.fk(rob, qo[t, 0].astype(np.float64))
                    tgt = _fk_targets(rob, paths[s][t:t + 1])[0].astype(np.float64)
                    e = O.residual(tgt[:3], tgt[3:], f["p_ee"], f["R_ee"])
                    assert abs(np.linalg.norm(e["rp"]) - ep[t, 0]) < 2e-5
        ch = np.asarray(chosen)
        step = np.abs(np.diff(ch, axis=0)).max(axis=2)  # [steps-1][T] largest joint move per step
        jumps[mode] = step
        say(f"  {mode}: solved {solved}/{T * (steps - 1)}, joint move per step: median {np.median(step):.4f}, "
            f"max {step.max():.3f} rad, steps moving > 0.5 rad: {int((step > 0.5).sum())}")
        assert solved >= 0.95 * T * (steps - 1)
    # the path moves each joint by at most 0.3 * 2 pi / 80 ~ 0.024 rad per step
    assert np.median(jumps["near"]) < 0.05
    assert (jumps["near"] > 0.5).sum() <= (jumps["cost"] > 0.5).sum()
    assert (jumps["near"] > 0.5).mean() < 0.02
