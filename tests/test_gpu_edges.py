"""GPU edge cases of the whole solve through the C ABI, against the oracle:
ragged and empty seed counts, top-k beyond the seed count, an empty batch,
the smallest and the largest chains, and a seed that already solves its
target."""
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


def _solve(H, ctx, rob, scene, tg, offs, params, seeds=None):
    import torch
    T, k, n = len(tg), params["top_k"], rob.dof
    o = dict(q=torch.zeros(max(T * k, 1), n, device="cuda"), ep=torch.zeros(max(T * k, 1), device="cuda"),
             eo=torch.zeros(max(T * k, 1), device="cuda"),
             fl=torch.zeros(max(T * k, 1), dtype=torch.uint8, device="cuda"),
             nf=torch.zeros(max(T, 1), dtype=torch.int32, device="cuda"),
             sv=torch.zeros(max(T, 1), dtype=torch.uint8, device="cuda"))
    rb = H.hjcd_load_robot(ctx, rob)
    sc = H.hjcd_load_scene(ctx, scene.spheres, scene.boxes)
    targets = torch.as_tensor(np.ascontiguousarray(np.asarray(tg, np.float32).reshape(-1, 7).T)).cuda() if T else \
        torch.zeros(7, 1, device="cuda")
    sd = None if seeds is None else torch.as_tensor(np.ascontiguousarray(seeds, np.float32)).cuda()
    H.hjcd_solve(ctx, [rb], sc, targets, offs, H.params_from_dict(params), o["q"], o["ep"], o["eo"], o["fl"],
                 o["nf"], o["sv"], seeds=sd)
    torch.cuda.synchronize()
    return {kk: v.cpu().numpy() for kk, v in o.items()}


def _check_against_oracle(rob, scene, tg, offs, params, g, max_disagree=0, seeds=None):
    T, k, n = len(tg), params["top_k"], rob.dof
    ref = O.solve(rob, scene, np.asarray(tg, np.float64), offs, params,
                  seeds=None if seeds is None else seeds[:n].T.astype(np.float64))
    disagree = int(np.sum(g["sv"][:T] != ref["solved"]))
    say(f"  solved gpu {g['sv'][:T].tolist()} oracle {ref['solved'].tolist()}")
    assert disagree <= max_disagree
    for t in range(T):
        M = int(offs[t + 1] - offs[t])
        for r in range(k):
            slot = t * k + r
            if r >= M:
                # fewer seeds than k: the remaining slots are empty
                assert g["fl"][slot] == 255 and np.isinf(g["ep"][slot])
                continue
            assert g["fl"][slot] in (0, 1)
            f = O.fk(rob, g["q"][slot].astype(np.float64))
            e = O.residual(np.asarray(tg[t][:3], np.float64), np.asarray(tg[t][3:], np.float64), f["p_ee"],
                           f["R_ee"])
            assert abs(np.linalg.norm(e["rp"]) - g["ep"][slot]) < 2e-5
        assert g["nf"][t] <= M
    return ref


def test_ragged_and_empty_targets(H, ctx):
    """Seed counts 0, 1, 63, 64, 65, 130 in one batch (waves straddle targets,
    a target with no seeds), top-4."""
    say("case: ragged and empty seed counts")
    b = W.config_tiny(host_seeds=False)
    rob = b.robots[0]
    counts = np.array([0, 1, 63, 64, 65, 130])
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    tg = O.targets_from_qstar(rob, b.q_star[:6])
    params = dict(b.params, top_k=4)
    g = _solve(H, ctx, rob, b.scene, tg, offs, params)
    assert g["sv"][0] == 0 and g["nf"][0] == 0 and np.all(g["fl"][0:4] == 255)
    _check_against_oracle(rob, b.scene, tg, offs, params, g, max_disagree=1)


def test_empty_batch_is_a_no_op(H, ctx):
    say("case: T = 0")
    b = W.config_tiny(host_seeds=False)
    g = _solve(H, ctx, b.robots[0], b.scene, np.zeros((0, 7), np.float32), np.zeros(1, np.int64), b.params)
    assert g["sv"].shape == (1,)


def test_one_joint_chain(H, ctx):
    """A single revolute joint with a 0.5 m link: every target on its circle
    is reachable exactly in position and orientation."""
    say("case: 1-DoF chain")
    rob = W.planar_chain([0.5], limit=3.0)
    rng = np.random.default_rng(5)
    qs = rng.uniform(-3, 3, size=(6, 1)).astype(np.float32)
    tg = O.targets_from_qstar(rob, qs)
    offs = np.arange(7, dtype=np.int64) * 64
    params = W.default_params(top_k=2, rng_seed=9)
    g = _solve(H, ctx, rob, W.empty_scene(), tg, offs, params)
    assert g["sv"].sum() == 6
    _check_against_oracle(rob, W.empty_scene(), tg, offs, params, g)
    best = g["q"].reshape(6, 2, 1)[:, 0, 0]
    assert np.all(np.abs(best - qs[:, 0]) < 1e-3)


def test_thirty_two_joint_chain(H, ctx):
    """The largest chain the ABI takes (32 joints, the 32-joint bucket)."""
    say("case: 32-DoF chain")
    rng = np.random.default_rng(32)
    rob = W.random_chain(rng, 32, "random32")
    tg = O.targets_from_qstar(rob, W.uniform_configs(rng, rob, 4))
    offs = np.arange(5, dtype=np.int64) * 96
    params = W.default_params(top_k=2, rng_seed=3, cd_sweeps=10, polish_iters=10)
    g = _solve(H, ctx, rob, W.empty_scene(), tg, offs, params)
    _check_against_oracle(rob, W.empty_scene(), tg, offs, params, g, max_disagree=1)


def test_seed_that_already_solves(H, ctx):
    """Seed 0 of each target is its q*: it passes both exit tests before the
    first iteration, so a collision-free one solves its target."""
    say("case: converged seed")
    b = W.config_tiny(host_seeds=True)
    rob = b.robots[0]
    seeds = b.seeds.copy()
    for t in range(b.T):
        seeds[:rob.dof, t * 64] = np.asarray(b.q_star[t], np.float32)
    tg = O.targets_from_qstar(rob, b.q_star)
    g = _solve(H, ctx, rob, b.scene, tg, b.seed_offsets, b.params, seeds=seeds)
    ref = _check_against_oracle(rob, b.scene, tg, b.seed_offsets, b.params, g, max_disagree=0, seeds=seeds)
    for t in range(b.T):
        if ref["flag_seed"][t * 64] == 0:
            assert g["sv"][t] == 1 and g["ep"][t] < 1e-5


def test_handles_outlive_their_context(H):
    """A robot and a scene destroyed after their context leave no HIP error
    behind in the caller's thread (the next torch kernel launch checks)."""
    import torch
    say("case: robot and scene destroyed after the context")
    b = W.config_tiny(host_seeds=False)
    c2 = H.hjcd_ctx_create(0)
    rb = H.hjcd_load_robot(c2, b.robots[0])
    sc = H.hjcd_load_scene(c2, b.scene.spheres, b.scene.boxes)
    c2.close()
    rb.close()
    sc.close()
    x = torch.ones(1000, device="cuda")
    assert float(x.sum().item()) == 1000.0


def test_bitwise_repeatable(H, ctx):
    """The same batch solved twice in one context, and once more in a fresh
    context on another stream, gives bit-identical outputs: no result depends
    on wave scheduling, atomics order or leftover device state."""
    import torch
    say("case: bitwise repeatability, 64 targets x 1024 seeds")
    b = W.config_batched(T=64, M=1024)
    rob = b.robots[0]
    tg = O.targets_from_qstar(rob, b.q_star)
    runs = [_solve(H, ctx, rob, b.scene, tg, b.seed_offsets, b.params) for _ in range(2)]
    c2 = H.hjcd_ctx_create(0)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        k, n, T = b.params["top_k"], rob.dof, b.T
        o = [torch.zeros(T * k, n, device="cuda"), torch.zeros(T * k, device="cuda"), torch.zeros(T * k, device="cuda"),
             torch.zeros(T * k, dtype=torch.uint8, device="cuda"), torch.zeros(T, dtype=torch.int32, device="cuda"),
             torch.zeros(T, dtype=torch.uint8, device="cuda")]
        rb = H.hjcd_load_robot(c2, rob)
        sc = H.hjcd_load_scene(c2, b.scene.spheres, b.scene.boxes)
        targets = torch.as_tensor(np.ascontiguousarray(np.asarray(tg, np.float32).T)).cuda()
        H.hjcd_solve(c2, [rb], sc, targets, b.seed_offsets, H.params_from_dict(b.params), *o, stream=s)
    s.synchronize()
    runs.append(dict(zip(("q", "ep", "eo", "fl", "nf", "sv"), [x.cpu().numpy() for x in o])))
    rb.close()
    sc.close()
    c2.close()
    say(f"  solved {int(runs[0]['sv'].sum())} of {T}")
    for r in runs[1:]:
        for key in ("q", "ep", "eo", "fl", "nf", "sv"):
            assert np.array_equal(runs[0][key], r[key]), key


@pytest.mark.parametrize("robot", ["panda", "random24"])
def test_statistics_modes_bit_identical(H, ctx, robot):
    """collect_stats 0 (no statistics), 1 (stage times and work counts: the
    per-seed kernels built with counters) and 2 (stage times only) return the
    same outputs bit for bit; counts are reported in mode 1 only."""
    import torch
    say(f"case: statistics modes, {robot}")
    if robot == "panda":
        b = W.config_batched(T=64, M=1024)
        rob, scene, params, offs = b.robots[0], b.scene, b.params, b.seed_offsets
        tg = O.targets_from_qstar(rob, b.q_star)
    else:
        rob = W.random_chain(np.random.default_rng(24), 24)
        scene = W.config_batched(T=1, M=1).scene
        params = W.default_params(top_k=4)
        T = 32
        tg = O.targets_from_qstar(rob, W.uniform_configs(np.random.default_rng(3), rob, T))
        offs = np.arange(T + 1, dtype=np.int64) * 512
    T, k, n = len(tg), params["top_k"], rob.dof
    rb = H.hjcd_load_robot(ctx, rob)
    sc = H.hjcd_load_scene(ctx, scene.spheres, scene.boxes)
    targets = torch.as_tensor(np.ascontiguousarray(np.asarray(tg, np.float32).reshape(-1, 7).T)).cuda()
    outs, stats = [], []
    for mode in (0, 1, 2):
        o = [torch.zeros(T * k, n, device="cuda"), torch.zeros(T * k, device="cuda"), torch.zeros(T * k, device="cuda"),
             torch.zeros(T * k, dtype=torch.uint8, device="cuda"), torch.zeros(T, dtype=torch.int32, device="cuda"),
             torch.zeros(T, dtype=torch.uint8, device="cuda")]
        H.hjcd_solve(ctx, [rb], sc, targets, offs, H.params_from_dict(params, collect_stats=mode), *o)
        stats.append(H.hjcd_get_stats(ctx) if mode else None)
        torch.cuda.synchronize()
        outs.append([x.cpu().numpy() for x in o])
    rb.close()
    sc.close()
    for r in outs[1:]:
        for a, c in zip(outs[0], r):
            assert np.array_equal(a, c)
    s1, s2 = stats[1], stats[2]
    say(f"  mode 1: ms_polish {s1['ms_polish']:.3f} pol_iters {s1['pol_iters']}; mode 2: ms_polish "
        f"{s2['ms_polish']:.3f} pol_iters {s2['pol_iters']}")
    assert s1["pol_iters"] > 0 and s1["cd_iters"] > 0 and s1["pol_trials"] >= s1["pol_iters"]
    assert s2["ms_polish"] > 0 and s2["ms_cd"] > 0
    assert all(s2[kk] == 0 for kk in ("cd_iters", "pol_iters", "pol_trials", "pol_dogleg", "coll_coarse"))
