"""GPU tests of reusable plans (hjcd_plan_*, through the C ABI): a graph
replay of an uneven multi-robot batch gives what the eager hjcd_solve gives,
on every replay, with and without autotuning."""
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


def _setup(H, ctx, b):
    import torch
    rbs = [H.hjcd_load_robot(ctx, r) for r in b.robots]
    sc = H.hjcd_load_scene(ctx, b.scene.spheres, b.scene.boxes)
    tg = np.concatenate([O.targets_from_qstar(b.robots[b.robot_of_target[t]], [b.q_star[t]]) for t in range(b.T)])
    targets = torch.as_tensor(np.ascontiguousarray(tg.T)).cuda()
    return rbs, sc, targets


def _outs(T, k, n_max):
    import torch
    return [torch.zeros(T * k, n_max, device="cuda"), torch.zeros(T * k, device="cuda"),
            torch.zeros(T * k, device="cuda"), torch.zeros(T * k, dtype=torch.uint8, device="cuda"),
            torch.zeros(T, dtype=torch.int32, device="cuda"), torch.zeros(T, dtype=torch.uint8, device="cuda")]


def _host(outs):
    import torch
    torch.cuda.synchronize()
    return [o.cpu().numpy().copy() for o in outs]


@pytest.mark.parametrize("tune", [False, True])
def test_plan_replays_equal_eager_solve(H, ctx, tune):
    import torch
    say(f"case: plan replay vs eager solve, tune={tune}")
    b = W.config_uneven(T=48, max_seeds=300)
    rbs, sc, targets = _setup(H, ctx, b)
    k, n_max = b.params["top_k"], b.n_max
    p = H.params_from_dict(b.params)
    ref = _outs(b.T, k, n_max)
    H.hjcd_solve(ctx, rbs, sc, targets, b.seed_offsets, p, *ref, robot_of_target=b.robot_of_target)
    ref = _host(ref)
    outs = _outs(b.T, k, n_max)
    plan = H.hjcd_plan_create(ctx, rbs, sc, targets, b.seed_offsets, p, *outs, robot_of_target=b.robot_of_target,
                              tune=tune)
    for r in range(len(b.robots)):
        ch = H.hjcd_plan_choice(plan, r)
        say(f"  robot {r}: {ch}")
        assert ch["variant"] in (0, 1) and ch["block_threads"] in (64, 128, 256)
        assert ch["seeds"] == sum(int(b.seed_offsets[t + 1] - b.seed_offsets[t]) for t in range(b.T)
                                  if b.robot_of_target[t] == r)
        if tune:
            assert ch["ms"] > 0
    for rep in range(3):
        for o in outs:
            o.zero_()
        H.hjcd_plan_execute(plan)
        got = _host(outs)
        # eager work between replays
        scratch = _outs(b.T, k, n_max)
        H.hjcd_solve(ctx, rbs, sc, targets, b.seed_offsets, p, *scratch, robot_of_target=b.robot_of_target)
        torch.cuda.synchronize()
        # the tuner picks launch shapes only: results are bit-identical
        for nm, g, e in zip(("q", "err_p", "err_o", "flag", "n_free", "solved"), got, ref):
            assert np.array_equal(g, e), (rep, nm)
    plan.close()


def test_plan_with_host_seeds(H, ctx):
    """Caller seeds in the caller's target order are regrouped by robot inside
    the graph (the gather node) exactly as hjcd_solve regroups them."""
    import torch
    say("case: plan with caller seeds")
    b = W.config_uneven(T=24, max_seeds=200, host_seeds=True)
    rbs, sc, targets = _setup(H, ctx, b)
    seeds = torch.as_tensor(np.ascontiguousarray(b.seeds)).cuda()
    k, n_max = b.params["top_k"], b.n_max
    p = H.params_from_dict(b.params)
    ref = _outs(b.T, k, n_max)
    H.hjcd_solve(ctx, rbs, sc, targets, b.seed_offsets, p, *ref, robot_of_target=b.robot_of_target, seeds=seeds)
    ref = _host(ref)
    outs = _outs(b.T, k, n_max)
    plan = H.hjcd_plan_create(ctx, rbs, sc, targets, b.seed_offsets, p, *outs, robot_of_target=b.robot_of_target,
                              seeds=seeds, tune=False)
    H.hjcd_plan_execute(plan)
    got = _host(outs)
    for g, e in zip(got, ref):
        assert np.array_equal(g, e)
    plan.close()


@pytest.mark.parametrize("tune", [False, True])
def test_plan_resampled_equals_eager(H, ctx, tune):
    """Paper-mode resampling (K = 16 best CD seeds per target, B = 40) in a
    plan over the uneven three-robot batch: each robot's branch ranks and
    replicates its own targets; replays equal the eager resampled solve bit
    for bit, with and without autotuning."""
    import torch
    say(f"case: resampled plan, tune={tune}")
    b = W.config_uneven(T=36, max_seeds=300)
    rbs, sc, targets = _setup(H, ctx, b)
    params = dict(b.params, resample_K=16, resample_B=40)
    k, n_max = params["top_k"], b.n_max
    p = H.params_from_dict(params)
    ref = _outs(b.T, k, n_max)
    H.hjcd_solve(ctx, rbs, sc, targets, b.seed_offsets, p, *ref, robot_of_target=b.robot_of_target)
    ref = _host(ref)
    outs = _outs(b.T, k, n_max)
    plan = H.hjcd_plan_create(ctx, rbs, sc, targets, b.seed_offsets, p, *outs, robot_of_target=b.robot_of_target,
                              tune=tune)
    for rep in range(2):
        for o in outs:
            o.zero_()
        H.hjcd_plan_execute(plan)
        got = _host(outs)
        scratch = _outs(b.T, k, n_max)
        H.hjcd_solve(ctx, rbs, sc, targets, b.seed_offsets, p, *scratch, robot_of_target=b.robot_of_target)
        torch.cuda.synchronize()
        for nm, g, e in zip(("q", "err_p", "err_o", "flag", "n_free", "solved"), got, ref):
            assert np.array_equal(g, e), (rep, nm)
    assert ref[4].max() <= 32  # n_free counts the B' = 32 polished slots
    say(f"  solved {int(ref[5].sum())} of {b.T}")
    plan.close()


def test_plan_rejects_resampling_without_seeds(H, ctx):
    b = W.config_uneven(T=8, max_seeds=64)
    rbs, sc, targets = _setup(H, ctx, b)
    p = H.params_from_dict(dict(b.params, resample_K=4, resample_B=16))
    offs = b.seed_offsets.copy()
    offs[3:] -= offs[3] - offs[2]  # target 2 has no seeds
    outs = _outs(b.T, b.params["top_k"], b.n_max)
    with pytest.raises(H.HJCDError) as e:
        H.hjcd_plan_create(ctx, rbs, sc, targets, offs, p, *outs, robot_of_target=b.robot_of_target)
    assert e.value.status == H.HJCD_E_INVALID


@pytest.mark.parametrize("tune", [False, True])
def test_plan_streaming_launch_equals_eager(H, ctx, tune):
    """A 20-joint batch large enough for the PJ-IK launch to stream seeds
    through its waves (4,200 x 256 seeds): a plan replay, autotuned or not,
    gives bit-identical results to the eager hjcd_solve."""
    import torch
    say(f"case: streaming PJ-IK in a plan, tune={tune}")
    b = W.config_large(T=4200)
    assert int(b.seed_offsets[-1]) >= 2 * 8192 * 64
    rbs, sc, targets = _setup(H, ctx, b)
    k, n_max = b.params["top_k"], b.n_max
    p = H.params_from_dict(b.params)
    ref = _outs(b.T, k, n_max)
    H.hjcd_solve(ctx, rbs, sc, targets, b.seed_offsets, p, *ref, robot_of_target=b.robot_of_target)
    ref = _host(ref)
    outs = _outs(b.T, k, n_max)
    plan = H.hjcd_plan_create(ctx, rbs, sc, targets, b.seed_offsets, p, *outs, robot_of_target=b.robot_of_target,
                              tune=tune)
    ch = H.hjcd_plan_choice(plan, 0)
    say(f"  choice {ch}")
    for rep in range(2):
        for o in outs:
            o.zero_()
        H.hjcd_plan_execute(plan)
        got = _host(outs)
        for nm, g, e in zip(("q", "err_p", "err_o", "flag", "n_free", "solved"), got, ref):
            assert np.array_equal(g, e), (rep, nm)
    say(f"  solved {int(ref[5].sum())} of {b.T}")
    plan.close()
