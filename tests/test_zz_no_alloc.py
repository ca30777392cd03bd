"""hjcd_solve_noalloc (the static-workspace variant of hjcd_solve, for callers
that cannot allocate) through the C ABI: bit-identical to hjcd_solve on two
calls in a row, the second with a smaller input, on single-robot, uneven
multi-robot (caller seeds regrouped) and resampled batches; requests beyond
the workspace are refused before any device work."""
import numpy as np
import pytest

import oracle as O
from gpu_common import cuda, say, targets_soa
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


def _outs(T, k, n_max):
    import torch
    return [torch.zeros(T * k, n_max, device="cuda"), torch.zeros(T * k, device="cuda"),
            torch.zeros(T * k, device="cuda"), torch.zeros(T * k, dtype=torch.uint8, device="cuda"),
            torch.zeros(T, dtype=torch.int32, device="cuda"), torch.zeros(T, dtype=torch.uint8, device="cuda")]


def _both(H, ctx, b, params=None, seeds=False):
    import torch
    params = params or b.params
    rbs = [H.hjcd_load_robot(ctx, r) for r in b.robots]
    sc = H.hjcd_load_scene(ctx, b.scene.spheres, b.scene.boxes)
    tg = np.concatenate([O.targets_from_qstar(b.robots[b.robot_of_target[t]], [b.q_star[t]]) for t in range(b.T)])
    targets = targets_soa(tg)
    sd = cuda(b.seeds) if seeds else None
    rot = b.robot_of_target if len(b.robots) > 1 else None
    p = H.params_from_dict(params)
    res = []
    for fn in (H.hjcd_solve, H.hjcd_solve_noalloc):
        o = _outs(b.T, params["top_k"], b.n_max)
        fn(ctx, rbs, sc, targets, b.seed_offsets, p, *o, robot_of_target=rot, seeds=sd)
        torch.cuda.synchronize()
        res.append([x.cpu().numpy() for x in o])
    for nm, a, g in zip(("q", "err_p", "err_o", "flag", "n_free", "solved"), res[0], res[1]):
        assert np.array_equal(a, g), nm
    return res[1]


def test_noalloc_equals_solve_twice_smaller_second(H, ctx):
    say("case: noalloc vs solve, batched 300 x 1024 then 40 x 200")
    big = W.config_batched(T=300, M=1024)
    g1 = _both(H, ctx, big)
    small = W.config_batched(T=40, M=200)
    g2 = _both(H, ctx, small)
    say(f"  solved {int(g1[5].sum())}/300, {int(g2[5].sum())}/40")


def test_noalloc_uneven_and_resampled(H, ctx):
    say("case: noalloc vs solve, uneven with caller seeds, then resampled tiny")
    _both(H, ctx, W.config_uneven(T=48, max_seeds=300, host_seeds=True), seeds=True)
    b = W.config_tiny()
    _both(H, ctx, b, params=dict(b.params, resample_K=8, resample_B=20, top_k=3), seeds=True)
    _both(H, ctx, W.config_uneven(T=12, max_seeds=100))


def test_noalloc_refuses_beyond_workspace(H, ctx):
    import torch
    say("case: noalloc limits")
    b = W.config_batched(T=2, M=1)
    rb = H.hjcd_load_robot(ctx, b.robots[0])
    o = _outs(2, 8, 7)
    p = H.params_from_dict(b.params)
    tg = targets_soa(O.targets_from_qstar(b.robots[0], b.q_star))
    too_many = np.array([0, 1, 2_000_001], np.int64)  # 2 M seeds x 41 bytes > 64 MiB
    with pytest.raises(H.HJCDError) as e:
        H.hjcd_solve_noalloc(ctx, [rb], None, tg, too_many, p, *o)
    assert e.value.status == H.HJCD_E_INVALID
    with pytest.raises(H.HJCDError) as e:
        H.hjcd_solve_noalloc(ctx, [rb], None, tg, np.array([0, 4, 8], np.int64), H.params_from_dict(b.params, True),
                             *o)
    assert e.value.status == H.HJCD_E_UNSUPPORTED
    torch.cuda.synchronize()
