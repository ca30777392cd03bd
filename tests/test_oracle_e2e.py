"""End-to-end pins of the oracle's HJCD-IK pipeline (Alg. HJCD-IK): returned
solutions hit their targets, and on planar 2R/3R chains they are the
analytic law-of-cosines solutions and beat a brute-force joint grid.  CPU only."""
import math

import numpy as np
from scipy.spatial.transform import Rotation

from paper_2510_07514_amd import workload as W


def test_returned_errors_recompute_and_hit_targets(oracle_lib):
    O = oracle_lib
    b = W.config_tiny()
    rob = b.robots[0]
    tg = O.targets_from_qstar(rob, b.q_star).astype(np.float64)
    out = O.solve(rob, b.scene, tg, b.seed_offsets, b.params, seeds=b.seeds[:7].T, nthreads=4)
    assert out["solved"].sum() >= 6
    for t in range(b.T):
        for i in range(b.params["top_k"]):
            q = out["q_out"][t, i]
            f = O.fk(rob, q)
            ep = np.linalg.norm(tg[t, :3] - f["p_ee"])
            Rt = Rotation.from_quat([tg[t, 4], tg[t, 5], tg[t, 6], tg[t, 3]])
            eo = np.linalg.norm((Rt * Rotation.from_matrix(f["R_ee"]).inv()).as_rotvec())
            assert abs(ep - out["err_p"][t, i]) < 1e-12
            assert abs(eo - out["err_o"][t, i]) < 1e-7
            assert np.all(q >= rob.q_min) and np.all(q <= rob.q_max)
            if out["solved"][t]:
                assert out["flag_out"][t, i] == 0 or i > 0
        if out["solved"][t]:
            assert out["err_p"][t, 0] <= 1e-3 and out["err_o"][t, 0] <= math.pi / 180


def _wrap(x):
    return (np.asarray(x) + math.pi) % (2 * math.pi) - math.pi


def _planar_batch(O, lengths, T, M, seed):
    rob = W.planar_chain(lengths)
    rng = np.random.default_rng(seed)
    qs = [W.uniform_configs(rng, rob, 1)[0] for _ in range(T)]
    tg = O.targets_from_qstar(rob, qs).astype(np.float64)
    offs = np.arange(T + 1, dtype=np.int64) * M
    seeds = W.uniform_configs(rng, rob, T * M)
    p = W.default_params(top_k=4, rng_seed=seed)
    out = O.solve(rob, W.empty_scene(), tg, offs, p, seeds=seeds, nthreads=4)
    return rob, tg, out


def _two_r_branches(x, y, l1, l2):
    c2 = np.clip((x * x + y * y - l1 * l1 - l2 * l2) / (2 * l1 * l2), -1, 1)
    sols = []
    for s in (1.0, -1.0):
        q2 = s * math.acos(c2)
        q1 = math.atan2(y, x) - math.atan2(l2 * math.sin(q2), l1 + l2 * math.cos(q2))
        sols.append(np.array([q1, q2]))
    return sols


def test_planar_2r_matches_analytic_branch_and_grid(oracle_lib):
    """With a full pose target the planar 2R solution is the law-of-cosines
    branch whose q1 + q2 equals the target heading; a 0.25 deg joint grid never
    beats the solver's best cost."""
    O = oracle_lib
    l1, l2 = 0.6, 0.4
    rob, tg, out = _planar_batch(O, [l1, l2], T=6, M=32, seed=3)
    g = np.deg2rad(np.arange(-180, 180, 0.25))
    G1, G2 = np.meshgrid(g, g, indexing="ij")
    for t in range(tg.shape[0]):
        x, y = tg[t, 0], tg[t, 1]
        head = 2 * math.atan2(tg[t, 6], tg[t, 3])
        sols = _two_r_branches(x, y, l1, l2)
        assert out["solved"][t] == 1
        best = out["q_out"][t, 0]
        err = [np.max(np.abs(_wrap(best - s))) for s in sols]
        i = int(np.argmin(err))
        assert err[i] < 1e-5
        assert abs(_wrap(sols[i].sum() - head)) < 1e-5
        # grid: cost = 0.5 (|dp|^2 + dpsi^2) on the plane
        px = l1 * np.cos(G1) + l2 * np.cos(G1 + G2)
        py = l1 * np.sin(G1) + l2 * np.sin(G1 + G2)
        cost = 0.5 * ((px - x) ** 2 + (py - y) ** 2 + _wrap(G1 + G2 - head) ** 2)
        best_cost = 0.5 * (out["err_p"][t, 0] ** 2 + out["err_o"][t, 0] ** 2)
        assert best_cost <= cost.min() + 1e-12
        assert cost.min() < 1e-4


def test_planar_3r_solutions_lie_on_analytic_branches(oracle_lib):
    """Planar 3R with a pose target: the wrist point is the target minus the
    last link along the heading, then a 2R problem; every successful returned
    solution is one of the two branches, and a 1 deg grid does not beat it."""
    O = oracle_lib
    L = [0.5, 0.4, 0.25]
    rob, tg, out = _planar_batch(O, L, T=5, M=48, seed=4)
    g = np.deg2rad(np.arange(-180, 180, 1.0))
    G1, G2, G3 = np.meshgrid(g, g, g, indexing="ij")
    for t in range(tg.shape[0]):
        head = 2 * math.atan2(tg[t, 6], tg[t, 3])
        wx = tg[t, 0] - L[2] * math.cos(head)
        wy = tg[t, 1] - L[2] * math.sin(head)
        sols = [np.array([s[0], s[1], head - s[0] - s[1]]) for s in _two_r_branches(wx, wy, L[0], L[1])]
        assert out["solved"][t] == 1
        for i in range(4):
            if out["err_p"][t, i] <= 1e-3 and out["err_o"][t, i] <= math.pi / 180:
                q = out["q_out"][t, i]
                err = min(np.max(np.abs(_wrap(q - s))) for s in sols)
                assert err < 1e-3
        px = L[0] * np.cos(G1) + L[1] * np.cos(G1 + G2) + L[2] * np.cos(G1 + G2 + G3)
        py = L[0] * np.sin(G1) + L[1] * np.sin(G1 + G2) + L[2] * np.sin(G1 + G2 + G3)
        cost = 0.5 * ((px - tg[t, 0]) ** 2 + (py - tg[t, 1]) ** 2 + _wrap(G1 + G2 + G3 - head) ** 2)
        best_cost = 0.5 * (out["err_p"][t, 0] ** 2 + out["err_o"][t, 0] ** 2)
        assert best_cost <= cost.min() + 1e-12


def test_resampling_shapes_and_consistency(oracle_lib):
    """Top-K + floor(B/K) noisy copies (Alg. HJCD-IK): the polished set has
    floor(B/K) K seeds per target and every reported error recomputes."""
    O = oracle_lib
    b = W.config_tiny()
    rob = b.robots[0]
    tg = O.targets_from_qstar(rob, b.q_star).astype(np.float64)
    p = dict(b.params, resample_K=8, resample_B=20, top_k=3)
    out = O.solve(rob, b.scene, tg, b.seed_offsets, p, seeds=b.seeds[:7].T, nthreads=4)
    assert out["q_seed"].shape == (8 * 16, 7)
    for s in range(0, 128, 9):
        f = O.fk(rob, out["q_seed"][s])
        t = s // 16
        assert abs(np.linalg.norm(tg[t, :3] - f["p_ee"]) - out["errp_seed"][s]) < 1e-12


def test_empty_and_short_targets(oracle_lib):
    """A target with no seeds returns empty slots (flag 255, infinite errors);
    one with fewer seeds than k fills the rest with empty slots."""
    O = oracle_lib
    b = W.config_tiny()
    rob = b.robots[0]
    tg = O.targets_from_qstar(rob, b.q_star[:3]).astype(np.float64)
    offs = np.array([0, 0, 2, 12], np.int64)
    p = dict(b.params, top_k=4)
    out = O.solve(rob, b.scene, tg, offs, p, seeds=b.seeds[:7, :12].T, nthreads=2)
    assert np.all(out["flag_out"][0] == 255) and np.all(np.isinf(out["err_p"][0]))
    assert out["n_free"][0] == 0 and out["solved"][0] == 0
    assert np.all(out["flag_out"][1, 2:] == 255) and np.all(out["flag_out"][1, :2] != 255)
    assert np.all(out["flag_out"][2] != 255)
