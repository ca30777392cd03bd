"""Pins of the oracle's top-K ranking and noisy replication (Alg. HJCD-IK)
and of the PJ-IK perturbation (Alg. PJ-IK, last fallback), rebuilt step by
step in numpy.  CPU only."""
import numpy as np

from paper_2510_07514_amd import workload as W


def _replicated(O, rob, q, cost, counts, K, B, mu, sigma, seed, keys):
    """numpy statement of the replication: per target, lexsort by (cost,
    index), copy i of rank k is clip(q[rank k mod M] + mu + sigma z(i K + k))."""
    n = rob.dof
    copies = B // K
    rows = []
    b0 = 0
    for t, M in enumerate(counts):
        order = np.lexsort((np.arange(M), cost[b0:b0 + M]))
        for i in range(copies):
            for k in range(K):
                src = b0 + order[k % M]
                z = O.normals(seed, i * K + k, int(keys[t]), O.ST_RESAMPLE, 0, n)
                rows.append(np.clip(q[src] + mu + sigma * z, rob.q_min, rob.q_max))
        b0 += M
    return np.asarray(rows)


def test_resample_matches_numpy_rebuild(oracle_lib):
    """Ranking by (cost, index) with ties, the copy layout t B' + i K + k, the
    RESAMPLE draw keys and the clip; one target has fewer seeds than K (its
    ranked seeds repeat cyclically) and one exactly K."""
    O = oracle_lib
    rob = W.panda_like()
    rng = np.random.default_rng(31)
    counts = [3, 8, 64, 100]
    S = sum(counts)
    q = W.uniform_configs(rng, rob, S).astype(np.float64)
    cost = rng.integers(0, 12, size=S) * 0.25  # ties on purpose
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    K, B = 8, 20
    p = W.default_params(resample_K=K, resample_B=B, rng_seed=77, mu=0.01, sigma=0.05)
    keys = np.array([5, 9, 2, 40], np.uint32)
    got = O.resample(rob, offs, q, cost, p, target_keys=keys)
    ref = _replicated(O, rob, q, cost, counts, K, B, 0.01, 0.05, 77, keys)
    assert got.shape == (len(counts) * (B // K) * K, rob.dof)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-15)
    # the best seed is the lowest-index one among the lowest cost
    t = 2
    b0 = offs[t]
    best = int(np.flatnonzero(cost[b0:b0 + counts[t]] == cost[b0:b0 + counts[t]].min())[0])
    z = O.normals(77, 0, int(keys[t]), O.ST_RESAMPLE, 0, rob.dof)
    Bp = (B // K) * K
    np.testing.assert_allclose(got[t * Bp], np.clip(q[b0 + best] + 0.01 + 0.05 * z, rob.q_min, rob.q_max),
                               atol=1e-15)


def test_resample_rejects_targets_without_seeds(oracle_lib):
    O = oracle_lib
    rob = W.panda_like()
    q = np.zeros((4, 7))
    p = W.default_params(resample_K=2, resample_B=4)
    import pytest
    with pytest.raises(ValueError):
        O.resample(rob, np.array([0, 4, 4], np.int64), q, np.zeros(4), p)


def test_solve_polishes_the_replicated_seeds(oracle_lib):
    """With no PO-CCD or PJ-IK iterations the whole solve's per-seed output is
    exactly the replicated set of the (clipped) input seeds, ranked by the
    cost at those seeds, in the layout t B' + i K + k (targets with fewer
    seeds than K included)."""
    O = oracle_lib
    b = W.config_tiny()
    rob = b.robots[0]
    rng = np.random.default_rng(5)
    counts = [3, 64, 10, 1]
    S = sum(counts)
    seeds = W.uniform_configs(rng, rob, S).astype(np.float64)
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    tg = O.targets_from_qstar(rob, W.uniform_configs(rng, rob, len(counts))).astype(np.float64)
    K, B = 4, 10
    p = dict(b.params, cd_sweeps=0, polish_iters=0, resample_K=K, resample_B=B, top_k=2)
    out = O.solve(rob, b.scene, tg, offs, p, seeds=seeds, nthreads=2)
    cost = np.zeros(S)
    for t in range(len(counts)):
        for s in range(offs[t], offs[t + 1]):
            f = O.fk(rob, seeds[s])
            cost[s] = O.residual(tg[t, :3], tg[t, 3:], f["p_ee"], f["R_ee"])["cost"]
    ref = _replicated(O, rob, seeds, cost, counts, K, B, p["mu"], p["sigma"], p["rng_seed"],
                      np.arange(len(counts)))
    np.testing.assert_allclose(out["q_seed"], ref, rtol=0, atol=1e-15)


def test_pjik_perturbation_when_every_step_fails(oracle_lib):
    """With a zero trust radius the LM, dogleg and single-coordinate steps are
    all zero, no trial lowers the cost, and every PJ-IK iteration takes the
    perturbation theta <- clip(theta + mu + sigma z), z drawn for (seed index,
    target key, POLISH, iteration)."""
    O = oracle_lib
    rob = W.panda_like()
    rng = np.random.default_rng(8)
    tg = O.targets_from_qstar(rob, W.uniform_configs(rng, rob, 1))[0].astype(np.float64)
    th0 = W.uniform_configs(rng, rob, 1)[0].astype(np.float64)
    p = W.default_params(trust_R=0.0, polish_iters=6, mu=0.02, sigma=0.07, rng_seed=123)
    m, key = 17, 9
    r = O.polish(rob, tg, p, m, key, th0)
    assert r["stats"]["n_perturb"] == 6 and r["stats"]["iters_run"] == 6
    assert r["stats"]["n_dogleg"] == 6 and r["stats"]["n_single"] == 6
    th = th0.copy()
    for it in range(6):
        np.testing.assert_allclose(r["traj"][it, :7], th, atol=1e-15)
        z = O.normals(123, m, key, O.ST_POLISH, it, 7)
        th = np.clip(th + 0.02 + 0.07 * z, rob.q_min, rob.q_max)
    np.testing.assert_allclose(r["theta"], th, atol=1e-15)
