"""Pins of the oracle's tracking pieces (warm start from the previous
solution set, selection nearest to a reference configuration), rebuilt step
by step in numpy.  CPU only."""
import numpy as np

from paper_2510_07514_amd import workload as W


def test_warm_seeds_match_numpy_rebuild(oracle_lib):
    O = oracle_lib
    rob = W.panda_like()
    rng = np.random.default_rng(3)
    T, k, M = 3, 4, 11
    q_prev = W.uniform_configs(rng, rob, T * k).astype(np.float64)
    q_prev[5, 2] = 9.0  # outside the limits: clipped
    keys = np.array([7, 0, 123456], np.uint32)
    p = W.default_params(rng_seed=55, sigma=0.03, mu=0.002)
    got = O.warm_seeds(rob, q_prev, k, M, p, target_keys=keys)
    for t in range(T):
        for m in range(M):
            x = np.clip(q_prev[t * k + m % k], rob.q_min, rob.q_max)
            if m >= k:
                z = O.normals(55, m, int(keys[t]), O.ST_WARM, 0, rob.dof)
                x = np.clip(x + 0.002 + 0.03 * z, rob.q_min, rob.q_max)
            np.testing.assert_allclose(got[t * M + m], x, rtol=0, atol=1e-15)
    # the first k seeds are the previous solutions themselves
    np.testing.assert_array_equal(got[M:M + k], np.clip(q_prev[k:2 * k], rob.q_min, rob.q_max))


def _near_ref(flag, cost, ep, eo, q, q_ref, k, sp, so):
    ok = (flag == 0) & (ep <= sp) & (eo <= so)
    cls = np.where(ok, 0, np.where(flag == 0, 1, 2))
    key = np.where(ok, ((q - q_ref) ** 2).sum(axis=1), cost)
    order = np.lexsort((np.arange(len(flag)), key, cls))
    out = -np.ones(k, np.int32)
    out[:min(k, len(flag))] = order[:k]
    return out


def test_select_near_matches_numpy_sort(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(9)
    for m in (0, 1, 7, 64, 300):
        n = 7
        flag = rng.integers(0, 2, size=m).astype(np.int32)
        cost = rng.integers(0, 20, size=m) * 0.25
        ep = rng.uniform(0, 2e-3, size=m)
        eo = rng.uniform(0, 0.03, size=m)
        q = rng.integers(-8, 8, size=(m, n)) / 8.0  # exact squared distances, ties on purpose
        q_ref = rng.integers(-8, 8, size=n) / 8.0
        for k in (1, 5, 400):
            got = O.select_near(flag, cost, ep, eo, q, q_ref, k, 1e-3, np.pi / 180)
            np.testing.assert_array_equal(got, _near_ref(flag, cost, ep, eo, q, q_ref, k, 1e-3, np.pi / 180))


def test_select_near_special_cases(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(10)
    m, n = 50, 6
    flag = np.zeros(m, np.int32)
    cost = rng.uniform(0, 1, size=m)
    ep = np.full(m, 1e-4)
    eo = np.full(m, 1e-3)
    q = rng.normal(size=(m, n))
    # the reference is one of the successful seeds: it comes first
    got = O.select_near(flag, cost, ep, eo, q, q[17], 3, 1e-3, np.pi / 180)
    assert got[0] == 17
    # no seed is within tolerance: the order is the cost order of select()
    ep_bad = np.full(m, 1.0)
    flag2 = rng.integers(0, 2, size=m).astype(np.int32)
    got = O.select_near(flag2, cost, ep_bad, eo, q, q[3], 10, 1e-3, np.pi / 180)
    np.testing.assert_array_equal(got, O.select(flag2, cost, 10))
