"""Pins of the oracle's random draws: Philox4x32-10 against the published
known-answer vectors, Box-Muller normals and uniform seeds.  CPU only."""
import os

import numpy as np

from paper_2510_07514_amd import workload as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        v = [int(x, 16) for x in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(oracle_lib):
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        np.testing.assert_array_equal(oracle_lib.philox(ctr, key), np.array(out, np.uint32))


def test_normals_moments_and_keys(oracle_lib):
    O = oracle_lib
    z = np.concatenate([O.normals(7, m, 3, O.ST_CD, 0, 8) for m in range(4000)])
    assert abs(z.mean()) < 0.03
    assert abs(z.var() - 1.0) < 0.05
    # different stage, iteration, seed or target key -> different draws
    a = O.normals(7, 1, 2, O.ST_CD, 5, 6)
    for other in (O.normals(7, 1, 2, O.ST_POLISH, 5, 6), O.normals(7, 1, 2, O.ST_CD, 6, 6),
                  O.normals(7, 2, 2, O.ST_CD, 5, 6), O.normals(7, 1, 3, O.ST_CD, 5, 6),
                  O.normals(8, 1, 2, O.ST_CD, 5, 6)):
        assert not np.allclose(a, other)
    # deterministic
    np.testing.assert_array_equal(a, O.normals(7, 1, 2, O.ST_CD, 5, 6))


def test_box_muller_pairs(oracle_lib):
    """Joints 2p and 2p+1 share one uniform pair: their squares add up to
    -2 ln u1, so the pair radius is the same for both."""
    O = oracle_lib
    z = O.normals(1, 0, 0, O.ST_CD, 0, 8)
    ctr = [0, 0, (O.ST_CD << 24), 0]
    x = O.philox(ctr, [1, 0])
    for p in range(2):
        u1 = ((int(x[2 * p]) >> 8) + 0.5) / 2 ** 24
        np.testing.assert_allclose(z[2 * p] ** 2 + z[2 * p + 1] ** 2, -2 * np.log(u1), rtol=1e-12)


def test_uniform_seed_in_limits(oracle_lib):
    O = oracle_lib
    rob = W.panda_like()
    th = np.array([O.uniform_seed(rob, 9, m, 1) for m in range(2000)])
    assert np.all(th >= rob.q_min) and np.all(th <= rob.q_max)
    u = (th - rob.q_min) / (rob.q_max - rob.q_min)
    assert abs(u.mean() - 0.5) < 0.02
