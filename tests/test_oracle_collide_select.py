"""Pins of the oracle's collision filter (Sec. IV-C) and final selection
(Alg. HJCD-IK, last line).  CPU only."""
import numpy as np

from paper_2510_07514_amd import workload as W


def _centres(O, rob, th):
    T = O.fk(rob, th)["link_T"]
    c = []
    for l, s in zip(rob.sphere_link, rob.sphere_xyzr):
        c.append(T[l][:, :3] @ s[:3] + T[l][:, 3])
    return np.array(c).reshape(-1, 3), rob.sphere_xyzr[:, 3]


def _brute(O, rob, scene, th):
    c, r = _centres(O, rob, th)
    flag, md = 0, np.inf
    for i in range(len(c)):
        for o in scene.spheres.astype(np.float64):
            d = np.linalg.norm(c[i] - o[:3]) - (r[i] + o[3])
            md = min(md, d)
            flag |= d < 0
        for b in scene.boxes.astype(np.float64):
            ex = np.maximum(0.0, np.abs(c[i] - b[:3]) - b[3:])
            d = np.linalg.norm(ex) - r[i]
            md = min(md, d)
            flag |= d < 0
    if rob.min_link_gap > 0:
        for i in range(len(c)):
            for j in range(i + 1, len(c)):
                if abs(int(rob.sphere_link[i]) - int(rob.sphere_link[j])) >= rob.min_link_gap:
                    d = np.linalg.norm(c[i] - c[j]) - (r[i] + r[j])
                    md = min(md, d)
                    flag |= d < 0
    return int(flag), md


def test_flags_match_numpy_brute_force(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(0)
    for b in (W.config_batched(T=2, M=4), W.config_large(T=2, M=4)):
        rob = b.robots[0]
        for th in W.uniform_configs(rng, rob, 15).astype(np.float64):
            f, md = O.collide(rob, b.scene, th)
            bf, bmd = _brute(O, rob, b.scene, th)
            assert f == bf
            assert abs(md - bmd) < 1e-12


def _one_sphere_robot(r=0.1, extra=None, gap=0):
    rob = W.Robot("s", W.DH_MODIFIED, np.zeros(3), np.zeros(3), np.zeros(3), np.zeros(3),
                  np.full(3, -3.0), np.full(3, 3.0), np.eye(4), min_link_gap=gap)
    rows = [[0, 0, 0, r]] + ([] if extra is None else [extra[1]])
    links = [0] + ([] if extra is None else [extra[0]])
    rob.sphere_link = np.array(links, np.int32)
    rob.sphere_xyzr = np.array(rows, np.float64)
    return rob


def test_contact_cases(oracle_lib):
    """Sphere-sphere and sphere-box contacts 2e-5 m inside and outside."""
    O = oracle_lib
    rob = _one_sphere_robot(0.1)
    th = np.zeros(3)
    for eps, expect in ((-2e-5, 1), (2e-5, 0)):
        sc = W.Scene(np.array([[0.1 + 0.05 + eps, 0, 0, 0.05]], np.float64), np.zeros((0, 6)))
        f, md = O.collide(rob, sc, th)
        assert f == expect and abs(md - eps) < 1e-12
        # face of a box at x = 0.1 + eps
        h = 0.2
        sc = W.Scene(np.zeros((0, 4)), np.array([[0.1 + eps + h, 0, 0, h, h, h]], np.float64))
        f, md = O.collide(rob, sc, th)
        assert f == expect and abs(md - eps) < 1e-12
        # corner of a box along the diagonal
        d = (0.1 + eps) / np.sqrt(3)
        sc = W.Scene(np.zeros((0, 4)), np.array([[d + h, d + h, d + h, h, h, h]], np.float64))
        f, md = O.collide(rob, sc, th)
        assert f == expect and abs(md - eps) < 1e-12
    # centre inside a box
    sc = W.Scene(np.zeros((0, 4)), np.array([[0.01, 0, 0, 0.05, 0.05, 0.05]], np.float64))
    assert O.collide(rob, sc, th)[0] == 1


def test_self_pairs_follow_link_gap(oracle_lib):
    O = oracle_lib
    # a sphere on link 2 that overlaps the base sphere at theta = 0
    for gap, expect in ((3, 0), (2, 1), (0, 0)):
        rob = _one_sphere_robot(0.1, extra=(2, [0.05, 0, 0, 0.1]), gap=gap)
        f, _ = O.collide(rob, W.empty_scene(), np.zeros(3))
        assert f == expect


def test_select_matches_full_sort(oracle_lib):
    O = oracle_lib
    rng = np.random.default_rng(3)
    for m in (0, 1, 7, 64, 1000):
        flag = rng.integers(0, 2, size=m).astype(np.int32)
        cost = rng.integers(0, 5, size=m).astype(np.float64) * 0.25  # many ties
        for k in (1, 8, 16):
            o = O.select(flag, cost, k)
            ref = np.lexsort((np.arange(m), cost, flag))[:k]
            got = o[: min(k, m)]
            np.testing.assert_array_equal(got, ref)
            assert np.all(o[min(k, m):] == -1)
