"""Pins of the oracle's PO-CCD (Sec. II-A, Sec. III, Sec. IV-A, Alg. PO-CCD)
against geometry computed independently in numpy/scipy.  CPU only."""
import copy
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from paper_2510_07514_amd import workload as W


def _wide(rob):
    r = copy.deepcopy(rob)
    r.q_min = np.full(rob.dof, -1e3)
    r.q_max = np.full(rob.dof, 1e3)
    return r


def _target(O, rob, q):
    f = O.fk(rob, q)
    return np.concatenate([f["p_ee"], f["quat"]])


def _proj(x, z):
    return x - np.dot(x, z) * z


@pytest.mark.parametrize("which", ["panda", "random12", "ur"])
def test_position_step_aligns_projections(oracle_lib, which):
    """eq. (vec_proj)/(theta_proj) with a sign: after turning joint j by dp_j the
    projection of P_ee - P_j onto the joint plane points along the projection
    of P_t - P_j; the score sp_j is |P_t - P_ee|^2 at that configuration."""
    O = oracle_lib
    rng = np.random.default_rng(21)
    base = {"panda": W.panda_like(), "random12": W.random_chain(rng, 12), "ur": W.ur_like()}[which]
    rob = _wide(base)
    p = W.default_params()
    for _ in range(5):
        th = W.uniform_configs(rng, base, 1)[0].astype(np.float64)
        tgt = _target(O, rob, W.uniform_configs(rng, base, 1)[0].astype(np.float64))
        c = O.cd_candidates(rob, tgt, p, th, 0)
        f = O.fk(rob, th)
        for j in range(rob.dof):
            z, P = f["joint_z"][j], f["joint_P"][j]
            v = _proj(tgt[:3] - P, z)
            u0 = _proj(f["p_ee"] - P, z)
            if np.linalg.norm(u0) < 1e-4 or np.linalg.norm(v) < 1e-4:
                continue
            t2 = th.copy()
            t2[j] += c["dp"][j]
            g = O.fk(rob, t2)
            u = _proj(g["p_ee"] - P, z)
            cosang = np.dot(u, v) / (np.linalg.norm(u) * np.linalg.norm(v))
            assert cosang > 1 - 1e-12
            assert abs(c["dp"][j]) <= math.pi + 1e-12
            np.testing.assert_allclose(c["sp"][j], np.sum((tgt[:3] - g["p_ee"]) ** 2), rtol=1e-12,
                                       atol=1e-15)


def test_planar_2r_position_step_is_textbook_ccd(oracle_lib):
    """For a planar chain the CCD angle of joint j is the difference of the
    polar angles of P_t - P_j and P_ee - P_j (wrapped to (-pi, pi])."""
    O = oracle_lib
    l1, l2 = 0.6, 0.4
    rob = _wide(W.planar_chain([l1, l2]))
    p = W.default_params()
    rng = np.random.default_rng(2)
    for _ in range(20):
        th = rng.uniform(-3, 3, size=2)
        tq = rng.uniform(-3, 3, size=2)
        tgt = _target(O, rob, tq)
        c = O.cd_candidates(rob, tgt, p, th, 0)
        joints = [np.zeros(2), l1 * np.array([math.cos(th[0]), math.sin(th[0])])]
        ee = joints[1] + l2 * np.array([math.cos(th[0] + th[1]), math.sin(th[0] + th[1])])
        for j in range(2):
            u, v = ee - joints[j], tgt[:2] - joints[j]
            d = math.atan2(v[1], v[0]) - math.atan2(u[1], u[0])
            d = (d + math.pi) % (2 * math.pi) - math.pi
            assert abs(c["dp"][j] - d) < 1e-12 or abs(abs(d) - math.pi) < 1e-9


def test_orientation_step(oracle_lib):
    """eq. (ori_update): dor_j = delta(k) sgn(a_hat . z_j) phi, with a_hat, phi the
    axis-angle of R_t R_ee^T and delta(k) = max(0.1, 0.9^k); score so_j =
    |rotvec(R_t R(theta + dor_j e_j)^T)|^2."""
    O = oracle_lib
    rob = _wide(W.panda_like())
    p = W.default_params()
    rng = np.random.default_rng(4)
    for k in (0, 3, 30):
        delta = max(0.1, 0.9 ** k)
        th = W.uniform_configs(rng, W.panda_like(), 1)[0].astype(np.float64)
        tgt = _target(O, rob, W.uniform_configs(rng, W.panda_like(), 1)[0].astype(np.float64))
        c = O.cd_candidates(rob, tgt, p, th, k)
        f = O.fk(rob, th)
        Rt = Rotation.from_quat([tgt[4], tgt[5], tgt[6], tgt[3]])
        rv = (Rt * Rotation.from_matrix(f["R_ee"]).inv()).as_rotvec()
        phi = np.linalg.norm(rv)
        ahat = rv / phi
        for j in range(rob.dof):
            ref = delta * np.sign(np.dot(ahat, f["joint_z"][j])) * phi
            assert abs(c["dor"][j] - ref) < 1e-10
            t2 = th.copy()
            t2[j] += c["dor"][j]
            g = O.fk(rob, t2)
            so = np.sum((Rt * Rotation.from_matrix(g["R_ee"]).inv()).as_rotvec() ** 2)
            assert abs(c["so"][j] - so) < 1e-9


def test_steps_respect_joint_limits(oracle_lib):
    O = oracle_lib
    rob = W.panda_like()
    p = W.default_params()
    rng = np.random.default_rng(8)
    for _ in range(20):
        th = W.uniform_configs(rng, rob, 1)[0].astype(np.float64)
        tgt = _target(O, rob, W.uniform_configs(rng, rob, 1)[0].astype(np.float64))
        c = O.cd_candidates(rob, tgt, p, th, 0)
        for key in ("dp", "dor"):
            moved = th + c[key]
            assert np.all(moved >= rob.q_min - 1e-12) and np.all(moved <= rob.q_max + 1e-12)


def test_one_dof_orientation_step_is_exact(oracle_lib):
    """A 1-DoF chain turning about z with a target rotated by psi about z: the
    first orientation step (delta(0) = 1) removes the whole error."""
    O = oracle_lib
    rob = W.Robot("one", W.DH_MODIFIED, np.zeros(1), np.zeros(1), np.zeros(1), np.zeros(1),
                  np.full(1, -3.0), np.full(1, 3.0), np.eye(4), min_link_gap=0)
    p = W.default_params(cd_sweeps=2)
    for psi in (-2.5, -0.3, 0.7, 2.9):
        q = Rotation.from_euler("z", psi).as_quat()
        tgt = np.array([0, 0, 0, q[3], q[0], q[1], q[2]])
        r = O.cd(rob, tgt, p, 0, 0, np.zeros(1))
        assert abs(r["traj"][1, 0] - psi) < 1e-12
        assert r["traj"][1, 2] < 1e-12
        assert r["stats"]["frozen_at"] == 1


def test_greedy_combination_and_acceptance(oracle_lib):
    """Alg. PO-CCD with the Sec. IV-A rule: best position joint and best
    orientation joint (the lowest joint within tie_eps of the best score) are
    both applied when they differ,
    else the larger step; an improvement > gamma in position or orientation
    accepts, otherwise the seed moves by N(mu, sigma^2 I) from the
    (stage=CD, iteration k) draw, clipped to the limits."""
    O = oracle_lib
    rob = W.panda_like()
    rng = np.random.default_rng(12)
    for trial in range(20):
        p = W.default_params(cd_sweeps=1, rng_seed=77)
        th = W.uniform_configs(rng, rob, 1)[0].astype(np.float64)
        tgt = _target(O, rob, W.uniform_configs(rng, rob, 1)[0].astype(np.float64))
        c = O.cd_candidates(rob, tgt, p, th, 0)
        sp, so = np.sqrt(c["sp"]), np.sqrt(c["so"])
        jp = int(np.nonzero(sp <= sp.min() + p["tie_eps"])[0][0])
        jo = int(np.nonzero(so <= so.min() + p["tie_eps"])[0][0])
        hat = th.copy()
        if jp != jo:
            hat[jp] += c["dp"][jp]
            hat[jo] += c["dor"][jo]
        elif abs(c["dp"][jp]) >= abs(c["dor"][jo]):
            hat[jp] += c["dp"][jp]
        else:
            hat[jo] += c["dor"][jo]
        f0, fh = O.fk(rob, th), O.fk(rob, hat)
        r0 = O.residual(tgt[:3], tgt[3:], f0["p_ee"], f0["R_ee"])
        rh = O.residual(tgt[:3], tgt[3:], fh["p_ee"], fh["R_ee"])
        imp = (np.sum(r0["rp"] ** 2) - np.sum(rh["rp"] ** 2) > p["gamma"]) or \
              (np.sum(r0["omega"] ** 2) - np.sum(rh["omega"] ** 2) > p["gamma"])
        r = O.cd(rob, tgt, p, 5, 9, th)
        if imp:
            np.testing.assert_allclose(r["theta"], hat, atol=1e-14)
            assert r["stats"]["n_perturb"] == 0
        else:
            z = O.normals(77, 5, 9, O.ST_CD, 0, rob.dof)
            np.testing.assert_allclose(r["theta"], np.clip(th + 0.05 * z, rob.q_min, rob.q_max),
                                       atol=1e-14)
        # forcing the perturbation path with a huge gamma
        p2 = dict(p, gamma=1e9)
        r2 = O.cd(rob, tgt, p2, 5, 9, th)
        z = O.normals(77, 5, 9, O.ST_CD, 0, rob.dof)
        np.testing.assert_allclose(r2["theta"], np.clip(th + 0.05 * z, rob.q_min, rob.q_max),
                                   atol=1e-14)
        assert r2["stats"]["n_perturb"] == 1


def test_converged_seed_freezes(oracle_lib):
    O = oracle_lib
    rob = W.panda_like()
    q = W.uniform_configs(np.random.default_rng(3), rob, 1)[0].astype(np.float64)
    tgt = _target(O, rob, q)
    r = O.cd(rob, tgt, W.default_params(), 0, 0, q)
    assert r["stats"]["frozen_at"] == 0 and r["stats"]["iters_run"] == 0
    np.testing.assert_array_equal(r["theta"], q)
    assert np.all(r["traj"][:, :7] == q)


def test_cd_reduces_error_on_average(oracle_lib):
    """Not a proof of anything, a sanity check that the greedy sweep moves
    seeds toward the target: the median error after 20 sweeps is below the
    median of the random seeds."""
    O = oracle_lib
    b = W.config_tiny()
    rob = b.robots[0]
    tg = O.targets_from_qstar(rob, b.q_star).astype(np.float64)
    e0, e1 = [], []
    for m in range(64):
        r = O.cd(rob, tg[m % 8], b.params, m, m % 8, b.seeds[:7, m].astype(np.float64))
        e0.append(r["traj"][0, 7])
        e1.append(r["traj"][-1, 7])
    assert np.median(e1) < 0.5 * np.median(e0)


def test_parallel_axes_tie_to_lowest_joint(oracle_lib):
    """Joints with parallel axes give the same orientation score (a planar
    chain: every joint turns about z); the pick is the lowest such joint, and
    an iteration with exactly tied scores records no near-tie margin."""
    O = oracle_lib
    rob = _wide(W.planar_chain([0.5, 0.4, 0.3]))  # no step is clipped
    p = W.default_params(cd_sweeps=1)
    rng = np.random.default_rng(3)
    for _ in range(10):
        th = rng.uniform(-2, 2, size=3)
        tgt = _target(O, rob, rng.uniform(-2, 2, size=3))
        c = O.cd_candidates(rob, tgt, p, th, 0)
        assert np.ptp(np.sqrt(c["so"])) < 1e-12
        r = O.cd(rob, tgt, p, 0, 0, th)
        moved = np.nonzero(np.abs(r["theta"] - th) > 0)[0]
        if r["stats"]["n_perturb"] == 0 and moved.size:
            jp = int(np.nonzero(np.sqrt(c["sp"]) <= np.sqrt(c["sp"]).min() + p["tie_eps"])[0][0])
            assert set(moved.tolist()) <= {jp, 0}
