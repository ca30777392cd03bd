"""ctypes front end of the FP64 CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of ``bench.py``.  The product path never imports it.

It takes robots / scenes / parameters as produced by the shared workload
generator and returns numpy float64 arrays.  Targets are defined as the FP64
forward kinematics of a float32 configuration q*, rounded once to float32
(``targets_from_qstar``).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hjcd_oracle.cpp")
# HJCD_ORACLE_LIBRARY selects another build of the same source (the tests'
# sanitizer build); it is used as given and never rebuilt here.
LIB_OVERRIDE = os.environ.get("HJCD_ORACLE_LIBRARY")
LIB = LIB_OVERRIDE or os.path.join(HERE, "liboracle.so")

ST_INIT, ST_CD, ST_RESAMPLE, ST_POLISH, ST_WARM = 0, 1, 2, 3, 4

# operation-count categories (hjcd_oracle.h, OR_OPS_*)
OPS_CATEGORIES = ("misc", "eval", "init", "cd_iter", "cd_perturb", "pj_iter", "pj_trial", "pj_dogleg",
                  "pj_single", "pj_perturb", "resample", "collide", "select", "instr")


def build() -> str:
    """Compile the oracle with g++ (plain IEEE double, no FMA contraction)."""
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared", "-Wall",
           "-o", LIB + ".tmp", SRC, "-lpthread"]
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(LIB + ".tmp", LIB)
    return LIB


class _Robot(C.Structure):
    _fields_ = [("dof", C.c_int32), ("convention", C.c_int32),
                ("a", C.POINTER(C.c_double)), ("d", C.POINTER(C.c_double)),
                ("alpha", C.POINTER(C.c_double)), ("offset", C.POINTER(C.c_double)),
                ("q_min", C.POINTER(C.c_double)), ("q_max", C.POINTER(C.c_double)),
                ("tool", C.POINTER(C.c_double)), ("n_spheres", C.c_int32),
                ("sphere_link", C.POINTER(C.c_int32)), ("sphere_xyzr", C.POINTER(C.c_double)),
                ("min_link_gap", C.c_int32)]


class _Scene(C.Structure):
    _fields_ = [("n_spheres", C.c_int32), ("spheres", C.POINTER(C.c_double)),
                ("n_boxes", C.c_int32), ("boxes", C.POINTER(C.c_double))]


class _Params(C.Structure):
    _fields_ = [("cd_sweeps", C.c_int32), ("polish_iters", C.c_int32),
                ("eps_cd", C.c_double), ("nu_cd", C.c_double), ("gamma", C.c_double),
                ("delta0", C.c_double), ("delta_decay", C.c_double), ("delta_min", C.c_double),
                ("proj_eps", C.c_double), ("tie_eps", C.c_double), ("lam", C.c_double), ("lambda_gn", C.c_double),
                ("trust_R", C.c_double), ("ls_beta", C.c_double),
                ("ls_A", C.c_int32), ("weight_mode", C.c_int32),
                ("eps_pol", C.c_double), ("ups_pol", C.c_double), ("sigma", C.c_double),
                ("mu", C.c_double), ("resample_K", C.c_int32), ("resample_B", C.c_int32),
                ("top_k", C.c_int32), ("succ_pos", C.c_double), ("succ_ori", C.c_double),
                ("rng_seed", C.c_uint64), ("shadow", C.c_uint64)]


class _Stats(C.Structure):
    _fields_ = [("iters_run", C.c_int32), ("frozen_at", C.c_int32), ("n_perturb", C.c_int32),
                ("n_trials", C.c_int32), ("n_dogleg", C.c_int32), ("n_single", C.c_int32),
                ("n_tie_pick", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not LIB_OVERRIDE and (not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC)):
            build()
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        up = C.POINTER(C.c_uint32)
        L.or_fk.argtypes = [C.POINTER(_Robot), dp, dp, dp, dp, dp, dp, dp, dp]
        L.or_quat_from_R.argtypes = [dp, dp]
        L.or_residual.argtypes = [dp, dp, dp, dp, dp]
        L.or_philox4x32_10.argtypes = [up, up, up]
        L.or_normals.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                 C.c_int, dp]
        L.or_uniform_seed.argtypes = [C.POINTER(_Robot), C.c_uint64, C.c_uint32, C.c_uint32, dp]
        stage = [C.POINTER(_Robot), dp, C.POINTER(_Params), C.c_uint32, C.c_uint32, dp, dp, dp,
                 C.POINTER(_Stats)]
        L.or_cd.argtypes = stage
        L.or_polish.argtypes = stage[:8] + [dp, C.POINTER(_Stats)]
        L.or_cd_candidates.argtypes = [C.POINTER(_Robot), dp, C.POINTER(_Params), dp, C.c_int32,
                                       dp, dp, dp, dp]
        L.or_pjik_steps.argtypes = [C.POINTER(_Robot), dp, C.POINTER(_Params), dp, dp, dp, dp,
                                    dp, dp, ip]
        L.or_collide.argtypes = [C.POINTER(_Robot), C.POINTER(_Scene), dp, ip, dp]
        L.or_select.argtypes = [C.c_int32, ip, dp, C.c_int32, ip]
        L.or_resample.argtypes = [C.POINTER(_Robot), C.c_int32, C.POINTER(C.c_int64), dp, dp, up,
                                  C.POINTER(_Params), dp]
        L.or_warm_seeds.argtypes = [C.POINTER(_Robot), C.c_int32, C.c_int32, dp, C.c_int32, up,
                                    C.POINTER(_Params), dp]
        L.or_select_near.argtypes = [C.c_int32, C.c_int32, ip, dp, dp, dp, dp, dp, C.c_double, C.c_double,
                                     C.c_int32, ip]
        L.or_ops_reset.argtypes = []
        L.or_ops_reset.restype = None
        L.or_ops_get.argtypes = [C.c_int32, C.POINTER(C.c_uint64)]
        L.or_solve.argtypes = [C.POINTER(_Robot), C.POINTER(_Scene), C.c_int32, dp,
                               C.POINTER(C.c_int64), dp, up, C.POINTER(_Params),
                               dp, dp, dp, dp, ip, dp, dp, dp, ip, ip, ip, C.c_int32]
        _lib = L
    return _lib


def _d(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _ptr(a, ct=C.c_double):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ct))


class RobotHandle:
    """Keeps the numpy buffers alive while the C struct points at them."""

    def __init__(self, robot):
        self.robot = robot
        self.bufs = [_d(robot.a), _d(robot.d), _d(robot.alpha), _d(robot.offset),
                     _d(robot.q_min), _d(robot.q_max), _d(np.asarray(robot.tool).reshape(16)),
                     np.ascontiguousarray(robot.sphere_link, dtype=np.int32),
                     _d(np.asarray(robot.sphere_xyzr).reshape(-1))]
        b = self.bufs
        self.c = _Robot(robot.dof, robot.convention, _ptr(b[0]), _ptr(b[1]), _ptr(b[2]),
                        _ptr(b[3]), _ptr(b[4]), _ptr(b[5]), _ptr(b[6]),
                        int(b[7].shape[0]), _ptr(b[7], C.c_int32), _ptr(b[8]),
                        int(robot.min_link_gap))
        self.n = robot.dof


class SceneHandle:
    def __init__(self, scene):
        self.s = _d(np.asarray(scene.spheres, dtype=np.float64).reshape(-1))
        self.b = _d(np.asarray(scene.boxes, dtype=np.float64).reshape(-1))
        self.c = _Scene(int(self.s.shape[0] // 4), _ptr(self.s), int(self.b.shape[0] // 6),
                        _ptr(self.b))


def params(p: dict) -> _Params:
    return _Params(int(p["cd_sweeps"]), int(p["polish_iters"]), p["eps_cd"], p["nu_cd"],
                   p["gamma"], p["delta0"], p["delta_decay"], p["delta_min"], p["proj_eps"], p["tie_eps"],
                   p["lam"], p["lambda_gn"], p["trust_R"], p["ls_beta"], int(p["ls_A"]),
                   int(p["weight_mode"]), p["eps_pol"], p["ups_pol"], p["sigma"], p["mu"],
                   int(p["resample_K"]), int(p["resample_B"]), int(p["top_k"]),
                   p["succ_pos"], p["succ_ori"], int(p["rng_seed"]) & 0xFFFFFFFFFFFFFFFF,
                   int(p.get("shadow", 0)))


def _rh(robot):
    return robot if isinstance(robot, RobotHandle) else RobotHandle(robot)


# ---------------------------------------------------------------------------
# kinematics
# ---------------------------------------------------------------------------

def fk(robot, theta):
    """FK at one configuration: dict with p_ee, R_ee, quat (w>=0), joint_P,
    joint_z, link_T ((n+1) x 3 x 4), J (6 x n)."""
    rh = _rh(robot)
    n = rh.n
    th = _d(theta)
    out = dict(p_ee=np.zeros(3), R_ee=np.zeros(9), quat=np.zeros(4), joint_P=np.zeros(3 * n),
               joint_z=np.zeros(3 * n), link_T=np.zeros(12 * (n + 1)), J=np.zeros(6 * n))
    rc = lib().or_fk(C.byref(rh.c), _ptr(th), *[_ptr(out[k]) for k in
                     ("p_ee", "R_ee", "quat", "joint_P", "joint_z", "link_T", "J")])
    if rc != 0:
        raise ValueError("or_fk rejected the robot")
    out["R_ee"] = out["R_ee"].reshape(3, 3)
    out["joint_P"] = out["joint_P"].reshape(n, 3)
    out["joint_z"] = out["joint_z"].reshape(n, 3)
    out["link_T"] = out["link_T"].reshape(n + 1, 3, 4)
    out["J"] = out["J"].reshape(6, n)
    return out


def quat_from_R(R):
    q = np.zeros(4)
    lib().or_quat_from_R(_ptr(_d(np.asarray(R).reshape(9))), _ptr(q))
    return q


def residual(p_t, q_t, p_ee, R_ee):
    out = np.zeros(11)
    lib().or_residual(_ptr(_d(p_t)), _ptr(_d(q_t)), _ptr(_d(p_ee)),
                      _ptr(_d(np.asarray(R_ee).reshape(9))), _ptr(out))
    return dict(rp=out[0:3], omega=out[3:6], phi=out[6], ahat=out[7:10], cost=out[10])


def targets_from_qstar(robot, q_star):
    """Target poses [T, 7] float32 (px py pz qw qx qy qz, w >= 0): FP64 FK of
    the float32 configurations, rounded once to float32."""
    rh = _rh(robot)
    out = np.zeros((len(q_star), 7), np.float32)
    for t, q in enumerate(q_star):
        f = fk(rh, np.asarray(q, np.float32).astype(np.float64))
        out[t, :3] = f["p_ee"]
        out[t, 3:] = f["quat"]
    return out


# ---------------------------------------------------------------------------
# random numbers
# ---------------------------------------------------------------------------

def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(o, C.c_uint32))
    return o


def normals(rng_seed, seed_idx, target_key, stage, it, n):
    z = np.zeros(n)
    lib().or_normals(rng_seed, seed_idx, target_key, stage, it, n, _ptr(z))
    return z


def uniform_seed(robot, rng_seed, seed_idx, target_key):
    rh = _rh(robot)
    th = np.zeros(rh.n)
    lib().or_uniform_seed(C.byref(rh.c), rng_seed, seed_idx, target_key, _ptr(th))
    return th


# ---------------------------------------------------------------------------
# stages on one seed
# ---------------------------------------------------------------------------

def _stage(fn, robot, target, p, seed_idx, target_key, theta, iters_key, with_sens=False):
    rh = _rh(robot)
    n = rh.n
    pr = params(p)
    K = int(p[iters_key])
    th = _d(np.asarray(theta, np.float64)).copy()
    traj = np.zeros((K + 1, n + 2))
    marg = np.zeros(max(K, 1))
    sens = np.zeros(max(K, 1))
    st = _Stats()
    extra = [_ptr(sens)] if with_sens else []
    rc = fn(C.byref(rh.c), _ptr(_d(target)), C.byref(pr), seed_idx, target_key, _ptr(th),
            _ptr(traj), _ptr(marg), *extra, C.byref(st))
    if rc != 0:
        raise ValueError("oracle stage rejected its input")
    return dict(theta=th, traj=traj, margin=marg[:K], sens=sens[:K], stats=st.as_dict())


def cd(robot, target, p, seed_idx, target_key, theta):
    """PO-CCD on one seed; returns theta, traj [(K+1), n+2], margin [K], stats."""
    return _stage(lib().or_cd, robot, target, p, seed_idx, target_key, theta, "cd_sweeps")


def polish(robot, target, p, seed_idx, target_key, theta):
    """PJ-IK on one seed; same layout as ``cd`` plus sens [K], the
    single-precision conditioning of each iteration's step (rad)."""
    return _stage(lib().or_polish, robot, target, p, seed_idx, target_key, theta, "polish_iters",
                  with_sens=True)


def cd_candidates(robot, target, p, theta, k):
    """Per-joint PO-CCD candidates at theta for iteration k."""
    rh = _rh(robot)
    n = rh.n
    out = {x: np.zeros(n) for x in ("dp", "dor", "sp", "so")}
    pr = params(p)
    rc = lib().or_cd_candidates(C.byref(rh.c), _ptr(_d(target)), C.byref(pr), _ptr(_d(theta)), k,
                                _ptr(out["dp"]), _ptr(out["dor"]), _ptr(out["sp"]),
                                _ptr(out["so"]))
    if rc != 0:
        raise ValueError("or_cd_candidates rejected its input")
    return out


def pjik_steps(robot, target, p, theta):
    """PJ-IK step vectors at theta: lm (unclipped), gd, gn, dogleg, single, single_idx."""
    rh = _rh(robot)
    n = rh.n
    out = {x: np.zeros(n) for x in ("lm", "gd", "gn", "dogleg", "single")}
    idx = C.c_int32(-1)
    pr = params(p)
    rc = lib().or_pjik_steps(C.byref(rh.c), _ptr(_d(target)), C.byref(pr), _ptr(_d(theta)),
                             _ptr(out["lm"]), _ptr(out["gd"]), _ptr(out["gn"]),
                             _ptr(out["dogleg"]), _ptr(out["single"]), C.byref(idx))
    if rc != 0:
        raise ValueError("or_pjik_steps rejected its input")
    out["single_idx"] = int(idx.value)
    return out


def collide(robot, scene, theta):
    rh = _rh(robot)
    sh = scene if isinstance(scene, SceneHandle) else SceneHandle(scene)
    f = C.c_int32(0)
    md = C.c_double(0)
    rc = lib().or_collide(C.byref(rh.c), C.byref(sh.c), _ptr(_d(theta)), C.byref(f), C.byref(md))
    if rc != 0:
        raise ValueError("or_collide rejected the robot")
    return int(f.value), float(md.value)


def select(flag, cost, k):
    fl = np.ascontiguousarray(flag, dtype=np.int32)
    c = _d(cost)
    o = np.zeros(k, np.int32)
    lib().or_select(int(fl.shape[0]), _ptr(fl, C.c_int32), _ptr(c), k, _ptr(o, C.c_int32))
    return o


def resample(robot, offsets, q_in, cost_in, p, target_keys=None):
    """Top-K ranking and floor(B/K) noisy copies per target (Alg. HJCD-IK):
    q_in [S, n], cost_in [S] -> q_out [T * B', n], B' = floor(B/K) K."""
    rh = _rh(robot)
    n = rh.n
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    T = offs.shape[0] - 1
    K, B = int(p["resample_K"]), int(p["resample_B"])
    Bp = (B // K) * K if K > 0 else 0
    q = _d(np.asarray(q_in, np.float64).reshape(-1))
    c = _d(cost_in)
    tk = None if target_keys is None else np.ascontiguousarray(target_keys, dtype=np.uint32)
    out = np.zeros((T * Bp, n))
    pr = params(p)
    rc = lib().or_resample(C.byref(rh.c), T, _ptr(offs, C.c_int64), _ptr(q), _ptr(c), _ptr(tk, C.c_uint32),
                           C.byref(pr), _ptr(out))
    if rc != 0:
        raise ValueError("or_resample rejected its input")
    return out


def warm_seeds(robot, q_prev, k, M, p, target_keys=None):
    """Tracking warm start: q_prev [T*k, n] previous solutions -> seeds
    [T*M, n] (seed m of target t from solution m mod k, perturbed for m >= k)."""
    rh = _rh(robot)
    n = rh.n
    qp = _d(np.asarray(q_prev, np.float64).reshape(-1))
    T = qp.shape[0] // (k * n)
    tk = None if target_keys is None else np.ascontiguousarray(target_keys, dtype=np.uint32)
    out = np.zeros((T * M, n))
    pr = params(p)
    rc = lib().or_warm_seeds(C.byref(rh.c), T, int(k), _ptr(qp), int(M), _ptr(tk, C.c_uint32), C.byref(pr),
                             _ptr(out))
    if rc != 0:
        raise ValueError("or_warm_seeds rejected its input")
    return out


def select_near(flag, cost, err_p, err_o, q, q_ref, k, succ_pos, succ_ori):
    """Order of the k seeds nearest to q_ref among the successful ones, then
    the rest by (flag, cost); q [m, n]."""
    f = np.ascontiguousarray(flag, dtype=np.int32)
    m = f.shape[0]
    qq = _d(np.asarray(q, np.float64).reshape(-1))
    n = qq.shape[0] // max(m, 1) if m else len(q_ref)
    o = np.zeros(k, np.int32)
    rc = lib().or_select_near(m, n, _ptr(f, C.c_int32), _ptr(_d(cost)), _ptr(_d(err_p)), _ptr(_d(err_o)), _ptr(qq),
                              _ptr(_d(q_ref)), float(succ_pos), float(succ_ori), k, _ptr(o, C.c_int32))
    if rc != 0:
        raise ValueError("or_select_near rejected its input")
    return o


# ---------------------------------------------------------------------------
# operation counts
# ---------------------------------------------------------------------------

def ops_reset():
    lib().or_ops_reset()


def ops_get():
    """{category: dict(add, mul, div, sqrt, trans, units, flops)} with flops =
    add + mul + div + sqrt (transcendental calls counted apart)."""
    out = {}
    buf = (C.c_uint64 * 6)()
    for i, name in enumerate(OPS_CATEGORIES):
        lib().or_ops_get(i, buf)
        d = dict(zip(("add", "mul", "div", "sqrt", "trans", "units"), [int(x) for x in buf]))
        d["flops"] = d["add"] + d["mul"] + d["div"] + d["sqrt"]
        out[name] = d
    return out


# ---------------------------------------------------------------------------
# whole pipeline
# ---------------------------------------------------------------------------

def solve(robot, scene, targets, offsets, p, seeds=None, target_keys=None, nthreads=0):
    """Full HJCD-IK solve on T targets (one robot).  ``targets`` [T, 7];
    ``offsets`` int64 [T+1]; ``seeds`` None (Philox) or [S, n] float;
    returns per-seed and per-target arrays."""
    rh = _rh(robot)
    sh = scene if isinstance(scene, SceneHandle) else SceneHandle(scene)
    n = rh.n
    tg = _d(np.asarray(targets, np.float64).reshape(-1, 7))
    T = tg.shape[0]
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    if p["resample_K"] > 0:
        K = p["resample_K"]
        Sp = T * (p["resample_B"] // K) * K
    else:
        Sp = int(offs[-1])
    k = int(p["top_k"])
    sd = None if seeds is None else _d(np.asarray(seeds, np.float64).reshape(-1))
    tk = None if target_keys is None else np.ascontiguousarray(target_keys, dtype=np.uint32)
    out = dict(q_seed=np.zeros((Sp, n)), errp_seed=np.zeros(Sp), erro_seed=np.zeros(Sp),
               cost_seed=np.zeros(Sp), flag_seed=np.zeros(Sp, np.int32),
               q_out=np.zeros((T, k, n)), err_p=np.zeros((T, k)), err_o=np.zeros((T, k)),
               flag_out=np.zeros((T, k), np.int32), n_free=np.zeros(T, np.int32),
               solved=np.zeros(T, np.int32))
    pr = params(p)
    ip = C.c_int32
    rc = lib().or_solve(C.byref(rh.c), C.byref(sh.c), T, _ptr(tg), _ptr(offs, C.c_int64),
                        _ptr(sd), _ptr(tk, C.c_uint32), C.byref(pr),
                        _ptr(out["q_seed"]), _ptr(out["errp_seed"]), _ptr(out["erro_seed"]),
                        _ptr(out["cost_seed"]), _ptr(out["flag_seed"], ip), _ptr(out["q_out"]),
                        _ptr(out["err_p"]), _ptr(out["err_o"]), _ptr(out["flag_out"], ip),
                        _ptr(out["n_free"], ip), _ptr(out["solved"], ip), int(nthreads))
    if rc != 0:
        raise ValueError("or_solve rejected its input")
    return out
