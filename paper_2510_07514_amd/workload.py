"""Seeded synthetic workloads for the batched HJCD-IK solve.

This module is shared by the GPU path (bench, tests) and by the FP64 oracle's
test harness, so it holds *no* arithmetic of the method: it draws robot
descriptions (DH tables, joint limits, link spheres), obstacle scenes, target
configurations q*, seeds and arrival streams with numpy's PCG64, and nothing
else.  A target pose is *defined* as FK(q*) and each side computes it with its
own forward kinematics.

Stand-ins: the paper evaluates on a Franka Panda and a Fetch with Halton-sampled
targets and on the MotionBenchMaker box_panda scene (Sec. V).  None of those
assets are used; the robots below are Panda-like / UR-like DH chains and random
DH chains, and the scenes are random sphere/box clutter of the same scale.

Every array that the solvers read is float32 (targets, seeds, tables are
rounded once here or by the FK that defines the target), so both sides see the
same bits.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

PI = math.pi

# DH convention codes (same numeric values in the C ABI and in the oracle).
DH_MODIFIED = 0
DH_STANDARD = 1


# ----------------------------------------------------------------------------
# Robots
# ----------------------------------------------------------------------------

@dataclass
class Robot:
    """A serial chain of revolute joints in DH form plus link spheres.

    a, d, alpha, offset, q_min, q_max: per-joint DH parameters and limits.
    tool: 4x4 row-major rigid transform from the last joint frame to the
    end effector.  Link l (0 = base, l = 1..n moves with joint l) carries
    spheres given in its own frame as rows (x, y, z, r) of ``sphere_xyzr``
    with link index ``sphere_link``.  Self-collision is tested between
    spheres of links whose indices differ by at least ``min_link_gap``
    (0 disables self-collision).
    """
    name: str
    convention: int
    a: np.ndarray
    d: np.ndarray
    alpha: np.ndarray
    offset: np.ndarray
    q_min: np.ndarray
    q_max: np.ndarray
    tool: np.ndarray
    sphere_link: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    sphere_xyzr: np.ndarray = field(default_factory=lambda: np.zeros((0, 4), np.float64))
    min_link_gap: int = 3

    @property
    def dof(self) -> int:
        return int(self.a.shape[0])


def _tool_tz(z: float) -> np.ndarray:
    t = np.eye(4)
    t[2, 3] = z
    return t


def panda_like() -> Robot:
    """7-DoF Panda-like chain in modified DH with a 0.107 m flange."""
    a = np.array([0.0, 0.0, 0.0, 0.0825, -0.0825, 0.0, 0.088])
    d = np.array([0.333, 0.0, 0.316, 0.0, 0.384, 0.0, 0.0])
    alpha = np.array([0.0, -PI / 2, PI / 2, PI / 2, -PI / 2, PI / 2, PI / 2])
    q_min = np.array([-2.8973, -1.7628, -2.8973, -3.0718, -2.8973, -0.0175, -2.8973])
    q_max = np.array([2.8973, 1.7628, 2.8973, -0.0698, 2.8973, 3.7525, 2.8973])
    return Robot("panda_like", DH_MODIFIED, a, d, alpha, np.zeros(7), q_min, q_max,
                 _tool_tz(0.107))


def ur_like() -> Robot:
    """6-DoF UR-like chain in standard DH, limits +-pi, no tool offset."""
    a = np.array([0.0, -0.425, -0.392, 0.0, 0.0, 0.0])
    d = np.array([0.163, 0.0, 0.0, 0.134, 0.100, 0.100])
    alpha = np.array([PI / 2, 0.0, 0.0, PI / 2, -PI / 2, 0.0])
    return Robot("ur_like", DH_STANDARD, a, d, alpha, np.zeros(6),
                 np.full(6, -PI), np.full(6, PI), np.eye(4))


def random_chain(rng: np.random.Generator, n: int, name: str | None = None) -> Robot:
    """Random modified-DH chain: alpha in {0, +-pi/2}, a, d ~ U[0.05, 0.3] m,
    limits +-2.9 rad, no tool offset."""
    alpha = rng.choice(np.array([0.0, PI / 2, -PI / 2]), size=n)
    a = rng.uniform(0.05, 0.3, size=n)
    d = rng.uniform(0.05, 0.3, size=n)
    return Robot(name or f"random{n}", DH_MODIFIED, a, d, alpha, np.zeros(n),
                 np.full(n, -2.9), np.full(n, 2.9), np.eye(4))


def chained_panda(copies: int) -> Robot:
    """6 x copies-DoF chain built from repeated copies of the Panda-like
    chain's first six joints (DH rows and limits), with the 0.107 m flange as
    the tool: the DoF-scaling robots of the paper's Sec. V study (12, 18 and
    24 DoF for 2, 3 and 4 copies).  No link spheres (open world)."""
    p = panda_like()
    rep = lambda x: np.tile(np.asarray(x[:6]), copies)
    return Robot(f"chained_panda{6 * copies}", DH_MODIFIED, rep(p.a), rep(p.d), rep(p.alpha),
                 np.zeros(6 * copies), rep(p.q_min), rep(p.q_max), _tool_tz(0.107), min_link_gap=0)


def planar_chain(lengths, limit: float = PI) -> Robot:
    """Planar nR chain (alpha = 0, d = 0, a = link lengths) in modified DH.
    The last link length is carried by the tool so the end effector sits at
    the tip of the last link."""
    lengths = np.asarray(lengths, dtype=np.float64)
    n = lengths.shape[0]
    a = np.concatenate([[0.0], lengths[:-1]])
    tool = np.eye(4)
    tool[0, 3] = lengths[-1]
    return Robot(f"planar{n}", DH_MODIFIED, a, np.zeros(n), np.zeros(n), np.zeros(n),
                 np.full(n, -limit), np.full(n, limit), tool, min_link_gap=0)


def _next_origin_in_link_frame(robot: Robot, link: int) -> np.ndarray:
    """Where the next joint's origin (or the tool origin for the last link)
    sits in link ``link``'s frame at the zero configuration.  This is robot
    *description* data (it places spheres along the link), not a solver
    step; it only reads the fixed DH constants."""
    n = robot.dof
    if link == n:
        return robot.tool[:3, 3].copy()
    j = link  # joint j+1 (0-based index j) connects link `link` to link+1
    a, d, al, off = robot.a[j], robot.d[j], robot.alpha[j], robot.offset[j]
    if robot.convention == DH_MODIFIED:
        return np.array([a, -d * math.sin(al), d * math.cos(al)])
    return np.array([a * math.cos(off), a * math.sin(off), d])


def place_link_spheres(robot: Robot, counts, radius) -> Robot:
    """Put ``counts[l]`` spheres on link l, evenly along the segment from the
    link frame origin to the next joint origin (Sec. IV-C uses offline
    bounding spheres; these synthetic ones stand in).  ``radius`` is a
    callable (link, i) -> r."""
    links, rows = [], []
    for link, cnt in enumerate(counts):
        end = _next_origin_in_link_frame(robot, link)
        for i in range(cnt):
            f = (i + 0.5) / cnt
            rows.append([end[0] * f, end[1] * f, end[2] * f, radius(link, i)])
            links.append(link)
    robot.sphere_link = np.asarray(links, dtype=np.int32)
    robot.sphere_xyzr = np.asarray(rows, dtype=np.float64).reshape(-1, 4)
    return robot


# ----------------------------------------------------------------------------
# Scenes
# ----------------------------------------------------------------------------

@dataclass
class Scene:
    """Obstacles in the world frame: spheres (x, y, z, r) and axis-aligned
    boxes (cx, cy, cz, hx, hy, hz), all float32."""
    spheres: np.ndarray
    boxes: np.ndarray


def _centres(rng, count, lo, hi, exclude_r):
    """Uniform centres in the box [lo, hi], rejecting a ball of radius
    exclude_r around the base and the column above it (|c_xy| < 0.25 m,
    c_z < 0.55 m) where the static base links stand."""
    out = []
    while len(out) < count:
        c = rng.uniform(lo, hi)
        if np.linalg.norm(c) < exclude_r:
            continue
        if math.hypot(c[0], c[1]) < 0.25 and c[2] < 0.55:
            continue
        out.append(c)
    return np.asarray(out).reshape(-1, 3)


def random_scene(rng, n_spheres, n_boxes, lo, hi, r_range=(0.02, 0.10),
                 half_range=(0.02, 0.15), exclude_r=0.3) -> Scene:
    sph = np.zeros((n_spheres, 4))
    if n_spheres:
        sph[:, :3] = _centres(rng, n_spheres, lo, hi, exclude_r)
        sph[:, 3] = rng.uniform(*r_range, size=n_spheres)
    box = np.zeros((n_boxes, 6))
    if n_boxes:
        box[:, :3] = _centres(rng, n_boxes, lo, hi, exclude_r)
        box[:, 3:] = rng.uniform(*half_range, size=(n_boxes, 3))
    return Scene(sph.astype(np.float32), box.astype(np.float32))


def empty_scene() -> Scene:
    return Scene(np.zeros((0, 4), np.float32), np.zeros((0, 6), np.float32))


# ----------------------------------------------------------------------------
# Solver parameters (defaults; every value the paper leaves open is a reading)
# ----------------------------------------------------------------------------

def default_params(**over) -> dict:
    """Parameters of PO-CCD (Alg. PO-CCD), PJ-IK (Alg. PJ-IK) and the outer loop (Alg. HJCD-IK).
    The paper prints none of these values except that lambda > 0."""
    p = dict(
        cd_sweeps=20, polish_iters=20,
        eps_cd=5e-3, nu_cd=5e-2,            # PO-CCD coarse exit (m, rad)
        gamma=1e-7,                          # PO-CCD improvement threshold (squared units)
        delta0=1.0, delta_decay=0.9, delta_min=0.1,   # annealing delta(k)
        proj_eps=1e-5,                       # min distance (m) of EE / target from a joint axis
        tie_eps=1e-5,                        # greedy picks: scores within this (m / rad) of the best tie
        lam=1e-3, lambda_gn=1e-4,            # LM damping; GN regulariser in the dogleg
        trust_R=0.2, ls_beta=2.0, ls_A=4,    # trust region, backtracking schedule
        weight_mode=0,                       # 0 = row-normalised W, 1 = identity
        eps_pol=1e-5, ups_pol=1e-5,          # PJ-IK exit (m, rad)
        sigma=0.05, mu=0.0,                  # perturbation N(mu, sigma^2 I)
        resample_K=0, resample_B=0,          # 0 = no top-K/replicate between stages
        top_k=1,
        succ_pos=1e-3, succ_ori=PI / 180.0,  # success at 1 mm / 1 deg
        rng_seed=0,
    )
    p.update(over)
    return p


# ----------------------------------------------------------------------------
# Draws
# ----------------------------------------------------------------------------

def uniform_configs(rng, robot: Robot, count: int) -> np.ndarray:
    """count x n configurations uniform within the joint limits, float32."""
    u = rng.uniform(size=(count, robot.dof))
    q = robot.q_min + (robot.q_max - robot.q_min) * u
    return q.astype(np.float32)


def log_uniform_int(rng, lo, hi, size):
    return np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), size=size))).astype(np.int64)


@dataclass
class Batch:
    """One batched solve: robots, per-target robot ids, target configurations
    q* (a target pose is FK(q*)), CSR seed offsets, optional host seeds
    (n_max x S float32 SoA, NaN-free, within limits), scene and parameters."""
    name: str
    robots: list
    robot_of_target: np.ndarray     # int32 [T]
    q_star: list                    # per target: float32 [n_robot]
    seed_offsets: np.ndarray        # int64 [T+1]
    seeds: np.ndarray | None        # float32 [n_max][S] or None (device RNG)
    scene: Scene
    params: dict
    rng_seed: int

    @property
    def T(self) -> int:
        return int(self.robot_of_target.shape[0])

    @property
    def S(self) -> int:
        return int(self.seed_offsets[-1])

    @property
    def n_max(self) -> int:
        return max(r.dof for r in self.robots)


def _seeds_soa(rng, robots, robot_of_target, offsets):
    n_max = max(r.dof for r in robots)
    S = int(offsets[-1])
    out = np.zeros((n_max, S), np.float32)
    for t in range(len(robot_of_target)):
        r = robots[robot_of_target[t]]
        b, e = int(offsets[t]), int(offsets[t + 1])
        out[: r.dof, b:e] = uniform_configs(rng, r, e - b).T
    return out


def config_tiny(host_seeds: bool = True) -> Batch:
    """Plain method, tiny: Panda-like chain, 8 targets x 64 seeds, self-collision
    only with one 6 cm sphere per link, 20 + 20 iterations, lambda = 1e-3."""
    rng = np.random.default_rng(1)
    robot = place_link_spheres(panda_like(), [1] * 8, lambda l, i: 0.06)
    T, M = 8, 64
    q_star = list(uniform_configs(rng, robot, T))
    offs = np.arange(T + 1, dtype=np.int64) * M
    seeds = _seeds_soa(rng, [robot], np.zeros(T, np.int32), offs) if host_seeds else None
    return Batch("tiny_panda_8x64", [robot], np.zeros(T, np.int32), q_star, offs, seeds,
                 empty_scene(), default_params(top_k=1, rng_seed=1), 1)


def _panda60(rng) -> Robot:
    r = rng.uniform(0.03, 0.08, size=60)
    counts = [8, 8, 8, 8, 7, 7, 7, 7]
    starts = np.cumsum([0] + counts)
    rob = place_link_spheres(panda_like(), counts, lambda l, i: float(r[starts[l] + i]))
    # Spheres reaching the link ends make links 4 and 7 (0.088 m apart) overlap
    # in every configuration; like an allowed-collision matrix, self pairs are
    # tested only four or more links apart.
    rob.min_link_gap = 4
    return rob


def config_batched(T: int = 1000, M: int = 1024, host_seeds: bool = False) -> Batch:
    """Batched Panda-like chain: T targets x M seeds, 60 link spheres (r 3-8 cm),
    32 obstacle spheres (r 2-10 cm) in [-.6,.6]^2 x [0,1.2] outside a 0.3 m ball
    around the base; top-8 per target."""
    rng = np.random.default_rng(2)
    robot = _panda60(rng)
    scene = random_scene(rng, 32, 0, np.array([-0.6, -0.6, 0.0]), np.array([0.6, 0.6, 1.2]))
    q_star = list(uniform_configs(rng, robot, T))
    offs = np.arange(T + 1, dtype=np.int64) * M
    seeds = _seeds_soa(rng, [robot], np.zeros(T, np.int32), offs) if host_seeds else None
    return Batch(f"batched_panda_{T}x{M}", [robot], np.zeros(T, np.int32), q_star, offs,
                 seeds, scene, default_params(top_k=8, rng_seed=2), 2)


def config_uneven(T: int = 4096, host_seeds: bool = False, max_seeds: int = 2048) -> Batch:
    """Uneven batch: T targets spread by a seeded permutation over a 6-DoF UR-like
    chain, the Panda-like chain and a random 12-DoF chain; seeds per target
    log-uniform in [16, max_seeds]; 64 obstacle spheres; top-8."""
    rng = np.random.default_rng(3)
    panda = _panda60(rng)
    ur = ur_like()
    r12 = random_chain(rng, 12, "random12")
    for rob in (ur, r12):
        nl = rob.dof + 1
        rr = rng.uniform(0.03, 0.08, size=4 * nl)
        place_link_spheres(rob, [4] * nl, lambda l, i, rr=rr: float(rr[4 * l + i]))
        rob.min_link_gap = 4
    scene = random_scene(rng, 64, 0, np.array([-0.6, -0.6, 0.0]), np.array([0.6, 0.6, 1.2]))
    robots = [ur, panda, r12]
    share = np.array([T - 2 * (T // 3), T // 3, T // 3])
    rot = np.repeat(np.arange(3, dtype=np.int32), share)
    rot = rot[rng.permutation(T)]
    counts = log_uniform_int(rng, 16, max_seeds, T)
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    q_star = [uniform_configs(rng, robots[rot[t]], 1)[0] for t in range(T)]
    seeds = _seeds_soa(rng, robots, rot, offs) if host_seeds else None
    return Batch(f"uneven_{T}", robots, rot, q_star, offs, seeds, scene,
                 default_params(top_k=8, rng_seed=3), 3)


def config_large(T: int = 100_000, M: int = 256, host_seeds: bool = False) -> Batch:
    """Large: random 20-DoF chain with 6 spheres per moving link (r 2-6 cm),
    128 spheres + 128 boxes in [-1,1]^3, T x M seeds, 40 + 40 iterations, top-16."""
    rng = np.random.default_rng(5)
    robot = random_chain(rng, 20, "random20")
    rr = rng.uniform(0.02, 0.06, size=120)
    place_link_spheres(robot, [0] + [6] * 20, lambda l, i: float(rr[6 * (l - 1) + i]))
    robot.min_link_gap = 4
    scene = random_scene(rng, 128, 128, np.full(3, -1.0), np.full(3, 1.0))
    q_star = list(uniform_configs(rng, robot, T))
    offs = np.arange(T + 1, dtype=np.int64) * M
    seeds = _seeds_soa(rng, [robot], np.zeros(T, np.int32), offs) if host_seeds else None
    return Batch(f"large_random20_{T}x{M}", [robot], np.zeros(T, np.int32), q_star, offs,
                 seeds, scene, default_params(cd_sweeps=40, polish_iters=40, top_k=16,
                                              rng_seed=5), 5)


def config_dof(dof: int, T: int = 1000, M: int = 1000, host_seeds: bool = False) -> Batch:
    """DoF scaling (Sec. V, the chained-Panda study): the Panda-like chain
    (dof = 7) or its chained first six joints (dof = 12, 18, 24), T targets x
    M seeds (the paper's B = 1,000), open world (no obstacles, no self test),
    20 + 20 iterations, top-1."""
    if dof == 7:
        robot = panda_like()
        robot.min_link_gap = 0
    elif dof in (12, 18, 24):
        robot = chained_panda(dof // 6)
    else:
        raise ValueError("dof must be 7, 12, 18 or 24")
    rng = np.random.default_rng(60 + dof)
    q_star = list(uniform_configs(rng, robot, T))
    offs = np.arange(T + 1, dtype=np.int64) * M
    seeds = _seeds_soa(rng, [robot], np.zeros(T, np.int32), offs) if host_seeds else None
    return Batch(f"dof_{robot.name}_{T}x{M}", [robot], np.zeros(T, np.int32), q_star, offs,
                 seeds, empty_scene(), default_params(top_k=1, rng_seed=60 + dof), 60 + dof)


def tracking_paths(robot: Robot, tracks: int, steps: int, seed: int = 7, amp: float = 0.3,
                   period: int = 100) -> np.ndarray:
    """Joint-space paths for the tracking workload (Sec. V demonstration: a
    pose that moves along a path): per track a centre uniform in the limits
    shrunk by amp, and q*(s) = centre + amp sin(2 pi s / period + phase) per
    joint, phase uniform; returns float32 [steps][tracks][n] (inside the
    limits).  A target on the path is FK(q*(s))."""
    rng = np.random.default_rng(seed)
    lo, hi = robot.q_min + amp, robot.q_max - amp
    centre = lo + (hi - lo) * rng.uniform(size=(tracks, robot.dof))
    phase = rng.uniform(0.0, 2.0 * PI, size=(tracks, robot.dof))
    s = np.arange(steps)[:, None, None]
    q = centre[None] + amp * np.sin(2.0 * PI * s / period + phase[None])
    return np.clip(q, robot.q_min, robot.q_max).astype(np.float32)


def serving_stream(rate: float, duration: float, seed: int = 4):
    """Poisson request stream for the serving workload: arrival times (s),
    targets per request U{1..16} (Panda-like, FK of uniform configs), a
    per-request seed budget log-uniform in [32, 1024] seeds per target, and
    the robot (60 link spheres) and 32-sphere scene of the batched workload."""
    rng2 = np.random.default_rng(2)
    robot = _panda60(rng2)
    scene = random_scene(rng2, 32, 0, np.array([-0.6, -0.6, 0.0]), np.array([0.6, 0.6, 1.2]))
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=int(rate * duration * 1.3) + 16)
    t = np.cumsum(gaps)
    t = t[t < duration]
    n_req = t.shape[0]
    n_tgt = rng.integers(1, 17, size=n_req)
    budget = log_uniform_int(rng, 32, 1024, n_req)
    q_all = uniform_configs(rng, robot, int(n_tgt.sum()))
    q_star = np.split(q_all, np.cumsum(n_tgt)[:-1])
    return dict(robot=robot, scene=scene, arrival=t, n_targets=n_tgt, seeds_per_target=budget,
                q_star=q_star, params=default_params(top_k=1, rng_seed=4))


CONFIGS = {
    "tiny": config_tiny,
    "batched": config_batched,
    "uneven": config_uneven,
    "large": config_large,
    "dof7": lambda **kw: config_dof(7, **kw),
    "dof12": lambda **kw: config_dof(12, **kw),
    "dof18": lambda **kw: config_dof(18, **kw),
    "dof24": lambda **kw: config_dof(24, **kw),
}
