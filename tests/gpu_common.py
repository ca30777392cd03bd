"""Shared helpers of the GPU tests: context, robots, data movement and the
decision-margin rule for trajectory parity."""
import math
import sys

import numpy as np

TAU_DEC = 1e-6       # decision margin (m or rad) below which a seed is tie-affected
TOL_TRAJ = 1e-4      # per-iteration trajectory tolerance: 1e-4 m / 1e-4 rad


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def cuda(x, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def soa(q_rows, n):
    """[S][n] -> float32 [n][S] on the device."""
    a = np.ascontiguousarray(np.asarray(q_rows, np.float32).reshape(-1, n).T)
    return cuda(a)


def targets_soa(tg):
    return cuda(np.ascontiguousarray(np.asarray(tg, np.float32).T))


def first_tie(margin):
    """Index of the first iteration whose decision margin is below TAU_DEC
    (len(margin) when there is none)."""
    bad = np.nonzero(np.asarray(margin) < TAU_DEC)[0]
    return int(bad[0]) if bad.size else len(margin)


SHADOW_FRAC = 0.25   # shadows must agree within TOL_TRAJ * SHADOW_FRAC
N_SHADOWS = 3


def shadow_horizon(orc, shadows):
    """Last row on which every FP64 shadow run (linearisations carrying
    single-precision-sized errors) stays within TOL_TRAJ * SHADOW_FRAC of
    the nominal oracle trajectory; rows beyond it are not reproducible in
    single precision and are not compared."""
    if not shadows:
        return orc["traj"].shape[0] - 1
    dv = np.max([np.abs(s["traj"] - orc["traj"]).max(axis=1) for s in shadows], axis=0)
    bad = np.nonzero(dv > TOL_TRAJ * SHADOW_FRAC)[0]
    return int(bad[0]) - 1 if bad.size else orc["traj"].shape[0] - 1


def compare_trajectories(gpu_traj, orc, n, shadows=None):
    """gpu_traj: [rows][n+2] float32 of one seed; orc: oracle stage dict.
    Compares rows 0..k* where k* is the first near-tie iteration (inclusive)
    or the shadow horizon, whichever comes first; returns (ok, k_star,
    worst_error).  k_star < number of iterations marks the seed as
    tie-affected."""
    k = min(first_tie(orc["margin"]), shadow_horizon(orc, shadows))
    rows = min(k + 1, gpu_traj.shape[0])
    g = gpu_traj[:rows].astype(np.float64)
    o = orc["traj"][:rows]
    d = np.abs(g - o)
    worst = float(d.max()) if d.size else 0.0
    return worst <= TOL_TRAJ, k, worst


def endpoint_ok(row, n, which, params):
    """The stage's own success test on the last trajectory row [theta, |r_p|,
    phi]: PO-CCD's exit tolerances (eps_cd, nu_cd) for CD, 1 mm / 1 deg for
    PJ-IK."""
    ep, phi = float(row[n]), float(row[n + 1])
    if which == "cd":
        return ep < params["eps_cd"] and phi < params["nu_cd"]
    return ep <= params["succ_pos"] and phi <= params["succ_ori"]


def quat_close(a, b):
    """Distance between unit quaternions up to sign."""
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return min(np.max(np.abs(a - b)), np.max(np.abs(a + b)))


__all__ = ["TAU_DEC", "TOL_TRAJ", "SHADOW_FRAC", "N_SHADOWS", "say", "cuda", "soa", "targets_soa",
           "first_tie", "shadow_horizon", "compare_trajectories", "endpoint_ok", "quat_close", "math"]
