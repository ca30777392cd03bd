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


def compare_trajectories(gpu_traj, orc, n, wrap=False):
    """gpu_traj: [rows][n+2] float32 of one seed; orc: oracle stage dict.
    Compares rows 0..k* (k* = first tie iteration, inclusive); returns
    (ok, k_star, worst_error)."""
    k = first_tie(orc["margin"])
    rows = min(k + 1, gpu_traj.shape[0])
    g = gpu_traj[:rows].astype(np.float64)
    o = orc["traj"][:rows]
    d = np.abs(g - o)
    worst = float(d.max()) if d.size else 0.0
    return worst <= TOL_TRAJ, k, worst


def quat_close(a, b):
    """Distance between unit quaternions up to sign."""
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return min(np.max(np.abs(a - b)), np.max(np.abs(a + b)))


__all__ = ["TAU_DEC", "TOL_TRAJ", "say", "cuda", "soa", "targets_soa", "first_tie",
           "compare_trajectories", "quat_close", "math"]
