"""Evaluation metrics over solver outputs (host numpy; not part of the solve).

Solution diversity (Sec. V, the MMD table): the maximum mean discrepancy
between a solver's returned joint configurations for one target and a
reference sample of independently seeded solutions of the same target.  The
paper does not state its kernel; this module uses the Gaussian kernel
k(x, y) = exp(-|x - y|^2 / (2 h^2)) on joint vectors (rad) with a fixed
bandwidth h, and the biased (V-statistic) estimate of MMD^2, which is >= 0.
"""
from __future__ import annotations

import numpy as np


def _gram(A, B, h):
    d = np.sum((A[:, None, :] - B[None, :, :]) ** 2, axis=-1)
    return np.exp(-d / (2.0 * h * h))


def mmd2(X, Y, h: float = 1.0) -> float:
    """Biased MMD^2 between samples X [m, n] and Y [k, n] (Gaussian kernel,
    bandwidth h)."""
    X = np.asarray(X, np.float64)
    Y = np.asarray(Y, np.float64)
    if X.shape[0] == 0 or Y.shape[0] == 0:
        raise ValueError("mmd2 needs non-empty samples")
    v = _gram(X, X, h).mean() + _gram(Y, Y, h).mean() - 2.0 * _gram(X, Y, h).mean()
    return float(max(v, 0.0))


def mmd(X, Y, h: float = 1.0) -> float:
    return float(np.sqrt(mmd2(X, Y, h)))
