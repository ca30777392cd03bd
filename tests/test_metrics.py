"""The diversity metric (MMD with a Gaussian kernel) against its closed forms
and invariants (CPU only)."""
import numpy as np

from paper_2510_07514_amd import metrics as M


def test_mmd_of_identical_samples_is_zero():
    rng = np.random.default_rng(0)
    X = rng.normal(size=(30, 7))
    assert M.mmd2(X, X) < 1e-15
    assert M.mmd2(X, X[::-1]) < 1e-15


def test_mmd_single_points_closed_form():
    # one point each: MMD^2 = 2 - 2 exp(-d^2 / (2 h^2))
    x, y = np.zeros((1, 3)), np.array([[0.3, 0.0, 0.4]])
    for h in (0.5, 1.0, 2.0):
        assert abs(M.mmd2(x, y, h) - (2 - 2 * np.exp(-0.25 / (2 * h * h)))) < 1e-14


def test_mmd_brute_force_definition():
    rng = np.random.default_rng(1)
    X, Y = rng.normal(size=(5, 2)), rng.normal(size=(4, 2))
    k = lambda a, b: np.exp(-np.sum((a - b) ** 2) / 2.0)
    ref = (sum(k(a, b) for a in X for b in X) / 25 + sum(k(a, b) for a in Y for b in Y) / 16
           - 2 * sum(k(a, b) for a in X for b in Y) / 20)
    assert abs(M.mmd2(X, Y, 1.0) - ref) < 1e-14


def test_mmd_symmetric_and_separates_shifts():
    rng = np.random.default_rng(2)
    X, Y = rng.normal(size=(40, 4)), rng.normal(size=(40, 4))
    assert abs(M.mmd2(X, Y) - M.mmd2(Y, X)) < 1e-14
    near = M.mmd2(X, Y)
    far = M.mmd2(X, Y + 3.0)
    assert far > 3 * near
    assert abs(M.mmd(X, Y) ** 2 - near) < 1e-14
