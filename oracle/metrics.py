"""Quality metrics (FP64).  TEST INFRASTRUCTURE ONLY.

The paper's metric section is not part of the available text; PSNR is the
usual peak signal-to-noise ratio it names in Section IV, with the peak taken
as the largest magnitude of the reference cube and the mean squared error
over every entry.
"""
from __future__ import annotations

import numpy as np


def psnr(est: np.ndarray, ref: np.ndarray) -> float:
    """10 log10(peak^2 / MSE), peak = max |ref| over the whole cube.

    Identical inputs give +inf."""
    est = np.asarray(est, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    mse = float(np.mean((est - ref) ** 2))
    peak = float(np.max(np.abs(ref)))
    if mse == 0.0:
        return float("inf")
    return 10.0 * np.log10(peak * peak / mse)


def rel_err(est: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Per-row ||est - ref||_2 / max(||ref||_2, 1e-30)."""
    est = np.asarray(est, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    num = np.linalg.norm(est - ref, axis=-1)
    den = np.maximum(np.linalg.norm(ref, axis=-1), 1e-30)
    return num / den


def lasso_objective(A: np.ndarray, Y: np.ndarray, X: np.ndarray, lam: float) -> np.ndarray:
    """H(x) = 1/2 ||A x - y||^2 + lam ||x||_1 per pixel (Eq. 2)."""
    A = np.asarray(A, dtype=np.float64)
    R = np.asarray(X, dtype=np.float64) @ A.T - np.asarray(Y, dtype=np.float64)
    return 0.5 * np.sum(R * R, axis=1) + lam * np.sum(np.abs(X), axis=1)


def lasso_kkt_residual(A: np.ndarray, Y: np.ndarray, X: np.ndarray, lam: float) -> np.ndarray:
    """Largest violation of the LASSO optimality conditions, per pixel.

    With g = A^T (A x - y): g_j + lam sign(x_j) = 0 where x_j != 0 and
    |g_j| <= lam where x_j = 0."""
    A = np.asarray(A, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    G = (X @ A.T - np.asarray(Y, dtype=np.float64)) @ A
    on = X != 0.0
    v_on = np.where(on, np.abs(G + lam * np.sign(X)), 0.0)
    v_off = np.where(on, 0.0, np.maximum(np.abs(G) - lam, 0.0))
    return np.max(np.maximum(v_on, v_off), axis=1)
