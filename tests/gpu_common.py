"""Shared helpers of the GPU parity tests (GPU side through the C-ABI binding,
reference side through the FP64 oracle, inputs from the workload generators)."""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2401_14762_amd as cs
    cs.library()     # raises if the HIP library is missing: no fallback
    return torch


def note(msg: str) -> None:
    """Print a progress line that names the case before a GPU step."""
    print(msg, file=sys.stderr, flush=True)


def to_dev(torch, a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def np_of(t):
    return t.detach().cpu().numpy()


def rel_err_rows(est, ref):
    dt = np.complex128 if (np.iscomplexobj(est) or np.iscomplexobj(ref)) else np.float64
    est = np.asarray(est, dtype=dt)
    ref = np.asarray(ref, dtype=dt)
    return np.linalg.norm(est - ref, axis=1) / np.maximum(np.linalg.norm(ref, axis=1), 1e-30)


# Near-tie thresholds for the greedy decisions.  A decision is counted as a
# near-tie when its gap to the next candidate is below either threshold:
#
# GAP, relative to the largest compared value.  An FP32 sum of M <= 96
# products carries a relative error of about sqrt(M) 2^-24 ~ 6e-7 of the
# largest correlation, and the FP32 normal-equations solve one of about
# kappa(B)^2 2^-24 ~ 3e-6 for the Gaussian sub-dictionaries met here
# (|c| <= 45 of M = 80 columns); 1e-5 is above both.
#
# GAP_ABS, relative to the scale on which rounding enters (the oracle's
# sel_gap_abs / prune_gap_abs).  The residual r = y - A x of Alg. 3 step 4 is
# formed by cancellation, so its rounding error is a multiple of 2^-24 ||y||,
# not of ||r||: late in a solve, when ||r|| << ||y||, a correlation gap that
# is large next to max|p| can still sit below FP32 resolution.  The typical
# error of a correlation is about (kappa(G_q) / sqrt(M) + 1 + sqrt(K / M))
# 2^-24 ||y|| (the coefficient error kappa 2^-24 ||s|| seen through one atom,
# the M-term dot product, the K-term residual sum) ~ 5.5 2^-24 ||y|| with
# kappa ~ 36, K = 20, M = 80; that of one least-squares coefficient about
# kappa 2^-24 ||s|| / sqrt(|c|) ~ 6 2^-24 ||s||.  Gaps below 8 2^-24 on these
# scales are counted as near-ties.
GAP = 1e-5
GAP_ABS = 8 * 2.0 ** -24
STOP_MARGIN = 1e-3
PIVOT = 1e-6


def assert_fista_parity(X_gpu, A, Y, lam, L, iters, floor=1e-5, **kw):
    """FISTA parity: per pixel, the GPU's relative error against the FP64
    oracle is at most max(floor, 30 x) that of a plain FP32 evaluation of the
    same iteration (the oracle's FP32 rounding model), and over the cube the
    largest and the median error are at most twice the rounding model's.
    Where the problem is well conditioned this is the 1e-5 bar; where a 2^-24
    perturbation already moves x by more (small lambda, many iterations), the
    bar is what FP32 arithmetic permits."""
    import oracle
    ref = oracle.fista(A, Y, lam, L, iters, **kw)
    r32 = oracle.fista(A, Y, lam, L, iters, dtype=np.float32, **kw)
    e = rel_err_rows(X_gpu, ref["X"])
    e32 = rel_err_rows(r32["X"], ref["X"])
    per_pixel = np.maximum(floor, 30.0 * e32)
    bad = np.nonzero(e > per_pixel)[0]
    assert len(bad) == 0, f"pixels {bad[:8]}: err {e[bad[:8]]} vs fp32 model {e32[bad[:8]]}"
    assert e.max() <= max(floor, 2.0 * e32.max()), (e.max(), e32.max())
    assert np.median(e) <= max(floor / 10, 2.0 * np.median(e32)), (np.median(e), np.median(e32))
    return ref, e


def assert_admm_parity(X_gpu, Z_gpu, A, Y, lam, alpha, iters, floor=1e-5, **kw):
    """ADMM parity, the bar of assert_fista_parity applied to x^I and z^I:
    per pixel at most max(floor, 30 x) the error of the oracle's FP32
    rounding model of Alg. 2 (which solves step 1 with an FP32 Cholesky
    factor), and cube-wide max and median at most twice the model's."""
    import oracle
    ref = oracle.admm(A, Y, lam, alpha, iters, **kw)
    r32 = oracle.admm(A, Y, lam, alpha, iters, dtype=np.float32, **kw)
    for name, got in (("X", X_gpu), ("Z", Z_gpu)):
        if got is None:
            continue
        e = rel_err_rows(got, ref[name])
        e32 = rel_err_rows(r32[name], ref[name])
        per_pixel = np.maximum(floor, 30.0 * e32)
        bad = np.nonzero(e > per_pixel)[0]
        assert len(bad) == 0, f"{name} pixels {bad[:8]}: err {e[bad[:8]]} vs fp32 model {e32[bad[:8]]}"
        assert e.max() <= max(floor, 2.0 * e32.max()), (name, e.max(), e32.max())
        assert np.median(e) <= max(floor / 10, 2.0 * np.median(e32)), (name, np.median(e), np.median(e32))
    return ref


def assert_cfista_parity(X_gpu, A, Y, lam, L, iters, floor=1e-5, **kw):
    """Complex FISTA parity: the bar of assert_fista_parity with the complex
    oracle (complex128) and its complex64 rounding model, errors measured in
    the complex 2-norm of each pixel's x."""
    import oracle
    ref = oracle.fista_complex(A, Y, lam, L, iters, **kw)
    r32 = oracle.fista_complex(A, Y, lam, L, iters, dtype=np.complex64, **kw)
    e = rel_err_rows(X_gpu, ref["X"])
    e32 = rel_err_rows(r32["X"], ref["X"])
    per_pixel = np.maximum(floor, 30.0 * e32)
    bad = np.nonzero(e > per_pixel)[0]
    assert len(bad) == 0, f"pixels {bad[:8]}: err {e[bad[:8]]} vs complex64 model {e32[bad[:8]]}"
    assert e.max() <= max(floor, 2.0 * e32.max()), (e.max(), e32.max())
    assert np.median(e) <= max(floor / 10, 2.0 * np.median(e32)), (np.median(e), np.median(e32))
    return ref, e


def assert_cadmm_parity(X_gpu, Z_gpu, A, Y, lam, alpha, iters, floor=1e-5, **kw):
    """Complex ADMM parity: the bar of assert_admm_parity with the complex
    oracle (complex128) and its complex64 rounding model, on x^I and z^I."""
    import oracle
    ref = oracle.admm_complex(A, Y, lam, alpha, iters, **kw)
    r32 = oracle.admm_complex(A, Y, lam, alpha, iters, dtype=np.complex64, **kw)
    for name, got in (("X", X_gpu), ("Z", Z_gpu)):
        if got is None:
            continue
        e = rel_err_rows(got, ref[name])
        e32 = rel_err_rows(r32[name], ref[name])
        per_pixel = np.maximum(floor, 30.0 * e32)
        bad = np.nonzero(e > per_pixel)[0]
        assert len(bad) == 0, f"{name} pixels {bad[:8]}: err {e[bad[:8]]} vs complex64 model {e32[bad[:8]]}"
        assert e.max() <= max(floor, 2.0 * e32.max()), (name, e.max(), e32.max())
        assert np.median(e) <= max(floor / 10, 2.0 * np.median(e32)), (name, np.median(e), np.median(e32))
    return ref


def ls_on_own_support(A, Y, S):
    """Per pixel, the FP64 least-squares solution of Alg. 3 step 2 on the
    pixel's own support (the non-negative entries of its row of S), as a
    dense P x N matrix: what x must be once a greedy solver has chosen that
    support, whatever the choice."""
    import oracle
    A = np.asarray(A, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    P, N = Y.shape[0], A.shape[1]
    X = np.zeros((P, N))
    sizes = (S >= 0).sum(axis=1)
    for k in np.unique(sizes):
        rows = np.nonzero(sizes == k)[0]
        if k == 0:
            continue
        cols = np.stack([np.sort(S[r][S[r] >= 0]) for r in rows])
        sol = oracle.lstsq_on_support(A, Y[rows], cols)
        X[rows[:, None], cols] = sol
    return X
