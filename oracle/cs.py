"""FP64 reference solvers, batched over independent pixels.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline of the benchmark, never by the product path, and sharing no code
with it.

Each solver follows the paper's algorithm step by step in its notation:

* ``fista``   -- Alg. 1 (FISTA for the LASSO of Eq. 2)
* ``gomp``    -- Alg. 3 (generalised OMP, G atoms per iteration, prune to kappa)
* ``biht``    -- Alg. 4 (backtracking IHT)
* ``cosamp``  -- Alg. 5 (CoSaMP)
* ``biht_one_bit`` -- binary IHT on 1-bit measurements.  Not an algorithm of
  the paper (its BIHT is the backtracking variant of Alg. 4); it is defined
  here as x <- H_K(x + mu A^T (y - sgn(A x))), output x / ||x||.

Inputs are upcast to float64; every product is a plain NumPy matmul, every
least-squares solve is a Householder QR of the selected columns (LAPACK via
``numpy.linalg.qr``), the QR analogue of MATLAB's backslash.  Pixels are
independent, so every solver vectorises over the pixels that are still
iterating; nothing is blocked, fused or reordered beyond that.

Readings of points the paper leaves open (all shared with the GPU path by
specification, not by code):

* x^0 = 0 unless given; r^0 = y (Alg. 1, 3, 4, 5 initialisation).
* Stop rule: a pixel stops after the iteration in which Delta < eps, or (greedy
  solvers) ||r|| <= res_tol ||y||, or when max_iter iterations are done.  The
  wall-clock cap t_conv of Section II is replaced by the iteration cap.
* argmax_k: the k largest magnitudes, ordered by (magnitude desc, index asc).
* gOMP Alg. 3 step 1 never re-selects an index already in c, so |c| grows by
  exactly G per iteration; step 3's argmax_kappa runs over c only and is a
  no-op while |c| <= kappa; default iteration cap min(kappa, floor(M / G)).
* CoSaMP keeps the least-squares values on the kappa kept atoms (no re-solve).
* BIHT step 3 zeroes the entries of s outside h.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

STOP_CONVERGED = 1   # stopped by Delta < eps or the residual tolerance
STOP_ITER_CAP = 2    # ran the full iteration budget
STOP_FALLBACK = 4    # (GPU only) least squares redone in FP64
STOP_NONFINITE = 8   # non-finite measurements: x = 0, no iterations


def round_to_format(v, fmt: str) -> np.ndarray:
    """v rounded to a shorter floating-point format, returned as float64: a
    rounding model of products whose operands a 16-bit MFMA receives.  The
    value is first rounded to IEEE binary32 (as FP32 data is), then
    'bf16': bfloat16 keeps the upper 16 bits of the binary32 encoding (sign,
    8 exponent bits, 7 significand bits), rounded to nearest, ties to even
    significand; 'f16': IEEE binary16, rounded to nearest even.  'f64' and
    'f32' return v rounded to that format."""
    v32 = np.asarray(v, dtype=np.float64).astype(np.float32)
    if fmt == "f64":
        return np.asarray(v, dtype=np.float64)
    if fmt == "f32":
        return v32.astype(np.float64)
    if fmt == "f16":
        return v32.astype(np.float16).astype(np.float64)
    if fmt != "bf16":
        raise ValueError(f"unknown format {fmt}")
    bits = v32.view(np.uint32).astype(np.uint64)
    keep = (bits >> 16) & 1                      # lowest kept bit: ties go to the even one
    rounded = ((bits + 0x7FFF + keep) >> 16) << 16
    finite = np.isfinite(v32)
    out = np.where(finite, (rounded & 0xFFFFFFFF).astype(np.uint32).view(np.float32), v32)
    return out.astype(np.float64)


def _f64(a) -> np.ndarray:
    return np.asarray(a, dtype=np.float64)


def soft_threshold(v: np.ndarray, thr: float) -> np.ndarray:
    """sign(v) * max(|v| - thr, 0) elementwise (Alg. 1 step 2)."""
    return np.sign(v) * np.maximum(np.abs(v) - thr, 0.0)


def lipschitz(A: np.ndarray) -> float:
    """L = lambda_max(A^* A) = ||A||_2^2 (Eq. 2), from the SVD."""
    return float(np.linalg.norm(_f64(A), 2) ** 2)


def top_indices(values: np.ndarray, k: int, allowed: Optional[np.ndarray] = None) -> np.ndarray:
    """Per row, the k indices of largest |value| ordered by (|value| desc,
    index asc).  Entries where ``allowed`` is False are never chosen while an
    allowed one remains."""
    key = np.abs(values)
    if allowed is not None:
        key = np.where(allowed, key, -1.0)
    order = np.argsort(-key, axis=1, kind="stable")
    return order[:, :k]


def _ordered_gap(values: np.ndarray, k: int, allowed: Optional[np.ndarray] = None,
                 scale: Optional[np.ndarray] = None) -> np.ndarray:
    """(|v|_(k) - |v|_(k+1)) / max|v| per row over the allowed entries:
    how far the k-th choice of ``top_indices`` is from a tie.  With ``scale``
    (one value per row) the gap is divided by it instead of by max|v|."""
    key = np.abs(values)
    if allowed is not None:
        key = np.where(allowed, key, -np.inf)
    srt = -np.sort(-key, axis=1)
    if srt.shape[1] <= k:
        return np.full(key.shape[0], np.inf)
    top = np.maximum(srt[:, 0] if scale is None else np.asarray(scale, dtype=np.float64), 1e-300)
    nxt = np.where(np.isfinite(srt[:, k]), srt[:, k], 0.0)
    return (srt[:, k - 1] - nxt) / top


def lstsq_on_support(A: np.ndarray, Y: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """s = B^+ y with B = A(:, cols) per pixel (Alg. 3 step 2, Alg. 5 step 2),
    for a batch of supports of one common size.  cols: P x k int; Y: P x M.
    Returns P x k.

    k <= M: Householder QR of each B (M x k, full column rank), then
    R s = Q^T y, the least-squares solution.
    k > M (CoSaMP's merged support when 3K > M): B has full row rank M and
    B^+ y is the minimum-norm solution of B s = y: with the QR of B^T
    (k x M, full column rank), B = R^T Q^T, so s = Q w with R^T w = y."""
    A = _f64(A)
    Y = _f64(Y)
    cols = np.asarray(cols)
    if cols.shape[1] == 0:
        return np.zeros((Y.shape[0], 0))
    B = np.transpose(A[:, cols], (1, 0, 2))          # P x M x k
    if cols.shape[1] > A.shape[0]:
        Q, R = np.linalg.qr(np.transpose(B, (0, 2, 1)))                   # P x k x M, P x M x M
        w = np.linalg.solve(np.transpose(R, (0, 2, 1)), Y[..., None])[..., 0]
        return np.einsum("pkm,pm->pk", Q, w)
    Q, R = np.linalg.qr(B)                            # P x M x k, P x k x k
    qty = np.einsum("pmk,pm->pk", Q, Y)
    return np.linalg.solve(R, qty[..., None])[..., 0]


def _lstsq_ragged(A: np.ndarray, Y: np.ndarray, supports: list) -> list:
    """lstsq_on_support for supports of different sizes: grouped by size."""
    out = [None] * len(supports)
    sizes = np.array([len(s) for s in supports])
    for k in np.unique(sizes):
        rows = np.nonzero(sizes == k)[0]
        cols = np.stack([supports[r] for r in rows]) if k > 0 else np.zeros((len(rows), 0), int)
        sol = lstsq_on_support(A, Y[rows], cols)
        for j, r in enumerate(rows):
            out[r] = sol[j]
    return out


def _finite_rows(Y: np.ndarray) -> np.ndarray:
    return np.all(np.isfinite(Y), axis=1)


def _pivot_ratio_min(A: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """min_j d_j / G_jj over the Cholesky factor of G = B^T B, B = A(:, cols):
    d_j is the squared j-th pivot, i.e. the squared distance of column j from
    the span of the columns before it, divided by its squared norm."""
    B = np.transpose(_f64(A)[:, cols], (1, 0, 2))
    G = np.einsum("pmi,pmj->pij", B, B)
    try:
        Lc = np.linalg.cholesky(G)
    except np.linalg.LinAlgError:
        return np.zeros(cols.shape[0])
    d = np.diagonal(Lc, axis1=1, axis2=2) ** 2
    g = np.diagonal(G, axis1=1, axis2=2)
    return np.min(d / np.maximum(g, 1e-300), axis=1)


# --------------------------------------------------------------------------
# Alg. 1 -- FISTA
# --------------------------------------------------------------------------

def fista(A, Y, lam: float, L: float, max_iter: int, eps: float = 0.0, X0=None,
          dtype=np.float64) -> dict:
    """FISTA for min 1/2||A x - y||^2 + lam ||x||_1 (Eq. 2, Alg. 1), every
    pixel (row of Y) independently.

    Per iteration i, for each pixel still running:
      1. aux = z^{i-1} - (1/L) A^T (A z^{i-1} - y)
      2. x^i = sign(aux) * max(|aux| - lam/L, 0)
      3. t^i = (1 + sqrt(1 + 4 (t^{i-1})^2)) / 2
      4. z^i = x^i + ((t^{i-1} - 1) / t^i) (x^i - x^{i-1})
      5. r^i = y - A x^i,  Delta = ||r^i - r^{i-1}||_2;  stop when Delta < eps
    with t^0 = 1, z^0 = x^0, r^0 = y.

    dtype=np.float32 evaluates the same steps with every array operation
    rounded to FP32: a rounding model used only to size the error a plain
    FP32 evaluation of Alg. 1 carries on a given problem (the parity
    reference is always the FP64 evaluation).

    Returns dict(X, iters, delta, resid, flags)."""
    A = np.asarray(A, dtype=dtype)
    Y = np.asarray(Y, dtype=dtype)
    P, M = Y.shape
    N = A.shape[1]
    fin = _finite_rows(Y)
    Yc = np.where(fin[:, None], Y, dtype(0.0))
    x = np.zeros((P, N), dtype=dtype) if X0 is None else np.asarray(X0, dtype=dtype).copy()
    x[~fin] = 0.0
    z = x.copy()
    r = Yc.copy()                    # r^0 = y
    t = 1.0
    iters = np.zeros(P, dtype=np.int64)
    delta = np.full(P, np.nan)
    flags = np.zeros(P, dtype=np.int64)
    flags[~fin] |= STOP_NONFINITE
    active = fin.copy()
    for i in range(1, max_iter + 1):
        if not active.any():
            break
        a = np.nonzero(active)[0]
        za, xa, ya = z[a], x[a], Yc[a]
        aux = za - dtype(1.0 / L) * ((za @ A.T - ya) @ A)       # step 1
        x_new = soft_threshold(aux, dtype(lam / L))             # step 2
        t_new = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0      # step 3
        z_new = x_new + dtype((t - 1.0) / t_new) * (x_new - xa)  # step 4
        r_new = ya - x_new @ A.T                                # step 5
        d = np.linalg.norm(r_new - r[a], axis=1)
        x[a], z[a], r[a] = x_new, z_new, r_new
        iters[a] = i
        delta[a] = d
        t = t_new
        stop = d < eps
        flags[a[stop]] |= STOP_CONVERGED
        active[a[stop]] = False
    flags[active] |= STOP_ITER_CAP
    resid = np.linalg.norm(Yc - x @ A.T, axis=1)
    return dict(X=x.astype(np.float64), iters=iters, delta=delta, resid=resid, flags=flags)


def soft_threshold_complex(v: np.ndarray, thr: float) -> np.ndarray:
    """sign(v) max(|v| - thr, 0) for complex v, sign(v) = v / |v| (0 at 0):
    the magnitude shrinks, the phase is kept (Alg. 1 step 2 on x in C^N)."""
    mag = np.abs(v)
    scale = np.where(mag > thr, (mag - thr) / np.where(mag > 0, mag, 1.0), 0.0)
    return v * scale.astype(v.real.dtype)


def fista_complex(A, Y, lam: float, L: float, max_iter: int, eps: float = 0.0, X0=None,
                  dtype=np.complex128) -> dict:
    """FISTA (Alg. 1) for the complex measurement model of Section II (a
    complex DFT basis makes A = Phi Psi and x complex): the steps of
    ``fista`` with A^* the conjugate transpose and the soft threshold acting
    on |x| (soft_threshold_complex).  L = lambda_max(A^* A).
    dtype=np.complex64 is the FP32 rounding model.

    Returns dict(X (complex128), iters, delta, resid, flags)."""
    A = np.asarray(A, dtype=dtype)
    Y = np.asarray(Y, dtype=dtype)
    rdt = A.real.dtype.type
    P, M = Y.shape
    N = A.shape[1]
    fin = _finite_rows(Y)
    Yc = np.where(fin[:, None], Y, dtype(0.0))
    Ah = np.conj(A)                  # rows v^T A^*^T = v^T conj(A): the row form of A^* v
    x = np.zeros((P, N), dtype=dtype) if X0 is None else np.asarray(X0, dtype=dtype).copy()
    x[~fin] = 0.0
    z = x.copy()
    r = Yc.copy()                    # r^0 = y
    t = 1.0
    iters = np.zeros(P, dtype=np.int64)
    delta = np.full(P, np.nan)
    flags = np.zeros(P, dtype=np.int64)
    flags[~fin] |= STOP_NONFINITE
    active = fin.copy()
    for i in range(1, max_iter + 1):
        if not active.any():
            break
        a = np.nonzero(active)[0]
        za, xa, ya = z[a], x[a], Yc[a]
        aux = za - rdt(1.0 / L) * ((za @ A.T - ya) @ Ah)           # step 1
        x_new = soft_threshold_complex(aux, rdt(lam / L))          # step 2
        t_new = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0         # step 3
        z_new = x_new + rdt((t - 1.0) / t_new) * (x_new - xa)      # step 4
        r_new = ya - x_new @ A.T                                   # step 5
        d = np.linalg.norm(r_new - r[a], axis=1)
        x[a], z[a], r[a] = x_new, z_new, r_new
        iters[a] = i
        delta[a] = d
        t = t_new
        stop = d < eps
        flags[a[stop]] |= STOP_CONVERGED
        active[a[stop]] = False
    flags[active] |= STOP_ITER_CAP
    resid = np.linalg.norm(Yc - x @ A.T, axis=1)
    return dict(X=x.astype(np.complex128), iters=iters, delta=delta, resid=resid, flags=flags)


def lipschitz_complex(A: np.ndarray) -> float:
    """L = lambda_max(A^* A) = ||A||_2^2 for a complex A (Eq. 2)."""
    return float(np.linalg.norm(np.asarray(A, dtype=np.complex128), 2) ** 2)


# --------------------------------------------------------------------------
# Alg. 2 -- ADMM
# --------------------------------------------------------------------------

ADMM_THRESHOLDS = ("paper", "standard")


def admm_threshold(lam: float, alpha: float, threshold: str = "paper") -> float:
    """The soft-threshold of Alg. 2 step 2.  The algorithm prints lam * alpha
    ("paper"); the textbook scaled-form ADMM for Eq. 2 uses lam / alpha
    ("standard").  With penalty alpha, a threshold tau makes the iteration
    solve Eq. 2 with regularisation tau * alpha, so "paper" solves it with
    lam * alpha^2 and "standard" with lam."""
    if threshold == "paper":
        return lam * alpha
    if threshold == "standard":
        return lam / alpha
    raise ValueError(f"threshold must be one of {ADMM_THRESHOLDS}")


def admm(A, Y, lam: float, alpha: float, max_iter: int, eps: float = 0.0, X0=None,
         threshold: str = "paper", dtype=np.float64) -> dict:
    """ADMM for the LASSO (Eq. 2 as the constrained problem x - z = 0; Alg. 2),
    every pixel (row of Y) independently.

    Per iteration i, for each pixel still running:
      1. x^i = (A^T A + alpha I)^{-1} (A^T y + alpha (z^{i-1} - w^{i-1}))
      2. z^i = sign(x^i + w^{i-1}) * max(|x^i + w^{i-1}| - thr, 0)
      3. w^i = w^{i-1} + x^i - z^i
      4. r^i = y - A x^i,  Delta = ||r^i - r^{i-1}||_2;  stop when Delta < eps
    with z^0 = w^0 = x^0 (the algorithm's initialisation), r^0 = y and thr =
    admm_threshold(lam, alpha, threshold).  Step 1 solves with a Cholesky
    factor of the N x N matrix A^T A + alpha I.

    dtype=np.float32 is the FP32 rounding model (as for fista).

    Returns dict(X = x^I, Z = z^I, iters, delta, resid (||y - A x^I||), flags)."""
    A = np.asarray(A, dtype=dtype)
    Y = np.asarray(Y, dtype=dtype)
    P, M = Y.shape
    N = A.shape[1]
    thr = dtype(admm_threshold(lam, alpha, threshold))
    fin = _finite_rows(Y)
    Yc = np.where(fin[:, None], Y, dtype(0.0))
    x = np.zeros((P, N), dtype=dtype) if X0 is None else np.asarray(X0, dtype=dtype).copy()
    x[~fin] = 0.0
    z = x.copy()
    w = x.copy()
    r = Yc.copy()                    # r^0 = y
    Lc = np.linalg.cholesky((A.T @ A + dtype(alpha) * np.eye(N, dtype=dtype)).astype(np.float64)).astype(dtype)
    Aty = Yc @ A
    iters = np.zeros(P, dtype=np.int64)
    delta = np.full(P, np.nan)
    flags = np.zeros(P, dtype=np.int64)
    flags[~fin] |= STOP_NONFINITE
    active = fin.copy()
    for i in range(1, max_iter + 1):
        if not active.any():
            break
        a = np.nonzero(active)[0]
        rhs = Aty[a] + dtype(alpha) * (z[a] - w[a])                      # step 1
        h = np.linalg.solve(Lc, rhs.T)
        x_new = np.linalg.solve(Lc.T, h).T.astype(dtype)
        zt = x_new + w[a]
        z_new = soft_threshold(zt, thr)                                  # step 2
        w_new = zt - z_new                                               # step 3
        r_new = Yc[a] - x_new @ A.T                                      # step 4
        d = np.linalg.norm(r_new - r[a], axis=1)
        x[a], z[a], w[a], r[a] = x_new, z_new, w_new, r_new
        iters[a] = i
        delta[a] = d
        stop = d < eps
        flags[a[stop]] |= STOP_CONVERGED
        active[a[stop]] = False
    flags[active] |= STOP_ITER_CAP
    resid = np.linalg.norm(Yc - x @ A.T, axis=1)
    return dict(X=x.astype(np.float64), Z=z.astype(np.float64), iters=iters, delta=delta, resid=resid,
                flags=flags)


def admm_complex(A, Y, lam: float, alpha: float, max_iter: int, eps: float = 0.0, X0=None,
                 threshold: str = "paper", dtype=np.complex128) -> dict:
    """ADMM (Alg. 2) for the complex measurement model of Section II (a
    complex DFT basis makes A = Phi Psi and x complex): the steps of ``admm``
    with A^* the conjugate transpose -- step 1 solves with the Hermitian
    positive definite A^* A + alpha I by its Cholesky factor C C^* -- and the
    soft threshold of step 2 acting on |x + w| (soft_threshold_complex).
    Threshold as admm_threshold.  dtype=np.complex64 is the FP32 rounding
    model.

    Returns dict(X = x^I, Z = z^I (complex128), iters, delta, resid, flags)."""
    A = np.asarray(A, dtype=dtype)
    Y = np.asarray(Y, dtype=dtype)
    rdt = A.real.dtype.type
    P, M = Y.shape
    N = A.shape[1]
    tau = rdt(admm_threshold(lam, alpha, threshold))
    fin = _finite_rows(Y)
    Yc = np.where(fin[:, None], Y, dtype(0.0))
    xc = np.zeros((P, N), dtype=dtype) if X0 is None else np.asarray(X0, dtype=dtype).copy()
    xc[~fin] = 0.0
    zc = xc.copy()
    wc = xc.copy()
    rc = Yc.copy()                   # r^0 = y
    A64 = A.astype(np.complex128)
    Cf = np.linalg.cholesky(np.conj(A64).T @ A64 + alpha * np.eye(N)).astype(dtype)   # A^* A + alpha I = C C^*
    Ahy = Yc @ np.conj(A)            # rows (A^* y)^T
    iters = np.zeros(P, dtype=np.int64)
    delta = np.full(P, np.nan)
    flags = np.zeros(P, dtype=np.int64)
    flags[~fin] |= STOP_NONFINITE
    live = fin.copy()
    for i in range(1, max_iter + 1):
        if not live.any():
            break
        a = np.nonzero(live)[0]
        b = Ahy[a] + rdt(alpha) * (zc[a] - wc[a])                        # step 1
        xn = np.linalg.solve(np.conj(Cf).T, np.linalg.solve(Cf, b.T)).T.astype(dtype)
        v = xn + wc[a]
        zn = soft_threshold_complex(v, tau)                              # step 2
        wn = v - zn                                                      # step 3
        rn = Yc[a] - xn @ A.T                                            # step 4
        d = np.linalg.norm(rn - rc[a], axis=1)
        xc[a], zc[a], wc[a], rc[a] = xn, zn, wn, rn
        iters[a] = i
        delta[a] = d
        stop = d < eps
        flags[a[stop]] |= STOP_CONVERGED
        live[a[stop]] = False
    flags[live] |= STOP_ITER_CAP
    resid = np.linalg.norm(Yc - xc @ A.T, axis=1)
    return dict(X=xc.astype(np.complex128), Z=zc.astype(np.complex128), iters=iters, delta=delta, resid=resid,
                flags=flags)


# --------------------------------------------------------------------------
# Alg. 3 -- gOMP
# --------------------------------------------------------------------------

def gomp(A, Y, K: int, S: int, max_iter: int = 0, res_tol: float = 0.0, eps: float = 0.0,
         prune: str = "each", diagnostics: bool = False, corr_format: str = "f64") -> dict:
    """Generalised OMP (Alg. 3): kappa = K, G = S atoms per iteration.

    Per iteration i, for each pixel still running:
      1. p = A^T r^{i-1};  Theta^i = argmax_S |p| over indices not in c;
         c^i = c^{i-1} followed by Theta^i
      2. B = A(:, c^i),  s = B^+ y,  x = 0, x(c^i) = s
      3. when |c^i| > K (prune='each'): q = argmax_K |x| over c^i,
         s = A(:, q)^+ y,  x = 0, x(q) = s
      4. r^i = y - A x,  Delta = ||r^i - r^{i-1}||
    Stop after the iteration where ||r^i|| <= res_tol ||y|| or Delta < eps, or
    after max_iter (default min(K, floor(M/S))) iterations.  prune='final'
    applies step 3 once, after the loop, instead of every iteration.

    Returns dict(X, support (P x K, ascending, -1 padded), iters, delta, resid,
    flags) and, with diagnostics=True, per-pixel minimum selection gap,
    prune gap, stop margin and pivot ratio.  The gaps come twice: relative to
    the largest compared value (sel_gap, prune_gap) and relative to the scale
    on which rounding perturbs the compared values -- ||y|| for the
    correlations, which are formed from a residual y - A x, and ||s|| for the
    least-squares coefficients (sel_gap_abs, prune_gap_abs).  sel_gap_l1 is
    the selection gap relative to max_n sum_m |A_mn| |r_m|, the scale of the
    error of a correlation whose operands are rounded to a shorter format:
    rounding A and r to a significand of p bits (unit roundoff u = 2^-p)
    moves each |p_n| by at most about 2u sum_m |A_mn| |r_m|.

    corr_format ('f64' by default, 'bf16', 'f16') is a rounding model of a
    correlation computed on 16-bit operands: step 1 uses A and r rounded to
    that format (round_to_format), their products summed in FP64; every
    other step is unchanged."""
    A = _f64(A)
    Y = _f64(Y)
    P, M = Y.shape
    N = A.shape[1]
    I_max = max_iter if max_iter > 0 else min(K, M // S)
    if S * I_max > M:
        raise ValueError("S * max_iter exceeds M: the least-squares problems would be underdetermined")
    fin = _finite_rows(Y)
    Yc = np.where(fin[:, None], Y, 0.0)
    ynorm = np.linalg.norm(Yc, axis=1)
    Acorr = round_to_format(A, corr_format) if corr_format != "f64" else A
    x = np.zeros((P, N))
    r = Yc.copy()
    c = np.full((P, S * I_max), -1, dtype=np.int64)
    in_c = np.zeros((P, N), dtype=bool)
    supp = np.full((P, K), -1, dtype=np.int64)      # support of the current x
    iters = np.zeros(P, dtype=np.int64)
    delta = np.full(P, np.nan)
    flags = np.zeros(P, dtype=np.int64)
    flags[~fin] |= STOP_NONFINITE
    sel_gap = np.full(P, np.inf)
    prune_gap = np.full(P, np.inf)
    sel_gap_abs = np.full(P, np.inf)
    sel_gap_l1 = np.full(P, np.inf)
    prune_gap_abs = np.full(P, np.inf)
    stop_margin = np.full(P, np.inf)
    min_pivot = np.full(P, np.inf)
    active = fin.copy()
    for i in range(1, I_max + 1):
        if not active.any():
            break
        a = np.nonzero(active)[0]
        ra, ya = r[a], Yc[a]
        if corr_format == "f64":
            p = ra @ A                                          # step 1: A^T r
        else:
            p = round_to_format(ra, corr_format) @ Acorr        # step 1 on rounded operands
        allowed = ~in_c[a]
        theta = top_indices(p, S, allowed)
        if diagnostics:
            sel_gap[a] = np.minimum(sel_gap[a], _ordered_gap(p, S, allowed))
            sel_gap_abs[a] = np.minimum(sel_gap_abs[a], _ordered_gap(p, S, allowed, ynorm[a]))
            l1 = np.max(np.abs(ra) @ np.abs(A), axis=1)
            sel_gap_l1[a] = np.minimum(sel_gap_l1[a], _ordered_gap(p, S, allowed, l1))
        c[a, (i - 1) * S:i * S] = theta
        in_c[a[:, None], theta] = True
        cur = c[a, :i * S]
        s = lstsq_on_support(A, ya, cur)                        # step 2
        if diagnostics:
            min_pivot[a] = np.minimum(min_pivot[a], _pivot_ratio_min(A, cur))
        xa = np.zeros((len(a), N))
        xa[np.arange(len(a))[:, None], cur] = s
        if prune == "each" and i * S > K:                       # step 3
            q = top_indices(xa, K, in_c[a])
            if diagnostics:
                prune_gap[a] = np.minimum(prune_gap[a], _ordered_gap(xa, K, in_c[a]))
                prune_gap_abs[a] = np.minimum(prune_gap_abs[a],
                                              _ordered_gap(xa, K, in_c[a], np.linalg.norm(s, axis=1)))
            sq = lstsq_on_support(A, ya, q)
            xa = np.zeros((len(a), N))
            xa[np.arange(len(a))[:, None], q] = sq
            supp[a] = np.sort(q, axis=1)
        else:
            w = min(i * S, K)
            supp[a, :w] = np.sort(cur, axis=1)[:, :w]
        r_new = ya - xa @ A.T                                   # step 4
        d = np.linalg.norm(r_new - ra, axis=1)
        rn = np.linalg.norm(r_new, axis=1)
        x[a], r[a] = xa, r_new
        iters[a] = i
        delta[a] = d
        if diagnostics and res_tol > 0:
            stop_margin[a] = np.minimum(stop_margin[a],
                                        np.abs(rn / np.maximum(ynorm[a], 1e-300) - res_tol) / res_tol)
        stop = (rn <= res_tol * ynorm[a]) | (d < eps)
        flags[a[stop]] |= STOP_CONVERGED
        active[a[stop]] = False
    flags[active] |= STOP_ITER_CAP
    if prune == "final":
        big = np.nonzero(fin & (iters * S > K))[0]
        if len(big):
            q = top_indices(x[big], K, in_c[big])
            if diagnostics:
                prune_gap[big] = np.minimum(prune_gap[big], _ordered_gap(x[big], K, in_c[big]))
                prune_gap_abs[big] = np.minimum(prune_gap_abs[big], _ordered_gap(
                    x[big], K, in_c[big], np.linalg.norm(x[big], axis=1)))
            sq = lstsq_on_support(A, Yc[big], q)
            x[big] = 0.0
            x[big[:, None], q] = sq
            supp[big] = np.sort(q, axis=1)
    support = supp
    resid = np.linalg.norm(Yc - x @ A.T, axis=1)
    out = dict(X=x, support=support, iters=iters, delta=delta, resid=resid, flags=flags)
    if diagnostics:
        out.update(sel_gap=sel_gap, prune_gap=prune_gap, stop_margin=stop_margin,
                   min_pivot=min_pivot, sel_gap_abs=sel_gap_abs, prune_gap_abs=prune_gap_abs,
                   sel_gap_l1=sel_gap_l1)
    return out


# --------------------------------------------------------------------------
# Alg. 5 -- CoSaMP
# --------------------------------------------------------------------------

def cosamp(A, Y, K: int, max_iter: int, eps: float = 0.0, res_tol: float = 0.0,
           diagnostics: bool = False) -> dict:
    """CoSaMP (Alg. 5), every pixel independently.

    Per iteration i:
      1. p = A^T r^{i-1};  Theta = argmax_2K |p|;  c = Theta U c^{i-1}
      2. s = A(:, c)^+ y  (the least-squares solution while |c| <= M, the
         minimum-norm solution of A(:, c) s = y once |c| > M, which the
         pseudo-inverse gives; |c| <= 3K)
      3. q = argmax_K |s|;  s = s(q);  c = c(q);  x = 0, x(c) = s
      4. r^i = y - A x,  Delta = ||r^i - r^{i-1}||;  stop when Delta < eps
    (the kept values are the least-squares values on the larger set, no
    second solve)."""
    A = _f64(A)
    Y = _f64(Y)
    P, M = Y.shape
    N = A.shape[1]
    if 3 * K > N:
        raise ValueError("3K exceeds N")
    fin = _finite_rows(Y)
    Yc = np.where(fin[:, None], Y, 0.0)
    ynorm = np.linalg.norm(Yc, axis=1)
    x = np.zeros((P, N))
    r = Yc.copy()
    cprev = [np.zeros(0, dtype=np.int64) for _ in range(P)]
    iters = np.zeros(P, dtype=np.int64)
    delta = np.full(P, np.nan)
    flags = np.zeros(P, dtype=np.int64)
    flags[~fin] |= STOP_NONFINITE
    sel_gap = np.full(P, np.inf)
    prune_gap = np.full(P, np.inf)
    ls_cond = np.full(P, np.nan)
    active = fin.copy()
    for i in range(1, max_iter + 1):
        if not active.any():
            break
        a = np.nonzero(active)[0]
        ra, ya = r[a], Yc[a]
        p = ra @ A                                                  # step 1
        theta = top_indices(p, 2 * K)
        if diagnostics:
            sel_gap[a] = np.minimum(sel_gap[a], _ordered_gap(p, 2 * K))
        cs = [np.union1d(theta[j], cprev[a[j]]) for j in range(len(a))]
        ss = _lstsq_ragged(A, ya, cs)                               # step 2
        if diagnostics:
            ls_cond[a] = [np.linalg.cond(A[:, cj]) for cj in cs]
        xa = np.zeros((len(a), N))
        for j in range(len(a)):
            full = np.zeros(N)
            full[cs[j]] = ss[j]
            inc = np.zeros(N, dtype=bool)
            inc[cs[j]] = True
            q = top_indices(full[None, :], K, inc[None, :])[0]      # step 3
            if diagnostics:
                g = _ordered_gap(full[None, :], K, inc[None, :])[0]
                prune_gap[a[j]] = min(prune_gap[a[j]], g)
            xa[j, q] = full[q]
            cprev[a[j]] = np.sort(q)
        r_new = ya - xa @ A.T                                       # step 4
        d = np.linalg.norm(r_new - ra, axis=1)
        rn = np.linalg.norm(r_new, axis=1)
        x[a], r[a] = xa, r_new
        iters[a] = i
        delta[a] = d
        stop = (d < eps) | (rn <= res_tol * ynorm[a])
        flags[a[stop]] |= STOP_CONVERGED
        active[a[stop]] = False
    flags[active] |= STOP_ITER_CAP
    support = np.full((P, K), -1, dtype=np.int64)
    for p_ in range(P):
        support[p_, :len(cprev[p_])] = cprev[p_]
    resid = np.linalg.norm(Yc - x @ A.T, axis=1)
    out = dict(X=x, support=support, iters=iters, delta=delta, resid=resid, flags=flags)
    if diagnostics:
        # ls_cond: condition number of A(:, c) of the last solve (step 2)
        out.update(sel_gap=sel_gap, prune_gap=prune_gap, ls_cond=ls_cond)
    return out


# --------------------------------------------------------------------------
# Alg. 4 -- BIHT (backtracking iterative hard thresholding)
# --------------------------------------------------------------------------

def biht(A, Y, K: int, max_iter: int, mu: float = 0.1, eps: float = 0.0,
         res_tol: float = 0.0, diagnostics: bool = False) -> dict:
    """Backtracking IHT (Alg. 4), every pixel independently.

    Per iteration i:
      1. u = x_a + mu A^T (y - A x_a);  Theta = argmax_K |u|;
         c = supp(x_a) U Theta
      2. s = A(:, c)^+ y
      3. h = argmax_K |s|;  s = 0 outside h;  x_a = 0, x_a(c) = s;  x = x_a
      4. r^i = y - A x,  Delta = ||r^i - r^{i-1}||;  stop when Delta < eps"""
    A = _f64(A)
    Y = _f64(Y)
    P, M = Y.shape
    N = A.shape[1]
    if 2 * K > M:
        raise ValueError("2K exceeds M: the merged support could make the least squares underdetermined")
    fin = _finite_rows(Y)
    Yc = np.where(fin[:, None], Y, 0.0)
    ynorm = np.linalg.norm(Yc, axis=1)
    x = np.zeros((P, N))
    r = Yc.copy()
    iters = np.zeros(P, dtype=np.int64)
    delta = np.full(P, np.nan)
    flags = np.zeros(P, dtype=np.int64)
    flags[~fin] |= STOP_NONFINITE
    sel_gap = np.full(P, np.inf)
    prune_gap = np.full(P, np.inf)
    active = fin.copy()
    for i in range(1, max_iter + 1):
        if not active.any():
            break
        a = np.nonzero(active)[0]
        xa_prev, ya, ra = x[a], Yc[a], r[a]
        u = xa_prev + mu * ((ya - xa_prev @ A.T) @ A)               # step 1
        theta = top_indices(u, K)
        if diagnostics:
            sel_gap[a] = np.minimum(sel_gap[a], _ordered_gap(u, K))
        cs = [np.union1d(np.nonzero(xa_prev[j])[0], theta[j]) for j in range(len(a))]
        ss = _lstsq_ragged(A, ya, cs)                               # step 2
        xa = np.zeros((len(a), N))
        for j in range(len(a)):
            full = np.zeros(N)
            full[cs[j]] = ss[j]
            inc = np.zeros(N, dtype=bool)
            inc[cs[j]] = True
            h = top_indices(full[None, :], K, inc[None, :])[0]      # step 3
            if diagnostics and len(cs[j]) > K:
                g = _ordered_gap(full[None, :], K, inc[None, :])[0]
                prune_gap[a[j]] = min(prune_gap[a[j]], g)
            xa[j, h] = full[h]
        r_new = ya - xa @ A.T                                       # step 4
        d = np.linalg.norm(r_new - ra, axis=1)
        rn = np.linalg.norm(r_new, axis=1)
        x[a], r[a] = xa, r_new
        iters[a] = i
        delta[a] = d
        stop = (d < eps) | (rn <= res_tol * ynorm[a])
        flags[a[stop]] |= STOP_CONVERGED
        active[a[stop]] = False
    flags[active] |= STOP_ITER_CAP
    support = np.full((P, K), -1, dtype=np.int64)
    for p_ in range(P):
        nz = np.nonzero(x[p_])[0][:K]
        support[p_, :len(nz)] = nz
    resid = np.linalg.norm(Yc - x @ A.T, axis=1)
    out = dict(X=x, support=support, iters=iters, delta=delta, resid=resid, flags=flags)
    if diagnostics:
        out.update(sel_gap=sel_gap, prune_gap=prune_gap)
    return out


def biht_one_bit(A, Ysign, K: int, max_iter: int, mu: float = 0.1,
                 diagnostics: bool = False) -> dict:
    """Binary IHT on sign measurements y in {-1, +1}^M (not from the paper).

    x^0 = 0; per iteration x = H_K(x + mu A^T (y - sgn(A x))), sgn(0) = 0,
    H_K keeping the K largest |.| (ties to the lower index).  Output x/||x||
    (a zero x stays zero).  Diagnostics: the smallest |(A x)_m| / ||x|| met by
    a sign decision and the smallest top-K gap of |u|."""
    A = _f64(A)
    Ys = _f64(Ysign)
    P, M = Ys.shape
    N = A.shape[1]
    x = np.zeros((P, N))
    sign_margin = np.full(P, np.inf)
    sel_gap = np.full(P, np.inf)
    rows = np.arange(P)[:, None]
    for i in range(1, max_iter + 1):
        ax = x @ A.T
        if diagnostics:
            xn = np.linalg.norm(x, axis=1)
            nzr = xn > 0
            m = np.min(np.abs(ax), axis=1)
            sign_margin[nzr] = np.minimum(sign_margin[nzr], m[nzr] / xn[nzr])
        u = x + mu * ((Ys - np.sign(ax)) @ A)
        h = top_indices(u, K)
        if diagnostics:
            sel_gap = np.minimum(sel_gap, _ordered_gap(u, K))
        x = np.zeros((P, N))
        x[rows, h] = u[rows, h]
    nrm = np.linalg.norm(x, axis=1, keepdims=True)
    x = np.where(nrm > 0, x / np.where(nrm > 0, nrm, 1.0), 0.0)
    support = np.sort(np.where(x != 0, np.arange(N)[None, :], N), axis=1)[:, :K]
    support = np.where(support == N, -1, support)
    out = dict(X=x, support=support, iters=np.full(P, max_iter, dtype=np.int64),
               flags=np.full(P, STOP_ITER_CAP, dtype=np.int64))
    if diagnostics:
        out.update(sign_margin=sign_margin, sel_gap=sel_gap)
    return out
