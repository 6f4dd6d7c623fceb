"""Pins for the FP64 oracle: facts fixed by the paper and by mathematics,
never by the oracle itself.

Every check takes the oracle module as an argument so that the same checks
can be run against deliberately broken copies of the oracle source (see
test_oracle_mutations.py): each plausible mistake must fail at least one.

Kinds of pin used here:
  closed forms  -- results computable by hand for special dictionaries
                   (identity, scaled identity, orthonormal, diagonal);
  library       -- scikit-learn's coordinate-descent LASSO and its OMP,
                   SciPy's DCT and symmetric eigen-solver, NumPy's SVD lstsq;
  brute force   -- exhaustive L0 search on tiny problems;
  invariants    -- KKT conditions, residual orthogonality, sparsity, norms.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.fft
import scipy.linalg

from paper_2401_14762_amd import workloads as W


def _rng(seed):
    return np.random.default_rng(seed)


def _orthonormal(n, seed):
    q, r = np.linalg.qr(_rng(seed).standard_normal((n, n)))
    return q * np.sign(np.diag(r))[None, :]


def _sparse_problem(M, N, K, P, seed, noise=0.0):
    rng = _rng(seed)
    A = rng.standard_normal((M, N)) / math.sqrt(M)
    X = np.zeros((P, N))
    for p in range(P):
        idx = rng.choice(N, K, replace=False)
        X[p, idx] = rng.choice([-1.0, 1.0], K) * (1.0 + rng.random(K))
    Y = X @ A.T + noise * rng.standard_normal((P, M))
    return A, X, Y


# ---------------------------------------------------------------- dictionary

def check_dft_basis():
    for N in (8, 100, 154):
        psi = W.dft_synthesis(N)
        assert np.max(np.abs(np.conj(psi.T) @ psi - np.eye(N))) < 1e-12
        f = _rng(N).standard_normal(N)
        # x = Psi^* f is the unitary DFT of f (numpy's forward FFT, scaled)
        assert np.allclose(np.conj(psi.T) @ f, np.fft.fft(f) / math.sqrt(N), atol=1e-12)


def check_dct_basis():
    for N in (8, 100, 200, 224):
        psi = W.dct_synthesis(N)
        assert np.max(np.abs(psi.T @ psi - np.eye(N))) < 1e-13
        f = _rng(N).standard_normal(N)
        assert np.allclose(psi.T @ f, scipy.fft.dct(f, type=2, norm="ortho"), atol=1e-12)
        assert np.allclose(psi @ f, scipy.fft.idct(f, type=2, norm="ortho"), atol=1e-12)


def check_lipschitz(orc):
    A = _rng(1).standard_normal((30, 70))
    lam_max = scipy.linalg.eigh(A.T @ A, eigvals_only=True)[-1]
    assert abs(orc.lipschitz(A) - lam_max) <= 1e-10 * lam_max
    # closed form: scaled orthonormal rows
    Q = _orthonormal(50, 2)[:20]
    assert abs(orc.lipschitz(3.0 * Q) - 9.0) < 1e-12


# ---------------------------------------------------------------- FISTA

def _soft(v, t):
    out = np.zeros_like(v)
    out[v > t] = v[v > t] - t
    out[v < -t] = v[v < -t] + t
    return out


def check_fista_identity(orc):
    """A = c I, L = c^2: every iterate equals soft(y / c, lam / c^2)."""
    Y = _rng(3).standard_normal((7, 12)) * 2.0
    for c, lam in ((1.0, 0.3), (2.0, 0.5), (0.5, 0.01)):
        A = c * np.eye(12)
        want = _soft(Y / c, lam / c ** 2)
        for it in (1, 2, 7):
            out = orc.fista(A, Y, lam, c * c, it)
            assert np.max(np.abs(out["X"] - want)) < 1e-12, (c, lam, it)


def check_fista_zero_solution(orc):
    """lam >= ||A^T y||_inf gives x = 0 from x^0 = 0; slightly below gives x != 0."""
    A, _, Y = _sparse_problem(20, 50, 4, 5, 4)
    L = orc.lipschitz(A)
    lam0 = np.max(np.abs(Y @ A), axis=1)
    for p in range(Y.shape[0]):
        out = orc.fista(A, Y[p:p + 1], lam0[p] * 1.0000001, L, 30)
        assert np.all(out["X"] == 0.0)
        out = orc.fista(A, Y[p:p + 1], lam0[p] * 0.9, L, 30)
        assert np.any(out["X"] != 0.0)


def check_fista_diagonal_momentum(orc):
    """lam = 0 and A = diag(sigma): each coordinate's error e = x - x* obeys
    the scalar recursion e^i = q (e^{i-1} + b_{i-1}(e^{i-1} - e^{i-2})),
    q = 1 - sigma^2 / L, b_i = (t_{i-1} - 1) / t_i, t_0 = 1, from x^0 = 0."""
    sig = np.array([1.0, 0.8, 0.5, 0.3, 0.1])
    A = np.diag(sig)
    xstar = np.array([1.0, -2.0, 0.5, 3.0, -1.0])
    Y = (A @ xstar)[None, :]
    L = 1.0
    for n_it in (1, 2, 3, 10, 40):
        out = orc.fista(A, Y, 0.0, L, n_it)
        e_prev = -xstar.copy()      # e^{-1} = e^0 = -x*
        e = -xstar.copy()
        t = 1.0
        b = 0.0
        for _ in range(n_it):
            zerr = e + b * (e - e_prev)
            e_new = (1.0 - sig ** 2 / L) * zerr
            t_new = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
            b = (t - 1.0) / t_new
            t = t_new
            e_prev, e = e, e_new
        assert np.max(np.abs(out["X"][0] - (xstar + e))) < 1e-12, n_it


def check_fista_matches_sklearn_lasso(orc):
    """At convergence FISTA reaches the LASSO minimiser of Eq. 2, computed
    independently by scikit-learn's coordinate descent (alpha = lam / M)."""
    from sklearn.linear_model import Lasso
    A, _, Y = _sparse_problem(20, 35, 3, 3, 5, noise=0.01)
    lam = 0.02
    L = orc.lipschitz(A)
    out = orc.fista(A, Y, lam, L, 6000)
    for p in range(Y.shape[0]):
        m = Lasso(alpha=lam / A.shape[0], fit_intercept=False, tol=1e-14, max_iter=200000)
        m.fit(A, Y[p])
        assert np.max(np.abs(out["X"][p] - m.coef_)) < 1e-7, p


def check_fista_kkt_and_rate(orc):
    """KKT residual of Eq. 2 vanishes at convergence; along the way the
    objective gap obeys Beck-Teboulle's bound 2 L ||x0 - x*||^2 / (k+1)^2."""
    from oracle import metrics
    A, _, Y = _sparse_problem(15, 30, 3, 2, 6, noise=0.05)
    lam = 0.05
    L = orc.lipschitz(A)
    xs = orc.fista(A, Y, lam, L, 20000)["X"]
    kkt = metrics.lasso_kkt_residual(A, Y, xs, lam)
    assert np.all(kkt < 1e-9), kkt
    Hs = metrics.lasso_objective(A, Y, xs, lam)
    for k in (1, 2, 5, 20, 100):
        xk = orc.fista(A, Y, lam, L, k)["X"]
        gap = metrics.lasso_objective(A, Y, xk, lam) - Hs
        bound = 2.0 * L * np.sum(xs ** 2, axis=1) / (k + 1) ** 2
        assert np.all(gap <= bound * (1 + 1e-9) + 1e-12), (k, gap, bound)


def check_fista_stop_rule(orc):
    """Delta = ||r^i - r^{i-1}||, r^0 = y: a huge eps stops after iteration 1,
    eps = 0 runs the full budget; Delta at iteration 1 is ||A x^1||."""
    A, _, Y = _sparse_problem(20, 40, 3, 4, 7)
    L = orc.lipschitz(A)
    out = orc.fista(A, Y, 0.01, L, 50, eps=1e30)
    assert np.all(out["iters"] == 1)
    assert np.allclose(out["delta"], np.linalg.norm(out["X"] @ A.T, axis=1), rtol=1e-12)
    out = orc.fista(A, Y, 0.01, L, 50, eps=0.0)
    assert np.all(out["iters"] == 50)
    # a single converged pixel freezes while the others continue
    Y2 = Y.copy()
    Y2[0] = 0.0
    out = orc.fista(A, Y2, 0.01, L, 50, eps=1e-300)
    assert out["iters"][0] == 1 and np.all(out["iters"][1:] == 50)


def check_fista_nonfinite(orc):
    A, _, Y = _sparse_problem(10, 20, 2, 3, 8)
    Y[1, 3] = np.nan
    out = orc.fista(A, Y, 0.01, orc.lipschitz(A), 5)
    assert np.all(out["X"][1] == 0) and out["flags"][1] & orc.STOP_NONFINITE
    assert np.all(np.isfinite(out["X"]))


# ---------------------------------------------------------------- least squares

def check_lstsq(orc):
    rng = _rng(9)
    A = rng.standard_normal((30, 60))
    Y = rng.standard_normal((6, 30))
    cols = np.stack([rng.choice(60, 11, replace=False) for _ in range(6)])
    s = orc.lstsq_on_support(A, Y, cols)
    for p in range(6):
        B = A[:, cols[p]]
        ref = np.linalg.lstsq(B, Y[p], rcond=None)[0]       # SVD-based LAPACK gelsd
        assert np.max(np.abs(s[p] - ref)) < 1e-11
        assert np.max(np.abs(B.T @ (Y[p] - B @ s[p]))) < 1e-11   # normal equations


def check_lstsq_min_norm(orc):
    """More columns than rows (CoSaMP's merged support when 3K > M): the
    pseudo-inverse solution, i.e. the minimum-norm solution of B s = y --
    against numpy's SVD pseudo-inverse, and by its two defining properties:
    B s = y exactly, and s orthogonal to the null space of B (SciPy's SVD
    null-space basis)."""
    from scipy.linalg import null_space
    rng = _rng(31)
    A = rng.standard_normal((9, 40))
    Y = rng.standard_normal((5, 9))
    for k in (10, 13):
        cols = np.stack([np.sort(rng.choice(40, k, replace=False)) for _ in range(5)])
        s = orc.lstsq_on_support(A, Y, cols)
        for p in range(5):
            B = A[:, cols[p]]
            assert np.max(np.abs(s[p] - np.linalg.pinv(B) @ Y[p])) < 1e-11
            assert np.max(np.abs(B @ s[p] - Y[p])) < 1e-11
            assert np.max(np.abs(null_space(B).T @ s[p])) < 1e-11


def check_cosamp_wide(orc):
    """CoSaMP with 3K > M: a replay of Alg. 5 with numpy's SVD pseudo-inverse
    as step 2 (two iterations, at least one pixel reaching |c| > M) gives the
    same x; the iterate with |c| > M fits y exactly on c before the prune."""
    rng = _rng(32)
    M, N, K = 10, 40, 4
    A = rng.standard_normal((M, N))
    Y = rng.standard_normal((6, M))
    out = orc.cosamp(A, Y, K=K, max_iter=2)
    wide = 0
    for p in range(6):
        x = np.zeros(N)
        prev = np.zeros(0, dtype=int)
        for _ in range(2):
            r = Y[p] - A @ x
            theta = np.argsort(-np.abs(A.T @ r), kind="stable")[:2 * K]
            c = np.union1d(theta, prev)
            s = np.linalg.pinv(A[:, c]) @ Y[p]
            if len(c) > M:
                wide += 1
                assert np.max(np.abs(A[:, c] @ s - Y[p])) < 1e-10
            keep = np.argsort(-np.abs(s), kind="stable")[:K]
            x = np.zeros(N)
            x[c[keep]] = s[keep]
            prev = np.sort(c[keep])
        assert np.max(np.abs(out["X"][p] - x)) < 1e-10
    assert wide > 0


def check_top_indices(orc):
    v = np.array([[0.5, -2.0, 2.0, 1.0, -2.0, 0.1]])
    assert orc.top_indices(v, 3).tolist() == [[1, 2, 4]]
    allowed = np.array([[True, False, True, True, True, True]])
    assert orc.top_indices(v, 3, allowed).tolist() == [[2, 4, 3]]
    assert orc.top_indices(np.zeros((1, 5)), 2).tolist() == [[0, 1]]


# ---------------------------------------------------------------- gOMP

def check_gomp_is_omp_when_S1(orc):
    """G = 1 without pruning is textbook OMP (scikit-learn's Cholesky OMP)."""
    from sklearn.linear_model import OrthogonalMatchingPursuit
    A, _, Y = _sparse_problem(40, 90, 6, 6, 10, noise=0.02)
    K = 6
    out = orc.gomp(A, Y, K=K, S=1, max_iter=K)
    for p in range(Y.shape[0]):
        m = OrthogonalMatchingPursuit(n_nonzero_coefs=K, fit_intercept=False).fit(A, Y[p])
        assert np.max(np.abs(out["X"][p] - m.coef_)) < 1e-9, p
        assert out["support"][p].tolist() == np.sort(np.nonzero(m.coef_)[0]).tolist()


def check_gomp_orthonormal(orc):
    """Orthonormal A (M = N): after the loop and the prune the support is the K
    largest |A^T y| and the values are A^T y there."""
    N = 24
    Q = _orthonormal(N, 11)
    Y = _rng(12).standard_normal((5, N))
    for K, S, it in ((5, 2, 4), (4, 1, 0), (6, 3, 3), (3, 2, 5)):
        out = orc.gomp(Q, Y, K=K, S=S, max_iter=it)
        c = Y @ Q
        for p in range(5):
            top = np.argsort(-np.abs(c[p]), kind="stable")[:K]
            want = np.zeros(N)
            want[top] = c[p, top]
            assert np.max(np.abs(out["X"][p] - want)) < 1e-12, (K, S, it, p)
            assert out["support"][p].tolist() == np.sort(top).tolist()


def check_gomp_exact_recovery(orc):
    A, X, Y = _sparse_problem(40, 100, 5, 20, 13)
    out = orc.gomp(A, Y, K=5, S=2, res_tol=1e-10)
    ok = np.max(np.abs(out["X"] - X), axis=1) < 1e-10
    assert ok.mean() >= 0.9, ok.mean()
    for p in np.nonzero(ok)[0]:
        assert out["support"][p].tolist() == np.sort(np.nonzero(X[p])[0]).tolist()
        assert out["flags"][p] & orc.STOP_CONVERGED


def check_gomp_brute_force(orc):
    """N=12, K=2: gOMP's residual is never below the exhaustive L0 minimum and
    reaches it on exactly 2-sparse noiseless data when it finds the support."""
    rng = _rng(14)
    M, N, K = 8, 12, 2
    A = rng.standard_normal((M, N))
    for trial in range(20):
        y = rng.standard_normal(M)
        best = min(np.linalg.norm(y - A[:, list(s)] @ np.linalg.lstsq(A[:, list(s)], y, rcond=None)[0])
                   for s in itertools.combinations(range(N), K))
        out = orc.gomp(A, y[None, :], K=K, S=1, max_iter=2)
        assert out["resid"][0] >= best - 1e-12
        assert np.count_nonzero(out["X"][0]) <= K
    x = np.zeros(N)
    x[[3, 9]] = [1.5, -2.0]
    out = orc.gomp(A, (A @ x)[None, :], K=K, S=1, max_iter=2)
    assert out["resid"][0] < 1e-12 and np.allclose(out["X"][0], x, atol=1e-12)


def check_gomp_prune_invariants(orc):
    """With |c| > K: output is K-sparse, its support is inside the grown set,
    and the residual is orthogonal to the kept columns (values re-solved)."""
    A, _, Y = _sparse_problem(40, 80, 6, 8, 15, noise=0.1)
    K, S, it = 6, 2, 8
    out = orc.gomp(A, Y, K=K, S=S, max_iter=it)
    for p in range(Y.shape[0]):
        sup = out["support"][p]
        assert np.all(sup >= 0) and len(sup) == K
        assert np.count_nonzero(out["X"][p]) == K
        r = Y[p] - A @ out["X"][p]
        assert np.max(np.abs(A[:, sup].T @ r)) < 1e-10
        assert out["iters"][p] == it


def check_gomp_no_reselect(orc):
    """Indices already in c are never selected again: with A = I the support
    grows through the S largest |y| entries in order, ties to lower index."""
    y = np.array([[3.0, 1.0, 3.0, 2.0, 2.0, 0.5, 1.0, 0.0]])
    out = orc.gomp(np.eye(8), y, K=3, S=2, max_iter=3)
    assert out["support"][0].tolist() == [0, 2, 3]
    assert np.allclose(out["X"][0], [3, 0, 3, 2, 0, 0, 0, 0])


def check_gomp_stop(orc):
    A, X, Y = _sparse_problem(40, 100, 4, 6, 16)
    out = orc.gomp(A, Y, K=10, S=2, res_tol=1e-8)
    # exact 4-sparse data: stops no later than two iterations after the
    # support is covered, well before the cap of 10
    assert np.all(out["iters"] < 10) and np.all(out["flags"] & orc.STOP_CONVERGED)
    out = orc.gomp(A, Y, K=10, S=2, res_tol=0.0, eps=0.0, max_iter=7)
    assert np.all(out["iters"] == 7) and np.all(out["flags"] & orc.STOP_ITER_CAP)
    # the residual rule is relative: scaling y scales x and keeps the iterations
    base = orc.gomp(A, Y, K=10, S=2, res_tol=1e-8)
    for c in (1e-9, 1e9):
        sc = orc.gomp(A, c * Y, K=10, S=2, res_tol=1e-8)
        assert np.array_equal(sc["iters"], base["iters"])
        assert np.allclose(sc["X"], c * base["X"], rtol=1e-9,
                           atol=1e-12 * c * np.abs(base["X"]).max())


def check_gomp_final_prune(orc):
    """prune='final' (Alg. 3 step 3 applied once, after the loop).

    With G = 1 the loop without a prune is textbook OMP, so the grown set
    after I iterations and its values are scikit-learn's OMP with I atoms; the
    final step keeps the K largest of those values (ties to the lower index)
    and solves the least squares again on them (NumPy's SVD lstsq).  The
    orthonormal closed form of the per-iteration prune holds as well, and a
    run that never grows past K is not pruned."""
    from sklearn.linear_model import OrthogonalMatchingPursuit
    A, _, Y = _sparse_problem(40, 90, 6, 6, 41, noise=0.05)
    K, I = 4, 9
    out = orc.gomp(A, Y, K=K, S=1, max_iter=I, prune="final")
    each = orc.gomp(A, Y, K=K, S=1, max_iter=I, prune="each")
    differs = 0
    for p in range(Y.shape[0]):
        coef = OrthogonalMatchingPursuit(n_nonzero_coefs=I, fit_intercept=False).fit(A, Y[p]).coef_
        grown = np.nonzero(coef)[0]
        assert len(grown) == I
        q = grown[np.argsort(-np.abs(coef[grown]), kind="stable")[:K]]
        want = np.zeros(A.shape[1])
        want[q] = np.linalg.lstsq(A[:, q], Y[p], rcond=None)[0]
        assert np.max(np.abs(out["X"][p] - want)) < 1e-9, p
        assert out["support"][p].tolist() == np.sort(q).tolist()
        assert np.linalg.norm(want - coef) > 1e-6       # the re-solve changes the values
        differs += np.max(np.abs(each["X"][p] - want)) > 1e-9
    assert differs > 0                                    # the two placements are different methods
    # orthonormal A: the K largest |A^T y| with the values A^T y
    N = 24
    Q = _orthonormal(N, 42)
    Yq = _rng(43).standard_normal((4, N))
    cq = Yq @ Q
    for K2, S2, it in ((5, 2, 4), (3, 3, 2)):
        o = orc.gomp(Q, Yq, K=K2, S=S2, max_iter=it, prune="final")
        for p in range(4):
            top = np.argsort(-np.abs(cq[p]), kind="stable")[:K2]
            want = np.zeros(N)
            want[top] = cq[p, top]
            assert np.max(np.abs(o["X"][p] - want)) < 1e-12
            assert o["support"][p].tolist() == np.sort(top).tolist()
    # |c| never exceeds K: no prune, the OMP solution with I atoms
    o = orc.gomp(A, Y, K=6, S=1, max_iter=5, prune="final")
    for p in range(Y.shape[0]):
        coef = OrthogonalMatchingPursuit(n_nonzero_coefs=5, fit_intercept=False).fit(A, Y[p]).coef_
        assert np.max(np.abs(o["X"][p] - coef)) < 1e-9


def check_gomp_diagnostics_by_hand(orc):
    """The near-tie diagnostics of gOMP on cases worked by hand.

    A = I (M = N = 8), y = (4, 1, 2.5, 0.5, -2, 0, 0.25, 1.5), G = 1, K = 2,
    4 iterations.  The correlations are the residual, which is y with the
    selected entries removed:
      i=1: |p| sorted 4, 2.5, ...            gap 1.5 / 4
      i=2: over the unselected 2.5, 2, ...    gap 0.5 / 2.5
      i=3: 2, 1.5, ...                        gap 0.5 / 2
      i=4: 1.5, 1, ...                        gap 0.5 / 1.5
    so the selection gap is 0.2 (relative to the largest compared value) and
    0.5 / ||y|| on the ||y|| scale.  Prunes (|c| > 2) at i = 3, 4 rank
    |s| = (4, 2.5, 2) and (4, 2.5, 2, 1.5): gap 0.5 / 4, and on the ||s||
    scale 0.5 / sqrt(28.5) (the larger s).  The residual keeps y's entries
    1, 3, 5, 6, 7 and 4 (pruned back) from i = 2 on, ||r||^2 = 7.5625 of
    ||y||^2 = 29.8125; with res_tol = 0.1 the stop margin is
    |sqrt(7.5625 / 29.8125) - 0.1| / 0.1.  Every pivot ratio of an
    orthonormal support is 1.

    Pivot ratio: a0 = 2 e0 and a1 = 3 (cos t, sin t, 0) at angle t: the
    second Cholesky pivot squared of their Gram matrix is the second atom's
    squared norm times sin^2 t, so the ratio to its diagonal entry is
    sin^2 t whichever atom comes first."""
    y = np.array([[4.0, 1.0, 2.5, 0.5, -2.0, 0.0, 0.25, 1.5]])
    ny2 = float(np.sum(y * y))
    assert ny2 == 29.8125
    o = orc.gomp(np.eye(8), y, K=2, S=1, max_iter=4, res_tol=0.1, diagnostics=True)
    assert abs(o["sel_gap"][0] - 0.2) < 1e-15
    assert abs(o["sel_gap_abs"][0] - 0.5 / math.sqrt(ny2)) < 1e-15
    assert abs(o["prune_gap"][0] - 0.125) < 1e-15
    assert abs(o["prune_gap_abs"][0] - 0.5 / math.sqrt(28.5)) < 1e-15
    assert abs(o["stop_margin"][0] - abs(math.sqrt(7.5625 / ny2) - 0.1) / 0.1) < 1e-12
    assert abs(o["min_pivot"][0] - 1.0) < 1e-15
    assert o["support"][0].tolist() == [0, 2]
    # A = I: sum_m |A_mn| |r_m| = |r_n| = |p_n|, so the l1-scaled gap is sel_gap
    assert abs(o["sel_gap_l1"][0] - 0.2) < 1e-15
    # columns (3, -3) and (1, 1), y = (1, 1): p = (0, 2) but sum_m |A_mn| |y_m| =
    # (6, 2); the one selection's gap 2 - 0 is 1 of max |p| and 1/3 of the l1 scale
    d = orc.gomp(np.array([[3.0, 1.0], [-3.0, 1.0]]), np.array([[1.0, 1.0]]), K=1, S=1, max_iter=1,
                 diagnostics=True)
    assert d["support"][0].tolist() == [1]
    assert abs(d["sel_gap"][0] - 1.0) < 1e-15
    assert abs(d["sel_gap_l1"][0] - 1.0 / 3.0) < 1e-15
    for t in (0.3, 1e-3):
        A = np.array([[2.0, 3.0 * math.cos(t), 0.0],
                      [0.0, 3.0 * math.sin(t), 0.0],
                      [0.0, 0.0, 1.0]])
        yy = (A[:, 0] + 0.5 * A[:, 1])[None, :]
        d = orc.gomp(A, yy, K=2, S=2, max_iter=1, diagnostics=True)
        assert sorted(d["support"][0].tolist()) == [0, 1]
        assert abs(d["min_pivot"][0] / math.sin(t) ** 2 - 1.0) < 1e-9
    # CoSaMP and BIHT report the same selection gap of their first step
    # (A = I: p = y, 2K resp. K largest)
    c = orc.cosamp(np.eye(8), y, K=1, max_iter=1, diagnostics=True)
    assert abs(c["sel_gap"][0] - 0.5 / 4.0) < 1e-15          # 2nd (2.5) vs 3rd (2)
    b = orc.biht(np.eye(8), y, K=2, max_iter=1, mu=1.0, diagnostics=True)
    assert abs(b["sel_gap"][0] - 0.5 / 4.0) < 1e-15          # u = mu y: 2nd (2.5) vs 3rd (2)


def check_round_to_format(orc):
    """The 16-bit rounding model of the correlation (round_to_format) and
    gOMP's corr_format.  BF16 keeps 8 significant bits: spacing 2^-7 on
    [1, 2), so 1 + 2^-9 rounds down, 1 + 2^-8 is a tie and goes to the even
    significand (1), 1 + 3 2^-8 is a tie between 1 + 2^-7 (odd) and 1 + 2^-6
    (even); pi is 3.140625; FP16 (11 bits) ties 1 + 2^-11 to 1 and
    1 + 3 2^-11 to 1 + 2^-9, and 65520 overflows to inf.  Random values agree
    with torch's float32 -> bfloat16 / float16 conversions (round to nearest
    even).  With A = I and y = (1, 1 + 2^-8) the FP64 correlation selects
    atom 1, the BF16 model sees a tie and selects atom 0 (ties to the lower
    index)."""
    bf = orc.round_to_format(np.array([1 + 2.0 ** -9, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, math.pi, -2.5, 2.0 ** -130]),
                             "bf16")
    assert bf.tolist() == [1.0, 1.0, 1 + 2.0 ** -6, 3.140625, -2.5, 2.0 ** -130]
    h = orc.round_to_format(np.array([1 + 2.0 ** -11, 1 + 3 * 2.0 ** -11, 65520.0]), "f16")
    assert h[0] == 1.0 and h[1] == 1 + 2.0 ** -9 and np.isinf(h[2])
    import torch
    v = np.random.default_rng(0).standard_normal(4096) * np.exp(np.random.default_rng(1).uniform(-20, 20, 4096))
    t = torch.from_numpy(v.astype(np.float32))
    assert np.array_equal(orc.round_to_format(v, "bf16"), t.to(torch.bfloat16).to(torch.float64).numpy())
    assert np.array_equal(orc.round_to_format(v, "f16"), t.to(torch.float16).to(torch.float64).numpy())
    y = np.array([[1.0, 1.0 + 2.0 ** -8]])
    assert orc.gomp(np.eye(2), y, K=1, S=1, max_iter=1)["support"][0].tolist() == [1]
    assert orc.gomp(np.eye(2), y, K=1, S=1, max_iter=1, corr_format="bf16")["support"][0].tolist() == [0]


# ------------------------------------------------- complex greedy solvers

def check_greedy_complex_real_case(orc):
    """With real A and y and every atom its own group, the complex gOMP,
    CoSaMP and BIHT are the real ones (same supports, same x to 1e-10)."""
    rng = np.random.default_rng(3)
    M, N, P = 24, 60, 12
    A = rng.standard_normal((M, N)) / math.sqrt(M)
    X = np.zeros((P, N))
    for p in range(P):
        X[p, rng.choice(N, 4, replace=False)] = rng.standard_normal(4)
    Y = X @ A.T + 0.01 * rng.standard_normal((P, M))
    pairs = ((orc.gomp_complex(A, Y, K=5, S=2, res_tol=1e-6), orc.gomp(A, Y, K=5, S=2, res_tol=1e-6)),
             (orc.cosamp_complex(A, Y, K=4, max_iter=6), orc.cosamp(A, Y, K=4, max_iter=6)),
             (orc.biht_complex(A, Y, K=4, max_iter=6, mu=0.3), orc.biht(A, Y, K=4, max_iter=6, mu=0.3)))
    for got, ref in pairs:
        assert np.array_equal(got["support"], ref["support"])
        assert np.abs(got["X"] - ref["X"]).max() < 1e-10
        assert np.abs(got["X"].imag).max() == 0.0
        assert np.array_equal(got["iters"], ref["iters"])


def check_greedy_complex_recovery_and_phase(orc):
    """Complex Gaussian A (M = 20, N = 40), noiseless y of a 3-sparse complex
    x: gOMP (S = 1, K = 3), CoSaMP (K = 3) and BIHT (K = 3, mu = 0.5) recover
    x exactly; y -> e^{i phi} y gives x -> e^{i phi} x with the same support
    (the correlation is A^* r, so |p| is phase-blind)."""
    rng = np.random.default_rng(8)
    M, N, P = 20, 40, 6
    A = (rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N))) / math.sqrt(2 * M)
    X = np.zeros((P, N), dtype=complex)
    for p in range(P):
        X[p, rng.choice(N, 3, replace=False)] = (1.0 + rng.random(3)) * np.exp(2j * np.pi * rng.random(3))
    Y = X @ A.T
    ph = np.exp(0.7j)
    for fn in (lambda y: orc.gomp_complex(A, y, K=3, S=1),
               lambda y: orc.cosamp_complex(A, y, K=3, max_iter=8),
               lambda y: orc.biht_complex(A, y, K=3, max_iter=60, mu=0.5)):
        o = fn(Y)
        assert np.abs(o["X"] - X).max() < 1e-9
        o2 = fn(Y * ph)
        assert np.array_equal(o2["support"], o["support"])
        assert np.abs(o2["X"] - o["X"] * ph).max() < 1e-9


def check_greedy_complex_unitary_dft(orc):
    """A = the unitary DFT synthesis (M = N = 16), a real y, conjugate pairs
    as groups: gOMP with S = 1 and K = max_iter = 3 picks the three groups of
    largest |Psi^* y| in order and returns x = Psi^* y on their bins (a
    unitary A makes every least squares a projection); the x is
    conjugate-symmetric and A x is real."""
    N = 16
    n = np.arange(N)
    Psi = np.exp(2j * np.pi * np.outer(n, n) / N) / math.sqrt(N)
    y = np.random.default_rng(4).standard_normal((1, N))
    groups = orc.conj_pair_groups(N)
    assert [g.tolist() for g in groups[:3]] == [[0], [1, 15], [2, 14]] and groups[-1].tolist() == [8]
    o = orc.gomp_complex(Psi, y, K=3, S=1, max_iter=3, groups=groups)
    p = (y @ np.conj(Psi))[0]
    score = np.array([np.sqrt(np.mean(np.abs(p[g]) ** 2)) for g in groups])
    top = np.argsort(-score, kind="stable")[:3]
    bins = np.sort(np.concatenate([groups[g] for g in top]))
    sup = o["support"][0]
    assert sup[sup >= 0].tolist() == bins.tolist()
    ref = np.zeros(N, dtype=complex)
    ref[bins] = p[bins]
    assert np.abs(o["X"][0] - ref).max() < 1e-12
    assert np.abs(o["X"][0][1:][::-1] - np.conj(o["X"][0][1:])).max() < 1e-12
    assert np.abs((o["X"] @ Psi.T).imag).max() < 1e-12
    # a pair scores |p_k| (the RMS over its two equal members), not less: with
    # x_0 = 1 and |x_2| = |x_14| = 1.2 the pair comes first
    xs = np.zeros(N, dtype=complex)
    xs[0], xs[2], xs[14] = 1.0, 1.2j, -1.2j
    f = (Psi @ xs).real[None, :]
    o = orc.gomp_complex(Psi, f, K=1, S=1, max_iter=1, groups=groups)
    assert o["support"][0].tolist() == [2, 14]


def check_greedy_complex_conjugate_pairs(orc):
    """A = Phi Psi for a real Phi (M = 14 of N = 24 bands) and the DFT basis,
    y = Phi f real: with conjugate pairs as groups, every solver returns a
    conjugate-symmetric x (x_{N-k} = conj(x_k)), a support closed under
    k <-> N-k, and a real A x; a spectrum of two pairs and the DC bin is
    recovered exactly by gOMP (S = 1, K = 3)."""
    N, M = 24, 14
    n = np.arange(N)
    Psi = np.exp(2j * np.pi * np.outer(n, n) / N) / math.sqrt(N)
    rows = np.sort(np.random.default_rng(5).choice(N, M, replace=False))
    A = Psi[rows]
    groups = orc.conj_pair_groups(N)
    xs = np.zeros((1, N), dtype=complex)
    xs[0, 0] = 1.5
    for k, v in ((3, 1.0 - 0.5j), (7, -0.8 + 0.3j)):
        xs[0, k], xs[0, N - k] = v, np.conj(v)
    f = (xs @ Psi.T).real
    o = orc.gomp_complex(A, f[:, rows], K=3, S=1, groups=groups)
    assert np.abs(o["X"] - xs).max() < 1e-10
    rng = np.random.default_rng(6)
    F = rng.standard_normal((5, N))
    Y = F[:, rows]
    for fn in (lambda y: orc.gomp_complex(A, y, K=3, S=1, groups=groups),
               lambda y: orc.cosamp_complex(A, y, K=1, max_iter=5, groups=groups),
               lambda y: orc.biht_complex(A, y, K=2, max_iter=5, mu=0.3, groups=groups)):
        o = fn(Y)
        X = o["X"]
        assert np.abs(X[:, 1:][:, ::-1] - np.conj(X[:, 1:])).max() < 1e-10
        assert np.abs((X @ A.T).imag).max() < 1e-10
        for row in o["support"]:
            s = set(int(v) for v in row if v >= 0)
            assert s == {(N - v) % N for v in s}


# ---------------------------------------------------------------- CoSaMP

def check_cosamp_orthonormal(orc):
    N = 30
    Q = _orthonormal(N, 17)
    Y = _rng(18).standard_normal((4, N))
    K = 4
    c = Y @ Q
    for it in (1, 2, 5):
        out = orc.cosamp(Q, Y, K=K, max_iter=it)
        for p in range(4):
            top = np.argsort(-np.abs(c[p]), kind="stable")[:K]
            want = np.zeros(N)
            want[top] = c[p, top]
            assert np.max(np.abs(out["X"][p] - want)) < 1e-12


def check_cosamp_recovery(orc):
    A, X, Y = _sparse_problem(60, 120, 6, 10, 19)
    out = orc.cosamp(A, Y, K=6, max_iter=15)
    assert np.mean(np.max(np.abs(out["X"] - X), axis=1) < 1e-10) >= 0.9
    assert np.all(np.count_nonzero(out["X"], axis=1) <= 6)


def check_cosamp_no_resolve(orc):
    """The kept values are the least-squares values on the merged support, not
    a second solve on the kept atoms: the residual is generally not
    orthogonal to the kept columns, but x equals the merged solution there."""
    A, _, Y = _sparse_problem(30, 60, 4, 6, 20, noise=0.2)
    K = 4
    out = orc.cosamp(A, Y, K=K, max_iter=1)
    p_all = Y @ A
    for p in range(Y.shape[0]):
        theta = np.argsort(-np.abs(p_all[p]), kind="stable")[:2 * K]
        c = np.sort(theta)
        s = np.linalg.lstsq(A[:, c], Y[p], rcond=None)[0]
        keep = np.argsort(-np.abs(s), kind="stable")[:K]
        want = np.zeros(A.shape[1])
        want[c[keep]] = s[keep]
        assert np.max(np.abs(out["X"][p] - want)) < 1e-10


# ---------------------------------------------------------------- BIHT

def check_biht_orthonormal(orc):
    N = 20
    Q = _orthonormal(N, 21)
    Y = _rng(22).standard_normal((4, N))
    K = 5
    c = Y @ Q
    for it in (1, 3):
        out = orc.biht(Q, Y, K=K, max_iter=it, mu=0.1)
        for p in range(4):
            top = np.argsort(-np.abs(c[p]), kind="stable")[:K]
            want = np.zeros(N)
            want[top] = c[p, top]
            assert np.max(np.abs(out["X"][p] - want)) < 1e-12


def check_biht_first_step(orc):
    """From x_a = 0, u = mu A^T y; with a non-orthonormal A the first iterate is
    the least squares on the K largest |A^T y| (the set is K, so nothing is
    pruned), independently of mu."""
    A, _, Y = _sparse_problem(30, 60, 4, 5, 23, noise=0.3)
    K = 4
    for mu in (0.1, 1.0):
        out = orc.biht(A, Y, K=K, max_iter=1, mu=mu)
        for p in range(Y.shape[0]):
            top = np.sort(np.argsort(-np.abs(Y[p] @ A), kind="stable")[:K])
            s = np.linalg.lstsq(A[:, top], Y[p], rcond=None)[0]
            want = np.zeros(60)
            want[top] = s
            assert np.max(np.abs(out["X"][p] - want)) < 1e-10


def check_biht_second_step_mu(orc):
    """The second candidate set depends on mu through u = x_a + mu A^T r:
    with a huge mu the gradient term decides the new atoms."""
    A, _, Y = _sparse_problem(30, 60, 4, 3, 24, noise=0.3)
    K = 4
    x1 = orc.biht(A, Y, K=K, max_iter=1)["X"]
    for mu in (1e6, 0.1):
        out = orc.biht(A, Y, K=K, max_iter=2, mu=mu)
        for p in range(Y.shape[0]):
            u = x1[p] + mu * (A.T @ (Y[p] - A @ x1[p]))
            theta = np.argsort(-np.abs(u), kind="stable")[:K]
            c = np.union1d(np.nonzero(x1[p])[0], theta)
            s = np.linalg.lstsq(A[:, c], Y[p], rcond=None)[0]
            h = np.argsort(-np.abs(s), kind="stable")[:K]
            want = np.zeros(60)
            want[c[h]] = s[h]
            assert np.max(np.abs(out["X"][p] - want)) < 1e-9


def check_biht_recovery(orc):
    # a step mu = 1 lets the gradient term bring in new atoms; with a small mu
    # the kept atoms dominate u and the candidate set can stall
    A, X, Y = _sparse_problem(50, 100, 5, 10, 25)
    out = orc.biht(A, Y, K=5, max_iter=30, mu=1.0)
    assert np.mean(np.max(np.abs(out["X"] - X), axis=1) < 1e-10) >= 0.9
    assert np.all(np.count_nonzero(out["X"], axis=1) <= 5)


def check_cosamp_biht_res_tol(orc):
    """The residual stop of CoSaMP and BIHT is relative, ||r|| <= res_tol ||y||
    (the reading shared with gOMP): on exact sparse data every pixel stops
    with CONVERGED before the cap, the stop is the first iteration meeting
    the rule, and scaling y by 1e-9 or 1e9 scales x and keeps the iteration
    counts."""
    A, X, Y = _sparse_problem(50, 100, 4, 8, 44)
    tol = 1e-8
    runs = (lambda y, it: orc.cosamp(A, y, K=4, max_iter=it, res_tol=tol),
            lambda y, it: orc.biht(A, y, K=4, max_iter=it, mu=1.0, res_tol=tol))
    for run in runs:
        base = run(Y, 40)
        assert np.all(base["iters"] < 40) and np.all(base["flags"] & orc.STOP_CONVERGED)
        ny = np.linalg.norm(Y, axis=1)
        assert np.all(base["resid"] <= tol * ny)
        for p in range(Y.shape[0]):
            k = int(base["iters"][p])
            if k > 1:
                prev = run(Y[p:p + 1], k - 1)
                assert prev["resid"][0] > tol * ny[p] and prev["flags"][0] & orc.STOP_ITER_CAP
        for c in (1e-9, 1e9):
            sc = run(c * Y, 40)
            assert np.array_equal(sc["iters"], base["iters"])
            assert np.allclose(sc["X"], c * base["X"], rtol=1e-9, atol=1e-12 * c * np.abs(base["X"]).max())


def check_one_bit(orc):
    rng = _rng(26)
    M, N, K = 400, 60, 4
    A = rng.standard_normal((M, N)) / math.sqrt(M)
    X = np.zeros((6, N))
    for p in range(6):
        X[p, rng.choice(N, K, replace=False)] = rng.standard_normal(K)
    Ys = np.where(X @ A.T >= 0, 1, -1).astype(np.int8)
    # one iteration from zero is H_K(mu A^T y), normalised
    out1 = orc.biht_one_bit(A, Ys, K, 1, mu=0.1)
    u = 0.1 * (Ys.astype(float) @ A)
    for p in range(6):
        top = np.argsort(-np.abs(u[p]), kind="stable")[:K]
        want = np.zeros(N)
        want[top] = u[p, top]
        want /= np.linalg.norm(want)
        assert np.max(np.abs(out1["X"][p] - want)) < 1e-12
    out = orc.biht_one_bit(A, Ys, K, 60, mu=0.1)
    nrm = np.linalg.norm(out["X"], axis=1)
    assert np.allclose(nrm, 1.0, atol=1e-12)
    assert np.all(np.count_nonzero(out["X"], axis=1) <= K)
    cosang = np.sum(out["X"] * X, axis=1) / np.linalg.norm(X, axis=1)
    assert np.median(cosang) > 0.95, cosang
    agree = np.mean(np.sign(out["X"] @ A.T) == Ys, axis=1)
    assert np.median(agree) > 0.95, agree


# ---------------------------------------------------------------- metrics

# ---------------------------------------------------------------- ADMM (Alg. 2)

def check_admm_matches_sklearn_lasso(orc):
    """At convergence ADMM reaches the LASSO minimiser of Eq. 2 with the
    regularisation its threshold implies (threshold * alpha): lam alpha^2 for
    the threshold the algorithm prints, lam for the textbook one.  Reference:
    scikit-learn's coordinate descent (alpha = lam_eff / M).  Both x and z
    converge to it."""
    from sklearn.linear_model import Lasso
    A, _, Y = _sparse_problem(20, 35, 3, 3, 31, noise=0.01)
    for lam, alpha, mode, lam_eff in ((0.01, 1.8, "paper", 0.01 * 1.8 ** 2), (0.03, 1.8, "standard", 0.03),
                                      (0.02, 0.7, "paper", 0.02 * 0.49)):
        out = orc.admm(A, Y, lam, alpha, 4000, threshold=mode)
        for p in range(Y.shape[0]):
            m = Lasso(alpha=lam_eff / A.shape[0], fit_intercept=False, tol=1e-14, max_iter=200000)
            m.fit(A, Y[p])
            assert np.max(np.abs(out["Z"][p] - m.coef_)) < 1e-7, (mode, p)
            assert np.max(np.abs(out["X"][p] - m.coef_)) < 1e-7, (mode, p)


def check_admm_identity(orc):
    """A = I: the fixed point is soft(y, lam_eff), and the first iterate is
    x^1 = y / (1 + alpha) (z^0 = w^0 = 0)."""
    y = _rng(32).standard_normal((4, 9))
    lam, alpha = 0.2, 1.8
    out1 = orc.admm(np.eye(9), y, lam, alpha, 1)
    assert np.max(np.abs(out1["X"] - y / (1.0 + alpha))) < 1e-14
    assert np.max(np.abs(out1["Z"] - _soft(y / (1.0 + alpha), lam * alpha))) < 1e-14
    out = orc.admm(np.eye(9), y, lam, alpha, 3000)
    assert np.max(np.abs(out["Z"] - _soft(y, lam * alpha * alpha))) < 1e-12
    outs = orc.admm(np.eye(9), y, lam, alpha, 3000, threshold="standard")
    assert np.max(np.abs(outs["Z"] - _soft(y, lam))) < 1e-12


def check_admm_kkt_and_dual(orc):
    """KKT residual of Eq. 2 at lam_eff vanishes for the converged z; the dual
    variable w^k = sum_{j <= k} (x^j - z^j) (step 3 from w^0 = 0) stays inside
    [-thr, thr] at every iteration, since it is what the soft threshold of
    step 2 cut off."""
    from oracle import metrics
    A, _, Y = _sparse_problem(15, 30, 3, 2, 33, noise=0.05)
    lam, alpha = 0.02, 1.8
    out = orc.admm(A, Y, lam, alpha, 6000)
    kkt = metrics.lasso_kkt_residual(A, Y, out["Z"], lam * alpha * alpha)
    assert np.all(kkt < 1e-9), kkt
    thr = lam * alpha
    w = np.zeros_like(Y @ A)
    for k in range(1, 9):
        o = orc.admm(A, Y, lam, alpha, k)
        w = w + o["X"] - o["Z"]
        assert np.all(np.abs(w) <= thr * (1 + 1e-9)), (k, np.abs(w).max(), thr)


def check_admm_stop_rule(orc):
    """Delta = ||r^i - r^{i-1}||, r^0 = y: Delta at iteration 1 is ||A x^1||; a
    huge eps stops after iteration 1."""
    A, _, Y = _sparse_problem(20, 40, 3, 4, 34)
    o = orc.admm(A, Y, 0.01, 1.8, 1)
    assert np.allclose(o["delta"], np.linalg.norm(o["X"] @ A.T, axis=1), rtol=1e-12)
    o = orc.admm(A, Y, 0.01, 1.8, 50, eps=1e9)
    assert np.all(o["iters"] == 1) and np.all(o["flags"] == orc.STOP_CONVERGED)


# ---------------------------------------------------------------- complex FISTA (Section II DFT basis)

def _complex_problem(M, N, K, P, seed):
    rng = _rng(seed)
    A = (rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N))) / math.sqrt(2 * M)
    X = np.zeros((P, N), dtype=complex)
    for p in range(P):
        idx = rng.choice(N, K, replace=False)
        X[p, idx] = (1.0 + rng.random(K)) * np.exp(2j * np.pi * rng.random(K))
    return A, X, X @ A.T


def check_fista_complex_real_case(orc):
    """Real A and y: the complex iteration is the real one (imaginary parts stay 0)."""
    A, _, Y = _sparse_problem(12, 30, 3, 5, 41)
    L = orc.lipschitz(A)
    r = orc.fista_complex(A, Y, 0.05, L, 60)
    assert np.max(np.abs(r["X"].imag)) == 0.0
    assert np.allclose(r["X"].real, orc.fista(A, Y, 0.05, L, 60)["X"], atol=1e-12)


def check_fista_complex_identity(orc):
    """A = c I, c complex: L = |c|^2 and from x^0 = 0 the first iterate is the
    minimiser x* = sign(u) max(|u| - lam / |c|^2, 0), u = conj(c) y / |c|^2;
    every later iterate stays there."""
    c = 0.8 * np.exp(0.7j)
    y = (_rng(42).standard_normal((4, 9)) + 1j * _rng(43).standard_normal((4, 9)))
    lam = 0.3
    u = np.conj(c) * y / abs(c) ** 2
    mag = np.abs(u)
    xs = np.where(mag > lam / abs(c) ** 2, u * (mag - lam / abs(c) ** 2) / np.where(mag > 0, mag, 1), 0)
    for it in (1, 25):
        r = orc.fista_complex(c * np.eye(9), y, lam, abs(c) ** 2, it)
        assert np.allclose(r["X"], xs, atol=1e-12), it


def check_fista_complex_phase_equivariance(orc):
    """A -> e^{i a} A maps every iterate x -> e^{-i a} x, and y -> e^{i b} y
    maps x -> e^{i b} x: the threshold acts on |x| only."""
    A, _, Y = _complex_problem(15, 40, 4, 6, 44)
    L = orc.lipschitz_complex(A)
    r0 = orc.fista_complex(A, Y, 0.05, L, 40)
    r1 = orc.fista_complex(np.exp(0.9j) * A, Y, 0.05, L, 40)
    r2 = orc.fista_complex(A, np.exp(-1.3j) * Y, 0.05, L, 40)
    assert np.allclose(r1["X"], np.exp(-0.9j) * r0["X"], atol=1e-10)
    assert np.allclose(r2["X"], np.exp(-1.3j) * r0["X"], atol=1e-10)


def check_fista_complex_kkt(orc):
    """Run long, x meets the complex LASSO optimality conditions:
    A^*(A x - y) + lam x / |x| = 0 on the support, |A^*(A x - y)| <= lam off it;
    and exact sparse data is recovered for small lam."""
    A, X, Y = _complex_problem(20, 50, 3, 5, 45)
    L = orc.lipschitz_complex(A)
    lam = 0.02
    x = orc.fista_complex(A, Y, lam, L, 4000)["X"]
    g = (x @ A.T - Y) @ np.conj(A)
    on = np.abs(x) > 0
    assert np.max(np.abs(g + lam * x / np.where(on, np.abs(x), 1))[on]) < 1e-8
    assert np.max(np.abs(g)[~on]) <= lam + 1e-8
    # the 3 largest |x| are the true support (lasso shrinks their values a little)
    top = np.sort(np.argsort(-np.abs(x), axis=1)[:, :3], axis=1)
    assert np.array_equal(top, np.sort(np.argsort(-np.abs(X), axis=1)[:, :3], axis=1))


def check_admm_complex_real_case(orc):
    """Real A and y: complex ADMM is the real one, both threshold readings."""
    A, _, Y = _sparse_problem(12, 30, 3, 5, 51)
    for mode in ("paper", "standard"):
        r = orc.admm_complex(A, Y, 0.05, 1.8, 60, threshold=mode)
        o = orc.admm(A, Y, 0.05, 1.8, 60, threshold=mode)
        assert np.max(np.abs(r["X"].imag)) == 0.0 and np.max(np.abs(r["Z"].imag)) == 0.0
        assert np.allclose(r["X"].real, o["X"], atol=1e-12) and np.allclose(r["Z"].real, o["Z"], atol=1e-12)
        assert np.allclose(r["delta"], o["delta"], rtol=1e-10)


def check_admm_complex_identity(orc):
    """A = c I, c complex: with threshold tau the iteration solves Eq. 2 with
    weight tau alpha, whose minimiser is x* = sign(u) max(|u| - tau alpha /
    |c|^2, 0), u = conj(c) y / |c|^2; z^I and x^I converge to it."""
    c = 0.8 * np.exp(0.7j)
    y = (_rng(52).standard_normal((4, 9)) + 1j * _rng(53).standard_normal((4, 9)))
    lam, alpha = 0.2, 1.8
    u = np.conj(c) * y / abs(c) ** 2
    mag = np.abs(u)
    for mode, tau in (("paper", lam * alpha), ("standard", lam / alpha)):
        w = tau * alpha / abs(c) ** 2
        xs = np.where(mag > w, u * (mag - w) / np.where(mag > 0, mag, 1), 0)
        r = orc.admm_complex(c * np.eye(9), y, lam, alpha, 3000, threshold=mode)
        assert np.allclose(r["Z"], xs, atol=1e-9) and np.allclose(r["X"], xs, atol=1e-9), mode


def check_admm_complex_matches_fista_complex(orc):
    """Both solve the complex LASSO: ADMM with the lam / alpha threshold and
    FISTA with weight lam reach the same minimiser; the paper's lam alpha
    threshold solves it with weight lam alpha^2."""
    A, _, Y = _complex_problem(15, 40, 3, 4, 54)
    L = orc.lipschitz_complex(A)
    lam, alpha = 0.03, 1.8
    xf = orc.fista_complex(A, Y, lam, L, 6000)["X"]
    xa = orc.admm_complex(A, Y, lam, alpha, 6000, threshold="standard")["Z"]
    assert np.allclose(xa, xf, atol=1e-7), np.abs(xa - xf).max()
    xf2 = orc.fista_complex(A, Y, lam * alpha * alpha, L, 6000)["X"]
    xa2 = orc.admm_complex(A, Y, lam, alpha, 6000, threshold="paper")["Z"]
    assert np.allclose(xa2, xf2, atol=1e-7), np.abs(xa2 - xf2).max()


def check_admm_complex_phase_equivariance(orc):
    """A -> e^{i a} A maps x -> e^{-i a} x, y -> e^{i b} y maps x -> e^{i b} x."""
    A, _, Y = _complex_problem(15, 40, 4, 6, 55)
    r0 = orc.admm_complex(A, Y, 0.05, 1.8, 40)
    r1 = orc.admm_complex(np.exp(0.9j) * A, Y, 0.05, 1.8, 40)
    r2 = orc.admm_complex(A, np.exp(-1.3j) * Y, 0.05, 1.8, 40)
    assert np.allclose(r1["X"], np.exp(-0.9j) * r0["X"], atol=1e-10)
    assert np.allclose(r2["X"], np.exp(-1.3j) * r0["X"], atol=1e-10)
    assert np.allclose(r2["delta"], r0["delta"], rtol=1e-9)


def check_sparsify_complex_basis(orc):
    """With a unitary complex basis x = Psi^* f: a spectrum of 5 large and 59
    tiny complex coefficients keeps exactly the large ones, with their values."""
    N = 64
    rng = _rng(46)
    q, r = np.linalg.qr(rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)))
    Psi = q * (np.diag(r) / np.abs(np.diag(r)))[None, :]
    Xt = 0.01 * (rng.standard_normal((10, N)) + 1j * rng.standard_normal((10, N)))
    sup = np.stack([rng.choice(N, 5, replace=False) for _ in range(10)])
    for p in range(10):
        Xt[p, sup[p]] = (5.0 + rng.random(5)) * np.exp(2j * np.pi * rng.random(5))
    res = orc.sparsify(Xt @ Psi.T, Psi, 0.1)
    for p in range(10):
        assert set(np.nonzero(res["X"][p])[0]) == set(sup[p])
        assert np.allclose(res["X"][p, sup[p]], Xt[p, sup[p]], atol=1e-12)


# ---------------------------------------------------------------- sparsification (Section II)

def check_sparsify_worked(orc):
    """Hand-computed cases of the rule |x_n| - mu_x < T sigma_x -> x_n = 0
    (Psi = I, so x = f)."""
    # |x| = (3, 1, 0.5, 2): mu = 6.5 / 4 = 1.625; squared deviations sum to
    # 1.890625 + 0.390625 + 1.265625 + 0.140625 = 3.6875, so sigma = sqrt(3.6875 / 3)
    # = 1.10867789 (N - 1) and sqrt(3.6875 / 4) = 0.96014322 (N)
    f = np.array([[3.0, -1.0, 0.5, 2.0]])
    r = orc.sparsify(f, np.eye(4), 0.1)
    assert abs(r["mu"][0] - 1.625) < 1e-15 and abs(r["sigma"][0] - math.sqrt(3.6875 / 3)) < 1e-15
    # T = 0.1: threshold 1.625 + 0.1109 = 1.7359 keeps 3 and 2
    assert np.array_equal(r["X"], [[3.0, 0.0, 0.0, 2.0]]) and r["kept"][0] == 2
    # the rule reads |x|: negated entries keep their places and signs
    assert np.array_equal(orc.sparsify(-f, np.eye(4), 0.1)["X"], [[-3.0, 0.0, 0.0, -2.0]])
    # T = 0.36: 1.625 + 0.36 sigma is 2.0241 with N - 1 (drops 2) and 1.9706 with N (keeps it)
    assert np.array_equal(orc.sparsify(f, np.eye(4), 0.36)["X"], [[3.0, 0.0, 0.0, 0.0]])
    assert np.array_equal(orc.sparsify(f, np.eye(4), 0.36, ddof=0)["X"], [[3.0, 0.0, 0.0, 2.0]])
    # the inequality is strict: with T = 0 an entry equal to the mean is kept
    r = orc.sparsify(np.array([[1.0, 2.0, 3.0]]), np.eye(3), 0.0)
    assert np.array_equal(r["X"], [[0.0, 2.0, 3.0]]) and r["kept"][0] == 2 and r["margin"][0] == 0.0
    # a non-finite spectrum sparsifies to zero, with nothing kept
    g = np.array([[1.0, np.nan, 2.0, 0.0], [4.0, 0.0, 0.0, 0.0]])
    r = orc.sparsify(g, np.eye(4), 0.1)
    assert np.all(r["X"][0] == 0.0) and r["kept"][0] == 0 and r["kept"][1] == 1


def check_sparsify_transform(orc):
    """x = Psi^T f for an orthonormal, non-symmetric Psi: a spectrum built
    from 5 large and 59 tiny coefficients keeps exactly the large ones, with
    their values; keep-all returns f (Parseval); positive scaling commutes;
    raising T never keeps more."""
    N = 64
    Psi = _orthonormal(N, 31)
    rng = _rng(32)
    Xt = 0.01 * rng.standard_normal((20, N))
    sup = np.stack([rng.choice(N, 5, replace=False) for _ in range(20)])
    for p in range(20):
        Xt[p, sup[p]] = rng.choice([-1.0, 1.0], 5) * (5.0 + rng.random(5))
    F = Xt @ Psi.T
    r = orc.sparsify(F, Psi, 0.1)
    for p in range(20):
        assert set(np.nonzero(r["X"][p])[0]) == set(sup[p])
        assert np.allclose(r["X"][p, sup[p]], Xt[p, sup[p]], atol=1e-12)
    assert np.allclose(r["F"], r["X"] @ Psi.T, atol=1e-12)
    assert np.allclose(np.linalg.norm(r["F"], axis=1), np.linalg.norm(r["X"], axis=1), rtol=1e-12)
    keep_all = orc.sparsify(F, Psi, -1e9)
    assert np.allclose(keep_all["F"], F, atol=1e-12) and np.all(keep_all["kept"] == N)
    assert np.allclose(orc.sparsify(7.5 * F, Psi, 0.1)["X"], 7.5 * r["X"], atol=1e-11)
    k = [orc.sparsify(F, Psi, T)["kept"] for T in (-0.5, 0.0, 0.1, 0.5, 2.0)]
    assert all(np.all(a >= b) for a, b in zip(k, k[1:]))


def check_metrics():
    from oracle import metrics
    ref = _rng(27).standard_normal((10, 20))
    ref[3, 4] = 5.0
    est = ref + 0.01
    assert abs(metrics.psnr(est, ref) - 20.0 * math.log10(5.0 / 0.01)) < 1e-9
    assert metrics.psnr(ref, ref) == float("inf")
    flags = np.array([1, 2, 1, 3, 8])
    assert metrics.psnr(ref, ref) == float("inf")
    from oracle import protocol
    assert protocol.convergence_ratio(flags, 1) == 3 / 5 and protocol.convergence_ratio(flags, 2) == 2 / 5
    e = np.zeros_like(ref)
    e[:, 0] = 1.0
    assert np.allclose(metrics.rel_err(ref + e, ref), 1.0 / np.linalg.norm(ref, axis=1))
    # KKT residual is zero at the closed-form LASSO solution for A = I
    y = _rng(28).standard_normal((3, 8))
    x = _soft(y, 0.4)
    assert np.max(metrics.lasso_kkt_residual(np.eye(8), y, x, 0.4)) < 1e-15
    assert np.min(metrics.lasso_kkt_residual(np.eye(8), y, y, 0.4)) > 0.0


ORACLE_CHECKS = [
    check_lipschitz, check_fista_identity, check_fista_zero_solution,
    check_fista_diagonal_momentum, check_fista_matches_sklearn_lasso, check_fista_kkt_and_rate,
    check_fista_stop_rule, check_fista_nonfinite, check_lstsq, check_lstsq_min_norm, check_top_indices,
    check_gomp_is_omp_when_S1, check_gomp_orthonormal, check_gomp_exact_recovery,
    check_gomp_brute_force, check_gomp_prune_invariants, check_gomp_no_reselect,
    check_gomp_stop, check_gomp_final_prune, check_gomp_diagnostics_by_hand, check_round_to_format,
    check_greedy_complex_real_case, check_greedy_complex_recovery_and_phase, check_greedy_complex_unitary_dft,
    check_greedy_complex_conjugate_pairs,
    check_cosamp_biht_res_tol,
    check_cosamp_orthonormal, check_cosamp_recovery, check_cosamp_no_resolve, check_cosamp_wide,
    check_biht_orthonormal, check_biht_first_step, check_biht_second_step_mu,
    check_biht_recovery, check_one_bit, check_admm_matches_sklearn_lasso, check_admm_identity,
    check_admm_kkt_and_dual, check_admm_stop_rule, check_sparsify_worked, check_sparsify_transform,
    check_fista_complex_real_case, check_fista_complex_identity, check_fista_complex_phase_equivariance,
    check_fista_complex_kkt, check_sparsify_complex_basis, check_admm_complex_real_case, check_admm_complex_identity,
    check_admm_complex_matches_fista_complex, check_admm_complex_phase_equivariance,
]
