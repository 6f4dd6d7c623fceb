"""FP64 greedy solvers (Alg. 3, 4, 5) for the complex measurement model of
Section II, where the DFT basis makes A = Phi Psi and x complex.

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU leg
of the benchmark, never by the product path, sharing no code with it.

The steps are those of ``cs.gomp``, ``cs.cosamp`` and ``cs.biht`` with A^*
the conjugate transpose, |.| the complex magnitude, and the least squares
complex (Householder QR).  One generalisation: the units of selection and
pruning are groups of atoms (default: every atom is its own group, and the
solvers are the printed algorithms).  The score of a group is the root mean
square of |v_i| over its members.

Real measurements (the paper's setting: a real Phi measures a real spectrum)
make the columns of A conjugate-symmetric, A[:, N-k] = conj(A[:, k]), and
|p_k| = |p_{N-k}| for p = A^* r of every real r: atoms k and N - k tie
exactly in every correlation, and the least squares on a support closed
under k <-> N-k keeps x conjugate-symmetric (so A x and r stay real).  With
``conj_pair_groups(N)`` -- {0}, {k, N-k} for 0 < k < N/2, {N/2} for even N
-- as the groups, a tie that exact arithmetic leaves to chance becomes one
decision: the pair is selected, kept or pruned together.  K and S then
count groups (a pair is one of the K, and holds two complex atoms)."""
from __future__ import annotations

from typing import Optional

import numpy as np

from .cs import STOP_CONVERGED, STOP_ITER_CAP, STOP_NONFINITE


def conj_pair_groups(N: int) -> list:
    """The groups of a conjugate-symmetric spectrum of N bins: [0], then
    [k, N-k] for 1 <= k < N/2, then [N/2] for even N; group g holds bin g."""
    out = [np.array([0])]
    for k in range(1, (N + 1) // 2):
        out.append(np.array([k, N - k]))
    if N % 2 == 0:
        out.append(np.array([N // 2]))
    return out


def _c128(a) -> np.ndarray:
    return np.asarray(a, dtype=np.complex128)


def _members(groups: list, N: int) -> tuple:
    """(G x gmax member table padded with -1, group of each atom)."""
    gmax = max(len(g) for g in groups)
    tab = np.full((len(groups), gmax), -1, dtype=np.int64)
    owner = np.full(N, -1, dtype=np.int64)
    for i, g in enumerate(groups):
        tab[i, :len(g)] = g
        owner[g] = i
    if np.any(owner < 0):
        raise ValueError("the groups must cover every atom")
    return tab, owner


def group_scores(v: np.ndarray, tab: np.ndarray) -> np.ndarray:
    """Per row, sqrt(mean |v_i|^2) over the members of each group."""
    a2 = np.abs(v) ** 2
    valid = tab >= 0
    s = np.where(valid[None], a2[:, np.where(valid, tab, 0)], 0.0).sum(axis=2)
    return np.sqrt(s / valid.sum(axis=1)[None, :])


def _top_groups(scores: np.ndarray, k: int, allowed: Optional[np.ndarray] = None) -> np.ndarray:
    """Per row, the k groups of largest score, ordered (score desc, index asc);
    groups where allowed is False come only after every allowed one."""
    key = scores if allowed is None else np.where(allowed, scores, -1.0)
    return np.argsort(-key, axis=1, kind="stable")[:, :k]


def _gap(scores: np.ndarray, k: int, allowed: Optional[np.ndarray] = None) -> np.ndarray:
    """(score_(k) - score_(k+1)) / max score over the allowed groups."""
    key = scores if allowed is None else np.where(allowed, scores, -np.inf)
    srt = -np.sort(-key, axis=1)
    if srt.shape[1] <= k:
        return np.full(key.shape[0], np.inf)
    nxt = np.where(np.isfinite(srt[:, k]), srt[:, k], 0.0)
    return (srt[:, k - 1] - nxt) / np.maximum(srt[:, 0], 1e-300)


def lstsq_complex(A: np.ndarray, y: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """s = A(:, cols)^+ y for one pixel: Householder QR of the selected
    columns (full column rank), then R s = Q^* y."""
    B = A[:, cols]
    if B.shape[1] == 0:
        return np.zeros(0, dtype=np.complex128)
    Q, R = np.linalg.qr(B)
    return np.linalg.solve(R, np.conj(Q).T @ y)


def _atoms_of(gsel, tab) -> np.ndarray:
    m = tab[np.asarray(gsel, dtype=np.int64)].ravel()
    return np.sort(m[m >= 0])


def _finite_rows(Y: np.ndarray) -> np.ndarray:
    return np.all(np.isfinite(Y), axis=1)


def _support_table(x: np.ndarray, width: int) -> np.ndarray:
    P, N = x.shape
    out = np.full((P, width), -1, dtype=np.int64)
    for p in range(P):
        nz = np.nonzero(x[p] != 0)[0][:width]
        out[p, :len(nz)] = nz
    return out


def gomp_complex(A, Y, K: int, S: int, max_iter: int = 0, res_tol: float = 0.0, eps: float = 0.0,
                 prune: str = "each", groups: Optional[list] = None, diagnostics: bool = False) -> dict:
    """gOMP (Alg. 3) for complex A and y (y may be real), groups as units.

    Per iteration, for each pixel still running:
      1. p = A^* r;  the S groups of largest score not in c join c
      2. s = A(:, atoms of c)^+ y;  x = 0, x(atoms of c) = s
      3. when c holds more than K groups (prune='each'): q = the K groups of
         c with the largest score of s;  s = A(:, atoms of q)^+ y;  x on q
      4. r = y - A x,  Delta = ||r - r_prev||;  stop when ||r|| <= res_tol ||y||
         or Delta < eps
    Default max_iter: min(K, floor(M / (S gmax))), gmax the largest group, so
    that the atoms of c never outnumber the measurements.  prune='final'
    applies step 3 once after the loop.  Returns dict(X (complex128),
    support (P x K gmax atom indices, ascending, -1 padded), iters, delta,
    resid, flags) and with diagnostics the smallest selection and prune gaps
    (relative to the largest compared score)."""
    A = _c128(A)
    Y = _c128(Y)
    P, M = Y.shape
    N = A.shape[1]
    groups = [np.array([n]) for n in range(N)] if groups is None else groups
    tab, owner = _members(groups, N)
    G, gmax = tab.shape
    I_max = max_iter if max_iter > 0 else min(K, M // (S * gmax))
    if S * gmax * I_max > M:
        raise ValueError("S * max_iter groups could hold more atoms than measurements")
    Ah = np.conj(A)
    fin = _finite_rows(Y)
    Yc = np.where(fin[:, None], Y, 0.0)
    ynorm = np.linalg.norm(Yc, axis=1)
    x = np.zeros((P, N), dtype=np.complex128)
    r = Yc.copy()
    c = [[] for _ in range(P)]                  # selected groups, in order
    iters = np.zeros(P, dtype=np.int64)
    delta = np.full(P, np.nan)
    flags = np.zeros(P, dtype=np.int64)
    flags[~fin] |= STOP_NONFINITE
    sel_gap = np.full(P, np.inf)
    prune_gap = np.full(P, np.inf)
    active = fin.copy()
    for i in range(1, I_max + 1):
        if not active.any():
            break
        a = np.nonzero(active)[0]
        p = r[a] @ Ah                                           # step 1: A^* r
        sc = group_scores(p, tab)
        allowed = np.ones((len(a), G), dtype=bool)
        for j, pix in enumerate(a):
            allowed[j, c[pix]] = False
        theta = _top_groups(sc, S, allowed)
        if diagnostics:
            sel_gap[a] = np.minimum(sel_gap[a], _gap(sc, S, allowed))
        for j, pix in enumerate(a):
            c[pix].extend(int(g) for g in theta[j])
            cols = _atoms_of(c[pix], tab)
            s = lstsq_complex(A, Yc[pix], cols)                 # step 2
            xp = np.zeros(N, dtype=np.complex128)
            xp[cols] = s
            if prune == "each" and len(c[pix]) > K:             # step 3
                inc = np.zeros(G, dtype=bool)
                inc[c[pix]] = True
                gs = group_scores(xp[None, :], tab)
                q = _top_groups(gs, K, inc[None, :])[0]
                if diagnostics:
                    prune_gap[pix] = min(prune_gap[pix], _gap(gs, K, inc[None, :])[0])
                qc = _atoms_of(q, tab)
                xp = np.zeros(N, dtype=np.complex128)
                xp[qc] = lstsq_complex(A, Yc[pix], qc)
            r_new = Yc[pix] - A @ xp                            # step 4
            d = np.linalg.norm(r_new - r[pix])
            x[pix], r[pix] = xp, r_new
            iters[pix] = i
            delta[pix] = d
            if np.linalg.norm(r_new) <= res_tol * ynorm[pix] or d < eps:
                flags[pix] |= STOP_CONVERGED
                active[pix] = False
    flags[active] |= STOP_ITER_CAP
    if prune == "final":
        for pix in np.nonzero(fin)[0]:
            if len(c[pix]) <= K:
                continue
            inc = np.zeros(G, dtype=bool)
            inc[c[pix]] = True
            gs = group_scores(x[pix][None, :], tab)
            q = _top_groups(gs, K, inc[None, :])[0]
            if diagnostics:
                prune_gap[pix] = min(prune_gap[pix], _gap(gs, K, inc[None, :])[0])
            qc = _atoms_of(q, tab)
            x[pix] = 0.0
            x[pix, qc] = lstsq_complex(A, Yc[pix], qc)
    resid = np.linalg.norm(Yc - x @ A.T, axis=1)
    out = dict(X=x, support=_support_table(x, K * gmax), iters=iters, delta=delta, resid=resid, flags=flags)
    if diagnostics:
        out.update(sel_gap=sel_gap, prune_gap=prune_gap)
    return out


def cosamp_complex(A, Y, K: int, max_iter: int, eps: float = 0.0, res_tol: float = 0.0,
                   groups: Optional[list] = None, diagnostics: bool = False) -> dict:
    """CoSaMP (Alg. 5) for complex A and y, groups as units: Theta = the 2K
    groups of largest score of p = A^* r, c = Theta U the previous support,
    s = least squares on the atoms of c, keep the K groups of largest score
    of s with their values (no second solve), r = y - A x, stop on Delta < eps
    or ||r|| <= res_tol ||y||."""
    A = _c128(A)
    Y = _c128(Y)
    P, M = Y.shape
    N = A.shape[1]
    groups = [np.array([n]) for n in range(N)] if groups is None else groups
    tab, owner = _members(groups, N)
    G, gmax = tab.shape
    if 3 * K * gmax > M:
        raise ValueError("3K groups could hold more atoms than measurements")
    Ah = np.conj(A)
    fin = _finite_rows(Y)
    Yc = np.where(fin[:, None], Y, 0.0)
    ynorm = np.linalg.norm(Yc, axis=1)
    x = np.zeros((P, N), dtype=np.complex128)
    r = Yc.copy()
    kept = [np.zeros(0, dtype=np.int64) for _ in range(P)]
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
        sc = group_scores(r[a] @ Ah, tab)                       # step 1
        theta = _top_groups(sc, 2 * K)
        if diagnostics:
            sel_gap[a] = np.minimum(sel_gap[a], _gap(sc, 2 * K))
        for j, pix in enumerate(a):
            cg = np.union1d(theta[j], kept[pix])
            cols = _atoms_of(cg, tab)
            full = np.zeros(N, dtype=np.complex128)
            full[cols] = lstsq_complex(A, Yc[pix], cols)        # step 2
            if diagnostics:
                ls_cond[pix] = np.linalg.cond(A[:, cols])
            inc = np.zeros(G, dtype=bool)
            inc[cg] = True
            gs = group_scores(full[None, :], tab)
            q = _top_groups(gs, K, inc[None, :])[0]             # step 3
            if diagnostics:
                prune_gap[pix] = min(prune_gap[pix], _gap(gs, K, inc[None, :])[0])
            qc = _atoms_of(q, tab)
            xp = np.zeros(N, dtype=np.complex128)
            xp[qc] = full[qc]
            kept[pix] = np.sort(q)
            r_new = Yc[pix] - A @ xp                            # step 4
            d = np.linalg.norm(r_new - r[pix])
            x[pix], r[pix] = xp, r_new
            iters[pix] = i
            delta[pix] = d
            if d < eps or np.linalg.norm(r_new) <= res_tol * ynorm[pix]:
                flags[pix] |= STOP_CONVERGED
                active[pix] = False
    flags[active] |= STOP_ITER_CAP
    resid = np.linalg.norm(Yc - x @ A.T, axis=1)
    out = dict(X=x, support=_support_table(x, K * gmax), iters=iters, delta=delta, resid=resid, flags=flags)
    if diagnostics:
        # ls_cond: condition number of A(:, c) of the last solve (step 2)
        out.update(sel_gap=sel_gap, prune_gap=prune_gap, ls_cond=ls_cond)
    return out


def biht_complex(A, Y, K: int, max_iter: int, mu: float = 0.1, eps: float = 0.0, res_tol: float = 0.0,
                 groups: Optional[list] = None, diagnostics: bool = False) -> dict:
    """Backtracking IHT (Alg. 4) for complex A and y, groups as units:
    u = x + mu A^* (y - A x), Theta = the K groups of largest score of u,
    c = the groups of x's support U Theta, s = least squares on the atoms of
    c, keep the K groups of largest score of s (zero elsewhere), r = y - A x,
    stop on Delta < eps or ||r|| <= res_tol ||y||."""
    A = _c128(A)
    Y = _c128(Y)
    P, M = Y.shape
    N = A.shape[1]
    groups = [np.array([n]) for n in range(N)] if groups is None else groups
    tab, owner = _members(groups, N)
    G, gmax = tab.shape
    if 2 * K * gmax > M:
        raise ValueError("2K groups could hold more atoms than measurements")
    Ah = np.conj(A)
    fin = _finite_rows(Y)
    Yc = np.where(fin[:, None], Y, 0.0)
    ynorm = np.linalg.norm(Yc, axis=1)
    x = np.zeros((P, N), dtype=np.complex128)
    r = Yc.copy()
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
        xa = x[a]
        u = xa + mu * ((Yc[a] - xa @ A.T) @ Ah)                 # step 1
        sc = group_scores(u, tab)
        theta = _top_groups(sc, K)
        if diagnostics:
            sel_gap[a] = np.minimum(sel_gap[a], _gap(sc, K))
        for j, pix in enumerate(a):
            prev = np.unique(owner[np.nonzero(x[pix] != 0)[0]])
            cg = np.union1d(prev, theta[j])
            cols = _atoms_of(cg, tab)
            full = np.zeros(N, dtype=np.complex128)
            full[cols] = lstsq_complex(A, Yc[pix], cols)        # step 2
            if diagnostics:
                ls_cond[pix] = np.linalg.cond(A[:, cols])
            inc = np.zeros(G, dtype=bool)
            inc[cg] = True
            gs = group_scores(full[None, :], tab)
            h = _top_groups(gs, K, inc[None, :])[0]             # step 3
            if diagnostics and len(cg) > K:
                prune_gap[pix] = min(prune_gap[pix], _gap(gs, K, inc[None, :])[0])
            hc = _atoms_of(h, tab)
            xp = np.zeros(N, dtype=np.complex128)
            xp[hc] = full[hc]
            r_new = Yc[pix] - A @ xp                            # step 4
            d = np.linalg.norm(r_new - r[pix])
            x[pix], r[pix] = xp, r_new
            iters[pix] = i
            delta[pix] = d
            if d < eps or np.linalg.norm(r_new) <= res_tol * ynorm[pix]:
                flags[pix] |= STOP_CONVERGED
                active[pix] = False
    flags[active] |= STOP_ITER_CAP
    resid = np.linalg.norm(Yc - x @ A.T, axis=1)
    out = dict(X=x, support=_support_table(x, K * gmax), iters=iters, delta=delta, resid=resid, flags=flags)
    if diagnostics:
        # ls_cond: condition number of A(:, c) of the last solve (step 2)
        out.update(sel_gap=sel_gap, prune_gap=prune_gap, ls_cond=ls_cond)
    return out
