"""Plant plausible mistakes in a copy of the oracle source (on the CPU) and
check that the pins catch every one of them.  The real oracle is untouched.

A mutant is the whole oracle: the mutated module's functions laid over the
real package's, so every check finds every function it calls and fails only
on wrong arithmetic.  An unmutated copy must pass every check, and a check
that raises anything but a wrong-value error is a bug of the harness, not a
catch."""
import os
import types

import numpy as np
import pytest

import oracle
import oracle_pins as pins

ORACLE_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")
SRC = os.path.join(ORACLE_DIR, "cs.py")
PROTOCOL_SRC = os.path.join(ORACLE_DIR, "protocol.py")
COMPLEX_SRC = os.path.join(ORACLE_DIR, "greedy_complex.py")

# (id, text to replace, replacement[, which occurrence (1 = first)])
MUTATIONS = [
    ("fista-threshold-lam", "soft_threshold(aux, dtype(lam / L))", "soft_threshold(aux, dtype(lam))"),
    ("fista-no-step-1/L", "(1.0 / L) * ((za @ A.T - ya) @ A)", "((za @ A.T - ya) @ A)"),
    ("fista-gradient-sign", "((za @ A.T - ya) @ A)", "((ya - za @ A.T) @ A)"),
    ("fista-no-momentum", "z_new = x_new + dtype((t - 1.0) / t_new) * (x_new - xa)", "z_new = x_new"),
    ("fista-t-recursion", "math.sqrt(1.0 + 4.0 * t * t)", "math.sqrt(1.0 + t * t)"),
    ("fista-momentum-index", "((t - 1.0) / t_new)", "((t_new - 1.0) / t_new)"),
    ("fista-delta-vs-y", "d = np.linalg.norm(r_new - r[a], axis=1)", "d = np.linalg.norm(r_new, axis=1)"),
    ("ties-to-higher-index", 'order = np.argsort(-key, axis=1, kind="stable")',
     'order = key.shape[1] - 1 - np.argsort(-key[:, ::-1], axis=1, kind="stable")'),
    ("lstsq-transposed-R", "np.linalg.solve(R, qty[..., None])",
     "np.linalg.solve(np.transpose(R, (0, 2, 1)), qty[..., None])"),
    ("min-norm-untransposed-R", "w = np.linalg.solve(np.transpose(R, (0, 2, 1)), Y[..., None])[..., 0]",
     "w = np.linalg.solve(R, Y[..., None])[..., 0]"),
    ("min-norm-ridge", "if cols.shape[1] > A.shape[0]:",
     "if cols.shape[1] > A.shape[0]:\n        G = np.einsum('pmi,pmj->pij', B, B) + 1e-6 * np.eye(cols.shape[1])\n"
     "        return np.linalg.solve(G, np.einsum('pmk,pm->pk', B, Y)[..., None])[..., 0]"),
    ("gomp-no-mask", "theta = top_indices(p, S, allowed)", "theta = top_indices(p, S)"),
    ("gomp-no-prune", 'if prune == "each" and i * S > K:', "if False:"),
    ("gomp-prune-no-resolve", "sq = lstsq_on_support(A, ya, q)",
     "sq = xa[np.arange(len(a))[:, None], q]"),
    ("gomp-wrong-ls-columns", "s = lstsq_on_support(A, ya, cur)",
     "s = lstsq_on_support(A, ya, cur)[:, ::-1]"),
    ("gomp-absolute-res-tol", "stop = (rn <= res_tol * ynorm[a]) | (d < eps)",
     "stop = (rn <= res_tol) | (d < eps)"),
    ("cosamp-K-not-2K", "theta = top_indices(p, 2 * K)", "theta = top_indices(p, K)"),
    ("cosamp-no-union", "np.union1d(theta[j], cprev[a[j]])", "np.sort(theta[j])"),
    ("biht-no-mu", "u = xa_prev + mu * ((ya - xa_prev @ A.T) @ A)",
     "u = xa_prev + ((ya - xa_prev @ A.T) @ A)"),
    ("biht-no-union", "np.union1d(np.nonzero(xa_prev[j])[0], theta[j])", "np.sort(theta[j])"),
    ("onebit-sgn0-plus", "u = x + mu * ((Ys - np.sign(ax)) @ A)",
     "u = x + mu * ((Ys - np.where(ax >= 0, 1.0, -1.0)) @ A)"),
    ("onebit-no-normalise", "x = np.where(nrm > 0, x / np.where(nrm > 0, nrm, 1.0), 0.0)", "x = x"),
    ("admm-threshold-over-alpha", "        return lam * alpha\n", "        return lam / alpha\n"),
    ("admm-no-alpha-identity", "(A.T @ A + dtype(alpha) * np.eye(N, dtype=dtype))", "(A.T @ A + np.eye(N, dtype=dtype))"),
    ("admm-dual-sign", "rhs = Aty[a] + dtype(alpha) * (z[a] - w[a])", "rhs = Aty[a] + dtype(alpha) * (z[a] + w[a])"),
    ("admm-no-dual-in-threshold", "zt = x_new + w[a]", "zt = x_new"),
    ("admm-dual-not-accumulated", "w_new = zt - z_new", "w_new = x_new - z_new"),
    ("cfista-transpose-not-adjoint", "Ah = np.conj(A) ", "Ah = A "),
    ("cfista-separable-shrink", "x_new = soft_threshold_complex(aux, rdt(lam / L))",
     "x_new = soft_threshold(aux.real, rdt(lam / L)) + 1j * soft_threshold(aux.imag, rdt(lam / L))"),
    ("cfista-phase-dropped", "    return v * scale.astype(v.real.dtype)", "    return np.abs(v) * scale.astype(v.real.dtype)"),
    ("cfista-no-momentum", "z_new = x_new + rdt((t - 1.0) / t_new) * (x_new - xa)", "z_new = x_new"),
    ("cadmm-transpose-not-adjoint", "Ahy = Yc @ np.conj(A) ", "Ahy = Yc @ A "),
    ("cadmm-gram-not-hermitian", "np.linalg.cholesky(np.conj(A64).T @ A64 + alpha * np.eye(N))",
     "np.linalg.cholesky(A64.T @ A64 + alpha * np.eye(N))"),
    ("cadmm-factor-not-conjugated", "np.linalg.solve(np.conj(Cf).T, ", "np.linalg.solve(Cf.T, "),
    ("cadmm-separable-shrink", "zn = soft_threshold_complex(v, tau)",
     "zn = soft_threshold(v.real, tau) + 1j * soft_threshold(v.imag, tau)"),
    ("cadmm-no-dual-in-threshold", "v = xn + wc[a]", "v = xn"),
    # gOMP's prune after the loop (Alg. 3 step 3 applied once)
    ("gomp-final-skipped", 'if prune == "final":', "if False:"),
    ("gomp-final-no-resolve", "sq = lstsq_on_support(A, Yc[big], q)", "sq = x[big[:, None], q]"),
    # the near-tie diagnostics that decide which pixels get exact parity
    ("ordered-gap-zero", "return (srt[:, k - 1] - nxt) / top", "return 0.0 * (srt[:, k - 1] - nxt) / top"),
    ("ordered-gap-scale-ignored",
     "top = np.maximum(srt[:, 0] if scale is None else np.asarray(scale, dtype=np.float64), 1e-300)",
     "top = np.maximum(srt[:, 0], 1e-300)"),
    ("ordered-gap-kth-vs-first", "return (srt[:, k - 1] - nxt) / top", "return (srt[:, 0] - nxt) / top"),
    ("sel-gap-l1-cancelling-sum", "l1 = np.max(np.abs(ra) @ np.abs(A), axis=1)",
     "l1 = np.max(np.abs(ra @ A), axis=1)"),
    ("sel-gap-l1-max-r", "l1 = np.max(np.abs(ra) @ np.abs(A), axis=1)", "l1 = np.max(np.abs(ra), axis=1)"),
    ("bf16-ties-away", "keep = (bits >> 16) & 1                      # lowest kept bit: ties go to the even one",
     "keep = 1 + 0 * bits"),
    ("bf16-truncate", "rounded = ((bits + 0x7FFF + keep) >> 16) << 16", "rounded = (bits >> 16) << 16"),
    ("corr-format-unrounded-r", "p = round_to_format(ra, corr_format) @ Acorr", "p = ra @ Acorr"),
    ("pivot-ratio-infinite", "return np.min(d / np.maximum(g, 1e-300), axis=1)",
     "return np.full(cols.shape[0], np.inf)"),
    ("pivot-ratio-unnormalised", "return np.min(d / np.maximum(g, 1e-300), axis=1)",
     "return np.min(d, axis=1)"),
    ("stop-margin-absolute", "np.abs(rn / np.maximum(ynorm[a], 1e-300) - res_tol) / res_tol)",
     "np.abs(rn - res_tol) / res_tol)"),
    # the relative residual stop of CoSaMP (first occurrence) and BIHT (second)
    ("cosamp-absolute-res-tol", "stop = (d < eps) | (rn <= res_tol * ynorm[a])",
     "stop = (d < eps) | (rn <= res_tol)", 1),
    ("biht-absolute-res-tol", "stop = (d < eps) | (rn <= res_tol * ynorm[a])",
     "stop = (d < eps) | (rn <= res_tol)", 2),
]

# mistakes planted in the sparsification (Section II)
PROTOCOL_MUTATIONS = [
    ("sparsify-population-std", "def sparsify(F, Psi, T: float, ddof: int = 1)",
     "def sparsify(F, Psi, T: float, ddof: int = 0)"),
    ("sparsify-signed-not-magnitude", "mag = np.abs(X)", "mag = X"),
    ("sparsify-non-strict", "zero = gap < 0.0", "zero = gap <= 0.0"),
    ("sparsify-transposed-basis", "X = Fc @ np.conj(Psi) ", "X = Fc @ np.conj(Psi).T "),
    ("sparsify-no-conjugate", "X = Fc @ np.conj(Psi) ", "X = Fc @ Psi "),
    ("sparsify-no-mean", "gap = (mag - mu[:, None]) - T * sigma[:, None]", "gap = mag - T * sigma[:, None]"),
    ("sparsify-keeps-nonfinite", "Fc = np.where(fin[:, None], F, 0.0)", "Fc = F"),
]


# mistakes planted in the complex greedy solvers (the DFT basis)
COMPLEX_MUTATIONS = [
    ("gompc-transpose-not-adjoint", "    Ah = np.conj(A)\n    fin = _finite_rows(Y)\n    Yc = np.where(fin[:, None], Y, 0.0)\n    ynorm = np.linalg.norm(Yc, axis=1)\n    x = np.zeros((P, N), dtype=np.complex128)\n    r = Yc.copy()\n    c = [",
     "    Ah = A\n    fin = _finite_rows(Y)\n    Yc = np.where(fin[:, None], Y, 0.0)\n    ynorm = np.linalg.norm(Yc, axis=1)\n    x = np.zeros((P, N), dtype=np.complex128)\n    r = Yc.copy()\n    c = ["),
    ("lstsq-complex-no-conj", "return np.linalg.solve(R, np.conj(Q).T @ y)", "return np.linalg.solve(R, Q.T @ y)"),
    ("group-score-one-member", "a2[:, np.where(valid, tab, 0)], 0.0).sum(axis=2)",
     "a2[:, np.where(valid, tab, 0)], 0.0)[:, :, :1].sum(axis=2)"),
    ("pair-groups-shifted", "out.append(np.array([k, N - k]))", "out.append(np.array([k, N - k - 1]))"),
    ("gompc-no-mask", "            allowed[j, c[pix]] = False\n", "            pass\n"),
    ("gompc-prune-no-resolve", "                xp[qc] = lstsq_complex(A, Yc[pix], qc)\n            r_new",
     "                xp[qc] = np.zeros(N, dtype=np.complex128)[qc] + 0 * xp[qc]\n            r_new"),
    ("cosampc-K-not-2K", "theta = _top_groups(sc, 2 * K)", "theta = _top_groups(sc, K)"),
    ("bihtc-no-mu", "u = xa + mu * ((Yc[a] - xa @ A.T) @ Ah)", "u = xa + ((Yc[a] - xa @ A.T) @ Ah)"),
]


# Errors a wrong oracle raises on its own (a failed comparison, a shape or
# value error of NumPy from a wrong index or operand, a floating-point trap);
# anything else (a missing name, a type error) means the check could not run.
CATCHES = (AssertionError, ValueError, IndexError, FloatingPointError, np.linalg.LinAlgError)


def _replace_nth(text, old, new, nth):
    at = -1
    for _ in range(nth):
        at = text.index(old, at + 1)
    return text[:at] + new + text[at + len(old):]


def _mutant(old, new, src=SRC, nth=1):
    """The oracle package with ``src`` replaced by a copy whose ``nth``
    occurrence of ``old`` reads ``new`` (old is None: an unmutated copy)."""
    with open(src) as f:
        text = f.read()
    if old is not None:
        assert text.count(old) >= nth, old
        text = _replace_nth(text, old, new, nth)
    mod = types.ModuleType("oracle_mutant")
    mod.__file__ = src
    mod.__package__ = "oracle"   # relative imports of the copy resolve in the package
    exec(compile(text, src + ":mutant", "exec"), mod.__dict__)
    whole = types.ModuleType("oracle_whole")
    for name in dir(oracle):
        if not name.startswith("__"):
            setattr(whole, name, getattr(oracle, name))
    for name, val in mod.__dict__.items():
        if not name.startswith("__"):
            setattr(whole, name, val)
    return whole


def _failing_checks(mod):
    """The first check that fails on ``mod`` (one catch is enough), as a list."""
    for check in pins.ORACLE_CHECKS:
        try:
            check(mod)
        except CATCHES:
            return [check.__name__]
    return []


@pytest.mark.parametrize("src", [SRC, PROTOCOL_SRC, COMPLEX_SRC], ids=["cs", "protocol", "greedy_complex"])
def test_unmutated_copy_passes_every_check(src):
    """The harness itself: a copy of the oracle with nothing planted passes
    every pin, so a failure under a mutation is the mutation's doing."""
    mod = _mutant(None, None, src)
    for check in pins.ORACLE_CHECKS:
        check(mod)          # any exception fails this test


@pytest.mark.parametrize("mut", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_mutation(mut):
    mid, old, new = mut[:3]
    nth = mut[3] if len(mut) > 3 else 1
    failed = _failing_checks(_mutant(old, new, SRC, nth))
    assert failed, f"no pin catches mutation {mid}"


@pytest.mark.parametrize("mid,old,new", PROTOCOL_MUTATIONS, ids=[m[0] for m in PROTOCOL_MUTATIONS])
def test_pins_catch_protocol_mutation(mid, old, new):
    failed = _failing_checks(_mutant(old, new, PROTOCOL_SRC))
    assert failed, f"no pin catches mutation {mid}"


@pytest.mark.parametrize("mid,old,new", COMPLEX_MUTATIONS, ids=[m[0] for m in COMPLEX_MUTATIONS])
def test_pins_catch_complex_mutation(mid, old, new):
    failed = _failing_checks(_mutant(old, new, COMPLEX_SRC))
    assert failed, f"no pin catches mutation {mid}"
