"""Plant plausible mistakes in a copy of the oracle source (on the CPU) and
check that the pins catch every one of them.  The real oracle is untouched."""
import importlib.util
import os
import sys
import types

import pytest

import oracle_pins as pins

ORACLE_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")
SRC = os.path.join(ORACLE_DIR, "cs.py")
PROTOCOL_SRC = os.path.join(ORACLE_DIR, "protocol.py")

# (id, text to replace (first occurrence), replacement)
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


def _mutant(old, new, src=SRC):
    with open(src) as f:
        text = f.read()
    assert text.count(old) >= 1, old
    text = text.replace(old, new, 1)
    mod = types.ModuleType("oracle_mutant")
    mod.__file__ = src
    exec(compile(text, src + ":mutant", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("mid,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_mutation(mid, old, new):
    mod = _mutant(old, new)
    failed = []
    for check in pins.ORACLE_CHECKS:
        try:
            check(mod)
        except (AssertionError, ValueError, IndexError, FloatingPointError, AttributeError):
            failed.append(check.__name__)
    assert failed, f"no pin catches mutation {mid}"


@pytest.mark.parametrize("mid,old,new", PROTOCOL_MUTATIONS, ids=[m[0] for m in PROTOCOL_MUTATIONS])
def test_pins_catch_protocol_mutation(mid, old, new):
    mod = _mutant(old, new, PROTOCOL_SRC)
    failed = []
    for check in (pins.check_sparsify_worked, pins.check_sparsify_transform, pins.check_sparsify_complex_basis):
        try:
            check(mod)
        except (AssertionError, ValueError, IndexError, FloatingPointError, AttributeError):
            failed.append(check.__name__)
    assert failed, f"no pin catches mutation {mid}"
