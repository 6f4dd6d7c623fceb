"""GPU parity of csrec_fista_complex (Alg. 1 with the complex DFT basis of
Section II) against the FP64 complex oracle.

The kernel runs the real iteration on the embedding [Re A, -Im A; Im A, Re A]
with the soft threshold applied to each pair (Re x_n, Im x_n) (the pair
kernel of the half-spectrum entry point in its complex-y mode).  Tolerance
(assert_cfista_parity): per-pixel relative error of x^I (complex 2-norm) at
most max(1e-5, 10x) that of the oracle's complex64 rounding model, cube-wide
max and median at most twice the model's.  Stats: the iteration count
exactly, the residual ||y - A x^I|| against the GPU's own x to FP32
resolution of ||y||."""
import numpy as np
import pytest

import oracle
from gpu_common import assert_cfista_parity, note, np_of, rel_err_rows, require_gpu, to_dev
from paper_2401_14762_amd import workloads as W

pytestmark = pytest.mark.gpu

LAM = 1e-2


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _run(torch, A, Y, lam, L, iters, **kw):
    import paper_2401_14762_amd as cs
    X0 = kw.pop("X0", None)
    if X0 is not None:
        kw["X0"] = to_dev(torch, X0.astype(np.complex64))
    X, st = cs.fista_complex(to_dev(torch, A), to_dev(torch, Y), lam=lam, L=L, max_iter=iters, **kw)
    torch.cuda.synchronize()
    return np_of(X), {k: np_of(v) for k, v in st.items()}


def _own_resid(A, Y, X):
    return np.linalg.norm(Y.astype(np.complex128) - X.astype(np.complex128) @ A.astype(np.complex128).T, axis=1)


def test_tiny_all_pixels(torch):
    c = W.complex_cube(256)
    L = oracle.lipschitz_complex(c["A"])
    note("fista_complex 16x16 N=100 M=40 300 it")
    X, st = _run(torch, c["A"], c["Y"], LAM, L, 300)
    assert_cfista_parity(X, c["A"], c["Y"], LAM, L, 300)
    assert np.all(st["iters"] == 300)
    assert np.all(st["flags"] == oracle.STOP_ITER_CAP)
    ynorm = np.linalg.norm(c["Y"].astype(np.complex128), axis=1)
    assert np.all(np.abs(st["resid"] - _own_resid(c["A"], c["Y"], X)) <= 1e-5 * ynorm + 1e-7)


@pytest.mark.parametrize("N,M,sampling", [(17, 5, "gaussian"), (30, 12, "subsample"), (32, 16, "gaussian"),
                                          (60, 24, "gaussian"), (64, 24, "subsample"), (80, 32, "gaussian"),
                                          (100, 40, "subsample"), (112, 40, "gaussian"), (112, 45, "subsample"),
                                          (128, 48, "gaussian")])
def test_shapes(torch, N, M, sampling):
    """Every kernel tile (2M up to 32, 48, 64, 80, 96 rows; N up to 32, 64,
    80, 112, 128) with ragged M and N and both samplings of Section IV."""
    c = W.complex_cube(130, N=N, M=M, K=max(2, M // 5), sampling=sampling, config_id=100 + N)
    L = oracle.lipschitz_complex(c["A"])
    note(f"fista_complex N={N} M={M} {sampling} 80 it")
    X, _ = _run(torch, c["A"], c["Y"], LAM, L, 80)
    assert_cfista_parity(X, c["A"], c["Y"], LAM, L, 80)


@pytest.mark.parametrize("P", [1, 15, 17, 64, 65, 1000])
def test_ragged_pixel_counts(torch, P):
    c = W.complex_cube(P)
    L = oracle.lipschitz_complex(c["A"])
    note(f"fista_complex ragged P={P}")
    X, _ = _run(torch, c["A"], c["Y"], LAM, L, 60)
    assert_cfista_parity(X, c["A"], c["Y"], LAM, L, 60)


def test_full_cube_sampled_and_kkt(torch):
    """256x256 pixels, N=100, M=40: the full launch, a seeded sample of 512
    pixels against the oracle after 200 iterations, and the optimality
    conditions of the complex LASSO on the sample after 1500: with
    g = A^*(y - A x), g_n = lambda x_n / |x_n| where x_n != 0 and
    |g_n| <= lambda where x_n = 0."""
    c = W.complex_cube(65536)
    L = oracle.lipschitz_complex(c["A"])
    note("fista_complex 256x256 N=100 M=40 200 it (full launch)")
    X, _ = _run(torch, c["A"], c["Y"], LAM, L, 200)
    idx = W.pixel_subset(c["P"], 512, 8)
    assert_cfista_parity(X[idx], c["A"], c["Y"][idx], LAM, L, 200)
    note("fista_complex 256x256 1500 it (KKT)")
    X15, _ = _run(torch, c["A"], c["Y"], LAM, L, 1500)
    A = c["A"].astype(np.complex128)
    x = X15[idx].astype(np.complex128)
    g = (c["Y"][idx].astype(np.complex128) - x @ A.T) @ np.conj(A)
    mag = np.abs(x)
    viol = np.where(mag > 0, np.abs(g - LAM * x / np.where(mag > 0, mag, 1.0)), np.maximum(np.abs(g) - LAM, 0.0))
    floor = 64 * 2.0 ** -24 * np.linalg.norm(c["Y"][idx], axis=1).max()
    assert viol.max() <= 2e-3 * LAM + floor, viol.max()


def test_eps_stop_and_x0(torch):
    """Per-pixel Delta < eps stop, and a caller-supplied starting point."""
    c = W.complex_cube(257)
    L = oracle.lipschitz_complex(c["A"])
    eps = 1e-3
    note("fista_complex eps stop")
    X, st = _run(torch, c["A"], c["Y"], LAM, L, 400, eps=eps)
    ref = oracle.fista_complex(c["A"], c["Y"], LAM, L, 400, eps=eps)
    same = st["iters"] == ref["iters"]
    assert np.mean(same) > 0.97
    assert_cfista_parity(X[same], c["A"], c["Y"][same], LAM, L, 400, eps=eps)
    assert np.all(st["flags"][st["iters"] < 400] & oracle.STOP_CONVERGED)
    assert np.all(st["flags"][st["iters"] == 400] & (oracle.STOP_ITER_CAP | oracle.STOP_CONVERGED))
    x0 = ref["X"].astype(np.complex64)
    note("fista_complex warm start X0")
    Xw, stw = _run(torch, c["A"], c["Y"], LAM, L, 20, X0=x0)
    refw, _ = assert_cfista_parity(Xw, c["A"], c["Y"], LAM, L, 20, X0=x0.astype(np.complex128))
    assert np.allclose(stw["delta"], refw["delta"], rtol=1e-3, atol=1e-6)


def test_nonfinite_pixel_and_zero(torch):
    c = W.complex_cube(40)
    Y = c["Y"].copy()
    Y[3, 5] = np.nan
    Y[7, 0] = complex(0.0, np.inf)
    Y[9] = 0.0
    L = oracle.lipschitz_complex(c["A"])
    note("fista_complex nonfinite pixels")
    X, st = _run(torch, c["A"], Y, LAM, L, 30)
    assert np.all(X[[3, 7, 9]] == 0.0)
    assert st["flags"][3] == oracle.STOP_NONFINITE and st["flags"][7] == oracle.STOP_NONFINITE
    assert st["iters"][3] == 0 and st["iters"][7] == 0
    good = np.setdiff1d(np.arange(40), [3, 7, 9])
    assert_cfista_parity(X[good], c["A"], Y[good], LAM, L, 30)


def test_real_dictionary_gives_real_fista(torch):
    """With Im A = 0 and real y the iteration never leaves the reals: the
    imaginary part of x stays exactly 0 and the real part is the real
    FISTA's (oracle.fista)."""
    pr = W.tiny_exact_sparse(100)
    A = pr.A.astype(np.complex64)
    Y = pr.Y.astype(np.complex64)
    L = oracle.lipschitz(pr.A)
    note("fista_complex with a real dictionary")
    X, _ = _run(torch, A, Y, LAM, L, 100)
    assert np.all(X.imag == 0.0)
    ref = oracle.fista(pr.A, pr.Y, LAM, L, 100)
    r32 = oracle.fista(pr.A, pr.Y, LAM, L, 100, dtype=np.float32)
    e = rel_err_rows(X.real, ref["X"])
    e32 = rel_err_rows(r32["X"], ref["X"])
    assert np.all(e <= np.maximum(1e-5, 30 * e32)), e.max()


def test_device_lipschitz(torch):
    """L = 0: the library estimates lambda_max(A^* A) on the device (power
    iteration on the real embedding, whose top eigenvalue is A^* A's)."""
    c = W.complex_cube(200)
    L = oracle.lipschitz_complex(c["A"])
    note("fista_complex device-estimated L")
    X, _ = _run(torch, c["A"], c["Y"], LAM, 0.0, 100)
    assert_cfista_parity(X, c["A"], c["Y"], LAM, L, 100, floor=1e-4)


def test_zero_iterations_and_empty(torch):
    import paper_2401_14762_amd as cs
    c = W.complex_cube(20)
    note("fista_complex max_iter=0")
    X, st = _run(torch, c["A"], c["Y"], LAM, 1.0, 0)
    assert np.all(X == 0) and np.all(st["iters"] == 0)
    A = to_dev(torch, c["A"])
    Y = torch.empty((0, c["M"]), dtype=torch.complex64, device="cuda")
    X0, _ = cs.fista_complex(A, Y, lam=LAM, L=1.0, max_iter=5)
    assert X0.shape == (0, c["N"])
