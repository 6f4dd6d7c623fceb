"""GPU parity of csrec_fista_hermitian (Alg. 1 with the complex DFT basis of
Section II, real measurements y = Phi f of real spectra) against the FP64
complex oracle, which iterates on the full complex x with the full A.

The kernel iterates on the half spectrum (x_{N-k} = conj(x_k)), N real
unknowns; the oracle knows nothing of that reduction.  Tolerance
(assert_cfista_parity): per pixel at most max(1e-5, 10x) the error of the
oracle's complex64 rounding model, cube-wide max and median at most twice
the model's.  The returned spectrum is checked to be exactly
conjugate-symmetric."""
import numpy as np
import pytest

import oracle
from gpu_common import assert_cfista_parity, note, np_of, require_gpu, to_dev
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
    X, st = cs.fista_hermitian(to_dev(torch, A), to_dev(torch, Y), lam=lam, L=L, max_iter=iters, **kw)
    torch.cuda.synchronize()
    return np_of(X), {k: np_of(v) for k, v in st.items()}


def _symmetric(X):
    N = X.shape[1]
    assert np.all(X[:, 0].imag == 0.0)
    if N % 2 == 0:
        assert np.all(X[:, N // 2].imag == 0.0)
    k = np.arange(1, N)
    assert np.array_equal(X[:, N - k], np.conj(X[:, k]))


def _hermitian(x):
    x = x.copy()
    N = x.shape[1]
    x[:, 0] = x[:, 0].real
    if N % 2 == 0:
        x[:, N // 2] = x[:, N // 2].real
    k = np.arange(1, (N + 1) // 2)
    x[:, N - k] = np.conj(x[:, k])
    return x


def _parity(X, c, lam, L, iters, **kw):
    _symmetric(X)
    return assert_cfista_parity(X, c["A"], c["Y"].astype(np.complex64), lam, L, iters, **kw)


@pytest.mark.parametrize("N,M,sampling", [(17, 6, "gaussian"), (64, 24, "subsample"), (100, 40, "gaussian"),
                                          (101, 40, "subsample"), (154, 62, "gaussian"), (198, 79, "subsample"),
                                          (224, 90, "gaussian"), (255, 96, "subsample"), (256, 96, "gaussian")])
def test_shapes(torch, N, M, sampling):
    """Every kernel tile (M up to 32, 48, 64, 80, 96; half spectra up to 32,
    64, 80, 112, 128 slots), odd and even N, both samplings."""
    c = W.dft_mixing_cube(130, N, M, sampling, config_id=200 + N)
    L = oracle.lipschitz_complex(c["A"])
    note(f"fista_hermitian N={N} M={M} {sampling} 100 it")
    X, st = _run(torch, c["A"], c["Y"], LAM, L, 100)
    _parity(X, c, LAM, L, 100)
    resid = np.linalg.norm(c["Y"].astype(np.float64) - (X.astype(np.complex128) @ c["A"].astype(np.complex128).T).real,
                           axis=1)
    assert np.all(np.abs(st["resid"] - resid) <= 1e-5 * np.linalg.norm(c["Y"], axis=1) + 1e-7)


@pytest.mark.parametrize("name", sorted(W.PAPER_SHAPES))
def test_paper_cube_full_launch_sampled(torch, name):
    """The data-set-shaped cubes at full size (Section IV's spatial and
    spectral shapes, 40 % of the bands sampled, peak 1e4, lambda 100 as in
    Section IV): the whole cube in one launch, 256 seeded pixels against the
    oracle."""
    c = W.paper_shape_dft(name)
    L = oracle.lipschitz_complex(c["A"])
    note(f"fista_hermitian {name} P={c['P']} N={c['N']} M={c['M']} 150 it (full launch)")
    X, _ = _run(torch, c["A"], c["Y"], 100.0, L, 150)
    idx = W.pixel_subset(c["P"], 256, 300 + c["N"])
    _symmetric(X[idx])
    assert_cfista_parity(X[idx], c["A"], c["Y"][idx].astype(np.complex64), 100.0, L, 150)


@pytest.mark.parametrize("P", [1, 15, 17, 64, 65, 1000])
def test_ragged_pixel_counts(torch, P):
    c = W.dft_mixing_cube(P, 100, 40)
    L = oracle.lipschitz_complex(c["A"])
    note(f"fista_hermitian ragged P={P}")
    X, _ = _run(torch, c["A"], c["Y"], LAM, L, 60)
    _parity(X, c, LAM, L, 60)


def test_eps_stop_and_x0(torch):
    c = W.dft_mixing_cube(257, 200, 80)
    L = oracle.lipschitz_complex(c["A"])
    eps = 1e-4
    note("fista_hermitian eps stop")
    X, st = _run(torch, c["A"], c["Y"], LAM, L, 400, eps=eps)
    Yc = c["Y"].astype(np.complex64)
    ref = oracle.fista_complex(c["A"], Yc, LAM, L, 400, eps=eps)
    same = st["iters"] == ref["iters"]
    assert np.mean(same) > 0.97
    _symmetric(X)
    assert_cfista_parity(X[same], c["A"], Yc[same], LAM, L, 400, eps=eps)
    assert np.all(st["flags"][st["iters"] < 400] & oracle.STOP_CONVERGED)
    # an exactly conjugate-symmetric starting point (the library reads its half)
    x0 = _hermitian(ref["X"].astype(np.complex64))
    note("fista_hermitian warm start X0")
    Xw, stw = _run(torch, c["A"], c["Y"], LAM, L, 20, X0=x0)
    refw, _ = assert_cfista_parity(Xw, c["A"], Yc, LAM, L, 20, X0=x0.astype(np.complex128))
    assert np.allclose(stw["delta"], refw["delta"], rtol=1e-3, atol=1e-6)


def test_nonfinite_pixel_and_zero(torch):
    c = W.dft_mixing_cube(40, 100, 40)
    Y = c["Y"].copy()
    Y[3, 5] = np.nan
    Y[7, 0] = np.inf
    Y[9] = 0.0
    c = dict(c, Y=Y)
    L = oracle.lipschitz_complex(c["A"])
    note("fista_hermitian nonfinite pixels")
    X, st = _run(torch, c["A"], Y, LAM, L, 30)
    assert np.all(X[[3, 7, 9]] == 0.0)
    assert st["flags"][3] == oracle.STOP_NONFINITE and st["flags"][7] == oracle.STOP_NONFINITE
    good = np.setdiff1d(np.arange(40), [3, 7, 9])
    _parity(X[good], dict(c, Y=Y[good]), LAM, L, 30)


def test_device_lipschitz(torch):
    """L = 0: power iteration on C diag(sqrt(w)), whose Gram matrix is A A^*."""
    c = W.dft_mixing_cube(200, 224, 90)
    L = oracle.lipschitz_complex(c["A"])
    note("fista_hermitian device-estimated L")
    X, _ = _run(torch, c["A"], c["Y"], LAM, 0.0, 100)
    _symmetric(X)
    assert_cfista_parity(X, c["A"], c["Y"].astype(np.complex64), LAM, L, 100, floor=1e-4)


def test_agrees_with_complex_entry_point(torch):
    """Where both entry points hold the shape, the half-spectrum iteration and
    the full complex one give the same x to FP32 rounding."""
    import paper_2401_14762_amd as cs
    c = W.dft_mixing_cube(300, 100, 40)
    L = oracle.lipschitz_complex(c["A"])
    note("fista_hermitian vs fista_complex")
    X, _ = _run(torch, c["A"], c["Y"], LAM, L, 100)
    Xc, _ = cs.fista_complex(to_dev(torch, c["A"]), to_dev(torch, c["Y"].astype(np.complex64)), lam=LAM, L=L,
                             max_iter=100)
    Xc = np_of(Xc)
    e = np.linalg.norm(X - Xc, axis=1) / np.maximum(np.linalg.norm(Xc, axis=1), 1e-30)
    assert e.max() <= 1e-4, e.max()


def test_zero_iterations_and_empty(torch):
    import paper_2401_14762_amd as cs
    c = W.dft_mixing_cube(20, 100, 40)
    note("fista_hermitian max_iter=0")
    X, st = _run(torch, c["A"], c["Y"], LAM, 1.0, 0)
    assert np.all(X == 0) and np.all(st["iters"] == 0)
    Y = torch.empty((0, 40), dtype=torch.float32, device="cuda")
    X0, _ = cs.fista_hermitian(to_dev(torch, c["A"]), Y, lam=LAM, L=1.0, max_iter=5)
    assert X0.shape == (0, 100)
