"""The seeded input generators (CPU): reproducibility, the measurement model
A = Phi Psi with both samplings, and the shapes and scale of the synthetic
stand-ins for the data sets of Section IV."""
import numpy as np
import pytest

from paper_2401_14762_amd import workloads as W


def test_seeded_and_reproducible():
    a = W.plain_cube(64)
    b = W.plain_cube(64)
    assert np.array_equal(a.A, b.A) and np.array_equal(a.Y, b.Y)
    assert not np.array_equal(W.mixing_spectra(8, 50, 40.0, 1), W.mixing_spectra(8, 50, 40.0, 2))


@pytest.mark.parametrize("N", [20, 154, 198, 224])
def test_dictionaries(N):
    M = W.m_for(N)
    assert M == int(round(N / 2.5))
    a64, a32, psi, phi = W.dictionary(N, M, 3)
    assert np.allclose(a64, phi @ psi) and a32.dtype == np.float32
    s64, s32, psi2, sel, rows = W.subsampled_dictionary(N, M, 3)
    # Phi selects M distinct bands; A = Psi[rows, :] has orthonormal rows
    assert len(set(rows.tolist())) == M and np.all(np.diff(rows) > 0)
    assert np.allclose(sel @ psi2, s64) and np.allclose(s64 @ s64.T, np.eye(M), atol=1e-12)
    f = np.random.default_rng(0).standard_normal(N)
    assert np.allclose(s64 @ (psi2.T @ f), f[rows])        # y = f at the kept bands


def test_paper_shape_cubes():
    for name, c in W.PAPER_SHAPES.items():
        cube = W.paper_shape_cube(name, P=500)
        assert cube["F"].shape == (500, c["N"]) and cube["A"].shape == (W.m_for(c["N"]), c["N"])
        assert np.isclose(np.max(np.abs(cube["F"])), W.PAPER_PEAK)
        g = W.paper_shape_cube(name, P=50, sampling="gaussian")
        assert g["A"].shape == cube["A"].shape and not np.allclose(g["A"], cube["A"])
    assert W.PAPER_SHAPES["salinas-like"]["rows"] * W.PAPER_SHAPES["salinas-like"]["cols"] == 111104
    with pytest.raises(ValueError):
        W.paper_shape_cube("jasper-like", P=4, sampling="other")


@pytest.mark.parametrize("N", [17, 64, 101, 224])
def test_dft_basis_inputs(N):
    """The DFT synthesis matrix is unitary; A = Phi Psi with a real Phi has
    conjugate-symmetric columns (column 0, and N/2 for even N, real), so the
    measurements Phi f of a real spectrum are real and equal A x for the
    conjugate-symmetric x = Psi^* f -- the structure the half-spectrum
    solvers rely on."""
    psi = W.dft_synthesis(N)
    assert np.allclose(psi @ np.conj(psi).T, np.eye(N), atol=1e-12)
    M = max(2, W.m_for(N))
    for sampling in ("gaussian", "subsample"):
        c = W.dft_mixing_cube(8, N, M, sampling, config_id=N)
        A = c["A64"]
        k = np.arange(1, N)
        assert np.allclose(A[:, N - k], np.conj(A[:, k]), atol=1e-12)
        assert np.max(np.abs(A[:, 0].imag)) <= 1e-12
        if N % 2 == 0:
            assert np.max(np.abs(A[:, N // 2].imag)) <= 1e-12
        x = c["F"] @ np.conj(psi)                          # x = Psi^* f per pixel
        assert np.allclose(x[:, N - k], np.conj(x[:, k]), atol=1e-10)
        assert c["Y"].dtype == np.float32
        assert np.allclose(x @ A.T, c["F"] @ c["Phi"].T, atol=1e-9)
        assert np.allclose(c["Y"], c["F"] @ c["Phi"].T, rtol=1e-5, atol=1e-6)


def test_complex_cube():
    """K-sparse complex coefficients, y = A x (+ noise at the stated SNR),
    complex64 inputs, reproducible from the seed."""
    c = W.complex_cube(50, snr_db=None)
    assert c["A"].dtype == np.complex64 and c["Y"].dtype == np.complex64
    assert np.all(np.count_nonzero(c["X_true"], axis=1) == W.COMPLEX["K"])
    assert np.allclose(c["Y"], c["X_true"] @ c["A64"].T, atol=1e-5)
    n = W.complex_cube(2000)
    noise = n["Y"].astype(np.complex128) - n["X_true"] @ n["A64"].T
    snr = 10 * np.log10(np.sum(np.abs(n["X_true"] @ n["A64"].T) ** 2) / np.sum(np.abs(noise) ** 2))
    assert abs(snr - W.COMPLEX["snr_db"]) < 0.5
    assert np.array_equal(W.complex_cube(20)["Y"], W.complex_cube(20)["Y"])


def test_paper_shape_dft():
    d = W.paper_shape_dft("china-like", P=100)
    c = W.paper_shape_cube("china-like", P=100)
    assert np.array_equal(d["F"], c["F"]) and np.array_equal(d["Phi"], c["Phi"])
    assert d["A"].shape == (c["M"], c["N"]) and d["A"].dtype == np.complex64
    assert d["Y"].dtype == np.float32 and np.allclose(d["Y"], c["F"] @ c["Phi"].T, rtol=1e-5, atol=1e-2)
