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
