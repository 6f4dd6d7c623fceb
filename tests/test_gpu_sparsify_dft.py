"""GPU parity of csrec_sparsify_dft (Section II sparsification with the
complex DFT basis, fused with the compression y = A x_s) against the FP64
oracle (oracle.sparsify on complex Psi: x = Psi^* f over the full spectrum).

The kernel works on the half spectrum of the conjugate-symmetric x and
counts each pair (k, N-k) twice in mu and sigma; the oracle knows nothing of
that.  Decisions are FP comparisons (FP32 on the GPU, FP64 in the oracle): a
pixel is compared exactly (same kept set, same count) when the oracle's
margin exceeds NEAR; elsewhere every kept value must be the pixel's own
coefficient.  Values within 1e-5 relative; y against A x_s of the GPU's own
x_s to FP32 rounding of the sum; the returned spectrum exactly
conjugate-symmetric."""
import numpy as np
import pytest

import oracle
from gpu_common import note, np_of, rel_err_rows, require_gpu, to_dev
from paper_2401_14762_amd import workloads as W

pytestmark = pytest.mark.gpu

NEAR = 1e-5


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _run(torch, psi, A, F, T=0.1, ddof=1):
    import paper_2401_14762_amd as cs
    Xs, Y, kept = cs.sparsify_dft(to_dev(torch, psi.astype(np.complex64)), to_dev(torch, A.astype(np.complex64)),
                                  to_dev(torch, F.astype(np.float32)), T=T, ddof=ddof)
    torch.cuda.synchronize()
    return np_of(Xs), np_of(Y), np_of(kept)


def _check(psi, A, F, Xs, Y, kept, T=0.1, ddof=1, min_clean=0.9):
    N = Xs.shape[1]
    k = np.arange(1, N)
    assert np.array_equal(Xs[:, N - k], np.conj(Xs[:, k]))
    assert np.all(Xs[:, 0].imag == 0.0)
    F32 = F.astype(np.float32).astype(np.float64)
    psi32 = psi.astype(np.complex64).astype(np.complex128)
    A32 = A.astype(np.complex64).astype(np.complex128)
    ref = oracle.sparsify(F32, psi32, T, ddof=ddof)
    clean = ref["margin"] > NEAR
    assert clean.mean() >= min_clean, clean.mean()
    same = (Xs != 0) == (ref["X"] != 0)
    assert np.all(same[clean]), np.nonzero(~same.all(axis=1) & clean)[0][:8]
    assert np.array_equal(kept[clean], ref["kept"][clean])
    assert rel_err_rows(Xs[clean], ref["X"][clean]).max() <= 1e-5
    # near-tie pixels: every kept value is the pixel's own coefficient
    full = F32 @ np.conj(psi32)
    on = Xs != 0
    tol = 1e-5 * (np.abs(full).max(axis=1, keepdims=True) + 1e-30)
    assert np.all((np.abs(Xs - full) <= tol)[on])
    assert np.array_equal(kept, on.sum(axis=1))
    # y = A x_s of the GPU's own x_s (real up to rounding)
    yc = Xs.astype(np.complex128) @ A32.T
    scale = np.abs(Xs.astype(np.complex128)) @ np.abs(A32).T
    assert np.all(np.abs(Y - yc.real) <= 16 * N * 2.0 ** -24 * scale + 1e-30)
    assert np.all(np.abs(yc.imag) <= 16 * N * 2.0 ** -24 * scale + 1e-30)
    return ref


@pytest.mark.parametrize("N", [20, 60, 100, 101, 154, 198, 224, 240, 255, 256])
def test_band_counts(torch, N):
    M = min(W.m_for(N), 96)
    c = W.dft_mixing_cube(300, N, M, "gaussian", config_id=700 + N)
    note(f"sparsify_dft band count N={N} M={M}")
    Xs, Y, kept = _run(torch, c["Psi"], c["A"], c["F"])
    _check(c["Psi"], c["A"], c["F"], Xs, Y, kept, min_clean=0.8)


@pytest.mark.parametrize("name", sorted(W.PAPER_SHAPES))
def test_paper_cube_full_launch_sampled(torch, name):
    """The data-set-shaped cubes at full size (40 % of the bands sampled,
    peak 1e4); 2048 seeded pixels checked."""
    c = W.paper_shape_dft(name)
    note(f"sparsify_dft {name} P={c['P']} N={c['N']} M={c['M']} (full launch)")
    Xs, Y, kept = _run(torch, c["Psi"], c["A"], c["F"])
    idx = W.pixel_subset(c["P"], 2048, 800 + c["N"])
    _check(c["Psi"], c["A"], c["F"][idx], Xs[idx], Y[idx], kept[idx])
    # T = 0.1 zeroes most coefficients, as in Section IV
    assert 0.8 <= 1.0 - kept.mean() / c["N"] <= 0.99


@pytest.mark.parametrize("P", [1, 15, 17, 65, 1000])
def test_ragged_pixel_counts(torch, P):
    c = W.dft_mixing_cube(P, 200, 80)
    note(f"sparsify_dft ragged P={P}")
    Xs, Y, kept = _run(torch, c["Psi"], c["A"], c["F"])
    _check(c["Psi"], c["A"], c["F"], Xs, Y, kept, min_clean=0.0)


def test_thresholds_and_ddof(torch):
    c = W.dft_mixing_cube(500, 200, 80)
    for T, ddof in ((0.0, 1), (0.5, 1), (1.5, 0), (-1e6, 1)):
        note(f"sparsify_dft T={T} ddof={ddof}")
        Xs, Y, kept = _run(torch, c["Psi"], c["A"], c["F"], T=T, ddof=ddof)
        _check(c["Psi"], c["A"], c["F"], Xs, Y, kept, T=T, ddof=ddof, min_clean=0.8)
    # keep-all: y is the compression of the whole pixel, A x = Phi f
    assert np.all(kept == 200)
    assert np.allclose(Y, c["F"] @ c["Phi"].T, rtol=1e-4, atol=1e-5 * np.abs(c["F"]).max())


def test_nonfinite_zero_and_empty(torch):
    import paper_2401_14762_amd as cs
    c = W.dft_mixing_cube(40, 100, 40)
    F = c["F"].copy()
    F[3, 7] = np.nan
    F[5, 0] = -np.inf
    F[9] = 0.0
    note("sparsify_dft nonfinite and zero spectra")
    Xs, Y, kept = _run(torch, c["Psi"], c["A"], F)
    assert np.all(Xs[[3, 5, 9]] == 0.0) and np.all(Y[[3, 5, 9]] == 0.0)
    assert kept[3] == 0 and kept[5] == 0
    # an all-zero spectrum: mu = sigma = 0, no entry is below the threshold
    assert kept[9] == 100 and oracle.sparsify(F[9:10], c["Psi"], 0.1)["kept"][0] == 100
    good = np.setdiff1d(np.arange(40), [3, 5, 9])
    _check(c["Psi"], c["A"], F[good], Xs[good], Y[good], kept[good], min_clean=0.8)
    Fe = torch.empty((0, 100), dtype=torch.float32, device="cuda")
    Xe, Ye, ke = cs.sparsify_dft(to_dev(torch, c["Psi"].astype(np.complex64)), to_dev(torch, c["A"]), Fe)
    assert Xe.shape == (0, 100) and Ye.shape == (0, 40) and ke.shape == (0,)
