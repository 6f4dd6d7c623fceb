"""Mixed precision (BF16 / FP16 operands on MFMA, FP32 accumulation and
state, optional FP32 correction pass): error against the FP64 oracle stated
per pixel, and equal quality against the plain FP32 form.

Bar: with the FP32 correction pass, PSNR of the reconstructed spectra
(F = Psi x) against the FP64 oracle >= 60 dB over the tested pixels, and the
PSNR against the ground-truth spectra within 0.1 dB of the FP32 form's."""
import numpy as np
import pytest

import oracle
from gpu_common import note, np_of, rel_err_rows, require_gpu, to_dev
from paper_2401_14762_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def cube():
    return W.precision_cube(4096)


def _fista(torch, pr, prec, iters, corr=0):
    import paper_2401_14762_amd as cs
    L = oracle.lipschitz(pr.A)
    X, st = cs.fista(to_dev(torch, pr.A), to_dev(torch, pr.Y), lam=1e-2, L=L, max_iter=iters, prec=prec,
                     correction_iters=corr)
    torch.cuda.synchronize()
    return np_of(X), {k: np_of(v) for k, v in st.items()}


@pytest.mark.parametrize("prec", ["bf16", "f16"])
def test_fista_mixed_precision(torch, cube, prec):
    pr = cube
    L = oracle.lipschitz(pr.A)
    idx = W.pixel_subset(pr.P, 512, 21)
    ref = oracle.fista(pr.A, pr.Y[idx], 1e-2, L, 200)
    note(f"fista {prec} 200 it, then +20 FP32 correction")
    Xl, stl = _fista(torch, pr, prec, 200)
    Xc, stc = _fista(torch, pr, prec, 200, corr=20)
    X32, _ = _fista(torch, pr, "f32", 200)
    F = lambda X: X @ pr.Psi.T
    e_low = rel_err_rows(Xl[idx], ref["X"])
    e_cor = rel_err_rows(Xc[idx], ref["X"])
    p_low = oracle.psnr(F(Xl[idx]), F(ref["X"]))
    p_cor = oracle.psnr(F(Xc[idx]), F(ref["X"]))
    note(f"  {prec}: psnr vs oracle {p_low:.1f} dB, corrected {p_cor:.1f} dB; "
         f"per-pixel rel err median {np.median(e_low):.2e} max {e_low.max():.2e}, "
         f"corrected median {np.median(e_cor):.2e} max {e_cor.max():.2e}")
    assert p_cor >= 60.0
    assert np.all(stc["iters"] == 220)
    # equal quality against the ground truth as the FP32 form
    truth = pr.F_true[idx]
    q32 = oracle.psnr(F(X32[idx]), truth)
    qc = oracle.psnr(F(Xc[idx]), truth)
    assert abs(qc - q32) <= 0.1, (qc, q32)
    assert np.all(np.isfinite(Xl))


def test_fista_mixed_ragged_and_shapes(torch):
    for N in (100, 154, 200):
        M = W.m_for(N)
        _, a32, _, phi = W.dictionary(N, M, 3)
        F = W.mixing_spectra(77, N, 40.0, 9)
        Y = (F @ phi.T).astype(np.float32)
        L = oracle.lipschitz(a32)
        import paper_2401_14762_amd as cs
        note(f"fista bf16 shape N={N} M={M} P=77")
        X, _ = cs.fista(to_dev(torch, a32), to_dev(torch, Y), lam=1e-2, L=L, max_iter=50, prec="bf16",
                        correction_iters=10)
        torch.cuda.synchronize()
        # the correction pass restarts the momentum from the 16-bit iterate
        ref0 = oracle.fista(a32, Y, 1e-2, L, 50)
        ref = oracle.fista(a32, Y, 1e-2, L, 10, X0=ref0["X"])
        p = oracle.psnr(np_of(X) @ W.dct_synthesis(N).T, ref["X"] @ W.dct_synthesis(N).T)
        assert p >= 60.0, p
