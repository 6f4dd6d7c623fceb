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


# The reference of the 16-bit correlation is the oracle's rounding model of
# it (corr_format: A and r rounded to BF16 / FP16, products summed in FP64).
# What still separates the GPU from the model is FP32 arithmetic, plus the
# rare residual entry r_m that FP32 and FP64 round to different 16-bit
# neighbours: that moves p_n by u |A_mn r_m| (u = 2^-8 for BF16, 2^-11 for
# FP16), about 2^-8 * 0.1 * 0.1 ||r|| / (0.3 ||r||) ~ 1.3e-4 of max |p| here.
# Selections with a gap above LOW_GAP (relative to max |p|) cannot flip.
LOW_GAP = {"bf16": 1e-3, "f16": 1.25e-4}


@pytest.mark.parametrize("prec", ["bf16", "f16"])
def test_gomp_mixed_precision(torch, cube, prec):
    """gOMP with the correlation on 16-bit MFMA.  Every pixel: x is the FP32
    least-squares solution on the support it selected (the FP32 correction:
    Alg. 3 steps 2-4 stay FP32), within 1e-5 of the FP64 one.  Against the
    oracle's 16-bit rounding model: the same support away from its near-ties,
    and on at least 95 % of all pixels.  Against the FP64 oracle: PSNR
    reported; against the ground truth: equal quality to the FP32 form."""
    import paper_2401_14762_amd as cs
    from gpu_common import GAP, GAP_ABS, STOP_MARGIN, ls_on_own_support
    pr = cube
    A, Y = to_dev(torch, pr.A), to_dev(torch, pr.Y)
    note(f"gomp {prec} correlation, 4096 pixels N=224 M=90")
    Xl, Sl, stl = cs.gomp(A, Y, K=20, S=2, res_tol=1e-3, prec=prec)
    X32, S32, _ = cs.gomp(A, Y, K=20, S=2, res_tol=1e-3)
    torch.cuda.synchronize()
    Xl, Sl, X32, S32 = np_of(Xl), np_of(Sl), np_of(X32), np_of(S32)
    assert np.all(np.isfinite(Xl)) and np.all((Sl >= 0).sum(axis=1) <= 20)
    # x on the chosen support, every pixel
    ls = ls_on_own_support(pr.A, pr.Y, Sl)
    e_ls = rel_err_rows(Xl, ls)
    assert e_ls.max() <= 1e-5, e_ls.max()
    # supports against the 16-bit rounding model
    idx = W.pixel_subset(pr.P, 512, 23)
    mdl = oracle.gomp(pr.A, pr.Y[idx], K=20, S=2, res_tol=1e-3, diagnostics=True, corr_format=prec)
    ref = oracle.gomp(pr.A, pr.Y[idx], K=20, S=2, res_tol=1e-3)
    clean = (mdl["sel_gap"] >= LOW_GAP[prec]) & (mdl["prune_gap"] >= GAP) & (mdl["stop_margin"] >= STOP_MARGIN)
    clean &= (mdl["sel_gap_abs"] >= GAP_ABS) & (mdl["prune_gap_abs"] >= GAP_ABS)
    same = np.array([np.array_equal(a, b) for a, b in zip(Sl[idx], mdl["support"])])
    same64 = np.array([np.array_equal(a, b) for a, b in zip(Sl[idx], ref["support"])])
    F = lambda X: X @ pr.Psi.T
    note(f"  {prec}: support equal to the 16-bit model's on {same.mean():.2%} of the sample "
         f"({clean.mean():.2%} away from its near-ties), to the FP64 oracle's on {same64.mean():.2%}; "
         f"psnr vs FP64 oracle {oracle.psnr(F(Xl[idx]), F(ref['X'])):.1f} dB")
    assert clean.sum() >= 10
    assert np.all(same[clean])
    assert same.mean() >= 0.95
    # equal quality against the ground truth
    q32 = oracle.psnr(F(X32), pr.F_true)
    ql = oracle.psnr(F(Xl), pr.F_true)
    note(f"  psnr vs truth: fp32 {q32:.2f} dB, {prec} {ql:.2f} dB")
    assert abs(ql - q32) <= 0.1, (ql, q32)


@pytest.mark.parametrize("prec", ["bf16", "f16"])
def test_cosamp_biht_mixed_precision(torch, prec):
    """CoSaMP and BIHT with the 16-bit correlation (their first correlation,
    A^T y, stays FP32) on the K = 15 sparse cube at 30 dB: the same supports
    as the FP32 form on at least 90 % of the pixels (each of CoSaMP's 30
    iterations selects 2K = 30 atoms, each a chance for a 16-bit near-tie;
    and their x is the least squares on the merged support, cut to K, so
    equal supports need not mean equal x), and recovery quality against the
    true coefficients within 0.5 dB of the FP32 form's.  (gOMP's bar is
    0.1 dB.  CoSaMP re-selects 2K atoms in every one of its 30 iterations
    and keeps values from a least squares on the merged 3K atoms, so a 16-bit
    near-tie anywhere can leave a worse support: BF16 costs it about 0.3 dB
    here, and a final FP32 iteration does not win that back.)"""
    import paper_2401_14762_amd as cs
    pr = W.other_solvers_cube(2048)
    A, Y = to_dev(torch, pr.A), to_dev(torch, pr.Y)
    for name, fn in (("cosamp", lambda p: cs.cosamp(A, Y, K=15, max_iter=30, prec=p)),
                     ("biht", lambda p: cs.biht(A, Y, K=15, max_iter=40, mu=0.1, prec=p))):
        note(f"{name} {prec} correlation, 2048 pixels")
        Xl, Sl, _ = fn(prec)
        X32, S32, _ = fn("f32")
        torch.cuda.synchronize()
        Xl, Sl, X32, S32 = np_of(Xl), np_of(Sl), np_of(X32), np_of(S32)
        same = np.array([np.array_equal(a, b) for a, b in zip(Sl, S32)])
        ql, q32 = oracle.psnr(Xl, pr.X_true), oracle.psnr(X32, pr.X_true)
        note(f"  {name} {prec}: same support as FP32 on {same.mean():.2%}; psnr vs truth {ql:.2f} dB "
             f"(fp32 {q32:.2f} dB)")
        assert same.mean() >= 0.90
        assert abs(ql - q32) <= 0.5, (ql, q32)
        assert np.all(np.isfinite(Xl))
