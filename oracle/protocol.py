"""The paper's evaluation protocol (Section II sparsification, Section IV
metrics) in FP64.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline of the benchmark, never by the product path, and sharing no code
with it.

Sparsification (Section II).  HSI spectra are compressible rather than
sparse, so before compression every pixel f is made kappa-sparse in the
transform domain: with x = Psi^{-1} f and mu_x, sigma_x the mean and the
standard deviation of the N magnitudes |x_n|, every x_n with
|x_n| - mu_x < T sigma_x is set to zero, the rest are kept.  T (0.1 in
Section IV) sets the sparsity.  Psi is orthonormal or unitary (the real
DCT-II, or the complex DFT basis of Section II), so Psi^{-1} = Psi^*.

Readings:
* sigma_x is the sample standard deviation (normalised by N - 1, the default
  of the MATLAB std the paper's experiments use); ddof = 0 gives the
  population form.
* A pixel with a non-finite spectrum sparsifies to x = 0 with no kept
  entries.

Metrics (Section IV): PSNR against the sparsified data (oracle.metrics.psnr
on the spectra Psi x), the convergence ratio (share of pixels whose Delta
fell below eps within the iteration cap, the cap replacing t_conv) and the
total number of iterations over the cube.
"""
from __future__ import annotations

import numpy as np


def sparsify(F, Psi, T: float, ddof: int = 1) -> dict:
    """Sparsification of Section II for every pixel (row of F).

    F: P x N spectra, Psi: N x N orthonormal synthesis basis (f = Psi x).
    Returns dict(X = sparsified coefficients (P x N), F = Psi x spectra
    (P x N), kept (P), mu, sigma (P), margin (P)): margin is the smallest
    | |x_n| - mu - T sigma | of the pixel over (mu + sigma), the distance of
    its closest keep/zero decision from the threshold."""
    F = np.asarray(F)
    F = F.astype(np.complex128 if np.iscomplexobj(F) else np.float64)
    Psi = np.asarray(Psi)
    Psi = Psi.astype(np.complex128 if np.iscomplexobj(Psi) else np.float64)
    P, N = F.shape
    fin = np.all(np.isfinite(F), axis=1)
    Fc = np.where(fin[:, None], F, 0.0)
    X = Fc @ np.conj(Psi)                          # x = Psi^* f, one row per pixel
    mag = np.abs(X)
    mu = mag.mean(axis=1)
    sigma = mag.std(axis=1, ddof=ddof) if N - ddof > 0 else np.zeros(P)
    gap = (mag - mu[:, None]) - T * sigma[:, None]
    zero = gap < 0.0                               # |x_n| - mu_x < T sigma_x
    Xs = np.where(zero, 0.0, X)                    # rows of non-finite spectra are 0 already
    kept = np.where(fin, np.count_nonzero(~zero, axis=1), 0)
    scale = np.maximum(mu + sigma, 1e-300)
    margin = np.where(fin, np.min(np.abs(gap), axis=1) / scale, np.inf)
    return dict(X=Xs, F=Xs @ Psi.T, kept=kept, mu=mu, sigma=sigma, margin=margin)


def convergence_ratio(flags, converged_bit: int) -> float:
    """Share of pixels whose stop was Delta < eps (Section IV's convergence
    column), the iteration cap replacing the wall-clock t_conv."""
    flags = np.asarray(flags)
    return float(np.mean((flags & converged_bit) != 0)) if flags.size else 0.0
