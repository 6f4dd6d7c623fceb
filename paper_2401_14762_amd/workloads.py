"""Seeded synthetic inputs for batched per-pixel sparse recovery.

This module builds problems, it solves nothing: the dictionary A = Phi Psi of
the measurement model (Section II, Eq. 1), synthetic hyperspectral spectra and
the measurements Y taken from them.  It holds none of the recovery arithmetic,
so the FP64 oracle and the HIP path can both be fed from it without sharing
any solver code.  Everything is NumPy only and importing it loads no GPU code.

Conventions (shared by every consumer):

* ``Psi`` is the N x N orthonormal DCT-II synthesis matrix, f = Psi x, so
  ``Psi.T @ f`` is the orthonormal DCT-II of f.  The paper uses a DFT basis;
  a real orthonormal basis keeps A real (A^* = A^T).
* ``Phi`` is M x N with i.i.d. N(0, 1/M) entries (the paper's randomised
  measurement matrix, Section II), M = round(N / 2.5) for the 2.5x
  compression of Section IV -- or, with ``subsampled_dictionary``, the
  random selection of M of the N spectral samples that Section IV applies
  to its data sets (A = the selected rows of Psi).
* Pixel-major layouts: Y is P x M, X is P x N, both row-major.
* Every random draw comes from ``numpy.random.default_rng`` seeded with a
  ``SeedSequence([config_id, stream_id])`` so a config is reproducible
  anywhere.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

# stream ids inside one config's SeedSequence
_S_PHI, _S_SUPPORT, _S_VALUES, _S_ENDMEMBERS, _S_ABUND, _S_NOISE, _S_PIXSEL = range(7)


def rng_for(config_id: int, stream_id: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(config_id), int(stream_id)]))


def dct_synthesis(N: int) -> np.ndarray:
    """Orthonormal DCT-II synthesis matrix Psi (N x N, FP64): f = Psi @ x.

    Psi[n, k] = a_k cos(pi (2n + 1) k / (2N)), a_0 = sqrt(1/N), a_k = sqrt(2/N).
    """
    n = np.arange(N, dtype=np.float64)[:, None]
    k = np.arange(N, dtype=np.float64)[None, :]
    psi = np.cos(np.pi * (2.0 * n + 1.0) * k / (2.0 * N))
    psi[:, 0] *= math.sqrt(1.0 / N)
    psi[:, 1:] *= math.sqrt(2.0 / N)
    return psi


def dft_synthesis(N: int) -> np.ndarray:
    """N x N unitary DFT synthesis matrix of Section II's complex basis:
    Psi[n, k] = exp(2 pi i n k / N) / sqrt(N), f = Psi x, x = Psi^* f."""
    n = np.arange(N)
    return np.exp(2j * np.pi * np.outer(n, n) / N) / math.sqrt(N)


def complex_dictionary(N: int, M: int, seed, sampling: str = "subsample") -> tuple:
    """A = Phi Psi with the complex DFT basis (complex128, complex64), the
    basis and Phi: "subsample" picks M of the N bands (Section IV),
    "gaussian" draws N(0, 1/M) entries."""
    psi = dft_synthesis(N)
    if sampling == "subsample":
        rows = np.sort(np.random.default_rng(seed).choice(N, M, replace=False))
        phi = np.zeros((M, N))
        phi[np.arange(M), rows] = 1.0
    elif sampling == "gaussian":
        phi = gaussian_phi(M, N, seed)
    else:
        raise ValueError(sampling)
    a = phi @ psi
    return a, a.astype(np.complex64), psi, phi


def gaussian_phi(M: int, N: int, seed) -> np.ndarray:
    """Phi with i.i.d. N(0, 1/M) entries (FP64)."""
    rng = seed if isinstance(seed, np.random.Generator) else np.random.default_rng(seed)
    return rng.standard_normal((M, N)) / math.sqrt(M)


def m_for(N: int, ratio: float = 2.5) -> int:
    """Measurements per pixel for a given compression ratio (2.5x in Section IV)."""
    return int(round(N / ratio))


@dataclasses.dataclass
class Problem:
    """One synthetic cube: A and Y exactly as the GPU receives them (FP32)
    plus FP64 ground truth kept for reporting."""
    name: str
    A: np.ndarray            # M x N float32
    Y: np.ndarray            # P x M float32
    A64: np.ndarray          # M x N float64 (before rounding)
    Psi: np.ndarray          # N x N float64
    X_true: Optional[np.ndarray] = None   # P x N float64 coefficients, if exactly sparse
    F_true: Optional[np.ndarray] = None   # P x N float64 spectra, if mixing model
    Ysign: Optional[np.ndarray] = None    # P x M int8, sign measurements
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def M(self) -> int:
        return self.A.shape[0]

    @property
    def N(self) -> int:
        return self.A.shape[1]

    @property
    def P(self) -> int:
        return self.Y.shape[0]


def dictionary(N: int, M: int, phi_seed) -> tuple:
    """A = Phi Psi in FP64 and its FP32 rounding."""
    psi = dct_synthesis(N)
    phi = gaussian_phi(M, N, phi_seed)
    a64 = phi @ psi
    return a64, a64.astype(np.float32), psi, phi


def subsampled_dictionary(N: int, M: int, seed) -> tuple:
    """A = Phi Psi with Phi the random selection of M of the N bands (sorted):
    y = f[rows], A = Psi[rows, :].  Returns (A64, A32, Psi, Phi, rows)."""
    psi = dct_synthesis(N)
    rows = np.sort(np.random.default_rng(seed).choice(N, M, replace=False))
    phi = np.zeros((M, N))
    phi[np.arange(M), rows] = 1.0
    a64 = psi[rows, :].copy()
    return a64, a64.astype(np.float32), psi, phi, rows


def sparse_coefficients(P: int, N: int, K: int, rng_support, rng_values) -> np.ndarray:
    """P x N coefficients, each row exactly K-sparse: uniform random support,
    N(0, 1) values."""
    X = np.zeros((P, N))
    # the K smallest of N i.i.d. uniform keys index a uniform random K-subset
    idx = np.argsort(rng_support.random((P, N)), axis=1, kind="stable")[:, :K]
    X[np.arange(P)[:, None], idx] = rng_values.standard_normal((P, K))
    return X


def endmembers(N: int, rng, n_end: int = 5, n_bumps: int = 3,
               width=(5.0, 30.0), amp=(0.2, 1.0)) -> np.ndarray:
    """n_end smooth spectra of N bands: each a sum of n_bumps Gaussians in band
    index, centre U[0, N), std-dev U[width], amplitude U[amp]."""
    n = np.arange(N, dtype=np.float64)
    E = np.zeros((n_end, N))
    for e in range(n_end):
        for _ in range(n_bumps):
            c = rng.uniform(0.0, N)
            w = rng.uniform(*width)
            a = rng.uniform(*amp)
            E[e] += a * np.exp(-((n - c) ** 2) / (2.0 * w * w))
    return E


def mixing_spectra(P: int, N: int, snr_db: float, config_id: int, n_end: int = 5) -> np.ndarray:
    """P x N spectra: Dirichlet(1,...,1) abundances over n_end endmembers plus
    white Gaussian noise whose power is the cube-mean signal power / 10^(snr/10)."""
    E = endmembers(N, rng_for(config_id, _S_ENDMEMBERS), n_end=n_end)
    ab = rng_for(config_id, _S_ABUND).dirichlet(np.ones(n_end), size=P)
    F = ab @ E
    sigma = math.sqrt(float(np.mean(F * F)) * 10.0 ** (-snr_db / 10.0))
    F = F + sigma * rng_for(config_id, _S_NOISE).standard_normal(F.shape)
    return F


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

TINY = dict(config_id=0, side=16, N=100, M=40, K=8, phi_seed=0)
PLAIN = dict(config_id=1, side=256, N=200, M=80, snr_db=40.0)
PRECISION = dict(config_id=2, side=1024, N=224, M=90, snr_db=40.0)
OTHER = dict(config_id=3, side=512, N=200, M=80, K=15, snr_db=30.0)
SERVING = dict(config_id=4, rate=200.0, side_min=64, side_max=512, bands=(100, 200, 224),
               snr_db=40.0)


def tiny_exact_sparse(P: Optional[int] = None) -> Problem:
    """16x16 pixels, N=100, M=40, Phi ~ N(0,1/M) from seed 0, every pixel
    exactly 8-sparse in the DCT, noiseless."""
    c = TINY
    P = c["side"] ** 2 if P is None else P
    a64, a32, psi, _ = dictionary(c["N"], c["M"], c["phi_seed"])
    X = sparse_coefficients(P, c["N"], c["K"], rng_for(c["config_id"], _S_SUPPORT),
                            rng_for(c["config_id"], _S_VALUES))
    Y = (X @ a64.T).astype(np.float32)
    return Problem("tiny-16x16-N100-M40-K8", a32, Y, a64, psi, X_true=X,
                   meta=dict(c, P=P))


def mixing_cube(cfg: dict, P: Optional[int] = None, name: str = "") -> Problem:
    N, M = cfg["N"], cfg["M"]
    P = cfg["side"] ** 2 if P is None else P
    a64, a32, psi, phi = dictionary(N, M, rng_for(cfg["config_id"], _S_PHI))
    F = mixing_spectra(P, N, cfg["snr_db"], cfg["config_id"])
    Y = (F @ phi.T).astype(np.float32)
    return Problem(name or f"mixing-{cfg['side']}x{cfg['side']}-N{N}-M{M}", a32, Y, a64, psi,
                   F_true=F, meta=dict(cfg, P=P))


def plain_cube(P: Optional[int] = None) -> Problem:
    """256x256 pixels, N=200, M=80, 5 endmembers, Dirichlet(1), 40 dB."""
    return mixing_cube(PLAIN, P, "plain-256x256-N200-M80")


def precision_cube(P: Optional[int] = None) -> Problem:
    """1024x1024 pixels, N=224, M=90, same generator as plain_cube."""
    return mixing_cube(PRECISION, P, "precision-1024x1024-N224-M90")


def other_solvers_cube(P: Optional[int] = None) -> Problem:
    """512x512 pixels, N=200, M=80, K=15-sparse DCT coefficients, 30 dB noise
    on y (per-pixel power), plus int8 signs of the noiseless A s."""
    c = OTHER
    N, M, K = c["N"], c["M"], c["K"]
    P = c["side"] ** 2 if P is None else P
    a64, a32, psi, _ = dictionary(N, M, rng_for(c["config_id"], _S_PHI))
    X = sparse_coefficients(P, N, K, rng_for(c["config_id"], _S_SUPPORT),
                            rng_for(c["config_id"], _S_VALUES))
    Y0 = X @ a64.T
    pw = np.sum(Y0 * Y0, axis=1, keepdims=True) / (M * 10.0 ** (c["snr_db"] / 10.0))
    Yn = Y0 + np.sqrt(pw) * rng_for(c["config_id"], _S_NOISE).standard_normal(Y0.shape)
    sign = np.where(Y0 >= 0.0, 1, -1).astype(np.int8)
    return Problem("other-512x512-N200-M80-K15", a32, Yn.astype(np.float32), a64, psi,
                   X_true=X, Ysign=sign, meta=dict(c, P=P))


# Synthetic stand-ins for the three data sets of Section IV (same spatial
# and spectral shapes; the mixing model of mixing_spectra, 40 dB), scaled to
# a peak of 1e4, the range of the 16-bit sensor counts of those data sets, so
# that the lambda values of Section IV (0.1 and 100) keep their weight, and
# the kappa pairs of Section IV for each.
PAPER_SHAPES = {
    "salinas-like": dict(config_id=5, rows=512, cols=217, N=224, kappas=(27, 33)),
    "jasper-like": dict(config_id=6, rows=100, cols=100, N=198, kappas=(18, 24)),
    "china-like": dict(config_id=7, rows=420, cols=140, N=154, kappas=(16, 22)),
}
PAPER_PEAK = 1.0e4


def paper_shape_cube(name: str, P: Optional[int] = None, sampling: str = "subsample") -> dict:
    """Spectra F (P x N, FP64) of a PAPER_SHAPES cube, the basis Psi and the
    dictionary A = Phi Psi (FP32) at M = round(N / 2.5); sampling
    "subsample" (Section IV: a random 40 % of the bands) or "gaussian"."""
    c = PAPER_SHAPES[name]
    N = c["N"]
    M = m_for(N)
    P = c["rows"] * c["cols"] if P is None else P
    if sampling == "subsample":
        _, a32, psi, phi, _ = subsampled_dictionary(N, M, rng_for(c["config_id"], _S_PHI))
    elif sampling == "gaussian":
        _, a32, psi, phi = dictionary(N, M, rng_for(c["config_id"], _S_PHI))
    else:
        raise ValueError(sampling)
    F = mixing_spectra(P, N, 40.0, c["config_id"])
    F *= PAPER_PEAK / float(np.max(np.abs(F)))
    return dict(name=name, F=F, A=a32, Psi=psi, Phi=phi, M=M, N=N, P=P, kappas=c["kappas"], sampling=sampling)


# Complex measurements with the DFT basis of Section II: K-sparse complex
# coefficients (circular complex Gaussian values), y = A x (+ circular
# complex white noise at snr_db).  Shapes within the complex-y kernels'
# limits (N <= 128, M <= 48).
COMPLEX = dict(config_id=8, side=64, N=100, M=40, K=8, snr_db=40.0)


def complex_cube(P: Optional[int] = None, N: int = COMPLEX["N"], M: int = COMPLEX["M"], K: int = COMPLEX["K"],
                 sampling: str = "gaussian", snr_db: Optional[float] = COMPLEX["snr_db"],
                 config_id: int = COMPLEX["config_id"]) -> dict:
    """A = Phi Psi with the unitary DFT synthesis Psi (complex64 A32 and
    complex128 A64), X_true (P x N complex128, K-sparse) and Y (P x M
    complex64).  sampling as complex_dictionary; snr_db None = noiseless."""
    P = COMPLEX["side"] ** 2 if P is None else P
    a64, a32, psi, phi = complex_dictionary(N, M, rng_for(config_id, _S_PHI), sampling)
    supp = sparse_coefficients(P, N, K, rng_for(config_id, _S_SUPPORT), rng_for(config_id, _S_VALUES)) != 0.0
    vals = rng_for(config_id, _S_ABUND).standard_normal((P, N, 2)) / math.sqrt(2.0)
    X = np.where(supp, vals[..., 0] + 1j * vals[..., 1], 0.0)
    Y0 = X @ a64.T
    if snr_db is not None:
        pw = np.sum(np.abs(Y0) ** 2, axis=1, keepdims=True) / (M * 10.0 ** (snr_db / 10.0))
        w = rng_for(config_id, _S_NOISE).standard_normal((P, M, 2))
        Y0 = Y0 + np.sqrt(pw / 2.0) * (w[..., 0] + 1j * w[..., 1])
    return dict(A=a32, A64=a64, Psi=psi, Phi=phi, X_true=X, Y=Y0.astype(np.complex64), M=M, N=N, P=P,
                sampling=sampling)


def paper_shape_dft(name: str, P: Optional[int] = None, sampling: str = "subsample") -> dict:
    """A PAPER_SHAPES cube measured for the complex DFT basis: the real
    spectra F and the real Phi of paper_shape_cube, Y = F Phi^T (real, FP32:
    y = Phi f), and A = Phi Psi with the unitary DFT synthesis Psi (complex64
    A, complex128 A64; its columns are conjugate-symmetric)."""
    c = paper_shape_cube(name, P, sampling)
    psi = dft_synthesis(c["N"])
    a64 = c["Phi"] @ psi
    Y = (c["F"] @ c["Phi"].T).astype(np.float32)
    return dict(c, A=a64.astype(np.complex64), A64=a64, Psi=psi, Y=Y)


def dft_mixing_cube(P: int, N: int, M: int, sampling: str = "gaussian", config_id: int = 9) -> dict:
    """Mixing-model spectra (40 dB) of N bands measured by a real Phi, with
    A = Phi Psi for the unitary DFT basis: Y (P x M float32) real,
    A (M x N complex64) conjugate-symmetric."""
    a64, a32, psi, phi = complex_dictionary(N, M, rng_for(config_id, _S_PHI), sampling)
    F = mixing_spectra(P, N, 40.0, config_id)
    return dict(A=a32, A64=a64, Psi=psi, Phi=phi, F=F, Y=(F @ phi.T).astype(np.float32), M=M, N=N, P=P,
                sampling=sampling)


def pixel_subset(P: int, n: int, config_id: int) -> np.ndarray:
    """Seeded sorted subset of n pixel indices out of P."""
    n = min(n, P)
    return np.sort(rng_for(config_id, _S_PIXSEL).choice(P, n, replace=False))


@dataclasses.dataclass
class Tile:
    tag: int
    t_arrival: float     # seconds from stream start
    side: int
    N: int
    M: int
    seed: int


def serving_stream(n_tiles: int, rate: float = SERVING["rate"], seed: int = 0) -> list:
    """Poisson arrivals (exponential gaps, mean 1/rate s) of square tiles whose
    side is log-uniform in [64, 512]; band count uniform over {100, 200, 224},
    M = round(N / 2.5)."""
    rng = rng_for(SERVING["config_id"], 100 + seed)
    t = 0.0
    out = []
    lo, hi = math.log(SERVING["side_min"]), math.log(SERVING["side_max"])
    for i in range(n_tiles):
        t += rng.exponential(1.0 / rate)
        side = int(round(math.exp(rng.uniform(lo, hi))))
        N = int(rng.choice(SERVING["bands"]))
        out.append(Tile(i, t, side, N, m_for(N), int(rng.integers(0, 2**31 - 1))))
    return out


def serving_dictionary(N: int) -> tuple:
    """One seeded Gaussian Phi per band count (seed = N)."""
    return dictionary(N, m_for(N), N)


def serving_tile_measurements(tile: Tile, phi_seed_N: Optional[int] = None) -> np.ndarray:
    """Y (P x M float32) for one serving tile: mixing-model spectra at 40 dB
    measured by the band count's shared Phi."""
    _, _, _, phi = serving_dictionary(tile.N)
    F = mixing_spectra(tile.side * tile.side, tile.N, SERVING["snr_db"], 1000 + tile.seed % 100000)
    return (F @ phi.T).astype(np.float32)
