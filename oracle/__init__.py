"""Plain FP64 CPU oracle for batched per-pixel sparse recovery.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links anything here; only the test-suite, the smoke check and the CPU leg of
the benchmark do.  It shares no code with the HIP path: it is written from
the paper's algorithms (Alg. 1 FISTA, Alg. 2 ADMM, Alg. 3 gOMP, Alg. 4
BIHT, Alg. 5 CoSaMP, Eq. 2 LASSO, the Section II sparsification and the
Section IV metrics; the greedy solvers also for the complex DFT basis) with NumPy/SciPy primitives only.
"""
from .cs import (round_to_format, fista, fista_complex, soft_threshold_complex, lipschitz_complex, admm, admm_complex, admm_threshold, gomp, cosamp, biht, biht_one_bit, lstsq_on_support, top_indices,
                 soft_threshold, lipschitz, STOP_CONVERGED, STOP_ITER_CAP, STOP_FALLBACK,
                 STOP_NONFINITE)
from .metrics import psnr, rel_err, lasso_objective, lasso_kkt_residual
from .protocol import sparsify, convergence_ratio
from .greedy_complex import (conj_pair_groups, gomp_complex, cosamp_complex, biht_complex, group_scores,
                             lstsq_complex)

__all__ = [
    "round_to_format", "conj_pair_groups", "gomp_complex", "cosamp_complex", "biht_complex", "group_scores",
    "lstsq_complex",
    "fista", "fista_complex", "soft_threshold_complex", "lipschitz_complex", "admm", "admm_complex", "admm_threshold", "gomp", "cosamp", "biht", "biht_one_bit", "lstsq_on_support", "top_indices",
    "soft_threshold", "lipschitz", "psnr", "rel_err", "lasso_objective",
    "lasso_kkt_residual", "sparsify", "convergence_ratio", "STOP_CONVERGED", "STOP_ITER_CAP", "STOP_FALLBACK", "STOP_NONFINITE",
]
