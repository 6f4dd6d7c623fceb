"""Shared helpers of the GPU parity tests (GPU side through the C-ABI binding,
reference side through the FP64 oracle, inputs from the workload generators)."""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2401_14762_amd as cs
    cs.library()     # raises if the HIP library is missing: no fallback
    return torch


def note(msg: str) -> None:
    """Print a progress line that names the case before a GPU step."""
    print(msg, file=sys.stderr, flush=True)


def to_dev(torch, a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def np_of(t):
    return t.detach().cpu().numpy()


def rel_err_rows(est, ref):
    est = np.asarray(est, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return np.linalg.norm(est - ref, axis=1) / np.maximum(np.linalg.norm(ref, axis=1), 1e-30)


# Near-tie thresholds for the greedy decisions (relative gaps).  FP32 sums of
# M <= 96 products carry a relative error below ~M * 2^-24 ~ 6e-6 of the
# largest magnitude, and the FP32 normal-equations solve one below
# kappa(B)^2 * 2^-24 ~ 2e-6 for the Gaussian sub-dictionaries met here, so a
# decision whose gap is above 1e-4 of the scale is taken identically in FP32
# and FP64.
GAP = 1e-4
STOP_MARGIN = 1e-3
PIVOT = 1e-6
