"""csrec -- batched per-pixel sparse recovery of compressed hyperspectral cubes
on AMD Instinct MI355X (gfx950).

Python binding of ``libcsrec.so`` (C ABI in ``include/csrec.h``).  The
functions take and return torch tensors that live on the GPU; torch provides
device memory and the stream, the library's HIP kernels do all the work.

    X, st = fista(A, Y, lam=1e-2, L=L, max_iter=200)           # Alg. 1
    X, S, st = gomp(A, Y, K=20, S=2, res_tol=1e-3)              # Alg. 3
    X, S, st = biht(A, Y, K=15, max_iter=100, mu=0.1)           # Alg. 4
    X, S, st = biht(A, None, K=15, max_iter=100, Ysign=Ys, mode="one_bit")
    X, S, st = cosamp(A, Y, K=15, max_iter=30)                  # Alg. 5
    X, st = fista_complex(Ac, Yc, lam=1e-2, max_iter=200)       # Alg. 1, complex A
    X, st = fista_hermitian(Ac, Y, lam=1e-2, max_iter=200)      # Alg. 1, DFT basis, real y
    X, Z, st = admm_hermitian(Ac, Y, lam=1e-2, alpha=1.8)       # Alg. 2, DFT basis, real y
    X, Z, st = admm_complex(Ac, Yc, lam=1e-2, alpha=1.8)        # Alg. 2, complex A and y

A: M x N float32, Y: P x M float32, both CUDA (HIP) tensors, contiguous.
``st`` is a dict of per-pixel tensors: iters, flags, resid, delta.
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import (CsrecError, FLAG_CONVERGED, FLAG_FP32_LIMIT, FLAG_FP64_FALLBACK, FLAG_ITER_CAP,
                   FLAG_NONFINITE, MAX_N)

__all__ = ["sparsify", "sparsify_dft", "fista", "fista_complex", "fista_hermitian", "admm", "admm_hermitian", "admm_complex", "gomp", "cosamp", "biht", "lipschitz", "Server", "CsrecError", "FLAG_CONVERGED",
           "FLAG_ITER_CAP", "FLAG_FP64_FALLBACK", "FLAG_NONFINITE", "FLAG_FP32_LIMIT", "MAX_N", "workspace_bytes",
           "library"]


def library():
    """The loaded ctypes library (raises if libcsrec.so is not built)."""
    return _lib.load()


def _torch():
    import torch
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _check_dev(name, t, dtype, shape=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _problem(A, Y, P, stream):
    torch = _torch()
    M, N = A.shape
    pb = _lib.Problem()
    pb.struct_size = ctypes.sizeof(_lib.Problem)
    pb.M, pb.N, pb.P = M, N, P
    pb.A = A.data_ptr()
    pb.Y = Y.data_ptr() if Y is not None else 0
    if stream is None:
        stream = torch.cuda.current_stream(A.device)
    pb.stream = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    return pb


def _stats_view(st):
    torch = _torch()
    return dict(iters=st[:, 0].clone(), flags=st[:, 1].clone(),
                resid=st[:, 2].view(torch.float32).clone(), delta=st[:, 3].view(torch.float32).clone())


def _workspace(lib, solver, pb, params, device):
    torch = _torch()
    nbytes = ctypes.c_size_t(0)
    _lib.check(lib.csrec_workspace_bytes(solver, ctypes.byref(pb), ctypes.byref(params),
                                         ctypes.byref(nbytes)), "csrec_workspace_bytes")
    ws = None
    if nbytes.value > 0:
        ws = torch.empty(nbytes.value, dtype=torch.uint8, device=device)
        pb.workspace = ws.data_ptr()
        pb.workspace_bytes = nbytes.value
    return ws


def workspace_bytes(solver: str, A, Y, **params) -> int:
    """Device scratch bytes a call of ``solver`` would allocate."""
    lib = library()
    P = Y.shape[0] if Y is not None else params.pop("P")
    pb = _problem(A, Y, P, None)
    prm, sid = _params(solver, A, P, params)
    nbytes = ctypes.c_size_t(0)
    _lib.check(lib.csrec_workspace_bytes(sid, ctypes.byref(pb), ctypes.byref(prm), ctypes.byref(nbytes)),
               "csrec_workspace_bytes")
    return nbytes.value


def _params(solver, A, P, kw):
    if solver in ("fista", "fista_complex", "fista_hermitian"):
        p = _lib.FistaParams()
        p.struct_size = ctypes.sizeof(p)
        p.max_iter = int(kw.get("max_iter", 100))
        p.lambda_ = float(kw.get("lam", 0.0))
        p.L = float(kw.get("L", 0.0))
        p.eps = float(kw.get("eps", 0.0))
        x0 = kw.get("X0")
        p.X0 = x0.data_ptr() if x0 is not None else 0
        p.prec = _lib.PREC[kw.get("prec", "f32")]
        p.correction_iters = int(kw.get("correction_iters", 0))
        return p, {"fista": _lib.SOLVER_FISTA, "fista_complex": _lib.SOLVER_FISTA_COMPLEX,
                   "fista_hermitian": _lib.SOLVER_FISTA_HERMITIAN}[solver]
    if solver in ("admm", "admm_hermitian", "admm_complex"):
        p = _lib.AdmmParams()
        p.struct_size = ctypes.sizeof(p)
        p.max_iter = int(kw.get("max_iter", 100))
        p.lambda_ = float(kw.get("lam", 0.0))
        p.alpha = float(kw.get("alpha", 1.8))
        p.eps = float(kw.get("eps", 0.0))
        x0 = kw.get("X0")
        p.X0 = x0.data_ptr() if x0 is not None else 0
        if kw.get("threshold", "paper") not in _lib.ADMM_THR:
            raise ValueError(f"threshold must be one of {sorted(_lib.ADMM_THR)}")
        p.threshold = _lib.ADMM_THR[kw.get("threshold", "paper")]
        return p, {"admm": _lib.SOLVER_ADMM, "admm_hermitian": _lib.SOLVER_ADMM_HERMITIAN,
                   "admm_complex": _lib.SOLVER_ADMM_COMPLEX}[solver]
    if solver == "gomp":
        p = _lib.GompParams()
        p.struct_size = ctypes.sizeof(p)
        p.K = int(kw["K"])
        p.S = int(kw.get("S", 1))
        p.max_iter = int(kw.get("max_iter", 0))
        p.res_tol = float(kw.get("res_tol", 0.0))
        p.eps = float(kw.get("eps", 0.0))
        p.prune = _lib.PRUNE[kw.get("prune", "each")]
        p.prec = _lib.PREC[kw.get("prec", "f32")]
        p.pivot_fallback = float(kw.get("pivot_fallback", 0.0))
        p.redo_tol = float(kw.get("redo_tol", 0.0))
        return p, _lib.SOLVER_GOMP
    if solver == "cosamp":
        p = _lib.CosampParams()
        p.struct_size = ctypes.sizeof(p)
        p.K = int(kw["K"])
        p.max_iter = int(kw.get("max_iter", 30))
        p.eps = float(kw.get("eps", 0.0))
        p.res_tol = float(kw.get("res_tol", 0.0))
        p.prec = _lib.PREC[kw.get("prec", "f32")]
        return p, _lib.SOLVER_COSAMP
    if solver == "biht":
        p = _lib.BihtParams()
        p.struct_size = ctypes.sizeof(p)
        p.K = int(kw["K"])
        p.max_iter = int(kw.get("max_iter", 100))
        p.mu = float(kw.get("mu", 0.1))
        p.eps = float(kw.get("eps", 0.0))
        p.res_tol = float(kw.get("res_tol", 0.0))
        p.mode = _lib.BIHT_MODE[kw.get("mode", "real")]
        ys = kw.get("Ysign")
        p.Ysign = ys.data_ptr() if ys is not None else 0
        p.prec = _lib.PREC[kw.get("prec", "f32")]
        return p, _lib.SOLVER_BIHT
    raise ValueError(solver)


def fista(A, Y, lam: float, L: float = 0.0, max_iter: int = 100, eps: float = 0.0, X0=None,
          prec: str = "f32", correction_iters: int = 0, stream=None, out=None):
    """FISTA (Alg. 1) on every pixel: returns (X (P x N), stats)."""
    torch = _torch()
    lib = library()
    _check_dev("A", A, torch.float32)
    M, N = A.shape
    _check_dev("Y", Y, torch.float32)
    P = Y.shape[0]
    if Y.shape[1] != M:
        raise ValueError("Y must be P x M")
    if X0 is not None:
        _check_dev("X0", X0, torch.float32, (P, N))
    pb = _problem(A, Y, P, stream)
    prm, sid = _params("fista", A, P, dict(lam=lam, L=L, max_iter=max_iter, eps=eps, X0=X0, prec=prec,
                                           correction_iters=correction_iters))
    ws = _workspace(lib, sid, pb, prm, A.device)
    X = out if out is not None else torch.empty((P, N), dtype=torch.float32, device=A.device)
    st = torch.empty((max(P, 1), 4), dtype=torch.int32, device=A.device)
    _lib.check(lib.csrec_fista(ctypes.byref(pb), ctypes.byref(prm), _ptr(X), _ptr(st)), "csrec_fista")
    _keep_alive(ws, A.device, stream)
    return X, _stats_view(st[:P])


def fista_complex(A, Y, lam: float, L: float = 0.0, max_iter: int = 100, eps: float = 0.0, X0=None,
                  stream=None, out=None):
    """FISTA (Alg. 1) for complex A (M x N) and Y (P x M), both complex64
    (the complex DFT basis of Section II): A^* in the gradient step, the soft
    threshold on |x_n|.  Returns (X (P x N complex64), stats)."""
    torch = _torch()
    lib = library()
    _check_dev("A", A, torch.complex64)
    M, N = A.shape
    _check_dev("Y", Y, torch.complex64)
    P = Y.shape[0]
    if Y.shape[1] != M:
        raise ValueError("Y must be P x M")
    if X0 is not None:
        _check_dev("X0", X0, torch.complex64, (P, N))
    pb = _problem(A, Y, P, stream)
    prm, sid = _params("fista_complex", A, P, dict(lam=lam, L=L, max_iter=max_iter, eps=eps, X0=X0))
    ws = _workspace(lib, sid, pb, prm, A.device)
    if out is not None:
        _check_dev("out", out, torch.complex64, (P, N))
    X = out if out is not None else torch.empty((P, N), dtype=torch.complex64, device=A.device)
    st = torch.empty((max(P, 1), 4), dtype=torch.int32, device=A.device)
    _lib.check(lib.csrec_fista_complex(ctypes.byref(pb), ctypes.byref(prm), _ptr(X), _ptr(st)),
               "csrec_fista_complex")
    _keep_alive(ws, A.device, stream)
    return X, _stats_view(st[:P])


def fista_hermitian(A, Y, lam: float, L: float = 0.0, max_iter: int = 100, eps: float = 0.0, X0=None,
                    stream=None, out=None):
    """FISTA (Alg. 1) with the DFT basis for real measurements: A (M x N
    complex64) with conjugate-symmetric columns (A = Phi Psi, Phi real), Y
    (P x M float32).  The iterate is conjugate-symmetric and the library
    iterates on its half (columns 0 .. N // 2 of A are read).  Returns
    (X (P x N complex64, the full spectrum), stats)."""
    torch = _torch()
    lib = library()
    _check_dev("A", A, torch.complex64)
    M, N = A.shape
    _check_dev("Y", Y, torch.float32)
    P = Y.shape[0]
    if Y.shape[1] != M:
        raise ValueError("Y must be P x M")
    if X0 is not None:
        _check_dev("X0", X0, torch.complex64, (P, N))
    pb = _problem(A, Y, P, stream)
    prm, sid = _params("fista_hermitian", A, P, dict(lam=lam, L=L, max_iter=max_iter, eps=eps, X0=X0))
    ws = _workspace(lib, sid, pb, prm, A.device)
    if out is not None:
        _check_dev("out", out, torch.complex64, (P, N))
    X = out if out is not None else torch.empty((P, N), dtype=torch.complex64, device=A.device)
    st = torch.empty((max(P, 1), 4), dtype=torch.int32, device=A.device)
    _lib.check(lib.csrec_fista_hermitian(ctypes.byref(pb), ctypes.byref(prm), _ptr(X), _ptr(st)),
               "csrec_fista_hermitian")
    _keep_alive(ws, A.device, stream)
    return X, _stats_view(st[:P])


def admm(A, Y, lam: float, alpha: float = 1.8, max_iter: int = 100, eps: float = 0.0, X0=None,
         threshold: str = "paper", want_z: bool = False, stream=None, out=None):
    """ADMM (Alg. 2) on every pixel: returns (X = x^I, Z = z^I or None, stats).
    threshold "paper" soft-thresholds at lam * alpha (Alg. 2 step 2 as
    printed), "standard" at lam / alpha."""
    torch = _torch()
    lib = library()
    _check_dev("A", A, torch.float32)
    M, N = A.shape
    _check_dev("Y", Y, torch.float32)
    P = Y.shape[0]
    if Y.shape[1] != M:
        raise ValueError("Y must be P x M")
    if X0 is not None:
        _check_dev("X0", X0, torch.float32, (P, N))
    pb = _problem(A, Y, P, stream)
    prm, sid = _params("admm", A, P, dict(lam=lam, alpha=alpha, max_iter=max_iter, eps=eps, X0=X0,
                                          threshold=threshold))
    ws = _workspace(lib, sid, pb, prm, A.device)
    X = out if out is not None else torch.empty((P, N), dtype=torch.float32, device=A.device)
    Z = torch.empty((P, N), dtype=torch.float32, device=A.device) if want_z else None
    st = torch.empty((max(P, 1), 4), dtype=torch.int32, device=A.device)
    _lib.check(lib.csrec_admm(ctypes.byref(pb), ctypes.byref(prm), _ptr(X), _ptr(Z),
                              _ptr(st)), "csrec_admm")
    _keep_alive(ws, A.device, stream)
    return X, Z, _stats_view(st[:P])


def admm_hermitian(A, Y, lam: float, alpha: float = 1.8, max_iter: int = 100, eps: float = 0.0, X0=None,
                   threshold: str = "paper", want_z: bool = False, stream=None, out=None):
    """ADMM (Alg. 2) with the DFT basis for real measurements: A (M x N
    complex64, conjugate-symmetric columns), Y (P x M float32).  Returns
    (X = x^I, Z = z^I or None (P x N complex64, full spectra), stats)."""
    torch = _torch()
    lib = library()
    _check_dev("A", A, torch.complex64)
    M, N = A.shape
    _check_dev("Y", Y, torch.float32)
    P = Y.shape[0]
    if Y.shape[1] != M:
        raise ValueError("Y must be P x M")
    if X0 is not None:
        _check_dev("X0", X0, torch.complex64, (P, N))
    pb = _problem(A, Y, P, stream)
    prm, sid = _params("admm_hermitian", A, P, dict(lam=lam, alpha=alpha, max_iter=max_iter, eps=eps, X0=X0,
                                                    threshold=threshold))
    ws = _workspace(lib, sid, pb, prm, A.device)
    if out is not None:
        _check_dev("out", out, torch.complex64, (P, N))
    X = out if out is not None else torch.empty((P, N), dtype=torch.complex64, device=A.device)
    Z = torch.empty((P, N), dtype=torch.complex64, device=A.device) if want_z else None
    st = torch.empty((max(P, 1), 4), dtype=torch.int32, device=A.device)
    _lib.check(lib.csrec_admm_hermitian(ctypes.byref(pb), ctypes.byref(prm), _ptr(X), _ptr(Z), _ptr(st)),
               "csrec_admm_hermitian")
    _keep_alive(ws, A.device, stream)
    return X, Z, _stats_view(st[:P])


def admm_complex(A, Y, lam: float, alpha: float = 1.8, max_iter: int = 100, eps: float = 0.0, X0=None,
                 threshold: str = "paper", want_z: bool = False, stream=None, out=None):
    """ADMM (Alg. 2) for complex A (M x N) and Y (P x M), both complex64:
    A^* in step 1, the soft threshold on |x + w|.  Returns (X = x^I,
    Z = z^I or None (P x N complex64), stats)."""
    torch = _torch()
    lib = library()
    _check_dev("A", A, torch.complex64)
    M, N = A.shape
    _check_dev("Y", Y, torch.complex64)
    P = Y.shape[0]
    if Y.shape[1] != M:
        raise ValueError("Y must be P x M")
    if X0 is not None:
        _check_dev("X0", X0, torch.complex64, (P, N))
    pb = _problem(A, Y, P, stream)
    prm, sid = _params("admm_complex", A, P, dict(lam=lam, alpha=alpha, max_iter=max_iter, eps=eps, X0=X0,
                                                  threshold=threshold))
    ws = _workspace(lib, sid, pb, prm, A.device)
    if out is not None:
        _check_dev("out", out, torch.complex64, (P, N))
    X = out if out is not None else torch.empty((P, N), dtype=torch.complex64, device=A.device)
    Z = torch.empty((P, N), dtype=torch.complex64, device=A.device) if want_z else None
    st = torch.empty((max(P, 1), 4), dtype=torch.int32, device=A.device)
    _lib.check(lib.csrec_admm_complex(ctypes.byref(pb), ctypes.byref(prm), _ptr(X), _ptr(Z), _ptr(st)),
               "csrec_admm_complex")
    _keep_alive(ws, A.device, stream)
    return X, Z, _stats_view(st[:P])


def sparsify(Psi, A, F, T: float = 0.1, ddof: int = 1, stream=None):
    """Section II sparsification of the spectra F (P x N) in the basis Psi
    (f = Psi x), fused with the compression of the sparsified pixels:
    returns (Xs (P x N), Y = Xs A^T (P x M), kept (P int32))."""
    torch = _torch()
    lib = library()
    _check_dev("A", A, torch.float32)
    M, N = A.shape
    _check_dev("Psi", Psi, torch.float32, (N, N))
    _check_dev("F", F, torch.float32)
    if F.shape[1] != N:
        raise ValueError("F must be P x N")
    P = F.shape[0]
    Xs = torch.empty((P, N), dtype=torch.float32, device=A.device)
    Y = torch.empty((P, M), dtype=torch.float32, device=A.device)
    kept = torch.empty((max(P, 1),), dtype=torch.int32, device=A.device)
    if stream is None:
        stream = torch.cuda.current_stream(A.device)
    sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    _lib.check(lib.csrec_sparsify(_ptr(Psi), _ptr(A), _ptr(F), M, N, P, float(T), int(ddof), _ptr(Xs), _ptr(Y),
                                  _ptr(kept), ctypes.c_void_p(sp)), "csrec_sparsify")
    return Xs, Y, kept[:P]


def sparsify_dft(Psi, A, F, T: float = 0.1, ddof: int = 1, stream=None):
    """Section II sparsification with the complex DFT basis Psi (N x N
    complex64, conjugate-symmetric columns) of the real spectra F (P x N
    float32), fused with the compression by A (M x N complex64, A = Phi Psi
    with Phi real): returns (Xs (P x N complex64), Y = Re(Xs A^T) (P x M
    float32), kept (P int32))."""
    torch = _torch()
    lib = library()
    _check_dev("A", A, torch.complex64)
    M, N = A.shape
    _check_dev("Psi", Psi, torch.complex64, (N, N))
    _check_dev("F", F, torch.float32)
    if F.shape[1] != N:
        raise ValueError("F must be P x N")
    P = F.shape[0]
    Xs = torch.empty((P, N), dtype=torch.complex64, device=A.device)
    Y = torch.empty((P, M), dtype=torch.float32, device=A.device)
    kept = torch.empty((max(P, 1),), dtype=torch.int32, device=A.device)
    if stream is None:
        stream = torch.cuda.current_stream(A.device)
    sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    _lib.check(lib.csrec_sparsify_dft(_ptr(Psi), _ptr(A), _ptr(F), M, N, P, float(T), int(ddof), _ptr(Xs), _ptr(Y),
                                      _ptr(kept), ctypes.c_void_p(sp)), "csrec_sparsify_dft")
    return Xs, Y, kept[:P]


def _keep_alive(ws, device, stream):
    # the workspace must outlive the enqueued kernels: tie it to the stream
    if ws is not None:
        torch = _torch()
        s = stream if stream is not None else torch.cuda.current_stream(device)
        if hasattr(s, "cuda_stream"):
            ws.record_stream(s)


def _greedy(solver, entry, A, Y, P, stream, kw):
    torch = _torch()
    lib = library()
    _check_dev("A", A, torch.float32)
    M, N = A.shape
    if Y is not None:
        _check_dev("Y", Y, torch.float32)
        if Y.shape[1] != M:
            raise ValueError("Y must be P x M")
    pb = _problem(A, Y, P, stream)
    prm, sid = _params(solver, A, P, kw)
    ws = _workspace(lib, sid, pb, prm, A.device)
    K = int(kw["K"])
    X = torch.empty((P, N), dtype=torch.float32, device=A.device)
    S = torch.empty((max(P, 1), K), dtype=torch.int32, device=A.device)
    st = torch.empty((max(P, 1), 4), dtype=torch.int32, device=A.device)
    fn = getattr(lib, entry)
    _lib.check(fn(ctypes.byref(pb), ctypes.byref(prm), _ptr(X), _ptr(S), _ptr(st)), entry)
    _keep_alive(ws, A.device, stream)
    return X, S[:P], _stats_view(st[:P])


def gomp(A, Y, K: int, S: int = 1, max_iter: int = 0, res_tol: float = 0.0, eps: float = 0.0,
         prune: str = "each", prec: str = "f32", pivot_fallback: float = 0.0, redo_tol: float = 0.0,
         stream=None):
    """gOMP (Alg. 3) on every pixel: returns (X, support (P x K, ascending, -1 padded), stats).
    pivot_fallback > 0 redoes in FP64 the pixels whose pivot ratio falls below
    it or whose FP32 error estimate exceeds redo_tol (0: the library's 1e-5)."""
    return _greedy("gomp", "csrec_gomp", A, Y, Y.shape[0], stream,
                   dict(K=K, S=S, max_iter=max_iter, res_tol=res_tol, eps=eps, prune=prune, prec=prec,
                        pivot_fallback=pivot_fallback, redo_tol=redo_tol))


def gomp_noalloc(A, Y, K: int, S: int = 1, max_iter: int = 0, res_tol: float = 0.0, eps: float = 0.0,
                 prune: str = "each", prec: str = "f32", pivot_fallback: float = 0.0, redo_tol: float = 0.0,
                 stream=None, out=None):
    """gOMP through csrec_gomp_noalloc: no workspace, the library's fixed
    per-device scratch instead (calls on one device must not overlap).
    out = (X (P x N float32), support (P x K int32), stats (P x 4 int32))
    receives the results when given, so that the call allocates nothing;
    otherwise they are allocated here.  Returns (X, support, stats)."""
    torch = _torch()
    lib = library()
    _check_dev("A", A, torch.float32)
    _check_dev("Y", Y, torch.float32)
    M, N = A.shape
    P = Y.shape[0]
    if Y.shape[1] != M:
        raise ValueError("Y must be P x M")
    pb = _problem(A, Y, P, stream)
    prm, _ = _params("gomp", A, P, dict(K=K, S=S, max_iter=max_iter, res_tol=res_tol, eps=eps, prune=prune,
                                         prec=prec, pivot_fallback=pivot_fallback, redo_tol=redo_tol))
    if out is None:
        X = torch.empty((P, N), dtype=torch.float32, device=A.device)
        Sp = torch.empty((max(P, 1), K), dtype=torch.int32, device=A.device)
        st = torch.empty((max(P, 1), 4), dtype=torch.int32, device=A.device)
    else:
        X, Sp, st = out
        if (X.shape[0] < P or X.shape[1] != N or Sp.shape[0] < P or Sp.shape[1] != K or st.shape[0] < P
                or st.shape[1] != 4 or not (X.is_contiguous() and Sp.is_contiguous() and st.is_contiguous())):
            raise ValueError("out must be contiguous (P x N float32, P x K int32, P x 4 int32) tensors")
        _check_dev("X", X, torch.float32)
        _check_dev("support", Sp, torch.int32)
        _check_dev("stats", st, torch.int32)
    _lib.check(lib.csrec_gomp_noalloc(ctypes.byref(pb), ctypes.byref(prm), _ptr(X), _ptr(Sp), _ptr(st)),
               "csrec_gomp_noalloc")
    return X[:P], Sp[:P], _stats_view(st[:P])


def gomp_hermitian(A, Y, K: int, S: int = 1, max_iter: int = 0, res_tol: float = 0.0, eps: float = 0.0,
                   prune: str = "each", prec: str = "f32", stream=None):
    """gOMP (Alg. 3) with the DFT basis for real measurements: A (M x N
    complex64) with conjugate-symmetric columns (A = Phi Psi, Phi real), Y
    (P x M float32).  K, S and max_iter count conjugate-pair groups ({0},
    {k, N-k}, {N/2}), selected and pruned together.  Returns (X (P x N
    complex64, conjugate-symmetric), support (P x 2K bins, ascending, -1
    padded), stats)."""
    torch = _torch()
    lib = library()
    _check_dev("A", A, torch.complex64)
    M, N = A.shape
    _check_dev("Y", Y, torch.float32)
    P = Y.shape[0]
    if Y.shape[1] != M:
        raise ValueError("Y must be P x M")
    pb = _problem(A, Y, P, stream)
    prm, _ = _params("gomp", A, P, dict(K=K, S=S, max_iter=max_iter, res_tol=res_tol, eps=eps, prune=prune,
                                         prec=prec, pivot_fallback=0.0))
    ws = _workspace(lib, _lib.SOLVER_GOMP_HERMITIAN, pb, prm, A.device)
    X = torch.empty((P, N), dtype=torch.complex64, device=A.device)
    Sp = torch.empty((max(P, 1), 2 * K), dtype=torch.int32, device=A.device)
    st = torch.empty((max(P, 1), 4), dtype=torch.int32, device=A.device)
    _lib.check(lib.csrec_gomp_hermitian(ctypes.byref(pb), ctypes.byref(prm), _ptr(X), _ptr(Sp), _ptr(st)),
               "csrec_gomp_hermitian")
    _keep_alive(ws, A.device, stream)
    return X, Sp[:P], _stats_view(st[:P])


def _greedy_hermitian(solver, entry, sid, A, Y, K, kw, stream):
    torch = _torch()
    lib = library()
    _check_dev("A", A, torch.complex64)
    M, N = A.shape
    _check_dev("Y", Y, torch.float32)
    P = Y.shape[0]
    if Y.shape[1] != M:
        raise ValueError("Y must be P x M")
    pb = _problem(A, Y, P, stream)
    prm, _ = _params(solver, A, P, dict(kw, K=K))
    ws = _workspace(lib, sid, pb, prm, A.device)
    X = torch.empty((P, N), dtype=torch.complex64, device=A.device)
    Sp = torch.empty((max(P, 1), 2 * K), dtype=torch.int32, device=A.device)
    st = torch.empty((max(P, 1), 4), dtype=torch.int32, device=A.device)
    fn = getattr(lib, entry)
    _lib.check(fn(ctypes.byref(pb), ctypes.byref(prm), _ptr(X), _ptr(Sp), _ptr(st)), entry)
    _keep_alive(ws, A.device, stream)
    return X, Sp[:P], _stats_view(st[:P])


def cosamp_hermitian(A, Y, K: int, max_iter: int = 30, eps: float = 0.0, res_tol: float = 0.0,
                     prec: str = "f32", stream=None):
    """CoSaMP (Alg. 5) with the DFT basis for real measurements, conjugate
    pairs as units (K counts groups): A (M x N complex64, conjugate-symmetric
    columns), Y (P x M float32).  Returns (X (P x N complex64), support
    (P x 2K bins), stats); FLAG_FP32_LIMIT as for cosamp."""
    return _greedy_hermitian("cosamp", "csrec_cosamp_hermitian", _lib.SOLVER_COSAMP_HERMITIAN, A, Y, K,
                             dict(max_iter=max_iter, eps=eps, res_tol=res_tol, prec=prec), stream)


def biht_hermitian(A, Y, K: int, max_iter: int = 100, mu: float = 0.1, eps: float = 0.0, res_tol: float = 0.0,
                   prec: str = "f32", stream=None):
    """Backtracking IHT (Alg. 4) with the DFT basis for real measurements,
    conjugate pairs as units (K counts groups).  As cosamp_hermitian."""
    return _greedy_hermitian("biht", "csrec_biht_hermitian", _lib.SOLVER_BIHT_HERMITIAN, A, Y, K,
                             dict(max_iter=max_iter, mu=mu, eps=eps, res_tol=res_tol, mode="real", Ysign=None,
                                  prec=prec), stream)


def cosamp(A, Y, K: int, max_iter: int = 30, eps: float = 0.0, res_tol: float = 0.0,
           prec: str = "f32", stream=None):
    """CoSaMP (Alg. 5) on every pixel: returns (X, support, stats).  On the
    FP32 path (3K <= M) a pixel whose least-squares solve meets a pivot ratio
    below 2^-20 stops with its previous iterate, flagged FLAG_FP32_LIMIT."""
    return _greedy("cosamp", "csrec_cosamp", A, Y, Y.shape[0], stream,
                   dict(K=K, max_iter=max_iter, eps=eps, res_tol=res_tol, prec=prec))


def biht(A, Y, K: int, max_iter: int = 100, mu: float = 0.1, eps: float = 0.0, res_tol: float = 0.0,
         mode: str = "real", Ysign=None, prec: str = "f32", stream=None):
    """BIHT: backtracking IHT (Alg. 4, mode='real') or binary IHT on int8
    signs (mode='one_bit', not from the paper).  Returns (X, support, stats)."""
    torch = _torch()
    if mode == "one_bit":
        _check_dev("Ysign", Ysign, torch.int8)
        P = Ysign.shape[0]
    else:
        P = Y.shape[0]
    return _greedy("biht", "csrec_biht", A, Y if mode != "one_bit" else None, P, stream,
                   dict(K=K, max_iter=max_iter, mu=mu, eps=eps, res_tol=res_tol, mode=mode, Ysign=Ysign,
                        prec=prec))


def lipschitz(A, stream=None):
    """L = lambda_max(A^T A) by power iteration on the GPU (float32 tensor of one element)."""
    torch = _torch()
    lib = library()
    _check_dev("A", A, torch.float32)
    M, N = A.shape
    out = torch.empty(1, dtype=torch.float32, device=A.device)
    s = stream if stream is not None else torch.cuda.current_stream(A.device)
    _lib.check(lib.csrec_lipschitz(_ptr(A), M, N, _ptr(out), ctypes.c_void_p(s.cuda_stream)),
               "csrec_lipschitz")
    return out


class Server:
    """Continuous-batching gOMP server (csrec_server_*): tiles of any band
    count are submitted from host memory, admitted by HBM budget, solved in
    batched launches with other admitted tiles, and polled back with their
    submit / admit / done times (seconds since creation)."""

    def __init__(self, K: int, S: int, res_tol: float = 0.0, max_iter: int = 0, prune: str = "each",
                 pivot_fallback: float = 0.0, prec: str = "f32", redo_tol: float = 0.0,
                 hbm_budget_bytes: int = 4 << 30,
                 batch_pixels: int = 262144, chunk_pixels: int = 65536, device: int = 0):
        import numpy as np  # noqa: F401
        lib = library()
        cfg = _lib.ServerCfg()
        cfg.struct_size = ctypes.sizeof(cfg)
        cfg.device = device
        cfg.hbm_budget_bytes = int(hbm_budget_bytes)
        cfg.batch_pixels = int(batch_pixels)
        cfg.chunk_pixels = int(chunk_pixels)
        self._defaults = dict(K=K, S=S, max_iter=max_iter, res_tol=res_tol, prune=prune,
                              pivot_fallback=pivot_fallback, prec=prec, redo_tol=redo_tol)
        g, _ = _params("gomp", None, 0, self._defaults)
        cfg.gomp = g
        h = ctypes.c_void_p(0)
        _lib.check(lib.csrec_server_create(ctypes.byref(cfg), ctypes.byref(h)), "csrec_server_create")
        self._lib, self._h, self.K = lib, h, K
        self._dicts = {}

    def add_dict(self, A) -> int:
        import numpy as np
        A = np.ascontiguousarray(A, dtype=np.float32)
        M, N = A.shape
        did = ctypes.c_int32(-1)
        _lib.check(self._lib.csrec_server_add_dict(self._h, A.ctypes.data, M, N, ctypes.byref(did)),
                   "csrec_server_add_dict")
        self._dicts[did.value] = (M, N)
        return did.value

    def submit(self, dict_id: int, Y, tag: int, **params) -> None:
        """Queues tile Y (P x M) under `tag`.  Keyword parameters (res_tol, eps,
        prune, pivot_fallback, redo_tol, max_iter, prec) override the server's for this
        tile; none given = the server's."""
        import numpy as np
        Y = np.ascontiguousarray(Y, dtype=np.float32)
        pp = None
        if params:
            kw = dict(self._defaults)
            kw.update(params)
            g, _ = _params("gomp", None, 0, kw)
            pp = ctypes.byref(g)
        _lib.check(self._lib.csrec_server_submit(self._h, dict_id, Y.ctypes.data, Y.shape[0], pp, tag),
                   "csrec_server_submit")

    def stats(self) -> dict:
        """Counters since creation: tiles, batches, pixels launched, pageable
        fallbacks, elapsed and busy seconds, time-averaged pixels in flight and
        device pool bytes in use."""
        st = _lib.ServerStats()
        st.struct_size = ctypes.sizeof(st)
        _lib.check(self._lib.csrec_server_get_stats(self._h, ctypes.byref(st)), "csrec_server_get_stats")
        return {name: getattr(st, name) for name, _ in _lib.ServerStats._fields_ if name != "struct_size"}

    def poll(self, max_results: int = 256, fetch: bool = True, release: bool = True) -> list:
        """Finished tiles as dicts (tag, status, X, support, iters, flags, t_submit, t_admit, t_done);
        arrays are copies, and the server's buffers are released unless
        release=False.  With fetch=False only the tag, status, pixel count and
        times are returned."""
        import numpy as np
        buf = (_lib.Result * max_results)()
        n = ctypes.c_int32(0)
        _lib.check(self._lib.csrec_server_poll(self._h, buf, max_results, ctypes.byref(n)), "csrec_server_poll")
        out = []
        for r in buf[:n.value]:
            P, N, K = r.P, r.N, r.K
            if not fetch:
                out.append(dict(tag=r.tag, status=r.status, dict_id=r.dict_id, P=P, t_submit=r.t_submit,
                                t_admit=r.t_admit, t_done=r.t_done))
                if release:
                    self._lib.csrec_server_release(self._h, r.tag)
                continue
            if P > 0 and r.status == 0:
                X = np.ctypeslib.as_array((ctypes.c_float * (P * N)).from_address(r.X)).reshape(P, N).copy()
                S = np.ctypeslib.as_array((ctypes.c_int32 * (P * K)).from_address(r.support)).reshape(P, K).copy()
                st = np.ctypeslib.as_array((ctypes.c_int32 * (P * 4)).from_address(r.stats)).reshape(P, 4).copy()
            else:
                X = np.zeros((P, N), np.float32)
                S = np.full((P, K), -1, np.int32)
                st = np.zeros((P, 4), np.int32)
            out.append(dict(tag=r.tag, status=r.status, dict_id=r.dict_id, X=X, support=S, iters=st[:, 0],
                            flags=st[:, 1].view(np.uint32), resid=st[:, 2].view(np.float32),
                            t_submit=r.t_submit, t_admit=r.t_admit, t_done=r.t_done))
            if release:
                self._lib.csrec_server_release(self._h, r.tag)
        return out

    def poll_held(self, max_results: int = 256) -> list:
        """Like poll(), but the server keeps each tile's host results until
        release(tag) is called (the arrays returned are still copies)."""
        return self.poll(max_results, release=False)

    def release(self, tag: int) -> None:
        _lib.check(self._lib.csrec_server_release(self._h, tag), "csrec_server_release")

    def drain(self) -> None:
        _lib.check(self._lib.csrec_server_drain(self._h), "csrec_server_drain")

    def close(self) -> None:
        if self._h:
            self._lib.csrec_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
