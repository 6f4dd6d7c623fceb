"""The C-ABI boundary on the CPU: the library loads, exports every symbol
include/csrec.h declares, the ctypes structs match the C layout, and
argument validation rejects bad calls before any GPU work (no kernel is
launched by these tests)."""
import ctypes
import os
import re
import shutil
import sys
import subprocess

import pytest

from paper_2401_14762_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "csrec.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libcsrec.so is not built (python -m paper_2401_14762_amd.build)")
    return L.load()


def _declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int32_t|const char\*)\s+(csrec_\w+)\s*\(", text, re.M)))


def test_header_declares_entry_points():
    names = _declared_functions()
    for must in ("csrec_fista", "csrec_gomp", "csrec_cosamp", "csrec_biht", "csrec_workspace_bytes"):
        assert must in names


def test_flag_values_match_the_header():
    """The binding's stats flags are the header's CSREC_FLAG_* values."""
    text = open(HEADER).read()
    flags = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define\s+CSREC_FLAG_(\w+)\s+(\d+)u", text)}
    assert set(flags) == {"CONVERGED", "ITER_CAP", "FP64_FALLBACK", "NONFINITE", "FP32_LIMIT"}
    for name, value in flags.items():
        assert getattr(L, "FLAG_" + name) == value, name
    assert len(set(flags.values())) == len(flags) and all(v & (v - 1) == 0 for v in flags.values())


def test_exports_every_declared_symbol(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name
        assert name in L.SIGNATURES, name
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True)
    exported = set(re.findall(r" T (csrec_\w+)", out.stdout))
    assert set(_declared_functions()) <= exported


def test_struct_layout_matches_c(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "sizes.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "csrec.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu\\n\","
        "sizeof(csrec_problem), sizeof(csrec_pixel_stats), sizeof(csrec_fista_params),"
        "sizeof(csrec_gomp_params), sizeof(csrec_cosamp_params), sizeof(csrec_biht_params),"
        "offsetof(csrec_problem, workspace_bytes), offsetof(csrec_biht_params, Ysign));"
        "printf(\"%zu %zu %zu\\n\", sizeof(csrec_server_cfg), sizeof(csrec_result), offsetof(csrec_result, t_done));"
        "printf(\"%zu %zu %zu\\n\", sizeof(csrec_admm_params), offsetof(csrec_admm_params, X0),"
        "offsetof(csrec_admm_params, threshold));"
        "printf(\"%zu %zu\\n\", offsetof(csrec_gomp_params, pivot_fallback), offsetof(csrec_gomp_params, redo_tol));"
        "return 0;}\n")
    exe = tmp_path / "sizes"
    subprocess.run([cc, "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    want = [ctypes.sizeof(L.Problem), ctypes.sizeof(L.PixelStats), ctypes.sizeof(L.FistaParams),
            ctypes.sizeof(L.GompParams), ctypes.sizeof(L.CosampParams), ctypes.sizeof(L.BihtParams),
            L.Problem.workspace_bytes.offset, L.BihtParams.Ysign.offset,
            ctypes.sizeof(L.ServerCfg), ctypes.sizeof(L.Result), L.Result.t_done.offset,
            ctypes.sizeof(L.AdmmParams), L.AdmmParams.X0.offset, L.AdmmParams.threshold.offset,
            L.GompParams.pivot_fallback.offset, L.GompParams.redo_tol.offset]
    assert got == want


def test_version_and_errors(lib):
    assert lib.csrec_abi_version() == L.CSREC_ABI_VERSION
    for code in (0, -1, -2, -3, -4, -5, -6, -99):
        assert isinstance(lib.csrec_strerror(code), bytes)


def _problem(M=40, N=100, P=10, A=0x1000, Y=0x2000):
    pb = L.Problem()
    pb.struct_size = ctypes.sizeof(L.Problem)
    pb.M, pb.N, pb.P = M, N, P
    pb.A, pb.Y = A, Y
    return pb


def _fista(**kw):
    p = L.FistaParams()
    p.struct_size = ctypes.sizeof(p)
    p.max_iter, p.lambda_, p.L, p.eps, p.prec = 10, 0.01, 1.0, 0.0, 0
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _gomp(**kw):
    p = L.GompParams()
    p.struct_size = ctypes.sizeof(p)
    p.K, p.S, p.max_iter, p.prune, p.prec = 8, 2, 0, 0, 0
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _admm(**kw):
    p = L.AdmmParams()
    p.struct_size = ctypes.sizeof(p)
    p.max_iter, p.lambda_, p.alpha, p.eps, p.threshold = 10, 0.01, 1.8, 0.0, 0
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _ws(lib, solver, pb, prm):
    n = ctypes.c_size_t(123)
    rc = lib.csrec_workspace_bytes(solver, ctypes.byref(pb), ctypes.byref(prm), ctypes.byref(n))
    return rc, n.value


def test_validation_shapes(lib):
    for M, N, P in ((0, 100, 1), (100, 100, 1), (120, 100, 1), (40, 257, 1), (40, 100, -1)):
        rc, _ = _ws(lib, L.SOLVER_FISTA, _problem(M, N, P), _fista())
        assert rc == L.E_SHAPE, (M, N, P)


def test_validation_params(lib):
    pb = _problem()
    assert _ws(lib, L.SOLVER_FISTA, pb, _fista(max_iter=-1))[0] == L.E_INVAL
    assert _ws(lib, L.SOLVER_FISTA, pb, _fista(lambda_=-1.0))[0] == L.E_INVAL
    assert _ws(lib, L.SOLVER_FISTA, pb, _fista(lambda_=float("nan")))[0] == L.E_INVAL
    assert _ws(lib, L.SOLVER_FISTA, pb, _fista(prec=7))[0] == L.E_INVAL
    bad = _fista()
    bad.struct_size = 8
    assert _ws(lib, L.SOLVER_FISTA, pb, bad)[0] == L.E_INVAL
    assert _ws(lib, L.SOLVER_GOMP, pb, _gomp(S=0))[0] == L.E_INVAL
    assert _ws(lib, L.SOLVER_GOMP, pb, _gomp(S=9))[0] == L.E_INVAL
    assert _ws(lib, L.SOLVER_GOMP, pb, _gomp(prune=5))[0] == L.E_INVAL
    # S * max_iter larger than M: the least squares would be underdetermined
    assert _ws(lib, L.SOLVER_GOMP, pb, _gomp(S=2, max_iter=21))[0] == L.E_SHAPE
    assert _ws(lib, 99, pb, _gomp())[0] == L.E_INVAL
    # null problem / null bytes
    n = ctypes.c_size_t(0)
    assert lib.csrec_workspace_bytes(L.SOLVER_FISTA, None, ctypes.byref(_fista()), ctypes.byref(n)) == L.E_INVAL
    assert lib.csrec_workspace_bytes(L.SOLVER_FISTA, ctypes.byref(pb), ctypes.byref(_fista()), None) == L.E_INVAL


def _cosamp(**kw):
    p = L.CosampParams()
    p.struct_size = ctypes.sizeof(p)
    p.K, p.max_iter, p.eps, p.res_tol, p.prec = 8, 10, 0.0, 0.0, 0
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_cosamp_3k_above_m_and_redo_tol(lib):
    """CoSaMP with 3K > M takes the FP64 path, which needs no workspace and
    computes in FP64 only (16-bit correlations refused); 3K must not exceed N
    nor 128.  gOMP's redo_tol must be finite and non-negative."""
    pb = _problem(40, 100, 16)
    rc, n = _ws(lib, L.SOLVER_COSAMP, pb, _cosamp(K=10))         # 3K = 30 <= M: on-chip path
    assert rc == L.OK and n > 0
    rc, n = _ws(lib, L.SOLVER_COSAMP, pb, _cosamp(K=15))         # 3K = 45 > M
    assert rc == L.OK and n == 0
    assert _ws(lib, L.SOLVER_COSAMP, pb, _cosamp(K=15, prec=1))[0] == L.E_UNSUPPORTED
    assert _ws(lib, L.SOLVER_COSAMP, pb, _cosamp(K=34))[0] == L.E_SHAPE          # 3K > N
    assert _ws(lib, L.SOLVER_COSAMP, _problem(40, 200, 16), _cosamp(K=43))[0] == L.E_SHAPE   # 3K > 128
    for bad in (-1.0, float("nan"), float("inf")):
        assert _ws(lib, L.SOLVER_GOMP, pb, _gomp(pivot_fallback=1e-6, redo_tol=bad))[0] == L.E_INVAL, bad
    rc, n = _ws(lib, L.SOLVER_GOMP, pb, _gomp(pivot_fallback=1e-6, redo_tol=1e-7))
    assert rc == L.OK and n > 0


def test_validation_entry_points_enqueue_nothing(lib):
    """Invalid calls return before touching the device (safe without a GPU)."""
    pb = _problem()
    assert lib.csrec_fista(ctypes.byref(pb), ctypes.byref(_fista(max_iter=-3)), None, None) == L.E_INVAL
    pb0 = _problem(P=0)
    assert lib.csrec_fista(ctypes.byref(pb0), ctypes.byref(_fista()), None, None) == L.OK
    assert lib.csrec_gomp(ctypes.byref(pb0), ctypes.byref(_gomp()), None, None, None) == L.OK
    # greedy without workspace -> E_WORKSPACE (checked before any launch)
    assert lib.csrec_gomp(ctypes.byref(pb), ctypes.byref(_gomp()), ctypes.c_void_p(0x3000), None,
                          None) == L.E_WORKSPACE
    # FISTA with L = 0 needs a workspace for the device estimate
    assert lib.csrec_fista(ctypes.byref(pb), ctypes.byref(_fista(L=0.0)), ctypes.c_void_p(0x3000),
                           None) == L.E_WORKSPACE
    # BIHT one-bit requires signs
    p = L.BihtParams()
    p.struct_size = ctypes.sizeof(p)
    p.K, p.max_iter, p.mu, p.mode = 5, 10, 0.1, 1
    assert lib.csrec_biht(ctypes.byref(pb), ctypes.byref(p), ctypes.c_void_p(0x3000), None, None) == L.E_INVAL


def test_admm_validation(lib):
    """ADMM: alpha must be a positive finite number (FP32 too), the threshold
    one of the two readings, the threshold value finite in FP32; M <= 96."""
    pb = _problem()
    assert _ws(lib, L.SOLVER_ADMM, pb, _admm()) == (L.OK, 40 * 40 * 4 // 256 * 256 + 256 * (40 * 40 * 4 % 256 > 0))
    for bad in (dict(alpha=0.0), dict(alpha=-1.0), dict(alpha=float("nan")), dict(alpha=float("inf")),
                dict(alpha=1e-50), dict(alpha=1e39), dict(lambda_=-1.0), dict(eps=float("nan")),
                dict(max_iter=-1), dict(threshold=2), dict(threshold=-1),
                dict(threshold=1, alpha=1e-30, lambda_=1e10)):
        assert _ws(lib, L.SOLVER_ADMM, pb, _admm(**bad))[0] == L.E_INVAL, bad
    wrong = _admm()
    wrong.struct_size = 8
    assert _ws(lib, L.SOLVER_ADMM, pb, wrong)[0] == L.E_INVAL
    assert _ws(lib, L.SOLVER_ADMM, _problem(M=96, N=240), _admm())[0] == L.OK
    assert _ws(lib, L.SOLVER_ADMM, _problem(M=97, N=240), _admm())[0] == L.E_UNSUPPORTED
    assert _ws(lib, L.SOLVER_ADMM, _problem(M=40, N=20), _admm())[0] == L.E_SHAPE
    assert _ws(lib, L.SOLVER_ADMM, _problem(P=0), _admm()) == (L.OK, 0)
    # entry point: invalid parameters, missing output or workspace return before any launch
    assert lib.csrec_admm(ctypes.byref(pb), ctypes.byref(_admm(alpha=0.0)), ctypes.c_void_p(0x3000), None,
                          None) == L.E_INVAL
    assert lib.csrec_admm(ctypes.byref(pb), ctypes.byref(_admm()), None, None, None) == L.E_INVAL
    assert lib.csrec_admm(ctypes.byref(pb), ctypes.byref(_admm()), ctypes.c_void_p(0x3000), None,
                          None) == L.E_WORKSPACE
    pb.workspace, pb.workspace_bytes = 0x4000, 40 * 40 * 4 - 4
    assert lib.csrec_admm(ctypes.byref(pb), ctypes.byref(_admm()), ctypes.c_void_p(0x3000), None,
                          None) == L.E_WORKSPACE
    assert lib.csrec_admm(ctypes.byref(_problem(P=0)), ctypes.byref(_admm()), None, None, None) == L.OK


def test_sparsify_validation(lib):
    """Shapes, ddof, T and pointers are checked before any launch."""
    v = ctypes.c_void_p(0x3000)
    ok = dict(Psi=v, A=v, F=v, M=40, N=100, P=10, T=0.1, ddof=1, Xs=v, Y=v)

    def call(**kw):
        a = dict(ok, **kw)
        return lib.csrec_sparsify(a["Psi"], a["A"], a["F"], a["M"], a["N"], a["P"], a["T"], a["ddof"], a["Xs"],
                                  a["Y"], None, None)
    for bad in (dict(M=0), dict(M=100), dict(N=257), dict(P=-1)):
        assert call(**bad) == L.E_SHAPE, bad
    for bad in (dict(ddof=2), dict(ddof=-1), dict(T=float("nan")), dict(T=1e39), dict(Psi=None), dict(A=None),
                dict(F=None), dict(Xs=None), dict(Y=None)):
        assert call(**bad) == L.E_INVAL, bad
    assert call(M=97, N=240) == L.E_UNSUPPORTED
    assert call(P=0, Psi=None, F=None, Xs=None, Y=None) == L.OK


def test_workspace_sizes(lib):
    pb = _problem(M=80, N=200, P=65536)
    rc, n = _ws(lib, L.SOLVER_FISTA, pb, _fista())
    assert rc == L.OK and n == 0
    rc, n = _ws(lib, L.SOLVER_FISTA, pb, _fista(L=0.0))
    assert rc == L.OK and n >= 4
    # gOMP in FP32 keeps every per-pixel quantity on chip: the workspace is
    # the Gram matrix, the padded A^T and nothing that grows with P
    rc, n1 = _ws(lib, L.SOLVER_GOMP, pb, _gomp(K=20, S=2))
    assert rc == L.OK and 200 * 200 * 4 + 200 * 128 * 4 <= n1 < 2 * 1024 * 1024
    # the FP64 fallback adds the FP64 Gram and per-pixel scratch for its redo
    rc, n2 = _ws(lib, L.SOLVER_GOMP, pb, _gomp(K=20, S=2, pivot_fallback=1e-6))
    assert rc == L.OK and n2 > n1 + 65536 * 4
    # CoSaMP keeps its state on chip too: the same Gram + dictionary copies
    p = L.CosampParams()
    p.struct_size = ctypes.sizeof(p)
    p.K, p.max_iter = 10, 20
    rc, n3 = _ws(lib, L.SOLVER_COSAMP, pb, p)
    assert rc == L.OK and n3 == n1


def test_one_hip_runtime_in_process():
    """Loading the library before torch must not map a second libamdhip64
    (torch bundles its own copy; two runtimes do not share devices)."""
    code = ("import sys; sys.path.insert(0, %r); from paper_2401_14762_amd import _lib; _lib.load(); "
            "import torch; print(len({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))"
            % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "1"


def test_fista_complex_validation(lib):
    """Complex FISTA: FP32 only, no correction pass, M <= 48 and N <= 128,
    a workspace for the real embedding of A (2M x 2N' floats, N' the
    multiple of 16 the kernel tile uses) plus the device L slot."""
    S = L.SOLVER_FISTA_COMPLEX
    pb = _problem(M=40, N=100)
    rc, n = _ws(lib, S, pb, _fista())
    assert rc == L.OK and 2 * 40 * 2 * 112 * 4 <= n <= 2 * 40 * 2 * 112 * 4 + 512
    assert _ws(lib, S, pb, _fista(L=0.0))[0] == L.OK
    assert _ws(lib, S, pb, _fista(prec=1))[0] == L.E_UNSUPPORTED
    assert _ws(lib, S, pb, _fista(correction_iters=5))[0] == L.E_UNSUPPORTED
    assert _ws(lib, S, pb, _fista(prec=7))[0] == L.E_INVAL
    assert _ws(lib, S, pb, _fista(lambda_=-1.0))[0] == L.E_INVAL
    assert _ws(lib, S, _problem(M=48, N=128), _fista())[0] == L.OK
    assert _ws(lib, S, _problem(M=49, N=128), _fista())[0] == L.E_UNSUPPORTED
    assert _ws(lib, S, _problem(M=40, N=129), _fista())[0] == L.E_UNSUPPORTED
    assert _ws(lib, S, _problem(M=5, N=17), _fista())[0] == L.OK
    assert _ws(lib, S, _problem(M=20, N=10), _fista())[0] == L.E_SHAPE
    assert _ws(lib, S, _problem(P=0), _fista()) == (L.OK, 0)
    # entry point: bad parameters, a missing output or workspace return before any launch
    v = ctypes.c_void_p(0x3000)
    assert lib.csrec_fista_complex(ctypes.byref(pb), ctypes.byref(_fista(max_iter=-1)), v, None) == L.E_INVAL
    assert lib.csrec_fista_complex(ctypes.byref(pb), ctypes.byref(_fista()), None, None) == L.E_INVAL
    assert lib.csrec_fista_complex(ctypes.byref(pb), ctypes.byref(_fista()), v, None) == L.E_WORKSPACE
    pb.workspace, pb.workspace_bytes = 0x4000, n - 4
    assert lib.csrec_fista_complex(ctypes.byref(pb), ctypes.byref(_fista()), v, None) == L.E_WORKSPACE
    assert lib.csrec_fista_complex(ctypes.byref(_problem(P=0)), ctypes.byref(_fista()), None, None) == L.OK


def test_fista_hermitian_validation(lib):
    """Half-spectrum FISTA: FP32 only, M <= 96, N <= 256; no workspace with
    a given L, C diag(sqrt(w)) (M x 2S floats, S = 16 ceil(ceil(N/2) / 16))
    plus the L slot for the device estimate."""
    S = L.SOLVER_FISTA_HERMITIAN
    pb = _problem(M=90, N=224)
    assert _ws(lib, S, pb, _fista()) == (L.OK, 0)
    rc, n = _ws(lib, S, pb, _fista(L=0.0))
    assert rc == L.OK and n == 90 * 2 * 112 * 4 // 256 * 256 + 256 * ((90 * 2 * 112 * 4) % 256 > 0) + 256
    assert _ws(lib, S, pb, _fista(prec=2))[0] == L.E_UNSUPPORTED
    assert _ws(lib, S, pb, _fista(correction_iters=1))[0] == L.E_UNSUPPORTED
    assert _ws(lib, S, pb, _fista(eps=-1.0))[0] == L.E_INVAL
    assert _ws(lib, S, _problem(M=96, N=256), _fista())[0] == L.OK
    assert _ws(lib, S, _problem(M=97, N=256), _fista())[0] == L.E_UNSUPPORTED
    assert _ws(lib, S, _problem(M=40, N=257), _fista())[0] == L.E_SHAPE
    assert _ws(lib, S, _problem(P=0), _fista(L=0.0)) == (L.OK, 0)
    v = ctypes.c_void_p(0x3000)
    assert lib.csrec_fista_hermitian(ctypes.byref(pb), ctypes.byref(_fista(lambda_=-1.0)), v, None) == L.E_INVAL
    assert lib.csrec_fista_hermitian(ctypes.byref(pb), ctypes.byref(_fista()), None, None) == L.E_INVAL
    assert lib.csrec_fista_hermitian(ctypes.byref(pb), ctypes.byref(_fista(L=0.0)), v, None) == L.E_WORKSPACE
    assert lib.csrec_fista_hermitian(ctypes.byref(_problem(P=0)), ctypes.byref(_fista()), None, None) == L.OK


def test_admm_hermitian_validation(lib):
    """Half-spectrum ADMM: the parameter checks of csrec_admm, M <= 96,
    N <= 256; workspace = the half-spectrum matrix (M x 2S) + R (M x M)."""
    S = L.SOLVER_ADMM_HERMITIAN
    pb = _problem(M=90, N=224)
    rc, n = _ws(lib, S, pb, _admm())
    assert rc == L.OK and n == 90 * 224 * 4 + (90 * 90 * 4 + 255) // 256 * 256
    for bad in (dict(alpha=0.0), dict(lambda_=-1.0), dict(threshold=3), dict(max_iter=-1)):
        assert _ws(lib, S, pb, _admm(**bad))[0] == L.E_INVAL, bad
    assert _ws(lib, S, _problem(M=96, N=256), _admm())[0] == L.OK
    assert _ws(lib, S, _problem(M=97, N=256), _admm())[0] == L.E_UNSUPPORTED
    assert _ws(lib, S, _problem(M=40, N=257), _admm())[0] == L.E_SHAPE
    assert _ws(lib, S, _problem(P=0), _admm()) == (L.OK, 0)
    v = ctypes.c_void_p(0x3000)
    assert lib.csrec_admm_hermitian(ctypes.byref(pb), ctypes.byref(_admm()), None, None, None) == L.E_INVAL
    assert lib.csrec_admm_hermitian(ctypes.byref(pb), ctypes.byref(_admm()), v, None, None) == L.E_WORKSPACE
    assert lib.csrec_admm_hermitian(ctypes.byref(_problem(P=0)), ctypes.byref(_admm()), None, None, None) == L.OK


def test_admm_complex_validation(lib):
    """Complex ADMM: the parameter checks of csrec_admm, M <= 48, N <= 128;
    workspace = the embedding (2M x 2N') + the embedded R (2M x 2M)."""
    S = L.SOLVER_ADMM_COMPLEX
    pb = _problem(M=40, N=100)
    rc, n = _ws(lib, S, pb, _admm())
    assert rc == L.OK and n == 80 * 224 * 4 + (80 * 80 * 4 + 255) // 256 * 256
    for bad in (dict(alpha=-1.0), dict(lambda_=float("nan")), dict(threshold=2)):
        assert _ws(lib, S, pb, _admm(**bad))[0] == L.E_INVAL, bad
    assert _ws(lib, S, _problem(M=48, N=128), _admm())[0] == L.OK
    assert _ws(lib, S, _problem(M=49, N=128), _admm())[0] == L.E_UNSUPPORTED
    assert _ws(lib, S, _problem(M=40, N=129), _admm())[0] == L.E_UNSUPPORTED
    assert _ws(lib, S, _problem(P=0), _admm()) == (L.OK, 0)
    v = ctypes.c_void_p(0x3000)
    assert lib.csrec_admm_complex(ctypes.byref(pb), ctypes.byref(_admm()), None, None, None) == L.E_INVAL
    assert lib.csrec_admm_complex(ctypes.byref(pb), ctypes.byref(_admm()), v, None, None) == L.E_WORKSPACE
    assert lib.csrec_admm_complex(ctypes.byref(_problem(P=0)), ctypes.byref(_admm()), None, None, None) == L.OK


def test_sparsify_dft_validation(lib):
    """DFT sparsification: shapes, ddof, T and pointers checked before any launch."""
    v = ctypes.c_void_p(0x3000)
    ok = dict(Psi=v, A=v, F=v, M=90, N=224, P=10, T=0.1, ddof=1, Xs=v, Y=v)

    def call(**kw):
        a = dict(ok, **kw)
        return lib.csrec_sparsify_dft(a["Psi"], a["A"], a["F"], a["M"], a["N"], a["P"], a["T"], a["ddof"], a["Xs"],
                                      a["Y"], None, None)
    for bad in (dict(M=0), dict(M=224), dict(N=257), dict(P=-1)):
        assert call(**bad) == L.E_SHAPE, bad
    for bad in (dict(ddof=2), dict(T=float("inf")), dict(Psi=None), dict(A=None), dict(F=None), dict(Xs=None),
                dict(Y=None)):
        assert call(**bad) == L.E_INVAL, bad
    assert call(M=97, N=240) == L.E_UNSUPPORTED
    assert call(P=0, Psi=None, F=None, Xs=None, Y=None) == L.OK
