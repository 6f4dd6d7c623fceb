// C-ABI entry points of libcsrec: argument validation, workspace sizing and
// dispatch to the kernels.  No device memory is allocated here.
#include <cmath>
#include <cstring>
#include <mutex>

#include "common.hpp"

namespace csrec {
namespace {
thread_local int32_t g_last_hip_error = 0;

bool finite_nonneg(double v) { return std::isfinite(v) && v >= 0.0; }

int check_problem(const csrec_problem* p, bool needs_Y) {
    if (!p) return CSREC_E_INVAL;
    if (p->struct_size != (int32_t)sizeof(csrec_problem)) return CSREC_E_INVAL;
    if (p->M < 1 || p->N > CSREC_MAX_N || p->M >= p->N || p->P < 0) return CSREC_E_SHAPE;
    if (p->P > 0 && (!p->A || (needs_Y && !p->Y))) return CSREC_E_INVAL;
    if (!p->A) return CSREC_E_INVAL;
    return CSREC_OK;
}

int check_prec(int32_t prec) {
    return (prec == CSREC_PREC_F32 || prec == CSREC_PREC_BF16 || prec == CSREC_PREC_F16) ? CSREC_OK
                                                                                           : CSREC_E_INVAL;
}

int check_fista(const csrec_problem* p, const csrec_fista_params* f) {
    int e = check_problem(p, true);
    if (e) return e;
    if (!f || f->struct_size != (int32_t)sizeof(csrec_fista_params)) return CSREC_E_INVAL;
    if (f->max_iter < 0 || !finite_nonneg(f->lambda) || !finite_nonneg(f->L) || !finite_nonneg(f->eps))
        return CSREC_E_INVAL;
    if (f->correction_iters < 0) return CSREC_E_INVAL;
    if ((e = check_prec(f->prec))) return e;
    return fista_supported(p->M, p->N, f->prec);
}

int check_fista_complex(const csrec_problem* p, const csrec_fista_params* f) {
    int e = check_problem(p, true);
    if (e) return e;
    if (!f || f->struct_size != (int32_t)sizeof(csrec_fista_params)) return CSREC_E_INVAL;
    if (f->max_iter < 0 || !finite_nonneg(f->lambda) || !finite_nonneg(f->L) || !finite_nonneg(f->eps))
        return CSREC_E_INVAL;
    if (f->correction_iters < 0) return CSREC_E_INVAL;
    if ((e = check_prec(f->prec))) return e;
    if (f->prec != CSREC_PREC_F32 || f->correction_iters != 0) return CSREC_E_UNSUPPORTED;
    return fista_complex_supported(p->M, p->N);
}

int check_fista_hermitian(const csrec_problem* p, const csrec_fista_params* f) {
    int e = check_fista_complex(p, f);
    if (e != CSREC_OK && e != CSREC_E_UNSUPPORTED) return e;
    if (f->prec != CSREC_PREC_F32 || f->correction_iters != 0) return CSREC_E_UNSUPPORTED;
    return fista_hermitian_supported(p->M, p->N);
}

int check_admm(const csrec_problem* p, const csrec_admm_params* q, float* thr) {
    int e = check_problem(p, true);
    if (e) return e;
    if (!q || q->struct_size != (int32_t)sizeof(csrec_admm_params)) return CSREC_E_INVAL;
    if (q->max_iter < 0 || !finite_nonneg(q->lambda) || !finite_nonneg(q->eps)) return CSREC_E_INVAL;
    if (!std::isfinite(q->alpha) || !((float)q->alpha > 0.f) || !std::isfinite((float)q->alpha)) return CSREC_E_INVAL;
    double t;
    if (q->threshold == CSREC_ADMM_THR_PAPER)
        t = q->lambda * q->alpha;
    else if (q->threshold == CSREC_ADMM_THR_STANDARD)
        t = q->lambda / q->alpha;
    else
        return CSREC_E_INVAL;
    if (!std::isfinite((float)t) || !std::isfinite((float)q->eps)) return CSREC_E_INVAL;
    *thr = (float)t;
    return admm_supported(p->M, p->N);
}

int check_admm_hermitian(const csrec_problem* p, const csrec_admm_params* q, float* thr) {
    int e = check_admm(p, q, thr);
    if (e != CSREC_OK && e != CSREC_E_UNSUPPORTED) return e;
    if (p->M > 96) return CSREC_E_UNSUPPORTED;
    return admm_hermitian_supported(p->M, p->N);
}

int check_admm_complex(const csrec_problem* p, const csrec_admm_params* q, float* thr) {
    int e = check_admm(p, q, thr);
    if (e != CSREC_OK && e != CSREC_E_UNSUPPORTED) return e;
    return admm_complex_supported(p->M, p->N);
}

int fill_gomp(const csrec_problem* p, const csrec_gomp_params* q, GreedyLaunch& l) {
    int e = check_problem(p, true);
    if (e) return e;
    if (!q || q->struct_size != (int32_t)sizeof(csrec_gomp_params)) return CSREC_E_INVAL;
    if (q->K < 1 || q->S < 1 || q->S > 8 || q->max_iter < 0) return CSREC_E_INVAL;
    if (!finite_nonneg(q->res_tol) || !finite_nonneg(q->eps) || !finite_nonneg(q->pivot_fallback) ||
        !finite_nonneg(q->redo_tol))
        return CSREC_E_INVAL;
    if (q->prune != CSREC_PRUNE_EACH && q->prune != CSREC_PRUNE_FINAL) return CSREC_E_INVAL;
    if ((e = check_prec(q->prec))) return e;
    const int imax = q->max_iter > 0 ? q->max_iter : (q->K < p->M / q->S ? q->K : p->M / q->S);
    if (imax < 1) return CSREC_E_INVAL;
    if (q->S * imax > p->M || q->S * imax > GOMP_CMAX || q->K > GOMP_CMAX) return CSREC_E_SHAPE;
    if (p->M > 96) return CSREC_E_UNSUPPORTED;
    if ((e = gomp_coop_supported(p->M, p->N, q->K, q->S, imax))) return e;
    l = GreedyLaunch{};
    l.kind = GREEDY_GOMP;
    l.K = q->K;
    l.S = q->S;
    l.max_iter = imax;
    l.prune = q->prune;
    l.prec = q->prec;
    l.res_tol = (float)q->res_tol;
    l.eps = (float)q->eps;
    l.pivot_fallback = q->pivot_fallback;
    l.redo_tol = q->redo_tol > 0.0 ? q->redo_tol : CSREC_REDO_TOL_DEFAULT;
    return CSREC_OK;
}

// gOMP with the DFT basis on real measurements: K, S and max_iter count
// conjugate-pair groups, each up to two real unknowns.
int fill_gomp_hermitian(const csrec_problem* p, const csrec_gomp_params* q, GreedyLaunch& l) {
    int e = check_problem(p, true);
    if (e) return e;
    if (!q || q->struct_size != (int32_t)sizeof(csrec_gomp_params)) return CSREC_E_INVAL;
    if (q->K < 1 || q->S < 1 || q->S > 8 || q->max_iter < 0) return CSREC_E_INVAL;
    if (!finite_nonneg(q->res_tol) || !finite_nonneg(q->eps) || !finite_nonneg(q->pivot_fallback))
        return CSREC_E_INVAL;
    if (q->prune != CSREC_PRUNE_EACH && q->prune != CSREC_PRUNE_FINAL) return CSREC_E_INVAL;
    if ((e = check_prec(q->prec))) return e;
    if (q->pivot_fallback > 0) return CSREC_E_UNSUPPORTED;
    if (p->M > 96 || pair_dict_atoms(p->N) > CSREC_MAX_N) return CSREC_E_UNSUPPORTED;
    const int imax = q->max_iter > 0 ? q->max_iter : (q->K < p->M / (2 * q->S) ? q->K : p->M / (2 * q->S));
    if (imax < 1) return CSREC_E_INVAL;
    if (2 * q->S * imax > p->M || 2 * q->S * imax > GOMP_CMAX || 2 * q->K > GOMP_CMAX) return CSREC_E_SHAPE;
    if ((e = gomp_coop_supported_grp(p->M, pair_dict_atoms(p->N), q->K, q->S, imax))) return e;
    l = GreedyLaunch{};
    l.kind = GREEDY_GOMP;
    l.K = q->K;
    l.S = q->S;
    l.max_iter = imax;
    l.prune = q->prune;
    l.prec = q->prec;
    l.res_tol = (float)q->res_tol;
    l.eps = (float)q->eps;
    l.pivot_fallback = 0.0;
    return CSREC_OK;
}

int fill_cosamp(const csrec_problem* p, const csrec_cosamp_params* q, GreedyLaunch& l) {
    int e = check_problem(p, true);
    if (e) return e;
    if (!q || q->struct_size != (int32_t)sizeof(csrec_cosamp_params)) return CSREC_E_INVAL;
    if (q->K < 1 || q->max_iter < 0 || !finite_nonneg(q->eps) || !finite_nonneg(q->res_tol))
        return CSREC_E_INVAL;
    if ((e = check_prec(q->prec))) return e;
    if (p->M > 96) return CSREC_E_UNSUPPORTED;
    if (3 * q->K > p->M) {
        // the merged support can outgrow M: the FP64 minimum-norm path
        if ((e = cosamp_wide_supported(p->M, p->N, q->K))) return e;
        if (q->prec != CSREC_PREC_F32) return CSREC_E_UNSUPPORTED;
    } else if (3 * q->K > GREEDY_CMAX) {
        return CSREC_E_SHAPE;
    }
    l = GreedyLaunch{};
    l.kind = GREEDY_COSAMP;
    l.K = q->K;
    l.S = 1;
    l.max_iter = q->max_iter;
    l.prec = q->prec;
    l.res_tol = (float)q->res_tol;
    l.eps = (float)q->eps;
    return CSREC_OK;
}

int fill_biht(const csrec_problem* p, const csrec_biht_params* q, GreedyLaunch& l) {
    if (!q || q->struct_size != (int32_t)sizeof(csrec_biht_params)) return CSREC_E_INVAL;
    const bool one = q->mode == CSREC_BIHT_ONE_BIT;
    if (!one && q->mode != CSREC_BIHT_REAL) return CSREC_E_INVAL;
    int e = check_problem(p, !one);
    if (e) return e;
    if (one && p->P > 0 && !q->Ysign) return CSREC_E_INVAL;
    if (q->K < 1 || q->max_iter < 0 || !std::isfinite(q->mu) || !finite_nonneg(q->eps) ||
        !finite_nonneg(q->res_tol))
        return CSREC_E_INVAL;
    if ((e = check_prec(q->prec))) return e;
    if (one ? (q->K > p->N || q->K > 64) : (2 * q->K > p->M || 2 * q->K > GREEDY_CMAX))
        return CSREC_E_SHAPE;
    if (p->M > 96) return CSREC_E_UNSUPPORTED;
    l = GreedyLaunch{};
    l.kind = one ? GREEDY_BIHT_ONE_BIT : GREEDY_BIHT;
    l.K = q->K;
    l.S = 1;
    l.max_iter = q->max_iter;
    l.prec = q->prec;
    l.res_tol = (float)q->res_tol;
    l.eps = (float)q->eps;
    l.mu = (float)q->mu;
    l.Ysign = q->Ysign;
    return CSREC_OK;
}

// CoSaMP and BIHT with the DFT basis on real measurements: K counts
// conjugate-pair groups (up to two atoms each).
int fill_other_hermitian(const csrec_problem* p, int kind, int32_t K, int32_t max_iter, double eps,
                         double res_tol, double mu, int32_t prec, GreedyLaunch& l) {
    int e = check_problem(p, true);
    if (e) return e;
    if (K < 1 || max_iter < 0 || !finite_nonneg(eps) || !finite_nonneg(res_tol) || !std::isfinite(mu))
        return CSREC_E_INVAL;
    if ((e = check_prec(prec))) return e;
    const int merged = (kind == GREEDY_COSAMP ? 3 : 2) * 2 * K;   // atoms of the merged support at most
    if (merged > p->M || merged > GREEDY_CMAX) return CSREC_E_SHAPE;
    if (p->M > 96 || pair_dict_atoms(p->N) > CSREC_MAX_N) return CSREC_E_UNSUPPORTED;
    if ((e = coop_other_supported_grp(kind, p->M, pair_dict_atoms(p->N), K))) return e;
    l = GreedyLaunch{};
    l.kind = static_cast<GreedyKind>(kind);
    l.K = K;
    l.S = 1;
    l.max_iter = max_iter;
    l.prec = prec;
    l.res_tol = (float)res_tol;
    l.eps = (float)eps;
    l.mu = (float)mu;
    return CSREC_OK;
}

int fill_cosamp_hermitian(const csrec_problem* p, const csrec_cosamp_params* q, GreedyLaunch& l) {
    if (!q || q->struct_size != (int32_t)sizeof(csrec_cosamp_params)) return CSREC_E_INVAL;
    return fill_other_hermitian(p, GREEDY_COSAMP, q->K, q->max_iter, q->eps, q->res_tol, 0.0, q->prec, l);
}

int fill_biht_hermitian(const csrec_problem* p, const csrec_biht_params* q, GreedyLaunch& l) {
    if (!q || q->struct_size != (int32_t)sizeof(csrec_biht_params)) return CSREC_E_INVAL;
    if (q->mode != CSREC_BIHT_REAL) return q->mode == CSREC_BIHT_ONE_BIT ? CSREC_E_UNSUPPORTED : CSREC_E_INVAL;
    return fill_other_hermitian(p, GREEDY_BIHT, q->K, q->max_iter, q->eps, q->res_tol, q->mu, q->prec, l);
}

void fill_problem(const csrec_problem* p, GreedyLaunch& l) {
    l.A = p->A;
    l.Y = p->Y;
    l.M = p->M;
    l.N = p->N;
    l.P = p->P;
    l.workspace = p->workspace;
    l.workspace_bytes = p->workspace_bytes;
    l.stream = reinterpret_cast<hipStream_t>(p->stream);
}

int run_greedy(GreedyLaunch& l, float* X, int32_t* support, csrec_pixel_stats* stats) {
    if (l.P > 0 && !X) return CSREC_E_INVAL;
    l.X = X;
    l.support = support;
    l.stats = stats;
    if (l.P == 0) return CSREC_OK;
    const size_t need = greedy_workspace(l);
    if (need > 0 && (!l.workspace || l.workspace_bytes < need)) return CSREC_E_WORKSPACE;
    return greedy_launch(l);
}
}  // namespace

void set_hip_error(hipError_t e) { g_last_hip_error = (int32_t)e; }

}  // namespace csrec

using namespace csrec;

extern "C" {

int32_t csrec_abi_version(void) { return CSREC_ABI_VERSION; }

const char* csrec_strerror(int32_t code) {
    switch (code) {
        case CSREC_OK: return "ok";
        case CSREC_E_INVAL: return "invalid argument";
        case CSREC_E_SHAPE: return "unsupported or invalid shape";
        case CSREC_E_WORKSPACE: return "workspace missing or too small";
        case CSREC_E_DEVICE: return "HIP runtime error";
        case CSREC_E_UNSUPPORTED: return "precision or mode not supported for this solver/shape";
        case CSREC_E_BUDGET: return "request exceeds the server's HBM budget";
        default: return "unknown error";
    }
}

int32_t csrec_last_hip_error(void) { return g_last_hip_error; }

int32_t csrec_workspace_bytes(int32_t solver, const csrec_problem* problem, const void* params,
                              size_t* bytes) {
    if (!bytes) return CSREC_E_INVAL;
    *bytes = 0;
    int e = CSREC_OK;
    GreedyLaunch l{};
    switch (solver) {
        case CSREC_SOLVER_FISTA: {
            const auto* f = static_cast<const csrec_fista_params*>(params);
            if ((e = check_fista(problem, f))) return e;
            *bytes = fista_workspace(problem->M, problem->N, problem->P, f->prec) + (f->L == 0.0 ? 256 : 0);
            return CSREC_OK;
        }
        case CSREC_SOLVER_ADMM: {
            float thr;
            if ((e = check_admm(problem, static_cast<const csrec_admm_params*>(params), &thr))) return e;
            *bytes = problem->P > 0 ? admm_workspace(problem->M) : 0;
            return CSREC_OK;
        }
        case CSREC_SOLVER_FISTA_COMPLEX:
            if ((e = check_fista_complex(problem, static_cast<const csrec_fista_params*>(params)))) return e;
            *bytes = problem->P > 0 ? fista_complex_workspace(problem->M, problem->N) : 0;
            return CSREC_OK;
        case CSREC_SOLVER_ADMM_COMPLEX: {
            float thr;
            if ((e = check_admm_complex(problem, static_cast<const csrec_admm_params*>(params), &thr))) return e;
            *bytes = problem->P > 0 ? admm_complex_workspace(problem->M, problem->N) : 0;
            return CSREC_OK;
        }
        case CSREC_SOLVER_ADMM_HERMITIAN: {
            float thr;
            if ((e = check_admm_hermitian(problem, static_cast<const csrec_admm_params*>(params), &thr))) return e;
            *bytes = problem->P > 0 ? admm_hermitian_workspace(problem->M, problem->N) : 0;
            return CSREC_OK;
        }
        case CSREC_SOLVER_FISTA_HERMITIAN: {
            const csrec_fista_params* f = static_cast<const csrec_fista_params*>(params);
            if ((e = check_fista_hermitian(problem, f))) return e;
            *bytes = problem->P > 0 ? fista_hermitian_workspace(problem->M, problem->N, !(f->L > 0.0)) : 0;
            return CSREC_OK;
        }
        case CSREC_SOLVER_GOMP:
            e = fill_gomp(problem, static_cast<const csrec_gomp_params*>(params), l);
            break;
        case CSREC_SOLVER_GOMP_HERMITIAN:
            if ((e = fill_gomp_hermitian(problem, static_cast<const csrec_gomp_params*>(params), l))) return e;
            *bytes = problem->P > 0 ? greedy_hermitian_workspace(problem->M, problem->N) : 0;
            return CSREC_OK;
        case CSREC_SOLVER_COSAMP_HERMITIAN:
            if ((e = fill_cosamp_hermitian(problem, static_cast<const csrec_cosamp_params*>(params), l))) return e;
            *bytes = problem->P > 0 ? greedy_hermitian_workspace(problem->M, problem->N) : 0;
            return CSREC_OK;
        case CSREC_SOLVER_BIHT_HERMITIAN:
            if ((e = fill_biht_hermitian(problem, static_cast<const csrec_biht_params*>(params), l))) return e;
            *bytes = problem->P > 0 ? greedy_hermitian_workspace(problem->M, problem->N) : 0;
            return CSREC_OK;
        case CSREC_SOLVER_COSAMP:
            e = fill_cosamp(problem, static_cast<const csrec_cosamp_params*>(params), l);
            break;
        case CSREC_SOLVER_BIHT:
            e = fill_biht(problem, static_cast<const csrec_biht_params*>(params), l);
            break;
        default: return CSREC_E_INVAL;
    }
    if (e) return e;
    fill_problem(problem, l);
    *bytes = problem->P > 0 ? greedy_workspace(l) : 0;
    return CSREC_OK;
}

int32_t csrec_fista(const csrec_problem* problem, const csrec_fista_params* params, float* X,
                    csrec_pixel_stats* stats) {
    int e = check_fista(problem, params);
    if (e) return e;
    if (problem->P == 0) return CSREC_OK;
    if (!X) return CSREC_E_INVAL;
    FistaLaunch l{};
    l.A = problem->A;
    l.Y = problem->Y;
    l.X0 = params->X0;
    l.X = X;
    l.stats = stats;
    l.M = problem->M;
    l.N = problem->N;
    l.P = problem->P;
    l.max_iter = params->max_iter;
    l.eps = (float)params->eps;
    l.lambda = params->lambda;
    l.prec = params->prec;
    l.correction_iters = params->correction_iters;
    l.stream = reinterpret_cast<hipStream_t>(problem->stream);
    l.workspace = problem->workspace;
    if (params->L > 0.0) {
        l.invL = (float)(1.0 / params->L);
        l.thr = (float)(params->lambda / params->L);
        l.L_dev = nullptr;
    } else {
        if (!problem->workspace || problem->workspace_bytes < 256) return CSREC_E_WORKSPACE;
        float* Ld = static_cast<float*>(problem->workspace);
        if ((e = lipschitz_launch(problem->A, problem->M, problem->N, Ld, l.stream))) return e;
        l.L_dev = Ld;
    }
    return fista_launch(l);
}

int32_t csrec_gomp(const csrec_problem* problem, const csrec_gomp_params* params, float* X,
                   int32_t* support, csrec_pixel_stats* stats) {
    GreedyLaunch l{};
    int e = fill_gomp(problem, params, l);
    if (e) return e;
    fill_problem(problem, l);
    return run_greedy(l, X, support, stats);
}

int32_t csrec_gomp_hermitian(const csrec_problem* problem, const csrec_gomp_params* params, float* X,
                             int32_t* support, csrec_pixel_stats* stats) {
    GreedyLaunch l{};
    int e = fill_gomp_hermitian(problem, params, l);
    if (e) return e;
    fill_problem(problem, l);
    if (l.P == 0) return CSREC_OK;
    if (!X) return CSREC_E_INVAL;
    l.X = X;
    l.support = support;
    l.stats = stats;
    if (!l.workspace || l.workspace_bytes < greedy_hermitian_workspace(l.M, l.N)) return CSREC_E_WORKSPACE;
    return gomp_hermitian_launch(l);
}

namespace {
int run_other_hermitian(GreedyLaunch& l, const csrec_problem* problem, float* X, int32_t* support,
                        csrec_pixel_stats* stats) {
    fill_problem(problem, l);
    if (l.P == 0) return CSREC_OK;
    if (!X) return CSREC_E_INVAL;
    l.X = X;
    l.support = support;
    l.stats = stats;
    if (!l.workspace || l.workspace_bytes < greedy_hermitian_workspace(l.M, l.N)) return CSREC_E_WORKSPACE;
    return other_hermitian_launch(l);
}
}  // namespace

int32_t csrec_cosamp_hermitian(const csrec_problem* problem, const csrec_cosamp_params* params, float* X,
                               int32_t* support, csrec_pixel_stats* stats) {
    GreedyLaunch l{};
    const int e = fill_cosamp_hermitian(problem, params, l);
    if (e) return e;
    return run_other_hermitian(l, problem, X, support, stats);
}

int32_t csrec_biht_hermitian(const csrec_problem* problem, const csrec_biht_params* params, float* X,
                             int32_t* support, csrec_pixel_stats* stats) {
    GreedyLaunch l{};
    const int e = fill_biht_hermitian(problem, params, l);
    if (e) return e;
    return run_other_hermitian(l, problem, X, support, stats);
}

}  // extern "C"

// The scratch of csrec_gomp_noalloc: one array per device, kept until the
// process ends.  In host code its name stands for the symbol, not a device
// address: every use goes through the address hipGetSymbolAddress returns
// for the current device, looked up once per device.
namespace {
constexpr size_t kNoallocScratchBytes = (size_t)CSREC_NOALLOC_SCRATCH_MB << 20;
static __device__ __align__(256) char csrec_noalloc_scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch (null and *err set on failure).
char* noalloc_scratch(int* err) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_hip_error(e);
        *err = CSREC_E_DEVICE;
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        *err = CSREC_E_DEVICE;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(csrec_noalloc_scratch));
        if (e != hipSuccess || !p) {
            set_hip_error(e);
            *err = CSREC_E_DEVICE;
            return nullptr;
        }
        g_scratch_ptr[dev] = static_cast<char*>(p);
    }
    return g_scratch_ptr[dev];
}
}  // namespace

extern "C" {

int32_t csrec_gomp_noalloc(const csrec_problem* problem, const csrec_gomp_params* params, float* X,
                           int32_t* support, csrec_pixel_stats* stats) {
    GreedyLaunch l{};
    int e = fill_gomp(problem, params, l);
    if (e) return e;
    fill_problem(problem, l);
    l.workspace = nullptr;
    l.workspace_bytes = 0;
    if (l.P > 0 && !X) return CSREC_E_INVAL;
    l.X = X;
    l.support = support;
    l.stats = stats;
    if (l.P == 0) return CSREC_OK;
    if (greedy_gomp_scratch_cols(l, kNoallocScratchBytes) < 0) return CSREC_E_WORKSPACE;
    char* scr = noalloc_scratch(&e);
    if (!scr) return e;
    return greedy_gomp_scratch_launch(l, scr, kNoallocScratchBytes);
}

int32_t csrec_cosamp(const csrec_problem* problem, const csrec_cosamp_params* params, float* X,
                     int32_t* support, csrec_pixel_stats* stats) {
    GreedyLaunch l{};
    int e = fill_cosamp(problem, params, l);
    if (e) return e;
    fill_problem(problem, l);
    return run_greedy(l, X, support, stats);
}

int32_t csrec_biht(const csrec_problem* problem, const csrec_biht_params* params, float* X,
                   int32_t* support, csrec_pixel_stats* stats) {
    GreedyLaunch l{};
    int e = fill_biht(problem, params, l);
    if (e) return e;
    fill_problem(problem, l);
    return run_greedy(l, X, support, stats);
}

int32_t csrec_admm(const csrec_problem* problem, const csrec_admm_params* params, float* X, float* Z,
                   csrec_pixel_stats* stats) {
    float thr = 0.f;
    int e = check_admm(problem, params, &thr);
    if (e) return e;
    if (problem->P == 0) return CSREC_OK;
    if (!X) return CSREC_E_INVAL;
    if (!problem->workspace || problem->workspace_bytes < admm_workspace(problem->M)) return CSREC_E_WORKSPACE;
    AdmmLaunch l{};
    l.A = problem->A;
    l.Y = problem->Y;
    l.X0 = params->X0;
    l.X = X;
    l.Z = Z;
    l.stats = stats;
    l.M = problem->M;
    l.N = problem->N;
    l.P = problem->P;
    l.max_iter = params->max_iter;
    l.alpha = params->alpha;
    l.thr = thr;
    l.eps = (float)params->eps;
    l.workspace = problem->workspace;
    l.stream = reinterpret_cast<hipStream_t>(problem->stream);
    return admm_launch(l);
}

int32_t csrec_fista_complex(const csrec_problem* problem, const csrec_fista_params* params, float* X,
                            csrec_pixel_stats* stats) {
    int e = check_fista_complex(problem, params);
    if (e) return e;
    if (problem->P == 0) return CSREC_OK;
    if (!X) return CSREC_E_INVAL;
    if (!problem->workspace || problem->workspace_bytes < fista_complex_workspace(problem->M, problem->N))
        return CSREC_E_WORKSPACE;
    FistaLaunch l{};
    l.A = problem->A;
    l.Y = problem->Y;
    l.X0 = params->X0;
    l.X = X;
    l.stats = stats;
    l.M = problem->M;
    l.N = problem->N;
    l.P = problem->P;
    l.max_iter = params->max_iter;
    l.eps = (float)params->eps;
    l.lambda = params->lambda;
    l.prec = CSREC_PREC_F32;
    l.workspace = problem->workspace;
    l.stream = reinterpret_cast<hipStream_t>(problem->stream);
    const bool power = !(params->L > 0.0);
    if (!power) {
        l.invL = (float)(1.0 / params->L);
        l.thr = (float)(params->lambda / params->L);
    }
    return fista_complex_launch(l, power);
}

int32_t csrec_fista_hermitian(const csrec_problem* problem, const csrec_fista_params* params, float* X,
                              csrec_pixel_stats* stats) {
    int e = check_fista_hermitian(problem, params);
    if (e) return e;
    if (problem->P == 0) return CSREC_OK;
    if (!X) return CSREC_E_INVAL;
    const bool power = !(params->L > 0.0);
    if (power && (!problem->workspace ||
                  problem->workspace_bytes < fista_hermitian_workspace(problem->M, problem->N, true)))
        return CSREC_E_WORKSPACE;
    FistaLaunch l{};
    l.A = problem->A;
    l.Y = problem->Y;
    l.X0 = params->X0;
    l.X = X;
    l.stats = stats;
    l.M = problem->M;
    l.N = problem->N;
    l.P = problem->P;
    l.max_iter = params->max_iter;
    l.eps = (float)params->eps;
    l.lambda = params->lambda;
    l.prec = CSREC_PREC_F32;
    l.workspace = problem->workspace;
    l.stream = reinterpret_cast<hipStream_t>(problem->stream);
    if (!power) {
        l.invL = (float)(1.0 / params->L);
        l.thr = (float)(params->lambda / params->L);
    }
    return fista_hermitian_launch(l, power);
}

int32_t csrec_admm_hermitian(const csrec_problem* problem, const csrec_admm_params* params, float* X, float* Z,
                             csrec_pixel_stats* stats) {
    float thr = 0.f;
    int e = check_admm_hermitian(problem, params, &thr);
    if (e) return e;
    if (problem->P == 0) return CSREC_OK;
    if (!X) return CSREC_E_INVAL;
    if (!problem->workspace || problem->workspace_bytes < admm_hermitian_workspace(problem->M, problem->N))
        return CSREC_E_WORKSPACE;
    AdmmLaunch l{};
    l.A = problem->A;
    l.Y = problem->Y;
    l.X0 = params->X0;
    l.X = X;
    l.Z = Z;
    l.stats = stats;
    l.M = problem->M;
    l.N = problem->N;
    l.P = problem->P;
    l.max_iter = params->max_iter;
    l.alpha = params->alpha;
    l.thr = thr;
    l.eps = (float)params->eps;
    l.workspace = problem->workspace;
    l.stream = reinterpret_cast<hipStream_t>(problem->stream);
    return admm_hermitian_launch(l);
}

int32_t csrec_admm_complex(const csrec_problem* problem, const csrec_admm_params* params, float* X, float* Z,
                           csrec_pixel_stats* stats) {
    float thr = 0.f;
    int e = check_admm_complex(problem, params, &thr);
    if (e) return e;
    if (problem->P == 0) return CSREC_OK;
    if (!X) return CSREC_E_INVAL;
    if (!problem->workspace || problem->workspace_bytes < admm_complex_workspace(problem->M, problem->N))
        return CSREC_E_WORKSPACE;
    AdmmLaunch l{};
    l.A = problem->A;
    l.Y = problem->Y;
    l.X0 = params->X0;
    l.X = X;
    l.Z = Z;
    l.stats = stats;
    l.M = problem->M;
    l.N = problem->N;
    l.P = problem->P;
    l.max_iter = params->max_iter;
    l.alpha = params->alpha;
    l.thr = thr;
    l.eps = (float)params->eps;
    l.workspace = problem->workspace;
    l.stream = reinterpret_cast<hipStream_t>(problem->stream);
    return admm_complex_launch(l);
}

int32_t csrec_sparsify(const float* Psi, const float* A, const float* F, int32_t M, int32_t N, int64_t P,
                       double T, int32_t std_ddof, float* Xs, float* Y, int32_t* kept, void* stream) {
    if (M < 1 || M >= N || N > CSREC_MAX_N || P < 0) return CSREC_E_SHAPE;
    if (std_ddof != 0 && std_ddof != 1) return CSREC_E_INVAL;
    if (!std::isfinite((float)T)) return CSREC_E_INVAL;
    if (P > 0 && (!Psi || !A || !F || !Xs || !Y)) return CSREC_E_INVAL;
    int e = sparsify_supported(M, N);
    if (e) return e;
    return sparsify_launch(Psi, A, F, M, N, P, (float)T, std_ddof, Xs, Y, kept, reinterpret_cast<hipStream_t>(stream));
}

int32_t csrec_sparsify_dft(const float* Psi, const float* A, const float* F, int32_t M, int32_t N, int64_t P,
                           double T, int32_t std_ddof, float* Xs, float* Y, int32_t* kept, void* stream) {
    if (M < 1 || M >= N || N > CSREC_MAX_N || P < 0) return CSREC_E_SHAPE;
    if (std_ddof != 0 && std_ddof != 1) return CSREC_E_INVAL;
    if (!std::isfinite((float)T)) return CSREC_E_INVAL;
    if (P > 0 && (!Psi || !A || !F || !Xs || !Y)) return CSREC_E_INVAL;
    int e = sparsify_dft_supported(M, N);
    if (e) return e;
    return sparsify_dft_launch(Psi, A, F, M, N, P, (float)T, std_ddof, Xs, Y, kept,
                               reinterpret_cast<hipStream_t>(stream));
}

int32_t csrec_lipschitz(const float* A, int32_t M, int32_t N, float* L_out, void* stream) {
    if (!A || !L_out) return CSREC_E_INVAL;
    if (M < 1 || M >= N || N > CSREC_MAX_N) return CSREC_E_SHAPE;
    return lipschitz_launch(A, M, N, L_out, reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
