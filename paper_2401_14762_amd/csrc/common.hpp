// Internal helpers shared by the HIP sources of libcsrec (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/csrec.h"

namespace csrec {

typedef float v4f __attribute__((ext_vector_type(4)));

// Records the last HIP error of the calling thread (see csrec_last_hip_error).
void set_hip_error(hipError_t e);

#define CSREC_HIP_TRY(expr)                     \
    do {                                        \
        hipError_t e_ = (expr);                 \
        if (e_ != hipSuccess) {                 \
            ::csrec::set_hip_error(e_);         \
            return CSREC_E_DEVICE;              \
        }                                       \
    } while (0)

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t a, size_t b) { return (a + b - 1) / b * b; }

// Entry (row, col) of the real M x 2S half-spectrum matrix of a complex
// M x N matrix A with conjugate-symmetric columns (S = 16 NTH, Ha = ceil(N/2)):
// columns [0, S) hold Re A[:, k] (k < Ha), column S holds Re A[:, N/2] (N
// even), columns S + s hold -Im A[:, s] (1 <= s < Ha); zero elsewhere.  With
// u the half-spectrum slots of a conjugate-symmetric x (a_s = Re x_s,
// b_s = Im x_s, x_{N/2} in b-slot 0), A x = C (w u) for w = 1 on x_0 and
// x_{N/2}, 2 on the pairs (k, N-k), and (Re, Im) of A^* v are C^T v for real v.
__device__ __forceinline__ float half_spectrum_entry(const float* __restrict__ A, int M, int N, int Ha, int S,
                                                    int row, int col) {
    if (row >= M) return 0.f;
    if (col < S) return col < Ha ? A[((size_t)row * N + col) * 2] : 0.f;
    const int s = col - S;
    if (s == 0) return (N & 1) ? 0.f : A[((size_t)row * N + N / 2) * 2];
    return s < Ha ? -A[((size_t)row * N + s) * 2 + 1] : 0.f;
}

// ---------------------------------------------------------------- launchers
// Each returns CSREC_OK or an error code; arguments are already validated.

struct FistaLaunch {
    const float* A;
    const float* Y;
    const float* X0;
    float* X;
    csrec_pixel_stats* stats;
    int M, N;
    int64_t P;
    int max_iter;
    float invL;           // 1 / L
    float thr;            // lambda / L
    float eps;
    const float* L_dev;   // device L when the host value is 0 (power iteration)
    double lambda;
    int prec;
    int correction_iters;
    void* workspace;
    hipStream_t stream;
};

int fista_supported(int M, int N, int prec);
size_t fista_workspace(int M, int N, int64_t P, int prec);
int fista_launch(const FistaLaunch& a);

int lipschitz_launch(const float* A, int M, int N, float* L_out, hipStream_t stream);

// Complex FISTA: A, Y, X0, X interleaved complex; invL / thr are used when
// `power` is false, otherwise L comes from a power iteration on the device.
int fista_complex_supported(int M, int N);
size_t fista_complex_workspace(int M, int N);
int fista_complex_launch(const FistaLaunch& a, bool power);
// Real y, conjugate-symmetric columns of A: the half-spectrum iteration.
int fista_hermitian_supported(int M, int N);
size_t fista_hermitian_workspace(int M, int N, bool power);
int fista_hermitian_launch(const FistaLaunch& a, bool power);
// A' = [Re A, -Im A; Im A, Re A] (2M x 2NP) of complex A (M x N)
int complex_embed_launch(const float* A, int M, int N, int NP, float* Ap, hipStream_t stream);
// Ch = C diag(sqrt(w)) (M x 2S) of the half-spectrum layout, S = 16 NTH
int herm_scaled_launch(const float* A, int M, int N, int S, float* Ch, hipStream_t stream);

struct AdmmLaunch {
    const float* A;
    const float* Y;
    const float* X0;
    float* X;
    float* Z;
    csrec_pixel_stats* stats;
    int M, N;
    int64_t P;
    int max_iter;
    double alpha;
    float thr;            // soft threshold of step 2
    float eps;
    void* workspace;      // >= admm_workspace(M) bytes: R = (alpha I + A A^T)^{-1}
    hipStream_t stream;
};

int admm_supported(int M, int N);
size_t admm_workspace(int M);
int admm_launch(const AdmmLaunch& a);
// R = (alpha I + A A^T)^{-1} (M x M) of an M x N matrix A
int admm_prepare_launch(const float* A, int M, int N, double alpha, float* R, hipStream_t stream);
// ADMM with the DFT basis on real y (half spectrum): A complex, X / Z complex
int admm_hermitian_supported(int M, int N);
size_t admm_hermitian_workspace(int M, int N);
int admm_hermitian_launch(const AdmmLaunch& a);
// ADMM with complex A and y (real embedding): A, Y, X0, X, Z complex
int admm_complex_supported(int M, int N);
size_t admm_complex_workspace(int M, int N);
int admm_complex_launch(const AdmmLaunch& a);

int sparsify_supported(int M, int N);
// Sparsification with a conjugate-symmetric complex basis (the DFT) of real
// spectra: Psi (N x N), A (M x N) complex; Xs (P x N) complex, Y real.
int sparsify_dft_supported(int M, int N);
int sparsify_dft_launch(const float* Psi, const float* A, const float* F, int M, int N, int64_t P, float T, int ddof,
                        float* Xs, float* Y, int32_t* kept, hipStream_t stream);
int sparsify_launch(const float* Psi, const float* A, const float* F, int M, int N, int64_t P, float T, int ddof,
                    float* Xs, float* Y, int32_t* kept, hipStream_t stream);

enum GreedyKind { GREEDY_GOMP = 0, GREEDY_COSAMP = 1, GREEDY_BIHT = 2, GREEDY_BIHT_ONE_BIT = 3 };

struct GreedyLaunch {
    GreedyKind kind;
    const float* A;
    const float* Y;
    const int8_t* Ysign;
    float* X;
    int32_t* support;
    csrec_pixel_stats* stats;
    int M, N;
    int64_t P;
    int K, S, max_iter;
    int prune;
    int prec;
    float res_tol, eps, mu;
    double pivot_fallback;
    double redo_tol;      // FP32 error estimate above which gOMP redoes a pixel in FP64
    void* workspace;
    size_t workspace_bytes;
    hipStream_t stream;
};

// Largest support the least-squares state can hold.
constexpr int GREEDY_CMAX = 96;   // CoSaMP and BIHT: largest merged support (3K, 2K)
constexpr int GOMP_CMAX = 96;     // gOMP: largest |c| = S * max_iter

size_t greedy_workspace(const GreedyLaunch& a);
int greedy_launch(const GreedyLaunch& a);
// CoSaMP with 3K > M (minimum-norm least squares once |c| > M; FP64, no workspace)
int cosamp_wide_supported(int M, int N, int K);
int cosamp_wide_launch(const GreedyLaunch& a);
inline bool cosamp_is_wide(const GreedyLaunch& a) { return a.kind == GREEDY_COSAMP && 3 * a.K > a.M; }
// gOMP on a fixed device scratch of cap bytes (a.workspace is not used):
// FP64 redo columns that fit (-1: the shape does not fit), and the launch
int64_t greedy_gomp_scratch_cols(const GreedyLaunch& a, size_t cap);
int greedy_gomp_scratch_launch(const GreedyLaunch& a, char* scratch, size_t cap);

// Grouped gOMP launches over pixel chunks of several tiles (serving).
struct GreedyTileItem {
    const float* A;
    const float* dict;    // gomp_coop_prepare output for A
    const float* Y;
    float* X;
    int32_t* support;
    csrec_pixel_stats* stats;
    const float* G32;
    const double* G64;
    int M, N, max_iter;
    int64_t p0, np;
};
int greedy_mmax_class(int M);
size_t greedy_group_item_bytes();
// bytes of the host and device item tables of one grouped launch of nitems
size_t greedy_group_table_bytes(int nitems);
size_t greedy_group_workspace(const GreedyLaunch& proto_max, int64_t batch_pixels);
int greedy_group_launch(const GreedyLaunch& proto_max, const GreedyTileItem* items, int nitems,
                        int64_t batch_pixels, void* ws, void* table_host, void* table_dev, hipStream_t stream);
int greedy_gram(const float* A, int M, int N, float* G32, double* G64, hipStream_t stream);
// gOMP with the DFT basis on real measurements: a.A is M x N complex
// (conjugate-symmetric columns), a.Y real, a.X P x N complex, a.support P x 2K
// bins; K, S, max_iter count conjugate-pair groups.  Workspace: the real
// dictionary of the groups (M x pair_dict_atoms(N)), its Gram matrix and the
// on-chip kernel's copies.
int pair_dict_atoms(int Nb);
size_t greedy_hermitian_workspace(int M, int Nb);
int gomp_hermitian_launch(const GreedyLaunch& a);
// CoSaMP (Alg. 5) and BIHT (Alg. 4) in the same setting (a.kind)
int other_hermitian_launch(const GreedyLaunch& a);

// gOMP with the least-squares state on chip (16 lanes per pixel, MFMA
// correlation).  Every solve reads a per-dictionary buffer of
// gomp_coop_dict_floats(M, N) floats built once by gomp_coop_prepare.
int gomp_coop_mp(int M);
size_t gomp_coop_lds_floats(int MP, int CM, int K);
size_t gomp_coop_dict_floats(int M, int N);
int gomp_coop_supported(int M, int N, int K, int S, int Imax);
void gomp_coop_prepare(const float* A, int M, int N, float* dictbuf, hipStream_t stream);
// Nb > 0: conjugate-pair groups of a half-spectrum dictionary (N = 2 (Nb / 2 + 1)
// real atoms; K, S and Imax count groups; X is P x Nb complex, support P x 2K bins)
int gomp_coop_launch(const float* Y, float* X, int32_t* support, csrec_pixel_stats* stats, const float* G32,
                     const float* dictbuf, uint32_t* fbflag, int M, int N, int64_t p0, int64_t P, int K, int S,
                     int Imax, int prune, float res_tol, float eps, double pivot_thr, float redo_tol, int prec, hipStream_t stream,
                     int Nb = 0);
int gomp_coop_supported_grp(int M, int N, int K, int S, int Imax);
struct GompCoopItem {
    const float* dict;    // gomp_coop_prepare output for this item's A
    const float* Y;
    const float* G32;
    float* X;
    int32_t* support;
    csrec_pixel_stats* stats;
    uint32_t* fbflag;
    int M, N, max_iter;
    int64_t p0, np;
};
size_t gomp_coop_item_bytes();
size_t gomp_coop_table_extra();      // bytes after a grouped launch's items (its work cursor)
int gomp_coop_class(int M, int N);   // items of one grouped launch share it (0..3)
// CoSaMP (Alg. 5), BIHT (Alg. 4) and one-bit BIHT on the same on-chip design.
size_t coop_other_lds_floats(int kind, int M, int N, int K);
int coop_other_supported(int kind, int M, int N, int K);
// Nb > 0: conjugate-pair groups (as gomp_coop_launch); CoSaMP and BIHT REAL only
int coop_other_launch(int kind, const float* Y, const int8_t* Ysign, float* X, int32_t* support,
                      csrec_pixel_stats* stats, const float* G32, const float* dictbuf, int M, int N, int64_t p0,
                      int64_t P, int K, int Imax, float mu, float res_tol, float eps, int prec, hipStream_t stream,
                      int Nb = 0);
int coop_other_supported_grp(int kind, int M, int N, int K);
int gomp_coop_group_launch(const GompCoopItem* items, int nitems, void* table_host, void* table_dev, int K, int S,
                           int prune, float res_tol, float eps, double pivot_thr, float redo_tol, int prec,
                           hipStream_t stream);

}  // namespace csrec
