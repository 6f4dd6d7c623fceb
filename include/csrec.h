/*
 * csrec.h -- batched per-pixel sparse recovery of compressed hyperspectral
 * cubes on AMD Instinct MI355X (gfx950).
 *
 * Every pixel spectrum is measured as y = Phi f = Phi Psi x = A x with one
 * dictionary A (M x N, M < N) shared by all pixels (Section II, Eq. 1).  The
 * entry points recover the sparse coefficients x of all P pixels of a cube
 * at once with the paper's algorithms:
 *
 *   csrec_fista   FISTA for the LASSO of Eq. 2            (Alg. 1)
 *   csrec_gomp    generalised OMP                          (Alg. 3)
 *   csrec_biht    backtracking IHT (Alg. 4), or binary IHT on 1-bit
 *                 measurements (mode CSREC_BIHT_ONE_BIT; not from the paper)
 *   csrec_cosamp  CoSaMP                                   (Alg. 5)
 *   csrec_admm    ADMM for the LASSO of Eq. 2             (Alg. 2)
 *   csrec_fista_complex  FISTA for complex A and y (Alg. 1 with the
 *                 complex DFT basis of Section II)
 *   csrec_fista_hermitian  the same for real y and conjugate-symmetric A
 *                 (a real Phi with the DFT basis): half-spectrum iteration
 *   csrec_admm_hermitian   ADMM (Alg. 2) in the same setting
 *   csrec_admm_complex     ADMM (Alg. 2) for complex A and y
 *
 * and the pre-stage of the paper's evaluation protocol:
 *
 *   csrec_sparsify  sparsification of Section II and the compression y = A x_s
 *   csrec_sparsify_dft  the same with the complex DFT basis (real spectra)
 *
 * Layout.  A is M x N row-major FP32.  Y is P x M row-major FP32 (pixel
 * major: the measurements of one pixel are contiguous).  X is P x N
 * row-major FP32.  All of A, Y, X, support, stats and workspace are DEVICE
 * pointers owned by the caller; the library never keeps them past the call's
 * stream work and never frees them.
 *
 * Asynchrony.  Arguments are checked synchronously on the host; the work is
 * then enqueued on problem->stream (a hipStream_t; NULL = the null stream)
 * and the call returns.  The caller synchronises the stream before reading
 * results.  Calls on different streams with disjoint outputs and workspaces
 * may run concurrently.
 *
 * Workspace.  csrec_workspace_bytes() reports the device scratch a call
 * needs; the caller allocates it and passes it in problem->workspace.  The
 * solve path itself allocates no device memory.
 *
 * Errors.  Every entry point returns CSREC_OK or a negative CSREC_E_* code
 * and enqueues nothing when it fails.  Per-pixel events (non-convergence,
 * FP64 fallback, non-finite input) are not errors: they are reported in the
 * per-pixel stats flags; a pixel with a non-finite measurement gets x = 0.
 */
#ifndef CSREC_H
#define CSREC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CSREC_ABI_VERSION 2

/* return codes */
#define CSREC_OK             0
#define CSREC_E_INVAL       -1  /* null pointer, bad parameter value, struct_size mismatch */
#define CSREC_E_SHAPE       -2  /* M >= N, N > CSREC_MAX_N, M < 1, P < 0, or shape the solver cannot hold */
#define CSREC_E_WORKSPACE   -3  /* workspace missing or smaller than csrec_workspace_bytes() */
#define CSREC_E_DEVICE      -4  /* a HIP call failed; see csrec_last_hip_error() */
#define CSREC_E_UNSUPPORTED -5  /* precision / mode not available for this solver or shape */
#define CSREC_E_BUDGET      -6  /* serving: a tile needs more than the server's HBM budget */

/* arithmetic of the dictionary products */
#define CSREC_PREC_F32  0   /* FP32 everywhere */
#define CSREC_PREC_BF16 1   /* BF16 operands on MFMA, FP32 accumulation and state */
#define CSREC_PREC_F16  2   /* FP16 operands on MFMA, FP32 accumulation and state */

/* gOMP's FP64 redo: default FP32 error-estimate threshold (csrec_gomp_params.redo_tol) */
#define CSREC_REDO_TOL_DEFAULT 1e-5

/* per-pixel flags (csrec_pixel_stats.flags) */
#define CSREC_FLAG_CONVERGED     1u  /* stopped by Delta < eps or the residual tolerance */
#define CSREC_FLAG_ITER_CAP      2u  /* ran max_iter iterations */
#define CSREC_FLAG_FP64_FALLBACK 4u  /* gOMP least squares redone in FP64 (pivot ratio) */
#define CSREC_FLAG_NONFINITE     8u  /* non-finite measurement: x = 0, no iterations */
#define CSREC_FLAG_FP32_LIMIT   16u  /* CoSaMP (FP32 path): a least-squares pivot ratio d / G_jj
                                        fell below 2^-20, so the FP32 solve on the merged support
                                        had no correct digit; the pixel stopped with the previous
                                        iterate (iters counts the iterations it completed) */

/* solver ids for csrec_workspace_bytes */
#define CSREC_SOLVER_FISTA  0
#define CSREC_SOLVER_GOMP   1
#define CSREC_SOLVER_COSAMP 2
#define CSREC_SOLVER_BIHT   3
#define CSREC_SOLVER_ADMM   4
#define CSREC_SOLVER_FISTA_COMPLEX 5
#define CSREC_SOLVER_FISTA_HERMITIAN 6
#define CSREC_SOLVER_ADMM_HERMITIAN 7
#define CSREC_SOLVER_ADMM_COMPLEX 8
#define CSREC_SOLVER_GOMP_HERMITIAN 9
#define CSREC_SOLVER_COSAMP_HERMITIAN 10
#define CSREC_SOLVER_BIHT_HERMITIAN 11

#define CSREC_MAX_N 256

/* gOMP prune placement (Alg. 3 step 3) */
#define CSREC_PRUNE_EACH  0  /* prune to K and re-solve in every iteration where |c| > K (Alg. 3 as printed) */
#define CSREC_PRUNE_FINAL 1  /* prune once after the loop (textbook gOMP) */

/* ADMM soft threshold (Alg. 2 step 2) */
#define CSREC_ADMM_THR_PAPER    0  /* lambda * alpha, as Alg. 2 prints it: the fixed point solves Eq. 2
                                      with l1 weight lambda * alpha^2 */
#define CSREC_ADMM_THR_STANDARD 1  /* lambda / alpha, scaled-form ADMM: solves Eq. 2 with weight lambda */

/* BIHT modes */
#define CSREC_BIHT_REAL    0 /* Alg. 4, backtracking IHT on real measurements Y */
#define CSREC_BIHT_ONE_BIT 1 /* binary IHT on int8 sign measurements Ysign */

/* One cube: P pixels, each y (M values) = A x (N values). */
typedef struct {
    int32_t struct_size;      /* sizeof(csrec_problem) */
    int32_t M, N;             /* 1 <= M < N <= CSREC_MAX_N */
    int64_t P;                /* pixels; 0 is a valid empty problem */
    const float* A;           /* device, M x N row-major */
    const float* Y;           /* device, P x M row-major (unused by BIHT ONE_BIT) */
    void* stream;             /* hipStream_t, NULL = null stream */
    void* workspace;          /* device scratch, >= csrec_workspace_bytes() */
    size_t workspace_bytes;
} csrec_problem;

/* Per-pixel result statistics (optional output, P entries). */
typedef struct {
    int32_t iters;            /* iterations run */
    uint32_t flags;           /* CSREC_FLAG_* */
    float resid;              /* ||y - A x||_2 of the returned x */
    float delta;              /* last Delta = ||r^i - r^{i-1}||_2 */
} csrec_pixel_stats;

/* Alg. 1.  Inputs y, A, x^0, L, lambda, eps (kappa is unused by FISTA). */
typedef struct {
    int32_t struct_size;      /* sizeof(csrec_fista_params) */
    int32_t max_iter;         /* >= 0; replaces the paper's wall-clock cap */
    double lambda;            /* >= 0, the l1 weight of Eq. 2 */
    double L;                 /* > 0: Lipschitz constant lambda_max(A^T A) (Eq. 2);
                                 0: the library estimates it on the device by power iteration */
    double eps;               /* a pixel stops after the iteration with Delta < eps; 0 disables */
    const float* X0;          /* device P x N starting point, NULL = 0 */
    int32_t prec;             /* CSREC_PREC_* */
    int32_t correction_iters; /* BF16/F16 only: FP32 iterations run after the low-precision
                                 ones, warm-started from their result (0 = none) */
} csrec_fista_params;

/* Alg. 3.  Inputs y, A, kappa (= K), G (= S), eps. */
typedef struct {
    int32_t struct_size;      /* sizeof(csrec_gomp_params) */
    int32_t K;                /* kappa: sparsity of the returned x, 1 <= K */
    int32_t S;                /* G: atoms added per iteration, 1 <= S <= 8 */
    int32_t max_iter;         /* 0 = min(K, floor(M / S)); S * max_iter <= min(M, 96) */
    double res_tol;           /* stop when ||r|| <= res_tol * ||y|| (0 disables) */
    double eps;               /* stop when Delta < eps (0 disables) */
    int32_t prune;            /* CSREC_PRUNE_EACH or CSREC_PRUNE_FINAL */
    int32_t prec;             /* precision of the correlation A^T r of step 1: CSREC_PREC_F32, or
                                 BF16 / F16 operands on MFMA with FP32 accumulation (r rounded to
                                 the format); the least squares, the prune and the residual stay in
                                 FP32, so x is the FP32 least-squares solution on the support the
                                 16-bit correlation selected */
    double pivot_fallback;    /* FP64 redo of a pixel when a Cholesky pivot ratio d_j / G_jj falls
                                 below this (e.g. 1e-6), or when the FP32 error estimate of its least
                                 squares on c, 2^-24 trace(G[c,c]) trace(G[c,c]^-1) / |c|, exceeds
                                 redo_tol (ill-conditioned supports, |c| near M); 0 disables both */
    double redo_tol;          /* >= 0; the FP32 error estimate that sends a pixel to the FP64 redo
                                 (0 = CSREC_REDO_TOL_DEFAULT); used only with pivot_fallback > 0.
                                 A smaller value redoes more pixels: at 1e-7 the supports near M of
                                 Section IV's operating points go to FP64 whole */
} csrec_gomp_params;

/* Alg. 5.  Inputs y, A, kappa (= K), eps. */
typedef struct {
    int32_t struct_size;      /* sizeof(csrec_cosamp_params) */
    int32_t K;                /* 1 <= K; 3K <= M (on-chip FP32 path, 3K <= 96), or 3K > M with
                                 3K <= min(N, 128) (the FP64 path: step 2's pseudo-inverse is the
                                 least-squares solution while |c| <= M and the minimum-norm solution
                                 of A(:, c) s = y once |c| > M; M <= 96) */
    int32_t max_iter;         /* >= 0 */
    double eps;               /* stop when Delta < eps (0 disables) */
    double res_tol;           /* stop when ||r|| <= res_tol * ||y|| (0 disables) */
    int32_t prec;             /* precision of the correlation A^T r (as csrec_gomp_params.prec; the
                                 first correlation, A^T y, the least-squares right-hand sides, is FP32);
                                 3K > M: CSREC_PREC_F32 only (that path computes in FP64) */
} csrec_cosamp_params;

/* Alg. 4 (REAL) or binary IHT (ONE_BIT).  Inputs y, A, kappa (= K), mu, eps. */
typedef struct {
    int32_t struct_size;      /* sizeof(csrec_biht_params) */
    int32_t K;                /* REAL: 1 <= K, 2K <= min(M, 96);  ONE_BIT: 1 <= K <= min(N, 64) */
    int32_t max_iter;         /* >= 0 */
    double mu;                /* gradient step (0.1 in Section IV) */
    double eps;               /* REAL: stop when Delta < eps (0 disables) */
    double res_tol;           /* REAL: stop when ||r|| <= res_tol * ||y|| (0 disables) */
    int32_t mode;             /* CSREC_BIHT_REAL or CSREC_BIHT_ONE_BIT */
    const int8_t* Ysign;      /* ONE_BIT: device P x M signs in {-1, +1}; REAL: ignored */
    int32_t prec;             /* precision of the correlation (as csrec_cosamp_params.prec; ONE_BIT
                                 has no least squares: its x carries the 16-bit rounding) */
} csrec_biht_params;

/* Alg. 2.  Inputs y, A, x^0, lambda, alpha, eps (kappa is unused by ADMM).
 * Initialisation z^0 = w^0 = x^0, r^0 = y; each iteration runs steps 1-4 and
 * a pixel stops after the iteration with Delta = ||r^i - r^{i-1}|| < eps. */
typedef struct {
    int32_t struct_size;      /* sizeof(csrec_admm_params) */
    int32_t max_iter;         /* >= 0; replaces the paper's wall-clock cap */
    double lambda;            /* >= 0 */
    double alpha;             /* > 0: the penalty of the augmented Lagrangian (1.8 in Section IV) */
    double eps;               /* 0 disables the Delta stop */
    const float* X0;          /* device P x N starting point, NULL = 0 */
    int32_t threshold;        /* CSREC_ADMM_THR_PAPER or CSREC_ADMM_THR_STANDARD */
} csrec_admm_params;

/* Library version and ABI. */
int32_t csrec_abi_version(void);
const char* csrec_strerror(int32_t code);
/* Last HIP error code seen by this thread (0 = none). */
int32_t csrec_last_hip_error(void);

/* Device scratch (bytes) a solve of `solver` on `problem` with `params` needs.
 * params points to the solver's params struct.  Returns CSREC_OK or an error
 * for invalid arguments; *bytes may be 0. */
int32_t csrec_workspace_bytes(int32_t solver, const csrec_problem* problem, const void* params,
                              size_t* bytes);

/* FISTA (Alg. 1): X (P x N) receives x^I; stats nullable. */
int32_t csrec_fista(const csrec_problem* problem, const csrec_fista_params* params, float* X,
                    csrec_pixel_stats* stats);

/* gOMP (Alg. 3): X (P x N) receives the K-sparse x; support (P x K int32, nullable) the
 * indices of its atoms in ascending order, -1 padded; stats nullable. */
int32_t csrec_gomp(const csrec_problem* problem, const csrec_gomp_params* params, float* X,
                   int32_t* support, csrec_pixel_stats* stats);

/* CoSaMP (Alg. 5): outputs as csrec_gomp.  With 3K > M the merged support can
 * hold more atoms than measurements; that case runs one pixel per workgroup in
 * FP64 and needs no workspace (csrec_workspace_bytes reports 0). */
int32_t csrec_cosamp(const csrec_problem* problem, const csrec_cosamp_params* params, float* X,
                     int32_t* support, csrec_pixel_stats* stats);

/* BIHT (Alg. 4 / binary IHT): outputs as csrec_gomp.  ONE_BIT returns x / ||x||. */
int32_t csrec_biht(const csrec_problem* problem, const csrec_biht_params* params, float* X,
                   int32_t* support, csrec_pixel_stats* stats);

/* gOMP (Alg. 3) with the complex DFT basis of Section II for REAL
 * measurements (a real Phi, real spectra): A = Phi Psi is M x N complex with
 * conjugate-symmetric columns, A[:, N-k] = conj(A[:, k]), so that for every
 * real residual r the correlations p = A^* r of bins k and N-k have equal
 * magnitude, and the least squares on a support closed under k <-> N-k keeps
 * x conjugate-symmetric.  The bins {k, N-k} are therefore selected, kept and
 * pruned together: params->K, S and max_iter count conjugate-pair groups
 * ({0}, {k, N-k} for 0 < k < N/2, {N/2} for even N), the score of a group is
 * |p_k|, the prune keeps the K groups of largest |x_k|.  max_iter 0 means
 * min(K, floor(M / (2 S))) (a pair holds two real unknowns); 2 S max_iter <=
 * min(M, 96), 2 K <= 96.  pivot_fallback must be 0 (CSREC_E_UNSUPPORTED
 * otherwise); prec as csrec_gomp.
 *
 * problem->A is M x N complex (interleaved (re, im) FP32 pairs; only columns
 * 0 .. floor(N/2) are read, and A[:, 0] (and A[:, N/2], N even) are taken as
 * real); problem->Y is P x M REAL.  X (P x N complex) receives the full
 * conjugate-symmetric x; support (P x 2K int32, nullable) its bins in
 * ascending order, -1 padded; stats as csrec_gomp.  Needs the workspace of
 * csrec_workspace_bytes(CSREC_SOLVER_GOMP_HERMITIAN, ...): the real M x
 * 2 (floor(N/2) + 1) dictionary of the groups, its Gram matrix and the
 * kernel's copies, formed on the device on every call.  M <= 96,
 * 2 (floor(N/2) + 1) <= CSREC_MAX_N. */
int32_t csrec_gomp_hermitian(const csrec_problem* problem, const csrec_gomp_params* params, float* X,
                             int32_t* support, csrec_pixel_stats* stats);

/* CoSaMP (Alg. 5) and backtracking IHT (Alg. 4) with the complex DFT basis
 * for REAL measurements, in the setting of csrec_gomp_hermitian: conjugate
 * pairs are the selection and prune units, params->K counts groups (CoSaMP
 * selects 2K groups and keeps K; BIHT selects K and keeps K), the scores are
 * |(A^* r)_k| (CoSaMP) and |x_k + mu (A^* r)_k| (BIHT), the merged support's
 * atoms at most 6K (CoSaMP) or 4K (BIHT) <= min(M, 96).  BIHT mode must be
 * CSREC_BIHT_REAL.  problem, X, support (P x 2K bins), stats and workspace
 * (csrec_workspace_bytes with CSREC_SOLVER_COSAMP_HERMITIAN /
 * CSREC_SOLVER_BIHT_HERMITIAN) as csrec_gomp_hermitian; prec as
 * csrec_cosamp / csrec_biht. */
int32_t csrec_cosamp_hermitian(const csrec_problem* problem, const csrec_cosamp_params* params, float* X,
                               int32_t* support, csrec_pixel_stats* stats);
int32_t csrec_biht_hermitian(const csrec_problem* problem, const csrec_biht_params* params, float* X,
                             int32_t* support, csrec_pixel_stats* stats);

/* gOMP (Alg. 3) without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  The same arguments and results as csrec_gomp
 * (bit-identical X, support and stats), but problem->workspace is not used:
 * the Gram matrices, the dictionary copies, the FP64 hand-off flags and the
 * FP64 redo state live in one fixed scratch array of
 * CSREC_NOALLOC_SCRATCH_MB MiB in device memory, one per device, held from
 * the first call on that device until the process ends.  Nothing in it must
 * start at zero: every call writes what it reads.  Pixels are solved in
 * chunks of up to 65,536, and the FP64 redo (pivot_fallback > 0) reuses as
 * many per-pixel state columns as fit.  CSREC_E_WORKSPACE when a shape needs
 * more than the scratch holds (the Gram matrices and flags, or 64 redo
 * columns).  All calls on one device share its scratch and keep the last
 * call's contents: calls that overlap on one device (two streams, two host
 * threads) race and give undefined results; serialise them. */
#define CSREC_NOALLOC_SCRATCH_MB 32
int32_t csrec_gomp_noalloc(const csrec_problem* problem, const csrec_gomp_params* params, float* X,
                           int32_t* support, csrec_pixel_stats* stats);

/* ADMM (Alg. 2): X (P x N) receives x^I, Z (P x N, nullable) z^I; stats nullable (resid is
 * ||y - A x^I||).  Needs a workspace of csrec_workspace_bytes() (the M x M matrix
 * (alpha I + A A^T)^{-1}, formed on the device in FP64 on every call).  FP32; M <= 96,
 * otherwise CSREC_E_UNSUPPORTED.  X may alias X0. */
int32_t csrec_admm(const csrec_problem* problem, const csrec_admm_params* params, float* X, float* Z,
                   csrec_pixel_stats* stats);

/* FISTA (Alg. 1) for the complex measurement model of Section II: with the
 * complex DFT basis, A = Phi Psi and x are complex; step 1 uses the conjugate
 * transpose A^*, and the soft threshold of step 2 shrinks the magnitude |x_n|
 * by lambda / L and keeps the phase (x_n = 0 when |x_n| <= lambda / L).
 * Delta and resid are the complex 2-norms.
 *
 * problem->A is M x N complex and problem->Y P x M complex; params->X0 (P x N
 * complex, nullable) and X (P x N complex) likewise.  Complex values are
 * interleaved (re, im) FP32 pairs, so A holds 2 M N floats.  params->L > 0
 * is lambda_max(A^* A); 0 estimates it on the device.  prec must be
 * CSREC_PREC_F32 and correction_iters 0.  Needs a workspace of
 * csrec_workspace_bytes(CSREC_SOLVER_FISTA_COMPLEX, ...) bytes (the real
 * 2M x 2N' embedding [Re A, -Im A; Im A, Re A] of A, N' >= N a multiple of
 * 16 chosen by the library, written on every call).  M <= 48 and N <= 128,
 * otherwise CSREC_E_UNSUPPORTED.  X may alias X0. */
int32_t csrec_fista_complex(const csrec_problem* problem, const csrec_fista_params* params, float* X,
                            csrec_pixel_stats* stats);

/* FISTA (Alg. 1) with the complex DFT basis of Section II for REAL
 * measurements: Phi real and the spectra real make y = Phi f real, and the
 * columns of A = Phi Psi conjugate-symmetric, A[:, N-k] = conj(A[:, k]).
 * Then every iterate of csrec_fista_complex started from a
 * conjugate-symmetric x^0 (0 is one) is conjugate-symmetric,
 * x_{N-k} = conj(x_k), and the library iterates on its half: the same x^I as
 * csrec_fista_complex up to rounding, with the work of a real FISTA on N
 * unknowns (the complex call iterates on 4 M N reals).
 *
 * problem->A is M x N complex (interleaved (re, im) FP32 pairs); only its
 * columns 0 .. floor(N/2) are read, and A[:, 0] (and A[:, N/2], N even) are
 * taken as real.  problem->Y is P x M REAL FP32.  params->X0 (P x N complex,
 * nullable) is read at entries 0 .. floor(N/2) only.  X (P x N complex)
 * receives the full conjugate-symmetric x^I.  params->L > 0 is
 * lambda_max(A^* A); 0 estimates it on the device (needs the workspace of
 * csrec_workspace_bytes(CSREC_SOLVER_FISTA_HERMITIAN, ...); none with L > 0).
 * prec must be CSREC_PREC_F32 and correction_iters 0.  M <= 96,
 * N <= CSREC_MAX_N.  X may alias X0. */
int32_t csrec_fista_hermitian(const csrec_problem* problem, const csrec_fista_params* params, float* X,
                              csrec_pixel_stats* stats);

/* ADMM (Alg. 2) with the complex DFT basis of Section II for REAL
 * measurements, the setting of csrec_fista_hermitian: step 1 with A^* (the
 * conjugate transpose), step 2's soft threshold on |x_k + w_k| (magnitude
 * shrunk, phase kept), threshold as params->threshold.  Every iterate from a
 * conjugate-symmetric x^0 is conjugate-symmetric, and the library iterates
 * on the half spectrum: the same x^I and z^I as the full complex iteration up
 * to rounding, with the work of a real ADMM on N unknowns.
 *
 * problem->A is M x N complex (interleaved (re, im) FP32 pairs); only its
 * columns 0 .. floor(N/2) are read, and A[:, 0] (and A[:, N/2], N even) are
 * taken as real.  problem->Y is P x M REAL FP32.  params->X0 (P x N complex,
 * nullable) is read at entries 0 .. floor(N/2).  X and Z (P x N complex, Z
 * nullable) receive the full conjugate-symmetric x^I and z^I; stats as
 * csrec_admm.  Needs the workspace of
 * csrec_workspace_bytes(CSREC_SOLVER_ADMM_HERMITIAN, ...): a real M x 2N'
 * matrix of the half-spectrum layout (N' >= ceil(N/2) a multiple of 16) and
 * the M x M matrix (alpha I + A A^*)^{-1}, formed on the device (the latter
 * in FP64) on every call.  M <= 96, N <= CSREC_MAX_N. */
int32_t csrec_admm_hermitian(const csrec_problem* problem, const csrec_admm_params* params, float* X, float* Z,
                             csrec_pixel_stats* stats);

/* ADMM (Alg. 2) for the complex measurement model of Section II (complex A
 * and y): step 1 with A^* (the conjugate transpose), step 2's soft threshold
 * on |x_n + w_n| (magnitude shrunk, phase kept).  A (M x N), Y (P x M),
 * params->X0, X and Z (P x N; X0, Z nullable) are complex, interleaved
 * (re, im) FP32 pairs; stats as csrec_admm.  Needs the workspace of
 * csrec_workspace_bytes(CSREC_SOLVER_ADMM_COMPLEX, ...): the real embedding
 * [Re A, -Im A; Im A, Re A] (2M x 2N' floats, N' >= N a multiple of 16) and
 * the 2M x 2M embedding of (alpha I + A A^*)^{-1}, formed on the device on
 * every call.  M <= 48, N <= 128, otherwise CSREC_E_UNSUPPORTED.  X may
 * alias X0. */
int32_t csrec_admm_complex(const csrec_problem* problem, const csrec_admm_params* params, float* X, float* Z,
                           csrec_pixel_stats* stats);

/* Sparsification (Section II) fused with the compression of the sparsified
 * pixels.  For each of the P spectra f (rows of F, P x N): x = Psi^T f, where
 * Psi (N x N row-major, f = Psi x) must be orthonormal; mu and sigma are the
 * mean and the standard deviation of the N values |x_n| (denominator
 * N - std_ddof: 1 is the sample form, 0 the population form); every x_n with
 * |x_n| - mu < T sigma is set to 0.  Writes Xs (P x N) = the sparsified x,
 * Y (P x M) = A Xs, and kept (P int32, nullable) = the entries kept.  A
 * spectrum with a non-finite value gives x_s = 0, y = 0, kept = 0.  Every
 * pointer is a device pointer; the decisions are taken in FP32.  Shapes as
 * csrec_problem, M <= 96.  No workspace. */
int32_t csrec_sparsify(const float* Psi, const float* A, const float* F, int32_t M, int32_t N, int64_t P,
                       double T, int32_t std_ddof, float* Xs, float* Y, int32_t* kept, void* stream);

/* Sparsification (Section II) with the complex DFT basis, fused with the
 * compression: for each real spectrum f (rows of F, P x N), x = Psi^* f,
 * where Psi (N x N complex) must be unitary with conjugate-symmetric
 * columns, Psi[:, N-k] = conj(Psi[:, k]) (the DFT), so that x is
 * conjugate-symmetric; mu and sigma are the mean and the standard deviation
 * of the N magnitudes |x_k| (denominator N - std_ddof); every x_k with
 * |x_k| - mu < T sigma is set to 0 (x_k and x_{N-k} share the decision).
 * Writes Xs (P x N complex) = the sparsified x, Y (P x M REAL) = A Xs for A
 * (M x N complex) with conjugate-symmetric columns (A = Phi Psi, Phi real;
 * Y is real), and kept (P int32, nullable) = the entries kept (of N).
 * Only columns 0 .. floor(N/2) of Psi and A are read.  Complex values are
 * interleaved (re, im) FP32 pairs; every pointer is a device pointer; the
 * decisions are taken in FP32.  A spectrum with a non-finite value gives
 * x_s = 0, y = 0, kept = 0.  Shapes as csrec_problem, M <= 96.  No
 * workspace. */
int32_t csrec_sparsify_dft(const float* Psi, const float* A, const float* F, int32_t M, int32_t N, int64_t P,
                           double T, int32_t std_ddof, float* Xs, float* Y, int32_t* kept, void* stream);

/* Lipschitz constant L = lambda_max(A^T A) of Eq. 2 by power iteration on the device:
 * writes one float to *L_out (device pointer) on `stream`. */
int32_t csrec_lipschitz(const float* A, int32_t M, int32_t N, float* L_out, void* stream);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of cube tiles (gOMP, Alg. 3).
 *
 * A server owns, on one device: a pool of `hbm_budget_bytes` for the tiles'
 * measurements and results, a batch workspace for `batch_pixels` pixels of
 * solver state, the registered dictionaries (A with its Gram matrix, resident
 * until destroy), a pinned host staging pool and a scheduler thread.
 *
 *   submit     the tile's measurements are copied into the pinned staging
 *              pool, or into pageable memory when the pool is full now;
 *   admission  tiles leave the arrival queue strictly in order when their
 *              device buffers (Y in; X, support, stats out) fit in the
 *              device pool; the input copy is enqueued at once and its
 *              staging freed when it has completed;
 *   batching   admitted tiles are cut into chunks of at most chunk_pixels;
 *              a batch takes chunks of any admitted tiles -- of any band
 *              count -- up to batch_pixels, and runs them as persistent
 *              grouped launches (one per parameter class and kernel
 *              variant): resident workgroups claim 4-pixel units of all the
 *              batch's tiles in admission order until none is left; two
 *              batches are in flight at most, so tiles admitted while one
 *              runs join the next;
 *   retirement a solved tile's results are copied into the pinned pool, or
 *              into pageable memory when it is full now; then its device
 *              buffers are freed.
 * No step waits for host memory, so every submitted tile finishes whatever
 * the caller does with polled results.  Each pixel's result depends only on
 * its own measurements, its dictionary and its tile's parameters: a tile's
 * result is bit-identical whether it runs alone or mixed with others.
 *
 * Threading: submit/poll/release/drain/stats may be called from any host
 * thread.  Host buffers passed to submit are copied before the call returns.
 * ---------------------------------------------------------------------- */
typedef struct csrec_server csrec_server;

typedef struct {
    int32_t struct_size;          /* sizeof(csrec_server_cfg) */
    int32_t device;               /* HIP device ordinal */
    size_t hbm_budget_bytes;      /* pool for admitted tiles (Y in, X/support/stats out) */
    int64_t batch_pixels;         /* pixels per batch (solver workspace capacity) */
    int64_t chunk_pixels;         /* largest piece of one tile in a batch */
    csrec_gomp_params gomp;       /* default parameters of a tile; their K, S and max_iter fix
                                     the batch workspace layout */
} csrec_server_cfg;

typedef struct {
    uint64_t tag;                 /* submit tag */
    int32_t status;               /* CSREC_OK or an error code */
    int32_t dict_id;
    int64_t P;
    int32_t N, K;
    const float* X;               /* host, P x N; valid until csrec_server_release(tag); NULL on error */
    const int32_t* support;       /* host, P x K */
    const csrec_pixel_stats* stats; /* host, P */
    double t_submit, t_admit, t_done; /* seconds since server creation */
} csrec_result;

/* Counters since creation.  Slot occupancy is mean_pixels_in_flight over
 * (2 x batch_pixels) (two batches in flight at most); pool occupancy is
 * mean_pool_bytes over hbm_budget_bytes. */
typedef struct {
    int32_t struct_size;          /* sizeof(csrec_server_stats), set by the caller */
    int64_t tiles_submitted, tiles_finished;
    int64_t batches, pixels_launched;
    int64_t host_in_pageable;     /* tiles whose measurements were staged in pageable memory */
    int64_t host_out_pageable;    /* tiles whose results went to pageable memory */
    double elapsed_s;             /* since creation */
    double busy_s;                /* time with at least one batch in flight */
    double mean_pixels_in_flight; /* time average of the pixels of the batches in flight */
    double mean_pool_bytes;       /* time average of the device pool bytes in use */
} csrec_server_stats;

/* Creates the server: allocates once its device pool (hbm_budget_bytes), its
 * batch workspace and a pinned host staging pool of min(max(budget, 64 MiB),
 * 4 GiB) for inputs and results, and starts its scheduler thread.  On an
 * error everything allocated so far is freed. */
int32_t csrec_server_create(const csrec_server_cfg* cfg, csrec_server** out);
/* Registers a dictionary (host A, M x N row-major, M <= 96); returns its id
 * (at most 64 dictionaries per server). */
int32_t csrec_server_add_dict(csrec_server* srv, const float* A_host, int32_t M, int32_t N, int32_t* dict_id);
/* Queues a tile of P pixels (host Y, P x M row-major) for dictionary dict_id.
 * params (nullable: the server's cfg.gomp) may change res_tol, eps, prune,
 * pivot_fallback (> 0 only on a server created with one) and max_iter (up to
 * the server's); K and S must be the server's (CSREC_E_UNSUPPORTED
 * otherwise).  CSREC_E_BUDGET if the tile alone exceeds the device pool;
 * CSREC_E_INVAL for a tag that is still queued, in flight, or polled and not
 * released. */
int32_t csrec_server_submit(csrec_server* srv, int32_t dict_id, const float* Y_host, int64_t P,
                            const csrec_gomp_params* params, uint64_t tag);
/* Moves up to max finished tiles into out; *n receives the count.  Their
 * results stay valid until csrec_server_release(tag). */
int32_t csrec_server_poll(csrec_server* srv, csrec_result* out, int32_t max, int32_t* n);
/* Frees the host results of a polled tile; its tag may then be reused. */
int32_t csrec_server_release(csrec_server* srv, uint64_t tag);
/* Blocks until every submitted tile has finished (results stay pollable). */
int32_t csrec_server_drain(csrec_server* srv);
/* Fills *stats (stats->struct_size set by the caller). */
int32_t csrec_server_get_stats(csrec_server* srv, csrec_server_stats* stats);
/* Waits for the submitted tiles, stops the scheduler and frees every
 * resource of the server. */
int32_t csrec_server_destroy(csrec_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* CSREC_H */
