// Sparsification pre-stage (Section II) fused with the compression y = A x_s.
//
// For every pixel spectrum f (N bands): x = Psi^T f (Psi orthonormal,
// f = Psi x); mu, sigma = mean and standard deviation (N - ddof in the
// denominator) of the N magnitudes |x_n|; every x_n with
// |x_n| - mu < T sigma is set to zero; then the measurements of the
// sparsified pixel, y = A x_s (= Phi Psi x_s).
//
// One wavefront owns 16 pixels, with the MFMA register layouts of the FISTA
// kernel (lane l = 16 h + j, pixel j):
//   n = 16 t + 4 r + h                          (x, x_s: D layout of Psi^T f)
//   k = 16 t + 8 (h & 1) + 4 (h >> 1) + r       (f: B layout of Psi^T f)
//   m = 16 t + 8 (h & 1) + 4 (h >> 1) + r       (y: D layout of A x_s)
// Psi^T f contracts over the band index k; Psi (N x N, up to 256 KiB) does
// not fit in LDS beside A, so it streams through LDS in double-buffered
// slices of 16 rows, each slice read by every wave of the workgroup.  A sits
// in LDS for the second product.  The per-pixel statistics are two passes
// over the pixel's N registers (mean, then centred squares), each closed by
// a 4-lane reduction.
#include "common.hpp"

#include <cmath>

namespace csrec {
namespace {

struct SparsifyArgs {
    const float* Psi;     // N x N row-major, f = Psi x
    const float* A;       // M x N row-major
    const float* F;       // P x N spectra
    float* Xs;            // P x N sparsified coefficients
    float* Y;             // P x M measurements of the sparsified pixels
    int32_t* kept;        // P, nullable
    int M, N;
    int64_t P;
    float T;
    int ddof;
};

__device__ __forceinline__ float quad_sum(float v) {
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

template <int MT, int NT, int WAVES>
__global__ __launch_bounds__(WAVES * 64, 1) void sparsify_kernel(SparsifyArgs a) {
    constexpr int PA = 16 * NT + 2;               // LDS row pitch (floats) of A and of the Psi slices
    constexpr int SLICE = 16 * PA;
    constexpr int THREADS = WAVES * 64;
    constexpr int STAGE = (SLICE + THREADS - 1) / THREADS;
    __shared__ float sA[16 * MT * PA];
    __shared__ float sP[2][SLICE];

    const int M = a.M, N = a.N;
    const int tid = threadIdx.x;
    for (int idx = tid; idx < 16 * MT * PA; idx += THREADS) {
        const int row = idx / PA, col = idx - (idx / PA) * PA;
        sA[idx] = (row < M && col < N) ? a.A[(size_t)row * N + col] : 0.f;
    }
    // rows 16 kt .. 16 kt + 15 of Psi, zero beyond N
    float stage[STAGE];
    auto load_slice = [&](int kt) {
#pragma unroll
        for (int u = 0; u < STAGE; ++u) {
            const int idx = tid + THREADS * u;
            const int row = idx / PA, col = idx - (idx / PA) * PA;
            const int k = 16 * kt + row;
            stage[u] = (idx < SLICE && k < N && col < N) ? a.Psi[(size_t)k * N + col] : 0.f;
        }
    };
    auto store_slice = [&](int buf) {
#pragma unroll
        for (int u = 0; u < STAGE; ++u) {
            const int idx = tid + THREADS * u;
            if (idx < SLICE) sP[buf][idx] = stage[u];
        }
    };
    load_slice(0);
    store_slice(0);

    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int h = lane >> 4;
    const int j = lane & 15;
    const int64_t pix = ((int64_t)blockIdx.x * WAVES + wave) * 16 + j;
    const bool valid = pix < a.P;
    const int mu_j = 8 * ((j >> 2) & 1) + 4 * (j >> 3) + (j & 3);
    const int nu_j = 4 * (j & 3) + (j >> 2);
    const int cm_h = 8 * (h & 1) + 4 * (h >> 1);

    // f in the contraction layout; a non-finite spectrum sparsifies to 0
    v4f Fr[NT];
    int bad = 0;
#pragma unroll
    for (int kt = 0; kt < NT; ++kt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int k = 16 * kt + cm_h + r;
            float v = 0.f;
            if (valid && k < N) {
                v = a.F[pix * N + k];
                if (!isfinite(v)) bad = 1;
            }
            Fr[kt][r] = v;
        }
    bad |= __shfl_xor(bad, 16);
    bad |= __shfl_xor(bad, 32);
    if (bad) {
#pragma unroll
        for (int kt = 0; kt < NT; ++kt) Fr[kt] = v4f{0.f, 0.f, 0.f, 0.f};
    }
    __syncthreads();

    // x = Psi^T f, one 16-row slice of Psi per step
    v4f X[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) X[nt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < NT; ++kt) {
        if (kt + 1 < NT) load_slice(kt + 1);
        const float* ps = sP[kt & 1] + cm_h * PA + nu_j;   // Psi[16 kt + cm_h + kk][16 nt + nu_j]
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                X[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ps[kk * PA + 16 * nt], Fr[kt][kk], X[nt], 0, 0, 0);
        if (kt + 1 < NT) store_slice((kt + 1) & 1);
        __syncthreads();
    }

    // mu and sigma of |x| over the N bands
    float s1 = 0.f;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (16 * nt + 4 * r + h < N) s1 += fabsf(X[nt][r]);
    const float mu = quad_sum(s1) / (float)N;
    float s2 = 0.f;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (16 * nt + 4 * r + h < N) {
                const float d = fabsf(X[nt][r]) - mu;
                s2 += d * d;
            }
    const float sigma = sqrtf(quad_sum(s2) / (float)(N - a.ddof));
    const float tsig = a.T * sigma;

    // |x_n| - mu < T sigma -> 0
    float cnt = 0.f;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const bool in = 16 * nt + 4 * r + h < N;
            const bool zero = !in || bad || (fabsf(X[nt][r]) - mu) - tsig < 0.f;
            X[nt][r] = zero ? 0.f : X[nt][r];
            cnt += zero ? 0.f : 1.f;
        }
    cnt = quad_sum(cnt);

    // y = A x_s
    const float* a1 = sA + mu_j * PA + h;
    v4f Yr[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) Yr[mt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                Yr[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[16 * mt * PA + 16 * nt + 4 * kk], X[nt][kk], Yr[mt],
                                                              0, 0, 0);

    if (valid) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int n = 16 * nt + 4 * r + h;
                if (n < N) a.Xs[pix * N + n] = X[nt][r];
            }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = 16 * mt + cm_h + r;
                if (m < M) a.Y[pix * M + m] = Yr[mt][r];
            }
        if (a.kept && h == 0) a.kept[pix] = (int32_t)cnt;
    }
}

typedef void (*sparsify_kernel_t)(SparsifyArgs);

struct SparsifyVariant {
    int MT, NT;
    sparsify_kernel_t fn;
};

constexpr int kSparsifyWaves = 4;

// LDS: 4 (16 MT + 32) (16 NT + 2) bytes, 132 KiB at (6, 16).
const SparsifyVariant kSparsifyVariants[] = {
    {1, 2, sparsify_kernel<1, 2, kSparsifyWaves>},
    {2, 4, sparsify_kernel<2, 4, kSparsifyWaves>},
    {3, 7, sparsify_kernel<3, 7, kSparsifyWaves>},
    {4, 8, sparsify_kernel<4, 8, kSparsifyWaves>},
    {4, 10, sparsify_kernel<4, 10, kSparsifyWaves>},
    {5, 13, sparsify_kernel<5, 13, kSparsifyWaves>},
    {6, 14, sparsify_kernel<6, 14, kSparsifyWaves>},
    {6, 16, sparsify_kernel<6, 16, kSparsifyWaves>},
};

const SparsifyVariant* sparsify_pick(int M, int N) {
    const int mt = (int)ceil_div(M, 16), nt = (int)ceil_div(N, 16);
    const SparsifyVariant* best = nullptr;
    for (const auto& v : kSparsifyVariants)
        if (v.MT >= mt && v.NT >= nt && (!best || v.MT * v.NT < best->MT * best->NT)) best = &v;
    return best;
}

}  // namespace

int sparsify_supported(int M, int N) { return sparsify_pick(M, N) ? CSREC_OK : CSREC_E_UNSUPPORTED; }

int sparsify_launch(const float* Psi, const float* A, const float* F, int M, int N, int64_t P, float T, int ddof,
                    float* Xs, float* Y, int32_t* kept, hipStream_t stream) {
    if (P == 0) return CSREC_OK;
    const SparsifyVariant* v = sparsify_pick(M, N);
    if (!v) return CSREC_E_UNSUPPORTED;
    SparsifyArgs a;
    a.Psi = Psi;
    a.A = A;
    a.F = F;
    a.Xs = Xs;
    a.Y = Y;
    a.kept = kept;
    a.M = M;
    a.N = N;
    a.P = P;
    a.T = T;
    a.ddof = ddof;
    const int64_t blocks = ceil_div(P, 16 * kSparsifyWaves);
    if (blocks > 0x7fffffff) return CSREC_E_SHAPE;
    hipLaunchKernelGGL(v->fn, dim3((unsigned)blocks), dim3(64 * kSparsifyWaves), 0, stream, a);
    CSREC_HIP_TRY(hipGetLastError());
    return CSREC_OK;
}

}  // namespace csrec
