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

// ---------------------------------------------------------------- the DFT basis
//
// With the unitary DFT basis (or any complex basis with conjugate-symmetric
// columns, Psi[:, N-k] = conj(Psi[:, k])) a real spectrum f has the
// conjugate-symmetric x = Psi^* f, x_{N-k} = conj(x_k).  Its half spectrum
// u (a_s = Re x_s in tile p, b_s = Im x_s in tile p + NTH, x_{N/2} in b-slot
// 0, as in the half-spectrum FISTA kernel) is T^T f for the real N x 2S
// half-spectrum matrix T of Psi (the conjugate of x_k contributes
// Re Psi[:, k] and -Im Psi[:, k]).  The statistics run over the N
// magnitudes |x_k| of the full spectrum: a pair (k, N-k) counts twice with
// |x_k| = |(a_k, b_k)|, x_0 and x_{N/2} once; a pair is kept or zeroed as a
// whole.  The measurements of the sparsified pixel, y = A x_s, are real:
// y = C (w u_s) with C the half-spectrum matrix of A (w = 2 on pairs, 1 on
// slot 0).  T streams through LDS in 16-row slices as Psi does above; C sits
// in LDS.

struct SparsifyDftArgs {
    const float* Psi;     // N x N complex
    const float* A;       // M x N complex
    const float* F;       // P x N real spectra
    float* Xs;            // P x N complex (full spectrum)
    float* Y;             // P x M real
    int32_t* kept;        // P, nullable
    int M, N, Ha;
    int64_t P;
    float T;
    int ddof;
};

template <int MT, int NTH, int WAVES>
__global__ __launch_bounds__(WAVES * 64, 1) void sparsify_dft_kernel(SparsifyDftArgs a) {
    constexpr int NT = 2 * NTH;                   // slot tiles; also the band tiles (N <= 32 NTH)
    constexpr int S = 16 * NTH;
    constexpr int PA = 16 * NT + 2;               // LDS row pitch (floats) of C and of the T slices
    constexpr int SLICE = 16 * PA;
    constexpr int THREADS = WAVES * 64;
    constexpr int STAGE = (SLICE + THREADS - 1) / THREADS;
    __shared__ float sA[16 * MT * PA];
    __shared__ float sP[2][SLICE];

    const int M = a.M, N = a.N, Ha = a.Ha;
    const int tid = threadIdx.x;
    for (int idx = tid; idx < 16 * MT * PA; idx += THREADS) {
        const int row = idx / PA, col = idx - (idx / PA) * PA;
        sA[idx] = col < 2 * S ? half_spectrum_entry(a.A, M, N, Ha, S, row, col) : 0.f;
    }
    // rows 16 kt .. 16 kt + 15 of T, zero beyond N
    float stage[STAGE];
    auto load_slice = [&](int kt) {
#pragma unroll
        for (int u = 0; u < STAGE; ++u) {
            const int idx = tid + THREADS * u;
            const int row = idx / PA, col = idx - (idx / PA) * PA;
            const int k = 16 * kt + row;
            stage[u] = (idx < SLICE && col < 2 * S) ? half_spectrum_entry(a.Psi, N, N, Ha, S, k, col) : 0.f;
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
    const bool h0 = h == 0;
    const bool even = !(N & 1);

    // a non-finite spectrum sparsifies to 0 (a first pass over f; the band
    // loop below reads f tile by tile, so no array of it is indexed by the
    // loop counter)
    int bad = 0;
    for (int k = cm_h; k < N; k += 16)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (valid && k + r < N && !isfinite(a.F[pix * N + k + r])) bad = 1;
    bad |= __shfl_xor(bad, 16);
    bad |= __shfl_xor(bad, 32);
    // band tile kt of f in the contraction layout (k = 16 kt + cm_h + r)
    auto load_f = [&](int kt) __attribute__((always_inline)) {
        v4f v;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int k = 16 * kt + cm_h + r;
            v[r] = (valid && !bad && k < N) ? a.F[pix * N + k] : 0.f;
        }
        return v;
    };
    v4f fk = load_f(0);
    __syncthreads();

    // u = T^T f, one 16-row slice of T per step
    v4f X[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) X[nt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < NT; ++kt) {
        v4f fn = {0.f, 0.f, 0.f, 0.f};
        if (kt + 1 < NT) {
            load_slice(kt + 1);
            fn = load_f(kt + 1);
        }
        const float* ps = sP[kt & 1] + cm_h * PA + nu_j;   // T[16 kt + cm_h + kk][16 nt + nu_j]
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                X[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ps[kk * PA + 16 * nt], fk[kk], X[nt], 0, 0, 0);
        if (kt + 1 < NT) store_slice((kt + 1) & 1);
        fk = fn;
        __syncthreads();
    }

    // |x_k| of the slot (the pair's, or slot 0's two real scalars) and its
    // multiplicity in the full spectrum
    auto mag_a = [&](int p, int r) __attribute__((always_inline)) {
        const int s = 16 * p + 4 * r + h;
        const float va = X[p][r], vb = X[p + NTH][r];
        return s == 0 ? fabsf(va) : sqrtf(va * va + vb * vb);
    };
    auto mult_a = [&](int p, int r) __attribute__((always_inline)) {
        const int s = 16 * p + 4 * r + h;
        return s == 0 ? 1.f : (s < Ha ? 2.f : 0.f);
    };
    // b-slot 0 (x_{N/2}), held by lane h = 0 in register 0 of tile NTH
    const float magN = fabsf(X[NTH][0]);
    const float multN = (h0 && even) ? 1.f : 0.f;

    float s1 = multN * magN;
#pragma unroll
    for (int p = 0; p < NTH; ++p)
#pragma unroll
        for (int r = 0; r < 4; ++r) s1 += mult_a(p, r) * mag_a(p, r);
    const float mu = quad_sum(s1) / (float)N;
    float s2 = multN * (magN - mu) * (magN - mu);
#pragma unroll
    for (int p = 0; p < NTH; ++p)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float d = mag_a(p, r) - mu;
            s2 += mult_a(p, r) * d * d;
        }
    const float sigma = sqrtf(quad_sum(s2) / (float)(N - a.ddof));
    const float tsig = a.T * sigma;

    // |x_k| - mu < T sigma -> 0 (a pair as a whole)
    float cnt = 0.f;
    const bool zeroN = multN == 0.f || bad || (magN - mu) - tsig < 0.f;
#pragma unroll
    for (int p = 0; p < NTH; ++p)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float m = mult_a(p, r);
            const bool zero = m == 0.f || bad || (mag_a(p, r) - mu) - tsig < 0.f;
            cnt += zero ? 0.f : m;
            if (p == 0 && r == 0) {
                // slot 0: x_0 in tile 0, x_{N/2} in tile NTH (lane h = 0)
                X[0][0] = zero ? 0.f : X[0][0];
                X[NTH][0] = h0 ? (zeroN ? 0.f : X[NTH][0]) : (zero ? 0.f : X[NTH][0]);
            } else {
                X[p][r] = zero ? 0.f : X[p][r];
                X[p + NTH][r] = zero ? 0.f : X[p + NTH][r];
            }
        }
    cnt += zeroN ? 0.f : multN;
    cnt = quad_sum(cnt);

    // y = C (w u_s)
    const float* a1 = sA + mu_j * PA + h;
    v4f Yr[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) Yr[mt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        v4f xw = X[nt] + X[nt];
        if (nt == 0 || nt == NTH) xw[0] = h0 ? X[nt][0] : xw[0];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                Yr[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[16 * mt * PA + 16 * nt + 4 * kk], xw[kk], Yr[mt],
                                                              0, 0, 0);
    }

    if (valid) {
        float* Xs = a.Xs + (size_t)pix * N * 2;
#pragma unroll
        for (int p = 0; p < NTH; ++p)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int s = 16 * p + 4 * r + h;
                const float va = X[p][r], vb = X[p + NTH][r];
                if (s == 0) {
                    Xs[0] = va;
                    Xs[1] = 0.f;
                    if (even) {
                        Xs[N] = vb;
                        Xs[N + 1] = 0.f;
                    }
                } else if (s < Ha) {
                    Xs[2 * s] = va;
                    Xs[2 * s + 1] = vb;
                    Xs[2 * (N - s)] = va;
                    Xs[2 * (N - s) + 1] = -vb;
                }
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

typedef void (*sparsify_dft_kernel_t)(SparsifyDftArgs);

struct SparsifyDftVariant {
    int MT, NTH;
    sparsify_dft_kernel_t fn;
};

// LDS: 4 (16 MT + 32) (32 NTH + 2) bytes, 132 KiB at (6, 8).
const SparsifyDftVariant kSparsifyDftVariants[] = {
    {1, 1, sparsify_dft_kernel<1, 1, kSparsifyWaves>}, {2, 2, sparsify_dft_kernel<2, 2, kSparsifyWaves>},
    {3, 4, sparsify_dft_kernel<3, 4, kSparsifyWaves>}, {4, 5, sparsify_dft_kernel<4, 5, kSparsifyWaves>},
    {5, 7, sparsify_dft_kernel<5, 7, kSparsifyWaves>}, {6, 7, sparsify_dft_kernel<6, 7, kSparsifyWaves>},
    {6, 8, sparsify_dft_kernel<6, 8, kSparsifyWaves>},
};

// band tiles (N <= 32 NTH) and half-spectrum slots (ceil(N/2) <= 16 NTH)
const SparsifyDftVariant* sparsify_dft_pick(int M, int N) {
    const int mt = (int)ceil_div(M, 16), nth = (int)ceil_div(N, 32);
    const SparsifyDftVariant* best = nullptr;
    for (const auto& v : kSparsifyDftVariants)
        if (v.MT >= mt && v.NTH >= nth && (!best || v.MT * v.NTH < best->MT * best->NTH)) best = &v;
    return best;
}

}  // namespace

int sparsify_supported(int M, int N) { return sparsify_pick(M, N) ? CSREC_OK : CSREC_E_UNSUPPORTED; }

int sparsify_dft_supported(int M, int N) { return sparsify_dft_pick(M, N) ? CSREC_OK : CSREC_E_UNSUPPORTED; }

int sparsify_dft_launch(const float* Psi, const float* A, const float* F, int M, int N, int64_t P, float T, int ddof,
                        float* Xs, float* Y, int32_t* kept, hipStream_t stream) {
    if (P == 0) return CSREC_OK;
    const SparsifyDftVariant* v = sparsify_dft_pick(M, N);
    if (!v) return CSREC_E_UNSUPPORTED;
    SparsifyDftArgs a;
    a.Psi = Psi;
    a.A = A;
    a.F = F;
    a.Xs = Xs;
    a.Y = Y;
    a.kept = kept;
    a.M = M;
    a.N = N;
    a.Ha = (N + 1) / 2;
    a.P = P;
    a.T = T;
    a.ddof = ddof;
    const int64_t blocks = ceil_div(P, 16 * kSparsifyWaves);
    if (blocks > 0x7fffffff) return CSREC_E_SHAPE;
    hipLaunchKernelGGL(v->fn, dim3((unsigned)blocks), dim3(64 * kSparsifyWaves), 0, stream, a);
    CSREC_HIP_TRY(hipGetLastError());
    return CSREC_OK;
}

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
