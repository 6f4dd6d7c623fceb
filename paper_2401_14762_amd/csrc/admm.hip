// ADMM (Alg. 2) for P independent LASSO problems (Eq. 2) sharing one A.
//
// Step 1 multiplies by (A^T A + alpha I)^{-1}, an N x N matrix.  By the
// matrix inversion lemma, with the M x M matrix R = (alpha I + A A^T)^{-1},
//   (A^T A + alpha I)^{-1} = (I - A^T R A) / alpha,
// and with q = R y and v = z^{i-1} - w^{i-1} step 1 becomes
//   x^i = v + A^T e,   e = q - R A v,
// because A^T R y = (A^T y - A^T R A A^T y) / alpha.  The same identity gives
// the residual of step 4 for free: A A^T R = I - alpha R, so
//   r^i = y - A x^i = alpha e
// and Delta = ||alpha e^i - r^{i-1}||_2 with r^0 = y.  An iteration therefore
// costs 4 M N + 2 M^2 flops per pixel (products A v, R t, A^T e), against
// 2 N^2 for a product with the N x N inverse plus 2 M N for the residual.
//
// R is formed once per call on the device in FP64 (Gram matrix of the rows
// of A, then Gauss-Jordan inversion, which needs no pivoting on a symmetric
// positive definite matrix) and stored as FP32, exactly symmetric.
//
// Work decomposition and MFMA mapping are those of the FISTA kernel: one
// wavefront owns 16 pixels for the whole solve, A and R sit in LDS, and the
// per-pixel vectors stay in VGPRs.  Lane l = 16 h + j holds, for pixel j,
//   n = 16 t + 4 r + h                               (z, w, x)
//   m = 16 t + 8 (h & 1) + 4 (h >> 1) + r            (q, t, e, r^{i-1})
// which is both the D layout of v_mfma_f32_16x16x4f32 and the B layout of
// the next product, so the three products chain register to register.  R is
// read through its symmetry, R[m][m'] = R[m'][m], which gives its operand
// reads the conflict-free pattern of the A^T reads.
#include "common.hpp"

#include <cmath>

namespace csrec {
namespace {

constexpr int ADMM_MAX_M = 96;

struct AdmmArgs {
    const float* A;
    const float* R;       // M x M row-major, symmetric
    const float* Y;
    const float* X0;
    float* X;
    float* Z;
    csrec_pixel_stats* stats;
    int M, N;
    int64_t P;
    int max_iter;
    float alpha, thr, eps;
};

__device__ __forceinline__ float quad_sum(float v) {
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

// R = (alpha I + A A^T)^{-1}, one workgroup of PREP_THREADS threads.
// Thread t owns the entries e = t + PREP_THREADS s of the M x M matrix in
// registers for the whole inversion; only the pivot row and column pass
// through LDS (double-buffered, one barrier per pivot).
constexpr int PREP_THREADS = 1024;
constexpr int PREP_SLOTS = (ADMM_MAX_M * ADMM_MAX_M + PREP_THREADS - 1) / PREP_THREADS;
constexpr int PREP_CH = 64;   // columns of A staged per pass of the Gram product

__global__ __launch_bounds__(PREP_THREADS) void admm_prepare_kernel(const float* __restrict__ A, int M, int N,
                                                                    double alpha, float* __restrict__ R) {
    __shared__ double G[ADMM_MAX_M * ADMM_MAX_M];
    __shared__ float sAc[ADMM_MAX_M * (PREP_CH + 1)];
    __shared__ double rowk[2][ADMM_MAX_M];
    __shared__ double colk[2][ADMM_MAX_M];
    const int tid = threadIdx.x;
    const int MM = M * M;
    int ei[PREP_SLOTS], ej[PREP_SLOTS];
    double g[PREP_SLOTS];
#pragma unroll
    for (int s = 0; s < PREP_SLOTS; ++s) {
        const int e = tid + PREP_THREADS * s;
        ei[s] = e < MM ? e / M : -1;
        ej[s] = e < MM ? e - (e / M) * M : -1;
        g[s] = 0.0;
    }
    // Gram matrix of the rows of A, PREP_CH columns at a time (the same
    // summation order for (i, j) and (j, i): exactly symmetric)
    for (int c0 = 0; c0 < N; c0 += PREP_CH) {
        const int nc = N - c0 < PREP_CH ? N - c0 : PREP_CH;
        __syncthreads();
        for (int idx = tid; idx < M * PREP_CH; idx += PREP_THREADS) {
            const int i = idx / PREP_CH, c = idx - (idx / PREP_CH) * PREP_CH;
            sAc[i * (PREP_CH + 1) + c] = c < nc ? A[(size_t)i * N + c0 + c] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < PREP_SLOTS; ++s) {
            if (ei[s] < 0) continue;
            const float* ai = sAc + ei[s] * (PREP_CH + 1);
            const float* aj = sAc + ej[s] * (PREP_CH + 1);
            double acc = 0.0;
            for (int c = 0; c < PREP_CH; ++c) acc += (double)ai[c] * (double)aj[c];
            g[s] += acc;
        }
    }
#pragma unroll
    for (int s = 0; s < PREP_SLOTS; ++s)
        if (ei[s] >= 0 && ei[s] == ej[s]) g[s] += alpha;
    // Gauss-Jordan, in place: after pivot k the pivoted rows/columns hold the
    // inverse of the leading block and the rest its Schur complement.
    for (int k = 0; k < M; ++k) {
        const int b = k & 1;
#pragma unroll
        for (int s = 0; s < PREP_SLOTS; ++s) {
            if (ei[s] == k) rowk[b][ej[s]] = g[s];
            if (ej[s] == k) colk[b][ei[s]] = g[s];
        }
        __syncthreads();
        const double inv = 1.0 / rowk[b][k];
#pragma unroll
        for (int s = 0; s < PREP_SLOTS; ++s) {
            const int i = ei[s], j = ej[s];
            if (i < 0) continue;
            if (i == k)
                g[s] = (j == k) ? inv : rowk[b][j] * inv;
            else if (j == k)
                g[s] = -colk[b][i] * inv;
            else
                g[s] -= colk[b][i] * rowk[b][j] * inv;
        }
    }
#pragma unroll
    for (int s = 0; s < PREP_SLOTS; ++s)
        if (ei[s] >= 0) G[ei[s] * M + ej[s]] = g[s];
    __syncthreads();
    for (int idx = tid; idx < MM; idx += PREP_THREADS) {
        const int i = idx / M, j = idx - (idx / M) * M;
        R[idx] = (float)(0.5 * (G[idx] + G[j * M + i]));
    }
}

template <int MT, int NT, int WAVES, int MINW>
__global__ __launch_bounds__(WAVES * 64, MINW) void admm_f32_kernel(AdmmArgs a) {
    constexpr int PA = 16 * NT + 2;   // LDS row pitch of A (floats)
    constexpr int PR = 16 * MT + 2;   // LDS row pitch of R
    constexpr int ROWS = 16 * MT;
    __shared__ float sA[ROWS * PA];
    __shared__ float sR[ROWS * PR];

    const int M = a.M, N = a.N;
    for (int idx = threadIdx.x; idx < ROWS * PA; idx += WAVES * 64) {
        const int row = idx / PA;
        const int col = idx - row * PA;
        sA[idx] = (row < M && col < N) ? a.A[(size_t)row * N + col] : 0.f;
    }
    for (int idx = threadIdx.x; idx < ROWS * PR; idx += WAVES * 64) {
        const int row = idx / PR;
        const int col = idx - row * PR;
        sR[idx] = (row < M && col < M) ? a.R[row * M + col] : 0.f;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int h = lane >> 4;
    const int j = lane & 15;
    const int64_t pix = ((int64_t)blockIdx.x * WAVES + wave) * 16 + j;
    const bool valid = pix < a.P;

    const int mu_j = 8 * ((j >> 2) & 1) + 4 * (j >> 3) + (j & 3);  // m of output row j (A v, R t)
    const int nu_j = 4 * (j & 3) + (j >> 2);                       // n of output row j (A^T e)
    const int cm_h = 8 * (h & 1) + 4 * (h >> 1);
    const float* a1 = sA + mu_j * PA + h;      // A[m][n]:  + 16 mt PA + 16 nt + 4 kk
    const float* a2 = sA + cm_h * PA + nu_j;   // A^T[n][m]: + (16 mt + kk) PA + 16 nt
    const float* a3 = sR + cm_h * PR + mu_j;   // R[m][m']:  + (16 mt' + kk) PR + 16 mt

    // ---- measurements, non-finite check
    v4f Rp[MT];   // r^{i-1}; r^0 = y
    int bad = 0;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int m = 16 * mt + cm_h + r;
            float v = 0.f;
            if (valid && m < M) {
                v = a.Y[pix * M + m];
                if (!isfinite(v)) bad = 1;
            }
            Rp[mt][r] = v;
        }
    bad |= __shfl_xor(bad, 16);
    bad |= __shfl_xor(bad, 32);
    if (bad) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) Rp[mt] = v4f{0.f, 0.f, 0.f, 0.f};
    }

    // q = R y
    v4f Q[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        Q[mt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ms = 0; ms < MT; ++ms)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                Q[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a3[(16 * ms + kk) * PR + 16 * mt], Rp[ms][kk], Q[mt],
                                                             0, 0, 0);
    }

    // z^0 = w^0 = x^0
    v4f Zr[NT], Wr[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int n = 16 * nt + 4 * r + h;
            float v = 0.f;
            if (a.X0 && valid && !bad && n < N) v = a.X0[pix * N + n];
            Zr[nt][r] = v;
            Wr[nt][r] = v;
        }

    // T = -A v^1 = A (w^0 - z^0) = 0
    v4f T[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) T[mt] = v4f{0.f, 0.f, 0.f, 0.f};

    bool active = valid && !bad;
    bool converged = false;
    int iters = 0;
    float last_d2 = __builtin_nanf("");
    const float alpha = a.alpha, thr = a.thr;
    const bool check_eps = a.eps > 0.f;

    for (int it = 0; it < a.max_iter; ++it) {
        // keeps the LDS operand reads inside the loop (they are loop-invariant,
        // and hoisting them would need every element of A and R in registers)
        asm volatile("" ::: "memory");
        // e = q - R A v = q + R T
        v4f E[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            E[mt] = Q[mt];
#pragma unroll
            for (int ms = 0; ms < MT; ++ms)
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    E[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a3[(16 * ms + kk) * PR + 16 * mt], T[ms][kk],
                                                                 E[mt], 0, 0, 0);
        }
        // step 4 ahead of the x update: r^i = alpha e, Delta = ||r^i - r^{i-1}||
        float d2 = 0.f;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float d = alpha * E[mt][r] - Rp[mt][r];
                d2 += d * d;
            }
        d2 = quad_sum(d2);
        const bool stop = check_eps && sqrtf(d2) < a.eps;
        const bool last = active && (stop || it + 1 == a.max_iter);

#pragma unroll
        for (int mt = 0; mt < MT; ++mt) T[mt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            // A^T e for 16 n-values of this tile
            v4f G = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    G = __builtin_amdgcn_mfma_f32_16x16x4f32(a2[(16 * mt + kk) * PA + 16 * nt], E[mt][kk], G, 0, 0,
                                                             0);
            v4f Vn;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float x = (Zr[nt][r] - Wr[nt][r]) + G[r];   // step 1
                const float zt = x + Wr[nt][r];
                const float zn = zt - __builtin_amdgcn_fmed3f(zt, -thr, thr);   // step 2: soft threshold
                const float wn = zt - zn;                          // step 3
                // a pixel's last iteration keeps x^i in place of w^i, which
                // no output needs: the frozen registers then hold x^I, z^I
                Vn[r] = wn - zn;
                Zr[nt][r] = active ? zn : Zr[nt][r];
                Wr[nt][r] = active ? (last ? x : wn) : Wr[nt][r];
            }
            // T = -A v of the next iteration, accumulated tile by tile
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    T[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[16 * mt * PA + 16 * nt + 4 * kk], Vn[kk], T[mt],
                                                                 0, 0, 0);
        }
        if (active) {
            iters = it + 1;
            last_d2 = d2;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) Rp[mt] = alpha * E[mt];
        }
        if (last) {
            active = false;
            converged = stop;
        }
        if (!__any(active)) break;
    }

    // ||y - A x^I||: r^I for pixels that iterated, y - A x^0 otherwise
    if (a.max_iter == 0) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    Rp[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[16 * mt * PA + 16 * nt + 4 * kk], -Zr[nt][kk],
                                                                  Rp[mt], 0, 0, 0);
    }
    float r2 = 0.f;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) r2 += Rp[mt][r] * Rp[mt][r];
    r2 = quad_sum(r2);

    if (valid) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int n = 16 * nt + 4 * r + h;
                if (n < N) {
                    // a pixel that never iterated returns x^0 (0 when its y is not finite)
                    a.X[pix * N + n] = iters == 0 ? Zr[nt][r] : Wr[nt][r];
                    if (a.Z) a.Z[pix * N + n] = Zr[nt][r];
                }
            }
        if (a.stats && h == 0) {
            csrec_pixel_stats s;
            s.iters = iters;
            s.flags = bad ? CSREC_FLAG_NONFINITE : (converged ? CSREC_FLAG_CONVERGED : CSREC_FLAG_ITER_CAP);
            s.resid = bad ? 0.f : sqrtf(r2);
            s.delta = bad ? __builtin_nanf("") : sqrtf(last_d2);
            a.stats[pix] = s;
        }
    }
}

// The same iteration with A (twice) and R in LDS pre-arranged in the MFMA
// operand order, as in the pre-arranged FISTA kernel: the four operand values
// a lane feeds to four consecutive MFMAs are 16 contiguous bytes (one
// ds_read_b128).  2 MT NT + MT^2 KiB of LDS: shapes with 2 MT NT + MT^2 <= 155.
template <int MT, int NT, int WAVES, int MINW>
__global__ __launch_bounds__(WAVES * 64, MINW) void admm_f32s_kernel(AdmmArgs a) {
    constexpr int BA = MT * NT * 64;
    constexpr int BR = MT * MT * 64;
    __shared__ v4f sA1[BA];   // [mt][nt][lane]: A[16 mt + mu_j][16 nt + 4 kk + h]
    __shared__ v4f sA2[BA];   // [nt][mt][lane]: A[16 mt + cm_h + kk][16 nt + nu_j]
    __shared__ v4f sR3[BR];   // [mt][ms][lane]: R[16 ms + cm_h + kk][16 mt + mu_j]

    const int M = a.M, N = a.N;
    for (int idx = threadIdx.x; idx < BA + BR; idx += WAVES * 64) {
        const int l = idx & 63;
        const int hh = l >> 4, jj = l & 15;
        const int mu = 8 * ((jj >> 2) & 1) + 4 * (jj >> 3) + (jj & 3);
        const int nu = 4 * (jj & 3) + (jj >> 2);
        const int cm = 8 * (hh & 1) + 4 * (hh >> 1);
        if (idx < BA) {
            const int blk = idx >> 6;
            v4f v1, v2;
            {
                const int mt = blk / NT, nt = blk - (blk / NT) * NT;
                const int row = 16 * mt + mu;
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int col = 16 * nt + 4 * kk + hh;
                    v1[kk] = (row < M && col < N) ? a.A[(size_t)row * N + col] : 0.f;
                }
            }
            {
                const int nt = blk / MT, mt = blk - (blk / MT) * MT;
                const int col = 16 * nt + nu;
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int row = 16 * mt + cm + kk;
                    v2[kk] = (row < M && col < N) ? a.A[(size_t)row * N + col] : 0.f;
                }
            }
            sA1[idx] = v1;
            sA2[idx] = v2;
        } else {
            const int blk = (idx - BA) >> 6;
            const int mt = blk / MT, ms = blk - (blk / MT) * MT;
            const int col = 16 * mt + mu;
            v4f v;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int row = 16 * ms + cm + kk;
                v[kk] = (row < M && col < M) ? a.R[row * M + col] : 0.f;
            }
            sR3[idx - BA] = v;
        }
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int h = lane >> 4;
    const int j = lane & 15;
    const int64_t pix = ((int64_t)blockIdx.x * WAVES + wave) * 16 + j;
    const bool valid = pix < a.P;

    const int mu_j = 8 * ((j >> 2) & 1) + 4 * (j >> 3) + (j & 3);  // m of output row j (A v, R t)
    const int nu_j = 4 * (j & 3) + (j >> 2);                       // n of output row j (A^T e)
    const int cm_h = 8 * (h & 1) + 4 * (h >> 1);
    const v4f* a1 = sA1 + lane;   // + (mt NT + nt) 64
    const v4f* a2 = sA2 + lane;   // + (nt MT + mt) 64
    const v4f* a3 = sR3 + lane;   // + (mt MT + ms) 64

    // ---- measurements, non-finite check
    v4f Rp[MT];   // r^{i-1}; r^0 = y
    int bad = 0;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int m = 16 * mt + cm_h + r;
            float v = 0.f;
            if (valid && m < M) {
                v = a.Y[pix * M + m];
                if (!isfinite(v)) bad = 1;
            }
            Rp[mt][r] = v;
        }
    bad |= __shfl_xor(bad, 16);
    bad |= __shfl_xor(bad, 32);
    if (bad) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) Rp[mt] = v4f{0.f, 0.f, 0.f, 0.f};
    }

    // q = R y
    v4f Q[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        Q[mt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ms = 0; ms < MT; ++ms) {
            const v4f rv = a3[(mt * MT + ms) * 64];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                Q[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(rv[kk], Rp[ms][kk], Q[mt], 0, 0, 0);
        }
    }

    // z^0 = w^0 = x^0
    v4f Zr[NT], Wr[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int n = 16 * nt + 4 * r + h;
            float v = 0.f;
            if (a.X0 && valid && !bad && n < N) v = a.X0[pix * N + n];
            Zr[nt][r] = v;
            Wr[nt][r] = v;
        }

    // T = -A v^1 = A (w^0 - z^0) = 0
    v4f T[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) T[mt] = v4f{0.f, 0.f, 0.f, 0.f};

    bool active = valid && !bad;
    bool converged = false;
    int iters = 0;
    float last_d2 = __builtin_nanf("");
    const float alpha = a.alpha, thr = a.thr;
    const bool check_eps = a.eps > 0.f;

    for (int it = 0; it < a.max_iter; ++it) {
        // keeps the LDS operand reads inside the loop (they are loop-invariant,
        // and hoisting them would need every element of A and R in registers)
        asm volatile("" ::: "memory");
        // e = q - R A v = q + R T
        v4f E[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            E[mt] = Q[mt];
#pragma unroll
            for (int ms = 0; ms < MT; ++ms) {
                const v4f rv = a3[(mt * MT + ms) * 64];
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    E[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(rv[kk], T[ms][kk], E[mt], 0, 0, 0);
            }
        }
        // step 4 ahead of the x update: r^i = alpha e, Delta = ||r^i - r^{i-1}||
        float d2 = 0.f;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float d = alpha * E[mt][r] - Rp[mt][r];
                d2 += d * d;
            }
        d2 = quad_sum(d2);
        const bool stop = check_eps && sqrtf(d2) < a.eps;
        const bool last = active && (stop || it + 1 == a.max_iter);

#pragma unroll
        for (int mt = 0; mt < MT; ++mt) T[mt] = v4f{0.f, 0.f, 0.f, 0.f};
        // A^T e of tile 0; tile nt + 1's is interleaved with tile nt's A v
        v4f Gn = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const v4f av = a2[mt * 64];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                Gn = __builtin_amdgcn_mfma_f32_16x16x4f32(av[kk], E[mt][kk], Gn, 0, 0, 0);
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            // A^T e for 16 n-values of this tile
            const v4f G = Gn;
            v4f Vn;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float x = (Zr[nt][r] - Wr[nt][r]) + G[r];   // step 1
                const float zt = x + Wr[nt][r];
                const float zn = zt - __builtin_amdgcn_fmed3f(zt, -thr, thr);   // step 2: soft threshold
                const float wn = zt - zn;                          // step 3
                // a pixel's last iteration keeps x^i in place of w^i, which
                // no output needs: the frozen registers then hold x^I, z^I
                Vn[r] = wn - zn;
                Zr[nt][r] = active ? zn : Zr[nt][r];
                Wr[nt][r] = active ? (last ? x : wn) : Wr[nt][r];
            }
            // T = -A v of the next iteration, accumulated tile by tile, with
            // the next tile's A^T e interleaved (its single accumulator chain
            // overlaps the MT independent ones of T)
            if (nt + 1 < NT) Gn = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const v4f av = a1[(mt * NT + nt) * 64];
                const v4f bv = a2[((nt + 1 < NT ? nt + 1 : nt) * MT + mt) * 64];
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    T[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[kk], Vn[kk], T[mt], 0, 0, 0);
                    if (nt + 1 < NT) Gn = __builtin_amdgcn_mfma_f32_16x16x4f32(bv[kk], E[mt][kk], Gn, 0, 0, 0);
                }
            }
        }
        if (active) {
            iters = it + 1;
            last_d2 = d2;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) Rp[mt] = alpha * E[mt];
        }
        if (last) {
            active = false;
            converged = stop;
        }
        if (!__any(active)) break;
    }

    // ||y - A x^I||: r^I for pixels that iterated, y - A x^0 otherwise
    if (a.max_iter == 0) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const v4f av = a1[(mt * NT + nt) * 64];
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    Rp[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[kk], -Zr[nt][kk], Rp[mt], 0, 0, 0);
            }
    }
    float r2 = 0.f;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) r2 += Rp[mt][r] * Rp[mt][r];
    r2 = quad_sum(r2);

    if (valid) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int n = 16 * nt + 4 * r + h;
                if (n < N) {
                    // a pixel that never iterated returns x^0 (0 when its y is not finite)
                    a.X[pix * N + n] = iters == 0 ? Zr[nt][r] : Wr[nt][r];
                    if (a.Z) a.Z[pix * N + n] = Zr[nt][r];
                }
            }
        if (a.stats && h == 0) {
            csrec_pixel_stats s;
            s.iters = iters;
            s.flags = bad ? CSREC_FLAG_NONFINITE : (converged ? CSREC_FLAG_CONVERGED : CSREC_FLAG_ITER_CAP);
            s.resid = bad ? 0.f : sqrtf(r2);
            s.delta = bad ? __builtin_nanf("") : sqrtf(last_d2);
            a.stats[pix] = s;
        }
    }
}

typedef void (*admm_kernel_t)(AdmmArgs);

struct AdmmVariant {
    int MT, NT, waves;
    admm_kernel_t fn;
};

// A and R together must fit in LDS: 4 (16 MT (16 NT + 2) + 16 MT (16 MT + 2))
// bytes, 136 KiB for the largest shape (M <= 96, N <= 256).
const AdmmVariant kAdmmVariants[] = {
    {1, 2, 4, admm_f32_kernel<1, 2, 4, 2>},
    {2, 4, 4, admm_f32_kernel<2, 4, 4, 2>},
    {3, 7, 4, admm_f32_kernel<3, 7, 4, 2>},
    {4, 8, 4, admm_f32_kernel<4, 8, 4, 2>},
    {4, 10, 4, admm_f32_kernel<4, 10, 4, 1>},
    {5, 13, 4, admm_f32_kernel<5, 13, 4, 1>},
    {6, 14, 4, admm_f32_kernel<6, 14, 4, 1>},
    {6, 16, 4, admm_f32_kernel<6, 16, 4, 1>},
};

const AdmmVariant kAdmmVariantsS[] = {
    {1, 2, 4, admm_f32s_kernel<1, 2, 4, 2>},
    {2, 4, 4, admm_f32s_kernel<2, 4, 4, 2>},
    {3, 7, 4, admm_f32s_kernel<3, 7, 4, 2>},
    {4, 8, 4, admm_f32s_kernel<4, 8, 4, 2>},
    {4, 10, 4, admm_f32s_kernel<4, 10, 4, 1>},
    {5, 13, 4, admm_f32s_kernel<5, 13, 4, 1>},
};

const AdmmVariant* admm_pick(int M, int N) {
    const int mt = (int)ceil_div(M, 16), nt = (int)ceil_div(N, 16);
    const AdmmVariant* best = nullptr;
    for (const auto& v : kAdmmVariants)
        if (v.MT >= mt && v.NT >= nt && (!best || v.MT * v.NT < best->MT * best->NT)) best = &v;
    for (const auto& v : kAdmmVariantsS)   // the pre-arranged form of the same tile shape, where it fits
        if (best && v.MT == best->MT && v.NT == best->NT) return &v;
    return best;
}

}  // namespace

int admm_supported(int M, int N) {
    if (M > ADMM_MAX_M || !admm_pick(M, N)) return CSREC_E_UNSUPPORTED;
    return CSREC_OK;
}

size_t admm_workspace(int M) { return align_up((size_t)M * M * sizeof(float), 256); }

int admm_prepare_launch(const float* A, int M, int N, double alpha, float* R, hipStream_t stream) {
    if (M > ADMM_MAX_M) return CSREC_E_UNSUPPORTED;
    hipLaunchKernelGGL(admm_prepare_kernel, dim3(1), dim3(PREP_THREADS), 0, stream, A, M, N, alpha, R);
    CSREC_HIP_TRY(hipGetLastError());
    return CSREC_OK;
}

int admm_launch(const AdmmLaunch& l) {
    if (l.P == 0) return CSREC_OK;
    const AdmmVariant* v = admm_pick(l.M, l.N);
    if (!v || l.M > ADMM_MAX_M) return CSREC_E_UNSUPPORTED;
    float* R = static_cast<float*>(l.workspace);
    int e = admm_prepare_launch(l.A, l.M, l.N, l.alpha, R, l.stream);
    if (e) return e;
    AdmmArgs a;
    a.A = l.A;
    a.R = R;
    a.Y = l.Y;
    a.X0 = l.X0;
    a.X = l.X;
    a.Z = l.Z;
    a.stats = l.stats;
    a.M = l.M;
    a.N = l.N;
    a.P = l.P;
    a.max_iter = l.max_iter;
    a.alpha = (float)l.alpha;
    a.thr = l.thr;
    a.eps = l.eps;
    const int64_t blocks = ceil_div(l.P, 16 * v->waves);
    if (blocks > 0x7fffffff) return CSREC_E_SHAPE;
    hipLaunchKernelGGL(v->fn, dim3((unsigned)blocks), dim3(64 * v->waves), 0, l.stream, a);
    CSREC_HIP_TRY(hipGetLastError());
    return CSREC_OK;
}

}  // namespace csrec
