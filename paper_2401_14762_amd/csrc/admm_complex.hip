// ADMM (Alg. 2) with the complex DFT basis of Section II for real
// measurements: y = Phi f of a real spectrum, A = Phi Psi with
// conjugate-symmetric columns, A[:, N-k] = conj(A[:, k]).
//
// As for FISTA, every iterate from a conjugate-symmetric start stays
// conjugate-symmetric (for real y, A^* y and (A^* A + alpha I)^{-1} map
// conjugate-symmetric vectors to conjugate-symmetric ones, and the soft
// threshold on |x_k| keeps |x_k| = |x_{N-k}|), so the iteration runs on the
// half spectrum.  Here in the scaled coordinates u' = sqrt(w) u, with u the
// half-spectrum slots of the FISTA kernel (a_s = Re x_s in tile p,
// b_s = Im x_s in tile p + NTH, x_{N/2} in b-slot 0) and w = 2 for the pairs
// (k, N-k), 1 for x_0 and x_{N/2}:
//   ||x||^2 = ||u'||^2  and  A x = Ch u',  Ch = C diag(sqrt(w)),
// so step 1, the minimiser of ||y - A x||^2 / 2 + alpha ||x - z + w||^2 / 2,
// is the real step on Ch, and the real kernel's Woodbury form applies with
// R = (alpha I + Ch Ch^T)^{-1} (Ch Ch^T = A A^*, real).  Step 2's threshold
// tau on |x_k| becomes sqrt(2) tau on the pair |(a'_s, b'_s)| and tau on the
// two real scalars of slot 0.  Steps 3 and 4 are linear.
//
// Ch and R are formed once per call on the device (Ch from complex A, R in
// FP64 by the real kernel's Gram and Gauss-Jordan pass) and read into LDS.
// The MFMA layouts, the chained products and the W-holds-x trick of the last
// iteration are those of the real kernel; the tile loop runs over the pairs
// (p, p + NTH), and the next pair's Ch^T e is interleaved with this pair's
// Ch v.
//
// Complex y (CY).  The same kernel runs ADMM on the real embedding
// A' = [Re A, -Im A; Im A, Re A] (2M x 2N', N' = 16 NTH): A' [Re x; Im x] =
// [Re Ax; Im Ax], A'^T [Re u; Im u] = [Re A^*u; Im A^*u], ||x|| is the
// 2-norm of [Re x; Im x], and (alpha I + A' A'^T)^{-1} is the embedding of
// (alpha I + A A^*)^{-1}.  Re x_n and Im x_n again sit in tiles p and
// p + NTH; the threshold is tau on every pair, and there is no mirrored
// half.
#include "common.hpp"

#include <cmath>

namespace csrec {
namespace {

constexpr float kSqrt2 = 1.41421356237309515f;
constexpr float kRsqrt2 = 0.707106781186547573f;

struct AdmmHArgs {
    const float* Ch;      // M x 2S row-major (S = 16 NTH); CY: the embedding A'
    const float* R;       // M x M row-major, symmetric
    const float* Y;       // P x M real; CY: P x Mc complex (M = 2 Mc)
    const float* X0;      // P x N complex, nullable; real y: entries 0 .. floor(N/2) are read
    float* X;             // P x N complex
    float* Z;             // P x N complex, nullable
    csrec_pixel_stats* stats;
    int M, N, Ha, Mc;
    int64_t P;
    int max_iter;
    float alpha, thr, eps;
};

__device__ __forceinline__ float quad_sum(float v) {
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

// fwd(mt, nt)[kk] = Ch[16 mt + mu_j][16 nt + 4 kk + h]; bwd(nt, mt)[kk] =
// Ch[16 mt + cm_h + kk][16 nt + nu_j]; rr(mt, ms)[kk] = R[16 ms + cm_h + kk][16 mt + mu_j]
template <int MT, int NT>
struct OpsPre {
    const v4f* a1;
    const v4f* a2;
    const v4f* a3;
    __device__ __forceinline__ v4f fwd(int mt, int nt) const { return a1[(mt * NT + nt) * 64]; }
    __device__ __forceinline__ v4f bwd(int nt, int mt) const { return a2[(nt * MT + mt) * 64]; }
    __device__ __forceinline__ v4f rr(int mt, int ms) const { return a3[(mt * MT + ms) * 64]; }
};

template <int MT, int NT>
struct OpsSingle {
    static constexpr int PA = 16 * NT + 2;   // even pitches with odd halves: conflict free
    static constexpr int PR = 16 * MT + 2;
    const float* a1;
    const float* a2;
    const float* a3;
    __device__ __forceinline__ v4f fwd(int mt, int nt) const {
        v4f v;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) v[kk] = a1[16 * mt * PA + 16 * nt + 4 * kk];
        return v;
    }
    __device__ __forceinline__ v4f bwd(int nt, int mt) const {
        v4f v;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) v[kk] = a2[(16 * mt + kk) * PA + 16 * nt];
        return v;
    }
    __device__ __forceinline__ v4f rr(int mt, int ms) const {
        v4f v;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) v[kk] = a3[(16 * ms + kk) * PR + 16 * mt];
        return v;
    }
};

template <int MT, int NTH, bool CY, class Ops>
__device__ __forceinline__ void admm_h_body(const AdmmHArgs& a, const Ops& ops, int h, int j, int64_t pix) {
    constexpr int NT = 2 * NTH;
    const int M = a.M, N = a.N, Ha = a.Ha;
    const bool valid = pix < a.P;
    const int cm_h = 8 * (h & 1) + 4 * (h >> 1);
    const bool h0 = h == 0;

    v4f Rp[MT];   // r^{i-1}; r^0 = y
    int bad = 0;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int m = 16 * mt + cm_h + r;
            float v = 0.f;
            if (valid && m < M) {
                if constexpr (CY) {
                    const int mc = m < a.Mc ? m : m - a.Mc;
                    v = a.Y[((size_t)pix * a.Mc + mc) * 2 + (m < a.Mc ? 0 : 1)];
                } else {
                    v = a.Y[pix * M + m];
                }
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
            const v4f rv = ops.rr(mt, ms);
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                Q[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(rv[kk], Rp[ms][kk], Q[mt], 0, 0, 0);
        }
    }

    // z^0 = w^0 = x^0 in the scaled half-spectrum coordinates
    v4f Zr[NT], Wr[NT];
#pragma unroll
    for (int p = 0; p < NTH; ++p)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int s = 16 * p + 4 * r + h;
            float va = 0.f, vb = 0.f;
            if (CY) {
                if (a.X0 && valid && !bad && s < N) {
                    va = a.X0[((size_t)pix * N + s) * 2];
                    vb = a.X0[((size_t)pix * N + s) * 2 + 1];
                }
            } else if (a.X0 && valid && !bad) {
                if (s == 0) {
                    va = a.X0[(size_t)pix * N * 2];
                    if (!(N & 1)) vb = a.X0[((size_t)pix * N + N / 2) * 2];
                } else if (s < Ha) {
                    va = kSqrt2 * a.X0[((size_t)pix * N + s) * 2];
                    vb = kSqrt2 * a.X0[((size_t)pix * N + s) * 2 + 1];
                }
            }
            Zr[p][r] = va;
            Wr[p][r] = va;
            Zr[p + NTH][r] = vb;
            Wr[p + NTH][r] = vb;
        }

    // T = -Ch v^1 = Ch (w^0 - z^0) = 0
    v4f T[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) T[mt] = v4f{0.f, 0.f, 0.f, 0.f};

    bool active = valid && !bad;
    bool converged = false;
    int iters = 0;
    float last_d2 = __builtin_nanf("");
    const float alpha = a.alpha, thr = a.thr, thr_pair = CY ? a.thr : a.thr * kSqrt2;
    const bool check_eps = a.eps > 0.f;

    for (int it = 0; it < a.max_iter; ++it) {
        // keeps the LDS operand reads inside the loop (loop-invariant; hoisted
        // they would need all of Ch and R in registers)
        asm volatile("" ::: "memory");
        // e = q - R Ch v = q + R T
        v4f E[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            E[mt] = Q[mt];
#pragma unroll
            for (int ms = 0; ms < MT; ++ms) {
                const v4f rv = ops.rr(mt, ms);
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
        // Ch^T e of the pair (0, NTH); each later pair's is interleaved with
        // the previous pair's Ch v
        v4f Ga = {0.f, 0.f, 0.f, 0.f}, Gb = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const v4f b0 = ops.bwd(0, mt);
            const v4f b1 = ops.bwd(NTH, mt);
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                Ga = __builtin_amdgcn_mfma_f32_16x16x4f32(b0[kk], E[mt][kk], Ga, 0, 0, 0);
                Gb = __builtin_amdgcn_mfma_f32_16x16x4f32(b1[kk], E[mt][kk], Gb, 0, 0, 0);
            }
        }
#pragma unroll
        for (int p = 0; p < NTH; ++p) {
            const v4f GA = Ga, GB = Gb;
            v4f Va, Vb;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float xa = (Zr[p][r] - Wr[p][r]) + GA[r];                 // step 1
                const float xb = (Zr[p + NTH][r] - Wr[p + NTH][r]) + GB[r];
                const float ta = xa + Wr[p][r];
                const float tb = xb + Wr[p + NTH][r];
                // step 2 on the pair's magnitude (sqrt(2) tau in these coordinates)
                const float mag = sqrtf(ta * ta + tb * tb);
                const float sc = mag > thr_pair ? (mag - thr_pair) / mag : 0.f;
                float za = ta * sc, zb = tb * sc;
                if (!CY && p == 0 && r == 0) {
                    // slot 0: x_0 and x_{N/2}, two real scalars, threshold tau
                    za = h0 ? ta - __builtin_amdgcn_fmed3f(ta, -thr, thr) : za;
                    zb = h0 ? tb - __builtin_amdgcn_fmed3f(tb, -thr, thr) : zb;
                }
                const float wa = ta - za, wb = tb - zb;                          // step 3
                Va[r] = wa - za;
                Vb[r] = wb - zb;
                // a pixel's last iteration keeps x^i in place of w^i
                Zr[p][r] = active ? za : Zr[p][r];
                Zr[p + NTH][r] = active ? zb : Zr[p + NTH][r];
                Wr[p][r] = active ? (last ? xa : wa) : Wr[p][r];
                Wr[p + NTH][r] = active ? (last ? xb : wb) : Wr[p + NTH][r];
            }
            const bool more = p + 1 < NTH;
            if (more) {
                Ga = v4f{0.f, 0.f, 0.f, 0.f};
                Gb = v4f{0.f, 0.f, 0.f, 0.f};
            }
            const int pn = more ? p + 1 : p;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const v4f av0 = ops.fwd(mt, p);
                const v4f av1 = ops.fwd(mt, p + NTH);
                const v4f b0 = ops.bwd(pn, mt);
                const v4f b1 = ops.bwd(pn + NTH, mt);
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    T[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av0[kk], Va[kk], T[mt], 0, 0, 0);
                    if (more) Ga = __builtin_amdgcn_mfma_f32_16x16x4f32(b0[kk], E[mt][kk], Ga, 0, 0, 0);
                    T[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av1[kk], Vb[kk], T[mt], 0, 0, 0);
                    if (more) Gb = __builtin_amdgcn_mfma_f32_16x16x4f32(b1[kk], E[mt][kk], Gb, 0, 0, 0);
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

    // ||y - A x^I||: r^I for pixels that iterated, y - Ch u'^0 otherwise
    if (a.max_iter == 0) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const v4f av = ops.fwd(mt, nt);
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
        // back to x = u' / sqrt(w), the full spectrum: x_s = (a, b),
        // x_{N-s} = (a, -b); slot 0 gives x_0 and (N even) x_{N/2}
        float* X = a.X + (size_t)pix * N * 2;
        float* Zo = a.Z ? a.Z + (size_t)pix * N * 2 : nullptr;
#pragma unroll
        for (int p = 0; p < NTH; ++p)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int s = 16 * p + 4 * r + h;
                // a pixel that never iterated returns x^0 (0 when its y is not finite)
                const float xa = iters == 0 ? Zr[p][r] : Wr[p][r];
                const float xb = iters == 0 ? Zr[p + NTH][r] : Wr[p + NTH][r];
                const float za = Zr[p][r], zb = Zr[p + NTH][r];
                if (CY) {
                    if (s < N) {
                        X[2 * s] = xa;
                        X[2 * s + 1] = xb;
                        if (Zo) {
                            Zo[2 * s] = za;
                            Zo[2 * s + 1] = zb;
                        }
                    }
                } else if (s == 0) {
                    X[0] = xa;
                    X[1] = 0.f;
                    if (!(N & 1)) {
                        X[N] = xb;
                        X[N + 1] = 0.f;
                    }
                    if (Zo) {
                        Zo[0] = za;
                        Zo[1] = 0.f;
                        if (!(N & 1)) {
                            Zo[N] = zb;
                            Zo[N + 1] = 0.f;
                        }
                    }
                } else if (s < Ha) {
                    X[2 * s] = kRsqrt2 * xa;
                    X[2 * s + 1] = kRsqrt2 * xb;
                    X[2 * (N - s)] = kRsqrt2 * xa;
                    X[2 * (N - s) + 1] = -kRsqrt2 * xb;
                    if (Zo) {
                        Zo[2 * s] = kRsqrt2 * za;
                        Zo[2 * s + 1] = kRsqrt2 * zb;
                        Zo[2 * (N - s)] = kRsqrt2 * za;
                        Zo[2 * (N - s) + 1] = -kRsqrt2 * zb;
                    }
                }
            }
        if (a.stats && h == 0) {
            csrec_pixel_stats st;
            st.iters = iters;
            st.flags = bad ? CSREC_FLAG_NONFINITE : (converged ? CSREC_FLAG_CONVERGED : CSREC_FLAG_ITER_CAP);
            st.resid = bad ? 0.f : sqrtf(r2);
            st.delta = bad ? __builtin_nanf("") : sqrtf(last_d2);
            a.stats[pix] = st;
        }
    }
}

// PRE: Ch twice and R once in LDS in the operand order ((4 MT NTH + MT^2)
// KiB); otherwise each once with padded pitches.
template <int MT, int NTH, int WAVES, int MINW, bool PRE, bool CY>
__global__ __launch_bounds__(WAVES * 64, MINW) void admm_h32_kernel(AdmmHArgs a) {
    constexpr int NT = 2 * NTH;
    constexpr int NC = 16 * NT;   // columns of Ch
    const int M = a.M;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int h = lane >> 4;
    const int j = lane & 15;
    const int64_t pix = ((int64_t)blockIdx.x * WAVES + wave) * 16 + j;
    const int mu_j = 8 * ((j >> 2) & 1) + 4 * (j >> 3) + (j & 3);
    const int nu_j = 4 * (j & 3) + (j >> 2);
    const int cm_h = 8 * (h & 1) + 4 * (h >> 1);
    if constexpr (PRE) {
        constexpr int BA = MT * NT * 64;
        constexpr int BR = MT * MT * 64;
        __shared__ v4f sA1[BA];
        __shared__ v4f sA2[BA];
        __shared__ v4f sR3[BR];
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
                    for (int kk = 0; kk < 4; ++kk)
                        v1[kk] = row < M ? a.Ch[(size_t)row * NC + 16 * nt + 4 * kk + hh] : 0.f;
                }
                {
                    const int nt = blk / MT, mt = blk - (blk / MT) * MT;
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) {
                        const int row = 16 * mt + cm + kk;
                        v2[kk] = row < M ? a.Ch[(size_t)row * NC + 16 * nt + nu] : 0.f;
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
        const OpsPre<MT, NT> ops{sA1 + lane, sA2 + lane, sR3 + lane};
        admm_h_body<MT, NTH, CY>(a, ops, h, j, pix);
    } else {
        using O = OpsSingle<MT, NT>;
        constexpr int PA = O::PA, PR = O::PR, ROWS = 16 * MT;
        __shared__ float sA[ROWS * PA];
        __shared__ float sR[ROWS * PR];
        for (int idx = threadIdx.x; idx < ROWS * PA; idx += WAVES * 64) {
            const int row = idx / PA, col = idx - (idx / PA) * PA;
            sA[idx] = (row < M && col < NC) ? a.Ch[(size_t)row * NC + col] : 0.f;
        }
        for (int idx = threadIdx.x; idx < ROWS * PR; idx += WAVES * 64) {
            const int row = idx / PR, col = idx - (idx / PR) * PR;
            sR[idx] = (row < M && col < M) ? a.R[row * M + col] : 0.f;
        }
        __syncthreads();
        const O ops{sA + mu_j * PA + h, sA + cm_h * PA + nu_j, sR + cm_h * PR + mu_j};
        admm_h_body<MT, NTH, CY>(a, ops, h, j, pix);
    }
}

typedef void (*admm_h_kernel_t)(AdmmHArgs);

struct AHVariant {
    int MT, NTH;
    admm_h_kernel_t fn;    // real y, half spectrum
    admm_h_kernel_t fnc;   // complex y, embedding
};

#define ADMM_H_VARIANT(MT, NTH, MINW, PRE) \
    { MT, NTH, admm_h32_kernel<MT, NTH, 4, MINW, PRE, false>, admm_h32_kernel<MT, NTH, 4, MINW, PRE, true> }
const AHVariant kAHVariants[] = {
    ADMM_H_VARIANT(2, 2, 2, true),  ADMM_H_VARIANT(3, 4, 2, true),  ADMM_H_VARIANT(4, 5, 1, true),
    ADMM_H_VARIANT(5, 7, 1, false), ADMM_H_VARIANT(6, 7, 1, false), ADMM_H_VARIANT(6, 8, 1, false),
};
#undef ADMM_H_VARIANT

// rows: M (real y) or 2M (complex y); pairs: ceil(N/2) slots (real y) or N (complex y)
const AHVariant* ahpick_rows(int rows, int pairs) {
    const int mt = (int)ceil_div(rows, 16), nth = (int)ceil_div(pairs, 16);
    const AHVariant* best = nullptr;
    for (const auto& v : kAHVariants)
        if (v.MT >= mt && v.NTH >= nth && (!best || v.MT * v.NTH < best->MT * best->NTH)) best = &v;
    return best;
}

const AHVariant* ahpick(int M, int N) { return ahpick_rows(M, (N + 1) / 2); }

}  // namespace

int admm_hermitian_supported(int M, int N) { return ahpick(M, N) ? CSREC_OK : CSREC_E_UNSUPPORTED; }

// Ch (M x 2S floats), then R (M x M floats)
size_t admm_hermitian_workspace(int M, int N) {
    const AHVariant* v = ahpick(M, N);
    if (!v) return 0;
    return align_up((size_t)M * 2 * 16 * v->NTH * sizeof(float), 256) + align_up((size_t)M * M * sizeof(float), 256);
}

int admm_hermitian_launch(const AdmmLaunch& l) {
    if (l.P == 0) return CSREC_OK;
    const AHVariant* v = ahpick(l.M, l.N);
    if (!v) return CSREC_E_UNSUPPORTED;
    const int S = 16 * v->NTH;
    char* ws = static_cast<char*>(l.workspace);
    float* Ch = reinterpret_cast<float*>(ws);
    float* R = reinterpret_cast<float*>(ws + align_up((size_t)l.M * 2 * S * sizeof(float), 256));
    int e = herm_scaled_launch(l.A, l.M, l.N, S, Ch, l.stream);
    if (e) return e;
    if ((e = admm_prepare_launch(Ch, l.M, 2 * S, l.alpha, R, l.stream))) return e;
    AdmmHArgs a;
    a.Ch = Ch;
    a.R = R;
    a.Y = l.Y;
    a.X0 = l.X0;
    a.X = l.X;
    a.Z = l.Z;
    a.stats = l.stats;
    a.M = l.M;
    a.Mc = l.M;
    a.N = l.N;
    a.Ha = (l.N + 1) / 2;
    a.P = l.P;
    a.max_iter = l.max_iter;
    a.alpha = (float)l.alpha;
    a.thr = l.thr;
    a.eps = l.eps;
    const int64_t blocks = ceil_div(l.P, 16 * 4);
    if (blocks > 0x7fffffff) return CSREC_E_SHAPE;
    hipLaunchKernelGGL(v->fn, dim3((unsigned)blocks), dim3(64 * 4), 0, l.stream, a);
    CSREC_HIP_TRY(hipGetLastError());
    return CSREC_OK;
}

int admm_complex_supported(int M, int N) {
    return (2 * M <= 96 && ahpick_rows(2 * M, N)) ? CSREC_OK : CSREC_E_UNSUPPORTED;
}

// A' (2M x 2S floats), then R (2M x 2M floats)
size_t admm_complex_workspace(int M, int N) {
    const AHVariant* v = ahpick_rows(2 * M, N);
    if (!v) return 0;
    return align_up((size_t)2 * M * 2 * 16 * v->NTH * sizeof(float), 256) +
           align_up((size_t)4 * M * M * sizeof(float), 256);
}

int admm_complex_launch(const AdmmLaunch& l) {
    if (l.P == 0) return CSREC_OK;
    const AHVariant* v = ahpick_rows(2 * l.M, l.N);
    if (!v || 2 * l.M > 96) return CSREC_E_UNSUPPORTED;
    const int S = 16 * v->NTH;
    char* ws = static_cast<char*>(l.workspace);
    float* Ap = reinterpret_cast<float*>(ws);
    float* R = reinterpret_cast<float*>(ws + align_up((size_t)2 * l.M * 2 * S * sizeof(float), 256));
    int e = complex_embed_launch(l.A, l.M, l.N, S, Ap, l.stream);
    if (e) return e;
    if ((e = admm_prepare_launch(Ap, 2 * l.M, 2 * S, l.alpha, R, l.stream))) return e;
    AdmmHArgs a;
    a.Ch = Ap;
    a.R = R;
    a.Y = l.Y;
    a.X0 = l.X0;
    a.X = l.X;
    a.Z = l.Z;
    a.stats = l.stats;
    a.M = 2 * l.M;
    a.Mc = l.M;
    a.N = l.N;
    a.Ha = l.N;
    a.P = l.P;
    a.max_iter = l.max_iter;
    a.alpha = (float)l.alpha;
    a.thr = l.thr;
    a.eps = l.eps;
    const int64_t blocks = ceil_div(l.P, 16 * 4);
    if (blocks > 0x7fffffff) return CSREC_E_SHAPE;
    hipLaunchKernelGGL(v->fnc, dim3((unsigned)blocks), dim3(64 * 4), 0, l.stream, a);
    CSREC_HIP_TRY(hipGetLastError());
    return CSREC_OK;
}

}  // namespace csrec
