// FISTA (Alg. 1) for the complex measurement model of Section II: with the
// DFT basis, A = Phi Psi (M x N) and x are complex, A^* is the conjugate
// transpose and the soft threshold shrinks |x_n| and keeps its phase.
//
// One kernel serves two entry points.  Both carry a real iterate in which
// the two parts of each complex unknown sit in tiles p and p + NTH with the
// same lane and register, so each lane holds the whole pair and the
// magnitude shrink is local; both multiply by one real matrix held in LDS
// (twice, pre-arranged in the MFMA operand order, where it fits; once with a
// padded pitch otherwise), and the next pair's transposed products are
// interleaved with this pair's forward products.
//
// Complex y: the real embedding
//   A' = [ Re A  -Im A ]   (2M x 2NP, column blocks of NP = 16 NTH),
//        [ Im A   Re A ]
// with A' [Re x; Im x] = [Re(A x); Im(A x)] and A'^T [Re u; Im u] =
// [Re(A^* u); Im(A^* u)]: the iteration is the real one on A' with the
// threshold on each (Re x_n, Im x_n).  ||r|| over the 2M real rows is the
// complex norm.  A' is written once per call into the workspace.
//
// Real y with conjugate-symmetric A: the half spectrum (below).
//
// Complex arrays are interleaved (re, im) FP32 pairs.
#include "common.hpp"

#include <cmath>

namespace csrec {
namespace {

__device__ __forceinline__ float quad_sum(float v) {
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

// A' from complex A (interleaved), zero in the padding columns N <= n < NP.
__global__ void embed_kernel(const float* __restrict__ A, int M, int N, int NP, float* __restrict__ Ap) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)2 * M * 2 * NP;
    if (idx >= total) return;
    const int row = (int)(idx / (2 * NP)), col = (int)(idx - (int64_t)row * 2 * NP);
    const int m = row < M ? row : row - M;
    const bool im_row = row >= M;
    const int n = col < NP ? col : col - NP;
    const bool im_col = col >= NP;
    float v = 0.f;
    if (n < N) {
        const float re = A[((size_t)m * N + n) * 2], im = A[((size_t)m * N + n) * 2 + 1];
        // [Re -Im; Im Re]
        v = im_row ? (im_col ? re : im) : (im_col ? -im : re);
    }
    Ap[idx] = v;
}

// ---------------------------------------------------------------- real y: the half spectrum
//
// When y is real and the columns of A are conjugate-symmetric,
// A[:, N-k] = conj(A[:, k]) with A[:, 0] (and A[:, N/2], N even) real -- the
// case A = Phi Psi of a real Phi with the DFT basis, whose measurements of a
// real spectrum are real -- every FISTA iterate started from a
// conjugate-symmetric x^0 stays conjugate-symmetric: A^* r of a real r is,
// the soft threshold keeps |x_k| = |x_{N-k}|, and A x is real.  The iteration
// is then carried on the half spectrum alone, N real unknowns u:
//   a-slot s < Ha = ceil(N/2):  a_s = Re x_s
//   b-slot 0:                   Re x_{N/2} (N even; nothing for odd N)
//   b-slot 1 <= s < Ha:         b_s = Im x_s
// with one real M x 2S matrix C (S = 16 NTH, a-slots in columns [0, S),
// b-slots in [S, 2S)): c_k = Re A[:, k] for a-slot k and the Nyquist column,
// -Im A[:, s] for b-slot s.  Then
//   A z = C (w u),  w = 1 for x_0 and x_{N/2}, 2 for the pairs (k, N-k),
//   (Re, Im) of A^* v = C^T v for real v,
// and the soft threshold acts on |x_s| = |(a_s, b_s)|, except in slot 0
// where a_0 and the Nyquist value are two real scalars.  The a- and b-slot
// of s sit in tiles p and p + NTH with the same lane and register, as in the
// complex kernel.  The weight 2 is exact in FP32.

struct HermArgs {
    const float* A;       // M x N complex (interleaved); columns 0 .. floor(N/2) are read
    const float* Ap;      // complex y: the embedding A' (M x 2S, M = 2 Mc)
    const float* Y;       // P x M real; complex y: P x Mc complex
    const float* X0;      // P x N complex, nullable; real y: entries 0 .. floor(N/2) are read
    float* X;             // P x N complex, written in full
    csrec_pixel_stats* stats;
    const float* L_dev;
    int M, N, Ha, Mc;
    int64_t P;
    int max_iter;
    float invL, thr, eps;
    double lambda;
};

// C[row][col] (S = 16 NTH), zero in the padding
__device__ __forceinline__ float herm_c(const float* __restrict__ A, int M, int N, int Ha, int S, int row, int col) {
    if (row >= M) return 0.f;
    if (col < S) return col < Ha ? A[((size_t)row * N + col) * 2] : 0.f;
    const int s = col - S;
    if (s == 0) return (N & 1) ? 0.f : A[((size_t)row * N + N / 2) * 2];
    return s < Ha ? -A[((size_t)row * N + s) * 2 + 1] : 0.f;
}

// C diag(sqrt(w)) for the power iteration: lambda_max of its Gram C w C^T is
// lambda_max(A A^*) = lambda_max(A^* A)
__global__ void herm_scaled_kernel(const float* __restrict__ A, int M, int N, int Ha, int S, float* __restrict__ Ch) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= M * 2 * S) return;
    const int row = idx / (2 * S), col = idx - row * 2 * S;
    const float v = herm_c(A, M, N, Ha, S, row, col);
    Ch[idx] = (col == 0 || col == S) ? v : v * 1.41421356237309515f;
}

// operand reads: fwd(mt, nt)[kk] = C[16 mt + mu_j][16 nt + 4 kk + h],
// bwd(nt, mt)[kk] = C[16 mt + cm_h + kk][16 nt + nu_j]
template <int MT, int NT>
struct OpsPre {
    const v4f* a1;
    const v4f* a2;
    __device__ __forceinline__ v4f fwd(int mt, int nt) const { return a1[(mt * NT + nt) * 64]; }
    __device__ __forceinline__ v4f bwd(int nt, int mt) const { return a2[(nt * MT + mt) * 64]; }
};

template <int NT>
struct OpsSingle {
    static constexpr int PA = 16 * NT + 2;   // even pitch with an odd half: conflict free for both reads
    const float* a1;
    const float* a2;
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
};

// YL: y kept in LDS (ysh: this wave's MT 64 v4f, each lane its own MT
// entries) instead of registers, and the scheduler held to one tile pair at a
// time: the eight-wave form.
template <int MT, int NTH, bool FREEZE, bool CY, class Ops, bool YL = false>
__device__ __forceinline__ void herm_body(const HermArgs& a, const Ops& ops, int h, int j, int64_t pix,
                                          v4f* ysh = nullptr) {
    constexpr int NT = 2 * NTH;
    const int M = a.M, N = a.N, Ha = a.Ha;
    float invL = a.invL, thr = a.thr;
    if (a.L_dev) {
        const float L = *a.L_dev;
        invL = 1.f / L;
        thr = (float)(a.lambda / (double)L);
    }
    const bool valid = pix < a.P;
    const int cm_h = 8 * (h & 1) + 4 * (h >> 1);
    const bool h0 = h == 0;

    v4f Yr[MT];
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
            Yr[mt][r] = v;
        }
    bad |= __shfl_xor(bad, 16);
    bad |= __shfl_xor(bad, 32);
    if (bad) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) Yr[mt] = v4f{0.f, 0.f, 0.f, 0.f};
    }

    // u^0 from the half of x^0
    v4f Xr[NT], Zr[NT];
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
                if (s < Ha) va = a.X0[((size_t)pix * N + s) * 2];
                if (s == 0) {
                    if (!(N & 1)) vb = a.X0[((size_t)pix * N + N / 2) * 2];
                } else if (s < Ha) {
                    vb = a.X0[((size_t)pix * N + s) * 2 + 1];
                }
            }
            Xr[p][r] = va;
            Zr[p][r] = va;
            Xr[p + NTH][r] = vb;
            Zr[p + NTH][r] = vb;
        }
    // w u of one tile: 2 u, except slot 0 (tile 0 / NTH, register 0, h = 0);
    // complex y: u itself
    auto wt = [&](const v4f& v, int p) {
        if constexpr (CY) return v;
        v4f o = v + v;
        if (p == 0) o[0] = h0 ? v[0] : o[0];
        return o;
    };

    v4f U1[MT], V[MT];
    v4f* const ylds = YL ? ysh + (threadIdx.x & 63) : nullptr;
    if constexpr (YL) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) ylds[mt * 64] = Yr[mt];
    }
    // y of tile mt inside the loop: from LDS (YL) or the registers
    auto yt = [&](int mt) -> v4f { if constexpr (YL) return ylds[mt * 64]; else return Yr[mt]; };
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) U1[mt] = -Yr[mt];
    if (a.X0) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const v4f xw = wt(Xr[nt], nt < NTH ? nt : nt - NTH);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const v4f av = ops.fwd(mt, nt);
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    U1[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[kk], xw[kk], U1[mt], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) V[mt] = U1[mt];

    bool active = valid && !bad;
    bool converged = false;
    int iters = 0;
    float last_d2 = __builtin_nanf("");
    double t = 1.0;
    float bprev = 0.f;
    const bool check_eps = a.eps > 0.f;

    for (int it = 0; it < a.max_iter; ++it) {
        // keeps the LDS operand reads inside the loop (loop-invariant; hoisted
        // they would need all of C in registers)
        asm volatile("" ::: "memory");
        const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));   // step 3
        const float bcur = (float)((t - 1.0) / tn);                  // step 4 coefficient
        t = tn;
        const float cp = 1.f + bprev;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) V[mt] = cp * U1[mt] - bprev * V[mt];
        v4f Un[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) Un[mt] = -yt(mt);

        v4f Wa = {0.f, 0.f, 0.f, 0.f}, Wb = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const v4f b0 = ops.bwd(0, mt);
            const v4f b1 = ops.bwd(NTH, mt);
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                Wa = __builtin_amdgcn_mfma_f32_16x16x4f32(b0[kk], V[mt][kk], Wa, 0, 0, 0);
                Wb = __builtin_amdgcn_mfma_f32_16x16x4f32(b1[kk], V[mt][kk], Wb, 0, 0, 0);
            }
        }
#pragma unroll
        for (int p = 0; p < NTH; ++p) {
            if constexpr (YL) __builtin_amdgcn_sched_barrier(0);
            const v4f Ga = Wa, Gb = Wb;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float va = Zr[p][r] - Ga[r] * invL;
                const float vb = Zr[p + NTH][r] - Gb[r] * invL;
                const float mag = sqrtf(va * va + vb * vb);
                const float sc = mag > thr ? (mag - thr) / mag : 0.f;
                float xa = va * sc, xb = vb * sc;
                if (!CY && p == 0 && r == 0) {
                    // slot 0: x_0 and x_{N/2} are real scalars
                    xa = h0 ? va - __builtin_amdgcn_fmed3f(va, -thr, thr) : xa;
                    xb = h0 ? vb - __builtin_amdgcn_fmed3f(vb, -thr, thr) : xb;
                }
                const float za = xa + bcur * (xa - Xr[p][r]);
                const float zb = xb + bcur * (xb - Xr[p + NTH][r]);
                const bool upd = !FREEZE || active;
                Xr[p][r] = upd ? xa : Xr[p][r];
                Xr[p + NTH][r] = upd ? xb : Xr[p + NTH][r];
                Zr[p][r] = upd ? za : Zr[p][r];
                Zr[p + NTH][r] = upd ? zb : Zr[p + NTH][r];
            }
            const bool more = p + 1 < NTH;
            if (more) {
                Wa = v4f{0.f, 0.f, 0.f, 0.f};
                Wb = v4f{0.f, 0.f, 0.f, 0.f};
            }
            const int pn = more ? p + 1 : p;
            const v4f xa = wt(Xr[p], p);
            const v4f xb = wt(Xr[p + NTH], p);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const v4f av0 = ops.fwd(mt, p);
                const v4f av1 = ops.fwd(mt, p + NTH);
                const v4f b0 = ops.bwd(pn, mt);
                const v4f b1 = ops.bwd(pn + NTH, mt);
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    Un[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av0[kk], xa[kk], Un[mt], 0, 0, 0);
                    if (more) Wa = __builtin_amdgcn_mfma_f32_16x16x4f32(b0[kk], V[mt][kk], Wa, 0, 0, 0);
                    Un[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av1[kk], xb[kk], Un[mt], 0, 0, 0);
                    if (more) Wb = __builtin_amdgcn_mfma_f32_16x16x4f32(b1[kk], V[mt][kk], Wb, 0, 0, 0);
                }
            }
        }

        // (without the stop only the last iteration's Delta is reported)
        float d2 = 0.f;
        if (FREEZE || it == a.max_iter - 1) {
            const float c0 = (it == 0 && a.X0) ? 1.f : 0.f;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const v4f y = yt(mt);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float ref = U1[mt][r] - c0 * (U1[mt][r] + y[r]);
                    const float d = Un[mt][r] - ref;
                    d2 += d * d;
                }
            }
            d2 = quad_sum(d2);
            if (active) last_d2 = d2;
        }
        if (active) iters = it + 1;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            V[mt] = U1[mt];
            U1[mt] = (!FREEZE || active) ? Un[mt] : U1[mt];
        }
        bprev = bcur;
        if (check_eps) {
            if (active && sqrtf(d2) < a.eps) {
                active = false;
                converged = true;
            }
            if (!__any(active)) break;
        }
    }

    float r2 = 0.f;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) r2 += U1[mt][r] * U1[mt][r];
    r2 = quad_sum(r2);

    if (valid) {
        // the full spectrum: x_s = (a, b) and x_{N-s} = (a, -b); slot 0 gives
        // x_0 = (a, 0) and, N even, x_{N/2} = (b-slot value, 0)
        float* X = a.X + (size_t)pix * N * 2;
#pragma unroll
        for (int p = 0; p < NTH; ++p)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int s = 16 * p + 4 * r + h;
                const float va = bad ? 0.f : Xr[p][r], vb = bad ? 0.f : Xr[p + NTH][r];
                if (CY) {
                    if (s < N) {
                        X[2 * s] = va;
                        X[2 * s + 1] = vb;
                    }
                } else if (s == 0) {
                    X[0] = va;
                    X[1] = 0.f;
                    if (!(N & 1)) {
                        X[N] = vb;
                        X[N + 1] = 0.f;
                    }
                } else if (s < Ha) {
                    X[2 * s] = va;
                    X[2 * s + 1] = vb;
                    X[2 * (N - s)] = va;
                    X[2 * (N - s) + 1] = -vb;
                }
            }
        if (a.stats && h == 0) {
            csrec_pixel_stats st;
            st.iters = bad ? 0 : iters;
            st.flags = bad ? CSREC_FLAG_NONFINITE : (converged ? CSREC_FLAG_CONVERGED : CSREC_FLAG_ITER_CAP);
            st.resid = bad ? 0.f : sqrtf(r2);
            st.delta = bad ? __builtin_nanf("") : sqrtf(last_d2);
            a.stats[pix] = st;
        }
    }
}

// PRE: C twice in LDS in the operand order (2 MT (2 NTH) KiB); otherwise
// once with the padded pitch (64 MT (32 NTH + 2) bytes).
template <int MT, int NTH, int WAVES, int MINW, bool PRE, bool CY>
__global__ __launch_bounds__(WAVES * 64, MINW) void fista_h32_kernel(HermArgs a) {
    constexpr int NT = 2 * NTH;
    constexpr int S = 16 * NTH;
    const int M = a.M, N = a.N, Ha = a.Ha;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int h = lane >> 4;
    const int j = lane & 15;
    const int64_t pix = ((int64_t)blockIdx.x * WAVES + wave) * 16 + j;
    const int mu_j = 8 * ((j >> 2) & 1) + 4 * (j >> 3) + (j & 3);
    const int nu_j = 4 * (j & 3) + (j >> 2);
    const int cm_h = 8 * (h & 1) + 4 * (h >> 1);
    auto cval = [&](int row, int col) {
        if constexpr (CY) return row < M ? a.Ap[(size_t)row * 2 * S + col] : 0.f;
        return herm_c(a.A, M, N, Ha, S, row, col);
    };
    if constexpr (PRE) {
        constexpr int BLK = MT * NT * 64;
        __shared__ v4f sA1[BLK];
        __shared__ v4f sA2[BLK];
        for (int idx = threadIdx.x; idx < BLK; idx += WAVES * 64) {
            const int l = idx & 63, blk = idx >> 6;
            const int hh = l >> 4, jj = l & 15;
            const int mu = 8 * ((jj >> 2) & 1) + 4 * (jj >> 3) + (jj & 3);
            const int nu = 4 * (jj & 3) + (jj >> 2);
            const int cm = 8 * (hh & 1) + 4 * (hh >> 1);
            v4f v1, v2;
            {
                const int mt = blk / NT, nt = blk - (blk / NT) * NT;
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) v1[kk] = cval(16 * mt + mu, 16 * nt + 4 * kk + hh);
            }
            {
                const int nt = blk / MT, mt = blk - (blk / MT) * MT;
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) v2[kk] = cval(16 * mt + cm + kk, 16 * nt + nu);
            }
            sA1[idx] = v1;
            sA2[idx] = v2;
        }
        __syncthreads();
        const OpsPre<MT, NT> ops{sA1 + lane, sA2 + lane};
        if (a.eps > 0.f)
            herm_body<MT, NTH, true, CY>(a, ops, h, j, pix);
        else
            herm_body<MT, NTH, false, CY>(a, ops, h, j, pix);
    } else {
        constexpr int PA = OpsSingle<NT>::PA;
        __shared__ float sA[16 * MT * PA];
        for (int idx = threadIdx.x; idx < 16 * MT * PA; idx += WAVES * 64) {
            const int row = idx / PA, col = idx - (idx / PA) * PA;
            sA[idx] = col < 2 * S ? cval(row, col) : 0.f;
        }
        __syncthreads();
        const OpsSingle<NT> ops{sA + mu_j * PA + h, sA + cm_h * PA + nu_j};
        if (a.eps > 0.f)
            herm_body<MT, NTH, true, CY>(a, ops, h, j, pix);
        else
            herm_body<MT, NTH, false, CY>(a, ops, h, j, pix);
    }
}

// The single-copy iteration without the Delta stop (only eps = 0 is
// dispatched here), eight waves per workgroup on the one LDS copy of C (two
// per SIMD) and y in LDS, which is what lets the state fit in 256 registers.
template <int MT, int NTH, bool CY>
__global__ __launch_bounds__(512, 1) void fista_h32i8_kernel(HermArgs a) {
    constexpr int NT = 2 * NTH;
    constexpr int S = 16 * NTH;
    constexpr int PA = OpsSingle<NT>::PA;
    __shared__ float sA[16 * MT * PA];
    __shared__ v4f sY[8 * MT * 64];
    const int M = a.M, N = a.N, Ha = a.Ha;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int h = lane >> 4;
    const int j = lane & 15;
    const int64_t pix = ((int64_t)blockIdx.x * 8 + wave) * 16 + j;
    const int mu_j = 8 * ((j >> 2) & 1) + 4 * (j >> 3) + (j & 3);
    const int nu_j = 4 * (j & 3) + (j >> 2);
    const int cm_h = 8 * (h & 1) + 4 * (h >> 1);
    for (int idx = threadIdx.x; idx < 16 * MT * PA; idx += 512) {
        const int row = idx / PA, col = idx - (idx / PA) * PA;
        float v = 0.f;
        if (col < 2 * S) {
            if constexpr (CY) v = row < M ? a.Ap[(size_t)row * 2 * S + col] : 0.f;
            else v = herm_c(a.A, M, N, Ha, S, row, col);
        }
        sA[idx] = v;
    }
    __syncthreads();
    const OpsSingle<NT> ops{sA + mu_j * PA + h, sA + cm_h * PA + nu_j};
    herm_body<MT, NTH, false, CY, OpsSingle<NT>, true>(a, ops, h, j, pix, sY + wave * MT * 64);
}

typedef void (*herm_kernel_t)(HermArgs);

struct HVariant {
    int MT, NTH;
    herm_kernel_t fn;    // real y, half spectrum
    herm_kernel_t fnc;   // complex y, embedding
    herm_kernel_t fn8 = nullptr;    // eps = 0, eight waves per workgroup (real y)
    herm_kernel_t fnc8 = nullptr;   // the same for complex y
};

#define FISTA_H_VARIANT(MT, NTH, MINW, PRE) \
    { MT, NTH, fista_h32_kernel<MT, NTH, 4, MINW, PRE, false>, fista_h32_kernel<MT, NTH, 4, MINW, PRE, true> }
#define FISTA_H_VARIANT8(MT, NTH, MINW, PRE)                                                               \
    { MT, NTH, fista_h32_kernel<MT, NTH, 4, MINW, PRE, false>, fista_h32_kernel<MT, NTH, 4, MINW, PRE, true>, \
      fista_h32i8_kernel<MT, NTH, false>, fista_h32i8_kernel<MT, NTH, true> }
// (4, 5) runs its solves without the Delta stop on eight waves (one copy of C
// plus y fit in LDS, and the state in 256 registers); the larger shapes would
// spill 40-70 registers there and keep four waves
const HVariant kHVariants[] = {
    FISTA_H_VARIANT(2, 2, 2, true),  FISTA_H_VARIANT(3, 4, 2, true),  FISTA_H_VARIANT8(4, 5, 1, true),
    FISTA_H_VARIANT(5, 7, 1, true),  FISTA_H_VARIANT(6, 7, 1, false), FISTA_H_VARIANT(6, 8, 1, false),
};
#undef FISTA_H_VARIANT
#undef FISTA_H_VARIANT8

// rows: M (real y) or 2M (complex y); pairs: ceil(N/2) slots (real y) or N (complex y)
const HVariant* hpick_rows(int rows, int pairs) {
    const int mt = (int)ceil_div(rows, 16), nth = (int)ceil_div(pairs, 16);
    const HVariant* best = nullptr;
    for (const auto& v : kHVariants)
        if (v.MT >= mt && v.NTH >= nth && (!best || v.MT * v.NTH < best->MT * best->NTH)) best = &v;
    return best;
}

const HVariant* hpick(int M, int N) { return hpick_rows(M, (N + 1) / 2); }

}  // namespace

int fista_complex_supported(int M, int N) {
    return (2 * M <= 96 && hpick_rows(2 * M, N)) ? CSREC_OK : CSREC_E_UNSUPPORTED;
}

int complex_embed_launch(const float* A, int M, int N, int NP, float* Ap, hipStream_t stream) {
    const int64_t total = (int64_t)2 * M * 2 * NP;
    hipLaunchKernelGGL(embed_kernel, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, stream, A, M, N, NP, Ap);
    CSREC_HIP_TRY(hipGetLastError());
    return CSREC_OK;
}

// A' has 2 NP columns with NP = 16 NTH of the chosen variant, so that the
// imaginary block starts at tile NTH.
// A' (2M x 2S floats, S = 16 NTH of the chosen tile), then the L slot
size_t fista_complex_workspace(int M, int N) {
    const HVariant* v = hpick_rows(2 * M, N);
    if (!v) return 0;
    return align_up((size_t)2 * M * 2 * 16 * v->NTH * sizeof(float), 256) + 256;
}

int fista_complex_launch(const FistaLaunch& l, bool power) {
    if (l.P == 0) return CSREC_OK;
    const HVariant* v = hpick_rows(2 * l.M, l.N);
    if (!v || 2 * l.M > 96) return CSREC_E_UNSUPPORTED;
    const int S = 16 * v->NTH;
    char* ws = static_cast<char*>(l.workspace);
    float* Ap = reinterpret_cast<float*>(ws);
    float* Ld = reinterpret_cast<float*>(ws + align_up((size_t)2 * l.M * 2 * S * sizeof(float), 256));
    int e = complex_embed_launch(l.A, l.M, l.N, S, Ap, l.stream);
    if (e) return e;
    HermArgs a;
    a.A = l.A;
    a.Ap = Ap;
    a.Y = l.Y;
    a.X0 = l.X0;
    a.X = l.X;
    a.stats = l.stats;
    a.L_dev = nullptr;
    a.M = 2 * l.M;
    a.Mc = l.M;
    a.N = l.N;
    a.Ha = l.N;
    a.P = l.P;
    a.max_iter = l.max_iter;
    a.invL = l.invL;
    a.thr = l.thr;
    a.eps = l.eps;
    a.lambda = l.lambda;
    if (power) {
        // L = lambda_max(A^* A) = lambda_max(A'^T A') by power iteration on A'
        if ((e = lipschitz_launch(Ap, 2 * l.M, 2 * S, Ld, l.stream))) return e;
        a.L_dev = Ld;
    }
    const bool w8 = a.eps <= 0.f && v->fnc8;
    const int waves = w8 ? 8 : 4;
    const int64_t blocks = ceil_div(l.P, 16 * waves);
    if (blocks > 0x7fffffff) return CSREC_E_SHAPE;
    hipLaunchKernelGGL(w8 ? v->fnc8 : v->fnc, dim3((unsigned)blocks), dim3(64 * waves), 0, l.stream, a);
    CSREC_HIP_TRY(hipGetLastError());
    return CSREC_OK;
}

int fista_hermitian_supported(int M, int N) { return hpick(M, N) ? CSREC_OK : CSREC_E_UNSUPPORTED; }

int herm_scaled_launch(const float* A, int M, int N, int S, float* Ch, hipStream_t stream) {
    const int total = M * 2 * S;
    hipLaunchKernelGGL(herm_scaled_kernel, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, stream, A, M, N,
                       (N + 1) / 2, S, Ch);
    CSREC_HIP_TRY(hipGetLastError());
    return CSREC_OK;
}

// the device L: C diag(sqrt(w)) then the L slot
size_t fista_hermitian_workspace(int M, int N, bool power) {
    const HVariant* v = hpick(M, N);
    if (!v || !power) return 0;
    return align_up((size_t)M * 2 * 16 * v->NTH * sizeof(float), 256) + 256;
}

int fista_hermitian_launch(const FistaLaunch& l, bool power) {
    if (l.P == 0) return CSREC_OK;
    const HVariant* v = hpick(l.M, l.N);
    if (!v) return CSREC_E_UNSUPPORTED;
    const int S = 16 * v->NTH;
    const int Ha = (l.N + 1) / 2;
    HermArgs a;
    a.A = l.A;
    a.Ap = nullptr;
    a.Y = l.Y;
    a.X0 = l.X0;
    a.X = l.X;
    a.stats = l.stats;
    a.L_dev = nullptr;
    a.M = l.M;
    a.Mc = l.M;
    a.N = l.N;
    a.Ha = Ha;
    a.P = l.P;
    a.max_iter = l.max_iter;
    a.invL = l.invL;
    a.thr = l.thr;
    a.eps = l.eps;
    a.lambda = l.lambda;
    if (power) {
        char* ws = static_cast<char*>(l.workspace);
        float* Ch = reinterpret_cast<float*>(ws);
        float* Ld = reinterpret_cast<float*>(ws + align_up((size_t)l.M * 2 * S * sizeof(float), 256));
        int e = herm_scaled_launch(l.A, l.M, l.N, S, Ch, l.stream);
        if (e) return e;
        e = lipschitz_launch(Ch, l.M, 2 * S, Ld, l.stream);
        if (e) return e;
        a.L_dev = Ld;
    }
    const bool w8 = a.eps <= 0.f && v->fn8;
    const int waves = w8 ? 8 : 4;
    const int64_t blocks = ceil_div(l.P, 16 * waves);
    if (blocks > 0x7fffffff) return CSREC_E_SHAPE;
    hipLaunchKernelGGL(w8 ? v->fn8 : v->fn, dim3((unsigned)blocks), dim3(64 * waves), 0, l.stream, a);
    CSREC_HIP_TRY(hipGetLastError());
    return CSREC_OK;
}

}  // namespace csrec
