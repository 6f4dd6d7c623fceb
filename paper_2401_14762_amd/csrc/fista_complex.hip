// FISTA (Alg. 1) for the complex measurement model of Section II: with the
// DFT basis, A = Phi Psi (M x N) and x are complex, A^* is the conjugate
// transpose and the soft threshold shrinks |x_n| and keeps its phase.
//
// The complex products run as real ones on the embedding
//   A' = [ Re A  -Im A ]   (2M x 2NP, column blocks of NP = 16 NTH),
//        [ Im A   Re A ]
// A' [Re x; Im x] = [Re(A x); Im(A x)] and A'^T [Re u; Im u] = [Re(A^* u);
// Im(A^* u)], so the iteration is the real kernel's on A' with one change:
// the threshold acts on the pair (Re x_n, Im x_n).  Column n of the real
// block and column NP + n of the imaginary block fall in tiles p and p + NTH
// with the same register and lane, so each lane holds both halves of its
// pixel's x_n.  ||r|| over the 2M real rows is the complex norm.
//
// A' is written once per call into the workspace and stored in LDS twice,
// pre-arranged in the MFMA operand order (one ds_read_b128 per four MFMAs),
// as in the pre-arranged real kernel; the next pair's A'^T products are
// interleaved with this pair's A' products.  Complex arrays are interleaved
// (re, im) FP32 pairs.
#include "common.hpp"

#include <cmath>

namespace csrec {
namespace {

struct CFistaArgs {
    const float* Ap;      // A', 2M x 2NP row-major
    const float* Y;       // P x M complex
    const float* X0;      // P x N complex, may be null
    float* X;             // P x N complex
    csrec_pixel_stats* stats;
    const float* L_dev;
    int M, N, NP;
    int64_t P;
    int max_iter;
    float invL, thr, eps;
    double lambda;
};

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

template <int MT, int NTH, int WAVES, int MINW, bool FREEZE>
__device__ __forceinline__ void cfista_body(const CFistaArgs& a, const v4f* __restrict__ sA1,
                                            const v4f* __restrict__ sA2) {
    constexpr int NT = 2 * NTH;
    const int M = a.M, N = a.N, NP = a.NP;
    const int M2 = 2 * M;
    float invL = a.invL, thr = a.thr;
    if (a.L_dev) {
        const float L = *a.L_dev;
        invL = 1.f / L;
        thr = (float)(a.lambda / (double)L);
    }
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int h = lane >> 4;
    const int j = lane & 15;
    const int64_t pix = ((int64_t)blockIdx.x * WAVES + wave) * 16 + j;
    const bool valid = pix < a.P;
    const int cm_h = 8 * (h & 1) + 4 * (h >> 1);
    const v4f* a1 = sA1 + lane;   // + (mt NT + nt) 64
    const v4f* a2 = sA2 + lane;   // + (nt MT + mt) 64

    // y' = [Re y; Im y] in the m-layout
    v4f Yr[MT];
    int bad = 0;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int m2 = 16 * mt + cm_h + r;
            float v = 0.f;
            if (valid && m2 < M2) {
                const int m = m2 < M ? m2 : m2 - M;
                v = a.Y[((size_t)pix * M + m) * 2 + (m2 < M ? 0 : 1)];
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

    // x^0 (z^0 = x^0): tile p holds Re x, tile p + NTH holds Im x
    v4f Xr[NT], Zr[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int n2 = 16 * nt + 4 * r + h;
            const int n = n2 < NP ? n2 : n2 - NP;
            float v = 0.f;
            if (a.X0 && valid && !bad && n < N) v = a.X0[((size_t)pix * N + n) * 2 + (n2 < NP ? 0 : 1)];
            Xr[nt][r] = v;
            Zr[nt][r] = v;
        }

    v4f U1[MT], V[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) U1[mt] = -Yr[mt];
    if (a.X0) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const v4f av = a1[(mt * NT + nt) * 64];
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    U1[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[kk], Xr[nt][kk], U1[mt], 0, 0, 0);
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
        // they would need all of A' in registers)
        asm volatile("" ::: "memory");
        const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));   // step 3
        const float bcur = (float)((t - 1.0) / tn);                  // step 4 coefficient
        t = tn;
        const float cp = 1.f + bprev;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) V[mt] = cp * U1[mt] - bprev * V[mt];
        v4f Un[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) Un[mt] = -Yr[mt];

        // A'^T V of the pair (0, NTH); each pair's is interleaved with the
        // previous pair's A' x products
        v4f Wre = {0.f, 0.f, 0.f, 0.f}, Wim = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const v4f b0 = a2[mt * 64];
            const v4f b1 = a2[(NTH * MT + mt) * 64];
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                Wre = __builtin_amdgcn_mfma_f32_16x16x4f32(b0[kk], V[mt][kk], Wre, 0, 0, 0);
                Wim = __builtin_amdgcn_mfma_f32_16x16x4f32(b1[kk], V[mt][kk], Wim, 0, 0, 0);
            }
        }
#pragma unroll
        for (int p = 0; p < NTH; ++p) {
            const v4f Gre = Wre, Gim = Wim;
            // steps 1, 2, 4 on the pair (Re, Im) of each x_n
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float re = Zr[p][r] - Gre[r] * invL;
                const float im = Zr[p + NTH][r] - Gim[r] * invL;
                const float mag = sqrtf(re * re + im * im);
                const float s = mag > thr ? (mag - thr) / mag : 0.f;
                const float xre = re * s, xim = im * s;
                const float zre = xre + bcur * (xre - Xr[p][r]);
                const float zim = xim + bcur * (xim - Xr[p + NTH][r]);
                const bool upd = !FREEZE || active;
                Xr[p][r] = upd ? xre : Xr[p][r];
                Xr[p + NTH][r] = upd ? xim : Xr[p + NTH][r];
                Zr[p][r] = upd ? zre : Zr[p][r];
                Zr[p + NTH][r] = upd ? zim : Zr[p + NTH][r];
            }
            // U += A'(:, tiles p, p + NTH) x, with the next pair's A'^T V interleaved
            const bool more = p + 1 < NTH;
            if (more) {
                Wre = v4f{0.f, 0.f, 0.f, 0.f};
                Wim = v4f{0.f, 0.f, 0.f, 0.f};
            }
            const int pn = more ? p + 1 : p;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const v4f av0 = a1[(mt * NT + p) * 64];
                const v4f av1 = a1[(mt * NT + p + NTH) * 64];
                const v4f b0 = a2[(pn * MT + mt) * 64];
                const v4f b1 = a2[((pn + NTH) * MT + mt) * 64];
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    Un[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av0[kk], Xr[p][kk], Un[mt], 0, 0, 0);
                    if (more) Wre = __builtin_amdgcn_mfma_f32_16x16x4f32(b0[kk], V[mt][kk], Wre, 0, 0, 0);
                    Un[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av1[kk], Xr[p + NTH][kk], Un[mt], 0, 0, 0);
                    if (more) Wim = __builtin_amdgcn_mfma_f32_16x16x4f32(b1[kk], V[mt][kk], Wim, 0, 0, 0);
                }
            }
        }

        // Delta^2 = ||r^i - r^{i-1}||^2 with r^0 = y
        const float c0 = (it == 0 && a.X0) ? 1.f : 0.f;
        float d2 = 0.f;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float ref = U1[mt][r] - c0 * (U1[mt][r] + Yr[mt][r]);
                const float d = Un[mt][r] - ref;
                d2 += d * d;
            }
        d2 = quad_sum(d2);
        if (active) {
            iters = it + 1;
            last_d2 = d2;
        }
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
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int n2 = 16 * nt + 4 * r + h;
                const int n = n2 < NP ? n2 : n2 - NP;
                if (n < N) a.X[((size_t)pix * N + n) * 2 + (n2 < NP ? 0 : 1)] = bad ? 0.f : Xr[nt][r];
            }
        if (a.stats && h == 0) {
            csrec_pixel_stats s;
            s.iters = bad ? 0 : iters;
            s.flags = bad ? CSREC_FLAG_NONFINITE : (converged ? CSREC_FLAG_CONVERGED : CSREC_FLAG_ITER_CAP);
            s.resid = bad ? 0.f : sqrtf(r2);
            s.delta = bad ? __builtin_nanf("") : sqrtf(last_d2);
            a.stats[pix] = s;
        }
    }
}

template <int MT, int NTH, int WAVES, int MINW>
__global__ __launch_bounds__(WAVES * 64, MINW) void fista_c32_kernel(CFistaArgs a) {
    constexpr int NT = 2 * NTH;
    constexpr int BLK = MT * NT * 64;
    __shared__ v4f sA1[BLK];   // [mt][nt][lane]: A'[16 mt + mu_j][16 nt + 4 kk + h]
    __shared__ v4f sA2[BLK];   // [nt][mt][lane]: A'[16 mt + cm_h + kk][16 nt + nu_j]
    const int M2 = 2 * a.M, N2 = 2 * a.NP;
    for (int idx = threadIdx.x; idx < BLK; idx += WAVES * 64) {
        const int l = idx & 63, blk = idx >> 6;
        const int hh = l >> 4, jj = l & 15;
        const int mu = 8 * ((jj >> 2) & 1) + 4 * (jj >> 3) + (jj & 3);
        const int nu = 4 * (jj & 3) + (jj >> 2);
        const int cm = 8 * (hh & 1) + 4 * (hh >> 1);
        v4f v1, v2;
        {
            const int mt = blk / NT, nt = blk - (blk / NT) * NT;
            const int row = 16 * mt + mu;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int col = 16 * nt + 4 * kk + hh;
                v1[kk] = (row < M2 && col < N2) ? a.Ap[(size_t)row * N2 + col] : 0.f;
            }
        }
        {
            const int nt = blk / MT, mt = blk - (blk / MT) * MT;
            const int col = 16 * nt + nu;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int row = 16 * mt + cm + kk;
                v2[kk] = (row < M2 && col < N2) ? a.Ap[(size_t)row * N2 + col] : 0.f;
            }
        }
        sA1[idx] = v1;
        sA2[idx] = v2;
    }
    __syncthreads();
    if (a.eps > 0.f)
        cfista_body<MT, NTH, WAVES, MINW, true>(a, sA1, sA2);
    else
        cfista_body<MT, NTH, WAVES, MINW, false>(a, sA1, sA2);
}

typedef void (*cfista_kernel_t)(CFistaArgs);

struct CVariant {
    int MT, NTH;
    cfista_kernel_t fn;
};

// 2 MT (2 NTH) KiB of LDS for the two copies of A'.
const CVariant kCVariants[] = {
    {2, 2, fista_c32_kernel<2, 2, 4, 2>},
    {3, 4, fista_c32_kernel<3, 4, 4, 2>},
    {4, 5, fista_c32_kernel<4, 5, 4, 1>},
    {5, 7, fista_c32_kernel<5, 7, 4, 1>},
};

const CVariant* cpick(int M, int N) {
    const int mt = (int)ceil_div(2 * M, 16), nth = (int)ceil_div(N, 16);
    const CVariant* best = nullptr;
    for (const auto& v : kCVariants)
        if (v.MT >= mt && v.NTH >= nth && (!best || v.MT * v.NTH < best->MT * best->NTH)) best = &v;
    return best;
}

}  // namespace

int fista_complex_supported(int M, int N) { return cpick(M, N) ? CSREC_OK : CSREC_E_UNSUPPORTED; }

// A' has 2 NP columns with NP = 16 NTH of the chosen variant, so that the
// imaginary block starts at tile NTH.
size_t fista_complex_workspace(int M, int N) {
    const CVariant* v = cpick(M, N);
    if (!v) return 0;
    const size_t np = 16 * (size_t)v->NTH;
    return align_up((size_t)2 * M * 2 * np * sizeof(float), 256) + 256;
}

int fista_complex_launch(const FistaLaunch& l, bool power) {
    if (l.P == 0) return CSREC_OK;
    const CVariant* v = cpick(l.M, l.N);
    if (!v) return CSREC_E_UNSUPPORTED;
    const int NP = 16 * v->NTH;
    char* ws = static_cast<char*>(l.workspace);
    float* Ap = reinterpret_cast<float*>(ws);
    float* Ld = reinterpret_cast<float*>(ws + align_up((size_t)2 * l.M * 2 * NP * sizeof(float), 256));
    const int64_t total = (int64_t)2 * l.M * 2 * NP;
    hipLaunchKernelGGL(embed_kernel, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, l.stream, l.A, l.M, l.N, NP,
                       Ap);
    CSREC_HIP_TRY(hipGetLastError());
    CFistaArgs a;
    a.Ap = Ap;
    a.Y = l.Y;
    a.X0 = l.X0;
    a.X = l.X;
    a.stats = l.stats;
    a.L_dev = nullptr;
    a.M = l.M;
    a.N = l.N;
    a.NP = NP;
    a.P = l.P;
    a.max_iter = l.max_iter;
    a.invL = l.invL;
    a.thr = l.thr;
    a.eps = l.eps;
    a.lambda = l.lambda;
    if (power) {
        // L = lambda_max(A^* A) = lambda_max(A'^T A') by power iteration on A'
        int e = lipschitz_launch(Ap, 2 * l.M, 2 * NP, Ld, l.stream);
        if (e) return e;
        a.L_dev = Ld;
    }
    const int64_t blocks = ceil_div(l.P, 16 * 4);
    if (blocks > 0x7fffffff) return CSREC_E_SHAPE;
    hipLaunchKernelGGL(v->fn, dim3((unsigned)blocks), dim3(64 * 4), 0, l.stream, a);
    CSREC_HIP_TRY(hipGetLastError());
    return CSREC_OK;
}

}  // namespace csrec
