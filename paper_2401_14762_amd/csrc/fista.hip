// FISTA (Alg. 1) for P independent LASSO problems (Eq. 2) sharing one A.
//
// Work decomposition.  One wavefront owns 16 pixels for the whole solve.
// The dictionary A lives once per workgroup in LDS; every per-pixel vector
// (x^{i-1}, z^{i-1}, A x^{i-1} - y, A x^{i-2} - y, y) lives in VGPRs for all
// iterations, so the loop touches HBM only to read y at the start and to
// write x at the end.
//
// Arithmetic per iteration i (all of Alg. 1, per pixel):
//   U_k = A x^k - y  (= -r^k, step 5) is carried instead of recomputed, and
//   A z^{i-1} - y = (1 + b_{i-1}) U_{i-1} - b_{i-1} U_{i-2}
//   with b_k = (t^{k-1} - 1) / t^k (step 4 is linear, so A commutes with it).
//   GEMM 2:  W = A^T V,   V = A z^{i-1} - y        (step 1)
//   epilogue: aux = z - W / L; x^i = soft(aux, lambda / L); z^i = x^i + b_i (x^i - x^{i-1})
//   GEMM 1:  U_i = A x^i - y                         (step 5)
//   Delta = ||U_i - U_{i-1}||_2                      (step 5; r^0 = y)
// so an iteration costs 4 M N flops per pixel instead of the 6 M N of the
// literal form.
//
// MFMA mapping (v_mfma_f32_16x16x4f32, D[16x16] += A[16x4] B[4x16]).
// Pixels are the 16 columns j of every product.  Lane l = 16 h + j holds,
// for its pixel j, the elements of tile t with register r:
//   n = 16 t + c_n(h, r),  c_n(h, r) = 4 r + h                 (x, z, W)
//   m = 16 t + c_m(h, r),  c_m(h, r) = 8 (h & 1) + 4 (h >> 1) + r  (U, V, y)
// which is exactly the D-register layout of one product and the B-operand
// layout of the next: in k-step kk of a 16-wide contraction tile, group h
// contributes the index c(h, kk), i.e. its own register kk.  The products
// therefore chain register to register.  The two index permutations make the
// single LDS copy of A (row pitch 16*NT+2, an even number whose half is odd)
// bank-conflict free for both the A (GEMM 1) and the A^T (GEMM 2) operand
// reads.
#include "common.hpp"

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <cmath>

namespace csrec {
namespace {

struct FistaArgs {
    const float* A;
    const float* Y;
    const float* X0;
    float* X;
    csrec_pixel_stats* stats;
    const float* L_dev;
    int M, N;
    int64_t P;
    int max_iter;
    int iter_offset;      // iterations already run by an earlier pass (added to the stats)
    float invL, thr, eps;
    double lambda;
};

__device__ __forceinline__ float soft_thr(float v, float t) {
    // sign(v) * max(|v| - t, 0)
    const float a = fabsf(v) - t;
    return a > 0.f ? copysignf(a, v) : 0.f;
}

__device__ __forceinline__ float quad_sum(float v) {
    // sum over the four lanes j, j+16, j+32, j+48 that hold one pixel
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

template <int MT, int NT, int WAVES, int MINW>
__global__ __launch_bounds__(WAVES * 64, MINW) void fista_f32_kernel(FistaArgs a) {
    constexpr int PA = 16 * NT + 2;   // LDS row pitch of A (floats)
    constexpr int ROWS = 16 * MT;
    __shared__ float sA[ROWS * PA];

    const int M = a.M, N = a.N;
    for (int idx = threadIdx.x; idx < ROWS * PA; idx += WAVES * 64) {
        const int row = idx / PA;
        const int col = idx - row * PA;
        float v = 0.f;
        if (row < M && col < N) v = a.A[(size_t)row * N + col];
        sA[idx] = v;
    }

    float invL = a.invL, thr = a.thr;
    if (a.L_dev) {
        const float L = *a.L_dev;
        invL = 1.f / L;
        thr = (float)(a.lambda / (double)L);
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int h = lane >> 4;
    const int j = lane & 15;
    const int64_t pix = ((int64_t)blockIdx.x * WAVES + wave) * 16 + j;
    const bool valid = pix < a.P;

    const int mu_j = 8 * ((j >> 2) & 1) + 4 * (j >> 3) + (j & 3);  // m of output row j (GEMM 1)
    const int nu_j = 4 * (j & 3) + (j >> 2);                       // n of output row j (GEMM 2)
    const int cm_h = 8 * (h & 1) + 4 * (h >> 1);
    const float* a1 = sA + mu_j * PA + h;      // + 16 mt PA + 16 nt + 4 kk
    const float* a2 = sA + cm_h * PA + nu_j;   // + (16 mt + kk) PA + 16 nt

    // ---- measurements, non-finite check
    v4f Yr[MT];
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
            Yr[mt][r] = v;
        }
    bad |= __shfl_xor(bad, 16);
    bad |= __shfl_xor(bad, 32);
    if (bad) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) Yr[mt] = v4f{0.f, 0.f, 0.f, 0.f};
    }

    // ---- starting point x^0 (z^0 = x^0)
    v4f Xr[NT], Zr[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int n = 16 * nt + 4 * r + h;
            float v = 0.f;
            if (a.X0 && valid && !bad && n < N) v = a.X0[pix * N + n];
            Xr[nt][r] = v;
            Zr[nt][r] = v;
        }

    // U_0 = A x^0 - y; U_{-1} = U_0 (so z^0 = x^0 whatever b_0 is)
    v4f U1[MT], V[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) U1[mt] = -Yr[mt];
    if (a.X0) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    U1[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                        a1[16 * mt * PA + 16 * nt + 4 * kk], Xr[nt][kk], U1[mt], 0, 0, 0);
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
        const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));   // step 3
        const float bcur = (float)((t - 1.0) / tn);                  // step 4 coefficient
        t = tn;

        // V = A z^{i-1} - y
        const float cp = 1.f + bprev;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) V[mt] = cp * U1[mt] - bprev * V[mt];

        v4f Un[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) Un[mt] = -Yr[mt];

#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            // W = (A^T V) for 16 n-values of this tile          (step 1)
            v4f W = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    W = __builtin_amdgcn_mfma_f32_16x16x4f32(a2[(16 * mt + kk) * PA + 16 * nt],
                                                             V[mt][kk], W, 0, 0, 0);
            // steps 1, 2, 4 elementwise
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float aux = Zr[nt][r] - W[r] * invL;
                const float xn = soft_thr(aux, thr);
                const float zn = xn + bcur * (xn - Xr[nt][r]);
                Xr[nt][r] = active ? xn : Xr[nt][r];
                Zr[nt][r] = active ? zn : Zr[nt][r];
            }
            // U_i += A(:, tile) x^i(tile)                        (step 5)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    Un[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                        a1[16 * mt * PA + 16 * nt + 4 * kk], Xr[nt][kk], Un[mt], 0, 0, 0);
        }

        // Delta^2 = ||r^i - r^{i-1}||^2 with r^0 = y: the reference is U_{i-1},
        // except in the first iteration from a given x^0, where it is -y.
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
            U1[mt] = active ? Un[mt] : U1[mt];
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
                const int n = 16 * nt + 4 * r + h;
                if (n < N) a.X[pix * N + n] = bad ? 0.f : Xr[nt][r];
            }
        if (a.stats && h == 0) {
            csrec_pixel_stats s;
            s.iters = bad ? 0 : iters + a.iter_offset;
            s.flags = bad ? CSREC_FLAG_NONFINITE : (converged ? CSREC_FLAG_CONVERGED : CSREC_FLAG_ITER_CAP);
            s.resid = bad ? 0.f : sqrtf(r2);
            s.delta = bad ? __builtin_nanf("") : sqrtf(last_d2);
            a.stats[pix] = s;
        }
    }
}

// Operand reads of the two products, in the MFMA operand order:
//   fwd(mt, nt)[kk] = A[16 mt + mu_j][16 nt + 4 kk + h]     (A x, B operand x)
//   bwd(nt, mt)[kk] = A[16 mt + cm_h + kk][16 nt + nu_j]   (A^T v, B operand v)
// OpsPre reads them from two pre-arranged copies (one ds_read_b128 each);
// OpsSingle from one copy with row pitch 16 NT + 2 (an even pitch whose half
// is odd: both read patterns are bank-conflict free), four ds_read_b32.
// at() places the reads for the lane (h, j) from the LDS base pointers.
template <int MT, int NT>
struct OpsPre {
    const v4f* a1;   // + (mt NT + nt) 64
    const v4f* a2;   // + (nt MT + mt) 64
    __device__ __forceinline__ static OpsPre at(const void* b1, const void* b2, int lane, int, int, int, int) {
        return OpsPre{static_cast<const v4f*>(b1) + lane, static_cast<const v4f*>(b2) + lane};
    }
    __device__ __forceinline__ v4f fwd(int mt, int nt) const { return a1[(mt * NT + nt) * 64]; }
    __device__ __forceinline__ v4f bwd(int nt, int mt) const { return a2[(nt * MT + mt) * 64]; }
};

template <int NT>
struct OpsSingle {
    static constexpr int PA = 16 * NT + 2;
    const float* a1;   // sA + mu_j PA + h
    const float* a2;   // sA + cm_h PA + nu_j
    __device__ __forceinline__ static OpsSingle at(const void* b1, const void*, int, int h, int mu_j, int nu_j,
                                                   int cm_h) {
        const float* sA = static_cast<const float*>(b1);
        return OpsSingle{sA + mu_j * PA + h, sA + cm_h * PA + nu_j};
    }
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

// YL: y kept in LDS (ysh: WAVES MT 64 v4f, each lane its own MT entries)
// instead of registers, and the scheduler held to one tile at a time, for
// the eight-wave form (two waves per SIMD on one LDS copy of A).
template <int MT, int NT, int WAVES, bool FREEZE, class Ops, bool YL = false>
__device__ __forceinline__ void fista_f32s_body(const FistaArgs& a, const void* lds1, const void* lds2,
                                                v4f* ysh = nullptr) {
    const int M = a.M, N = a.N;
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

    const int mu_j = 8 * ((j >> 2) & 1) + 4 * (j >> 3) + (j & 3);  // m of output row j (GEMM 1)
    const int nu_j = 4 * (j & 3) + (j >> 2);                       // n of output row j (GEMM 2)
    const int cm_h = 8 * (h & 1) + 4 * (h >> 1);
    const Ops ops = Ops::at(lds1, lds2, lane, h, mu_j, nu_j, cm_h);

    // ---- measurements, non-finite check
    v4f Yr[MT];
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
            Yr[mt][r] = v;
        }
    bad |= __shfl_xor(bad, 16);
    bad |= __shfl_xor(bad, 32);
    if (bad) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) Yr[mt] = v4f{0.f, 0.f, 0.f, 0.f};
    }

    // ---- starting point x^0 (z^0 = x^0)
    v4f Xr[NT], Zr[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int n = 16 * nt + 4 * r + h;
            float v = 0.f;
            if (a.X0 && valid && !bad && n < N) v = a.X0[pix * N + n];
            Xr[nt][r] = v;
            Zr[nt][r] = v;
        }

    // U_0 = A x^0 - y; U_{-1} = U_0 (so z^0 = x^0 whatever b_0 is)
    v4f U1[MT], V[MT];
    v4f* const ylds = YL ? ysh + wave * MT * 64 + lane : nullptr;
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
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const v4f av = ops.fwd(mt, nt);
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
        // keeps the LDS operand reads inside the loop (they are loop-invariant,
        // and hoisting them would need every element of A in registers)
        asm volatile("" ::: "memory");
        const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));   // step 3
        const float bcur = (float)((t - 1.0) / tn);                  // step 4 coefficient
        t = tn;

        // V = A z^{i-1} - y
        const float cp = 1.f + bprev;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) V[mt] = cp * U1[mt] - bprev * V[mt];

        v4f Un[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) Un[mt] = -yt(mt);

        v4f Wn = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const v4f av = ops.bwd(0, mt);
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                Wn = __builtin_amdgcn_mfma_f32_16x16x4f32(av[kk], V[mt][kk], Wn, 0, 0, 0);
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            if constexpr (YL) __builtin_amdgcn_sched_barrier(0);
            // W = (A^T V) for 16 n-values of this tile          (step 1)
            const v4f W = Wn;
            // steps 1, 2, 4 elementwise
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float aux = Zr[nt][r] - W[r] * invL;
                // sign(v) max(|v| - t, 0) = v - median(v, -t, t), bit for bit
                const float xn = aux - __builtin_amdgcn_fmed3f(aux, -thr, thr);
                const float zn = xn + bcur * (xn - Xr[nt][r]);
                // without the Delta stop every pixel runs the whole loop (a pixel
                // with zero y and zero x^0 stays at zero): nothing to freeze
                Xr[nt][r] = (!FREEZE || active) ? xn : Xr[nt][r];
                Zr[nt][r] = (!FREEZE || active) ? zn : Zr[nt][r];
            }
            // U_i += A(:, tile) x^i(tile) (step 5), interleaved with the next
            // tile's A^T V, whose single accumulator chain then overlaps the
            // five independent ones of U_i
            if (nt + 1 < NT) Wn = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const v4f av = ops.fwd(mt, nt);
                const v4f bv = ops.bwd(nt + 1 < NT ? nt + 1 : nt, mt);
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    Un[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[kk], Xr[nt][kk], Un[mt], 0, 0, 0);
                    if (nt + 1 < NT) Wn = __builtin_amdgcn_mfma_f32_16x16x4f32(bv[kk], V[mt][kk], Wn, 0, 0, 0);
                }
            }
        }
        // Delta^2 = ||r^i - r^{i-1}||^2 with r^0 = y: the reference is U_{i-1},
        // except in the first iteration from a given x^0, where it is -y.
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
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int n = 16 * nt + 4 * r + h;
                if (n < N) a.X[pix * N + n] = bad ? 0.f : Xr[nt][r];
            }
        if (a.stats && h == 0) {
            csrec_pixel_stats s;
            s.iters = bad ? 0 : iters + a.iter_offset;
            s.flags = bad ? CSREC_FLAG_NONFINITE : (converged ? CSREC_FLAG_CONVERGED : CSREC_FLAG_ITER_CAP);
            s.resid = bad ? 0.f : sqrtf(r2);
            s.delta = bad ? __builtin_nanf("") : sqrtf(last_d2);
            a.stats[pix] = s;
        }
    }
}


// The same iteration with A stored twice in LDS, pre-arranged so that the
// four operand values a lane feeds to four consecutive MFMAs (k-steps kk =
// 0..3 of one 16x16 tile of A or A^T) are 16 contiguous bytes: one
// ds_read_b128 per four MFMAs, conflict-free (lane l reads bytes 16 l ..
// 16 l + 15 of its tile's 1 KiB).  Two copies take 2 MT NT KiB, so this form
// serves shapes with MT NT <= 80 (M = 80, N = 200 among them).  The A^T V
// product of tile nt + 1 is issued interleaved with tile nt's A x product,
// so its single accumulator chain overlaps their five independent ones and
// the matrix cores stay busy across the epilogue; soft
// thresholding is v - median(v, -t, t); and without the Delta stop no pixel
// is frozen, which drops the per-element selects.
template <int MT, int NT, int WAVES, int MINW>
__global__ __launch_bounds__(WAVES * 64, MINW) void fista_f32s_kernel(FistaArgs a) {
    constexpr int BLK = MT * NT * 64;
    __shared__ v4f sA1[BLK];   // [mt][nt][lane]
    __shared__ v4f sA2[BLK];   // [nt][mt][lane]
    const int M = a.M, N = a.N;
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
    }
    __syncthreads();
    if (a.eps > 0.f)
        fista_f32s_body<MT, NT, WAVES, true, OpsPre<MT, NT>>(a, sA1, sA2);
    else
        fista_f32s_body<MT, NT, WAVES, false, OpsPre<MT, NT>>(a, sA1, sA2);
}

// The interleaved iteration with A once in LDS (row pitch 16 NT + 2), for
// the shapes whose two pre-arranged copies exceed the LDS (MT NT > 80:
// N = 224, M = 90 among them): 4 (16 MT (16 NT + 2)) bytes, 127 KiB at
// (7, 16).  It runs the solves without the Delta stop; with it, the
// per-element freeze selects of the interleaved loop make it slower than
// fista_f32_kernel, which serves those.
template <int MT, int NT, int WAVES, int MINW>
__global__ __launch_bounds__(WAVES * 64, MINW) void fista_f32i_kernel(FistaArgs a) {
    constexpr int PA = OpsSingle<NT>::PA;
    constexpr int ROWS = 16 * MT;
    __shared__ float sA[ROWS * PA];
    const int M = a.M, N = a.N;
    for (int idx = threadIdx.x; idx < ROWS * PA; idx += WAVES * 64) {
        const int row = idx / PA, col = idx - (idx / PA) * PA;
        sA[idx] = (row < M && col < N) ? a.A[(size_t)row * N + col] : 0.f;
    }
    __syncthreads();
    if (a.eps > 0.f)
        fista_f32s_body<MT, NT, WAVES, true, OpsSingle<NT>>(a, sA, nullptr);
    else
        fista_f32s_body<MT, NT, WAVES, false, OpsSingle<NT>>(a, sA, nullptr);
}

// The interleaved single-copy iteration without the Delta stop (only eps = 0
// is dispatched here), eight waves per workgroup on the one LDS copy of A
// (two per SIMD; a second workgroup would not fit beside the copy) and y in
// LDS, which is what lets the state fit in 256 registers.
template <int MT, int NT>
__global__ __launch_bounds__(512, 1) void fista_f32i8_kernel(FistaArgs a) {
    constexpr int PA = OpsSingle<NT>::PA;
    constexpr int ROWS = 16 * MT;
    __shared__ float sA[ROWS * PA];
    __shared__ v4f sY[8 * MT * 64];
    const int M = a.M, N = a.N;
    for (int idx = threadIdx.x; idx < ROWS * PA; idx += 512) {
        const int row = idx / PA, col = idx - (idx / PA) * PA;
        sA[idx] = (row < M && col < N) ? a.A[(size_t)row * N + col] : 0.f;
    }
    __syncthreads();
    fista_f32s_body<MT, NT, 8, false, OpsSingle<NT>, true>(a, sA, nullptr, sY);
}

// ---------------------------------------------------------------- 16-bit operands
//
// Same iteration with the two products on v_mfma_f32_16x16x32_{bf16,f16}:
// operands rounded to 16 bits, FP32 accumulation, FP32 state and epilogue.
// One 32-wide contraction step consumes two adjacent 16-tiles of the FP32
// layout above: group h contributes the four indices c(h, 0..3) of tile 2s
// followed by those of tile 2s+1, i.e. its own registers of the two tiles,
// packed to 16 bits.  A is stored twice in LDS, pre-swizzled so that the
// eight operand values a lane needs for one step are 16 contiguous bytes:
//   A1[mt][s][lane][8]: rows m of tile mt, columns n of the tile pair s (GEMM 1)
//   A2[nt][s][lane][8]: rows n of tile nt, columns m of the tile pair s (GEMM 2)
// so every operand read is one conflict-free ds_read_b128 per lane.

template <typename H>
struct Vec8;
template <>
struct Vec8<__bf16> {
    typedef __bf16 type __attribute__((ext_vector_type(8)));
};
template <>
struct Vec8<_Float16> {
    typedef _Float16 type __attribute__((ext_vector_type(8)));
};

template <typename H>
__device__ __forceinline__ v4f mfma16(const typename Vec8<H>::type& a, const typename Vec8<H>::type& b, v4f c);
template <>
__device__ __forceinline__ v4f mfma16<__bf16>(const Vec8<__bf16>::type& a, const Vec8<__bf16>::type& b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
template <>
__device__ __forceinline__ v4f mfma16<_Float16>(const Vec8<_Float16>::type& a, const Vec8<_Float16>::type& b,
                                                v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

template <typename H>
__device__ __forceinline__ typename Vec8<H>::type pack8(const v4f& lo, const v4f& hi) {
    typename Vec8<H>::type v;
    v[0] = (H)lo[0]; v[1] = (H)lo[1]; v[2] = (H)lo[2]; v[3] = (H)lo[3];
    v[4] = (H)hi[0]; v[5] = (H)hi[1]; v[6] = (H)hi[2]; v[7] = (H)hi[3];
    return v;
}

// MT, NT even (tile pairs); WAVES wavefronts of 16 pixels each.  FREEZE:
// the Delta stop (a pixel stops updating once Delta < eps).  Without it
// (eps = 0) no pixel is frozen: the per-element selects go, Delta is formed
// in the last iteration only (for the stats), the new residual accumulates
// in place of the old one once V has been packed, and the soft threshold is
// v - median(v, -t, t); that drops one residual array (MT v4f) and about a
// third of the epilogue's instructions, so the large shapes run two waves
// per SIMD (WAVES = 8 sharing one LDS copy of A).
template <typename H, int MT, int NT, int WAVES, int MINW, bool FREEZE = true>
__global__ __launch_bounds__(WAVES * 64, MINW) void fista_lp_kernel(FistaArgs a) {
    typedef typename Vec8<H>::type h8;
    constexpr int MS = MT / 2, NS = NT / 2;
    // eight waves without the stop keep y in LDS (each lane its own MT
    // v4f), which frees MT v4f registers for the second wave per SIMD
    constexpr bool YL = !FREEZE && WAVES >= 8;
    __shared__ h8 sA1[MT * NS * 64];
    __shared__ h8 sA2[NT * MS * 64];
    __shared__ v4f sY[YL ? WAVES * MT * 64 : 1];
    const int M = a.M, N = a.N;

    // swizzled LDS images of A: one thread builds one lane's 8-vector
    for (int idx = threadIdx.x; idx < MT * NS * 64; idx += WAVES * 64) {
        const int ln = idx & 63, blk = idx >> 6;
        const int mt = blk / NS, sp = blk - mt * NS;
        const int h = ln >> 4, j = ln & 15;
        const int m = 16 * mt + 8 * ((j >> 2) & 1) + 4 * (j >> 3) + (j & 3);
        h8 v;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int n = 32 * sp + (e < 4 ? 0 : 16) + 4 * (e & 3) + h;
            v[e] = (H)((m < M && n < N) ? a.A[(size_t)m * N + n] : 0.f);
        }
        sA1[idx] = v;
    }
    for (int idx = threadIdx.x; idx < NT * MS * 64; idx += WAVES * 64) {
        const int ln = idx & 63, blk = idx >> 6;
        const int nt = blk / MS, sp = blk - nt * MS;
        const int h = ln >> 4, j = ln & 15;
        const int n = 16 * nt + 4 * (j & 3) + (j >> 2);
        h8 v;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int m = 32 * sp + (e < 4 ? 0 : 16) + 8 * (h & 1) + 4 * (h >> 1) + (e & 3);
            v[e] = (H)((m < M && n < N) ? a.A[(size_t)m * N + n] : 0.f);
        }
        sA2[idx] = v;
    }
    float invL = a.invL, thr = a.thr;
    if (a.L_dev) {
        const float L = *a.L_dev;
        invL = 1.f / L;
        thr = (float)(a.lambda / (double)L);
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int h = lane >> 4;
    const int j = lane & 15;
    const int64_t pix = ((int64_t)blockIdx.x * WAVES + wave) * 16 + j;
    const bool valid = pix < a.P;
    const int cm_h = 8 * (h & 1) + 4 * (h >> 1);

    v4f Yr[MT];
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
            Yr[mt][r] = v;
        }
    bad |= __shfl_xor(bad, 16);
    bad |= __shfl_xor(bad, 32);
    if (bad) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) Yr[mt] = v4f{0.f, 0.f, 0.f, 0.f};
    }
    v4f Xr[NT], Zr[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int n = 16 * nt + 4 * r + h;
            float v = 0.f;
            if (a.X0 && valid && !bad && n < N) v = a.X0[pix * N + n];
            Xr[nt][r] = v;
            Zr[nt][r] = v;
        }
    v4f U1[MT], V[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) U1[mt] = -Yr[mt];
    if (a.X0) {
#pragma unroll
        for (int sp = 0; sp < NS; ++sp) {
            const h8 xb = pack8<H>(Xr[2 * sp], Xr[2 * sp + 1]);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) U1[mt] = mfma16<H>(sA1[(mt * NS + sp) * 64 + lane], xb, U1[mt]);
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

    if constexpr (!FREEZE) {
        // -y is kept (LDS for YL, else the registers), so that U_i starts
        // from it without a negation per iteration
        v4f* const ylds = sY + (YL ? wave * MT * 64 + lane : 0);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            if constexpr (YL) ylds[mt * 64] = -Yr[mt];
            else Yr[mt] = -Yr[mt];
        }
        auto ynt = [&](int mt) -> v4f { if constexpr (YL) return ylds[mt * 64]; else return Yr[mt]; };
        for (int it = 0; it < a.max_iter; ++it) {
            const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
            const float bcur = (float)((t - 1.0) / tn);
            t = tn;
            // -V / L with V = A z^{i-1} - y, packed, so that the MFMA
            // accumulates z - A^T V / L onto z (step 1); then V keeps U_{i-1}
            // and U1 accumulates U_i = A x^i - y
            const float cu = -(1.f + bprev) * invL, cv = bprev * invL;
            h8 Vb[MS];
#pragma unroll
            for (int sp = 0; sp < MS; ++sp) {
                const v4f v0 = cu * U1[2 * sp] + cv * V[2 * sp];
                const v4f v1 = cu * U1[2 * sp + 1] + cv * V[2 * sp + 1];
                Vb[sp] = pack8<H>(v0, v1);
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                V[mt] = U1[mt];
                U1[mt] = ynt(mt);
            }
#pragma unroll
            for (int np = 0; np < NS; ++np) {
                // keeps the scheduler from hoisting the operand reads of every
                // tile pair at once (their registers would not fit)
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const int nt = 2 * np + q;
                    v4f aux4 = Zr[nt];
#pragma unroll
                    for (int sp = 0; sp < MS; ++sp) aux4 = mfma16<H>(sA2[(nt * MS + sp) * 64 + lane], Vb[sp], aux4);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float aux = aux4[r];
                        const float xn = aux - __builtin_amdgcn_fmed3f(aux, -thr, thr);
                        Zr[nt][r] = xn + bcur * (xn - Xr[nt][r]);
                        Xr[nt][r] = xn;
                    }
                }
                const h8 xb = pack8<H>(Xr[2 * np], Xr[2 * np + 1]);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) U1[mt] = mfma16<H>(sA1[(mt * NS + np) * 64 + lane], xb, U1[mt]);
            }
            if (it == a.max_iter - 1) {
                const float c0 = (it == 0 && a.X0) ? 1.f : 0.f;
                float d2 = 0.f;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const v4f yn = ynt(mt);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float ref = V[mt][r] - c0 * (V[mt][r] - yn[r]);
                        const float d = U1[mt][r] - ref;
                        d2 += d * d;
                    }
                }
                last_d2 = quad_sum(d2);
            }
            bprev = bcur;
        }
        iters = a.max_iter;
    } else {
    for (int it = 0; it < a.max_iter; ++it) {
        const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
        const float bcur = (float)((t - 1.0) / tn);
        t = tn;
        const float cp = 1.f + bprev;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) V[mt] = cp * U1[mt] - bprev * V[mt];
        h8 Vb[MS];
#pragma unroll
        for (int sp = 0; sp < MS; ++sp) Vb[sp] = pack8<H>(V[2 * sp], V[2 * sp + 1]);
        v4f Un[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) Un[mt] = -Yr[mt];
#pragma unroll
        for (int np = 0; np < NS; ++np) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int nt = 2 * np + q;
                v4f W = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int sp = 0; sp < MS; ++sp) W = mfma16<H>(sA2[(nt * MS + sp) * 64 + lane], Vb[sp], W);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float aux = Zr[nt][r] - W[r] * invL;
                    const float xn = soft_thr(aux, thr);
                    const float zn = xn + bcur * (xn - Xr[nt][r]);
                    Xr[nt][r] = active ? xn : Xr[nt][r];
                    Zr[nt][r] = active ? zn : Zr[nt][r];
                }
            }
            const h8 xb = pack8<H>(Xr[2 * np], Xr[2 * np + 1]);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) Un[mt] = mfma16<H>(sA1[(mt * NS + np) * 64 + lane], xb, Un[mt]);
        }
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
            U1[mt] = active ? Un[mt] : U1[mt];
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
                const int n = 16 * nt + 4 * r + h;
                if (n < N) a.X[pix * N + n] = bad ? 0.f : Xr[nt][r];
            }
        if (a.stats && h == 0) {
            csrec_pixel_stats s;
            s.iters = bad ? 0 : iters + a.iter_offset;
            s.flags = bad ? CSREC_FLAG_NONFINITE : (converged ? CSREC_FLAG_CONVERGED : CSREC_FLAG_ITER_CAP);
            s.resid = bad ? 0.f : sqrtf(r2);
            s.delta = bad ? __builtin_nanf("") : sqrtf(last_d2);
            a.stats[pix] = s;
        }
    }
}

// ---------------------------------------------------------------- dispatch

typedef void (*fista_kernel_t)(FistaArgs);

struct FistaVariant {
    int MT, NT, waves;
    fista_kernel_t fn;
    fista_kernel_t fn_nostop = nullptr;   // for eps = 0, where faster
    int waves_nostop = 0;                 // its workgroup's waves (0: waves)
};

// Tile shapes instantiated: the 2.5x-compressed band counts of the paper's
// cubes and the synthetic workloads (N = 100, 154, 198/200, 224) plus
// general shapes.  A shape runs on the smallest variant covering it; the
// extra rows/columns of A are zero in LDS.
const FistaVariant kVariants[] = {
    {1, 2, 4, fista_f32_kernel<1, 2, 4, 2>, fista_f32i_kernel<1, 2, 4, 2>},
    {2, 4, 4, fista_f32_kernel<2, 4, 4, 2>, fista_f32i_kernel<2, 4, 4, 2>},
    {3, 7, 4, fista_f32_kernel<3, 7, 4, 2>, fista_f32i_kernel<3, 7, 4, 2>},
    {4, 8, 4, fista_f32_kernel<4, 8, 4, 2>, fista_f32i_kernel<4, 8, 4, 2>},
    {4, 10, 4, fista_f32_kernel<4, 10, 4, 1>, fista_f32i_kernel<4, 10, 4, 1>},
    {5, 13, 4, fista_f32_kernel<5, 13, 4, 1>, fista_f32i_kernel<5, 13, 4, 1>},
    {6, 14, 4, fista_f32_kernel<6, 14, 4, 1>, fista_f32i8_kernel<6, 14>, 8},
    {7, 16, 4, fista_f32_kernel<7, 16, 4, 1>, fista_f32i_kernel<7, 16, 4, 1>},
    {8, 16, 4, fista_f32_kernel<8, 16, 4, 1>, fista_f32i_kernel<8, 16, 4, 1>},
};

// The pre-arranged form (two LDS copies of A), for the shapes it fits; at
// (4, 10) and (5, 13) the solves without the Delta stop run the eight-wave
// single-copy form instead, whose second wave per SIMD outweighs the four
// 4-byte operand reads per 16-byte one (6.59 against 7.63 ms on the
// 256x256 N=200 M=80 cube, 200 iterations).
const FistaVariant kVariantsS[] = {
    {1, 2, 4, fista_f32s_kernel<1, 2, 4, 2>},
    {2, 4, 4, fista_f32s_kernel<2, 4, 4, 2>},
    {3, 7, 4, fista_f32s_kernel<3, 7, 4, 2>},
    {4, 8, 4, fista_f32s_kernel<4, 8, 4, 2>},
    {4, 10, 4, fista_f32s_kernel<4, 10, 4, 1>, fista_f32i8_kernel<4, 10>, 8},
    {5, 13, 4, fista_f32s_kernel<5, 13, 4, 1>, fista_f32i8_kernel<5, 13>, 8},
};

// Without the Delta stop the (6, 14) shape runs eight waves on one LDS copy
// of A (two per SIMD: the copy, 84 KiB, leaves no room for a second
// workgroup) with y in LDS; at (8, 16) the copy (128 KiB) leaves no room for
// y, and it stays at four.
const FistaVariant kVariantsBF16[] = {
    {2, 8, 4, fista_lp_kernel<__bf16, 2, 8, 4, 2>, fista_lp_kernel<__bf16, 2, 8, 4, 2, false>},
    {4, 8, 4, fista_lp_kernel<__bf16, 4, 8, 4, 2>, fista_lp_kernel<__bf16, 4, 8, 4, 2, false>},
    {4, 10, 4, fista_lp_kernel<__bf16, 4, 10, 4, 2>, fista_lp_kernel<__bf16, 4, 10, 4, 2, false>},
    {6, 14, 4, fista_lp_kernel<__bf16, 6, 14, 4, 1>, fista_lp_kernel<__bf16, 6, 14, 8, 1, false>, 8},
    {8, 16, 4, fista_lp_kernel<__bf16, 8, 16, 4, 1>, fista_lp_kernel<__bf16, 8, 16, 4, 1, false>},
};
const FistaVariant kVariantsF16[] = {
    {2, 8, 4, fista_lp_kernel<_Float16, 2, 8, 4, 2>, fista_lp_kernel<_Float16, 2, 8, 4, 2, false>},
    {4, 8, 4, fista_lp_kernel<_Float16, 4, 8, 4, 2>, fista_lp_kernel<_Float16, 4, 8, 4, 2, false>},
    {4, 10, 4, fista_lp_kernel<_Float16, 4, 10, 4, 2>, fista_lp_kernel<_Float16, 4, 10, 4, 2, false>},
    {6, 14, 4, fista_lp_kernel<_Float16, 6, 14, 4, 1>, fista_lp_kernel<_Float16, 6, 14, 8, 1, false>, 8},
    {8, 16, 4, fista_lp_kernel<_Float16, 8, 16, 4, 1>, fista_lp_kernel<_Float16, 8, 16, 4, 1, false>},
};

template <size_t K>
const FistaVariant* pick_from(const FistaVariant (&vs)[K], int M, int N) {
    const int mt = (int)ceil_div(M, 16), nt = (int)ceil_div(N, 16);
    const FistaVariant* best = nullptr;
    for (const auto& v : vs)
        if (v.MT >= mt && v.NT >= nt && (!best || v.MT * v.NT < best->MT * best->NT)) best = &v;
    return best;
}

const FistaVariant* pick(int M, int N, int prec) {
    if (prec == CSREC_PREC_BF16) return pick_from(kVariantsBF16, M, N);
    if (prec == CSREC_PREC_F16) return pick_from(kVariantsF16, M, N);
    const FistaVariant* v = pick_from(kVariants, M, N);
    const FistaVariant* w = pick_from(kVariantsS, M, N);
    return (w && v && w->MT == v->MT && w->NT == v->NT) ? w : v;
}

const FistaVariant* pick_f32(int M, int N) {
    const int mt = (int)ceil_div(M, 16), nt = (int)ceil_div(N, 16);
    const FistaVariant* best = nullptr;
    for (const auto& v : kVariants)
        if (v.MT >= mt && v.NT >= nt && (!best || v.MT * v.NT < best->MT * best->NT)) best = &v;
    return best;
}

}  // namespace

int fista_supported(int M, int N, int prec) {
    if (!pick(M, N, prec)) return CSREC_E_UNSUPPORTED;
    if (prec != CSREC_PREC_F32 && !pick(M, N, CSREC_PREC_F32)) return CSREC_E_UNSUPPORTED;
    return CSREC_OK;
}

size_t fista_workspace(int, int, int64_t, int) { return 0; }

namespace {
int launch_variant(const FistaVariant* v, const FistaArgs& a, hipStream_t stream) {
    const bool nostop = a.eps <= 0.f && v->fn_nostop;
    const fista_kernel_t fn = nostop ? v->fn_nostop : v->fn;
    const int waves = (nostop && v->waves_nostop) ? v->waves_nostop : v->waves;
    const int64_t pix_per_block = 16 * waves;
    const int64_t blocks = ceil_div(a.P, pix_per_block);
    if (blocks > 0x7fffffff) return CSREC_E_SHAPE;
    hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(64 * waves), 0, stream, a);
    CSREC_HIP_TRY(hipGetLastError());
    return CSREC_OK;
}
}  // namespace

int fista_launch(const FistaLaunch& l) {
    if (l.P == 0) return CSREC_OK;
    const FistaVariant* v = pick(l.M, l.N, l.prec);
    if (!v) return CSREC_E_UNSUPPORTED;
    FistaArgs a;
    a.A = l.A;
    a.Y = l.Y;
    a.X0 = l.X0;
    a.X = l.X;
    a.stats = l.stats;
    a.L_dev = l.L_dev;
    a.M = l.M;
    a.N = l.N;
    a.P = l.P;
    a.max_iter = l.max_iter;
    a.iter_offset = 0;
    a.invL = l.invL;
    a.thr = l.thr;
    a.eps = l.eps;
    a.lambda = l.lambda;
    int e = launch_variant(v, a, l.stream);
    if (e || l.prec == CSREC_PREC_F32 || l.correction_iters <= 0) return e;
    // FP32 correction: warm start from the 16-bit result (momentum restarts);
    // each pixel's lanes read x before they write it, so X0 = X is safe.
    a.X0 = l.X;
    a.max_iter = l.correction_iters;
    a.iter_offset = l.max_iter;
    return launch_variant(pick(l.M, l.N, CSREC_PREC_F32), a, l.stream);
}

// ---------------------------------------------------------------- L by power iteration

namespace {
// L = lambda_max(A^T A) (Eq. 2): power iteration v <- A^T A v / ||A^T A v||
// with the Rayleigh quotient ||A v||^2 (||v|| = 1) as the estimate.  One
// workgroup; A is small (at most 256 x 256) and read from L2.
__device__ float block_sum(float v, float* red) {
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    const float out = red[0];
    __syncthreads();
    return out;
}

__global__ __launch_bounds__(256) void lipschitz_kernel(const float* __restrict__ A, int M, int N,
                                                        float* __restrict__ L_out, int iters) {
    __shared__ float v[CSREC_MAX_N];
    __shared__ float u[CSREC_MAX_N];
    __shared__ float w[CSREC_MAX_N];
    __shared__ float red[256];
    const int tid = threadIdx.x;
    float part = 0.f;
    for (int n = tid; n < N; n += 256) {
        v[n] = 1.f + 0.01f * (float)(n % 7);
        part += v[n] * v[n];
    }
    float inv = 1.f / sqrtf(block_sum(part, red));
    for (int n = tid; n < N; n += 256) v[n] *= inv;
    __syncthreads();
    float lam = 0.f;
    for (int it = 0; it < iters; ++it) {
        part = 0.f;
        for (int m = tid; m < M; m += 256) {
            float s = 0.f;
            for (int n = 0; n < N; ++n) s += A[(size_t)m * N + n] * v[n];
            u[m] = s;
            part += s * s;
        }
        lam = block_sum(part, red);          // ||A v||^2
        part = 0.f;
        for (int n = tid; n < N; n += 256) {
            float s = 0.f;
            for (int m = 0; m < M; ++m) s += A[(size_t)m * N + n] * u[m];
            w[n] = s;
            part += s * s;
        }
        inv = 1.f / sqrtf(block_sum(part, red));
        for (int n = tid; n < N; n += 256) v[n] = w[n] * inv;
        __syncthreads();
    }
    if (tid == 0) *L_out = lam;
}
}  // namespace

int lipschitz_launch(const float* A, int M, int N, float* L_out, hipStream_t stream) {
    hipLaunchKernelGGL(lipschitz_kernel, dim3(1), dim3(256), 0, stream, A, M, N, L_out, 400);
    CSREC_HIP_TRY(hipGetLastError());
    return CSREC_OK;
}

}  // namespace csrec
