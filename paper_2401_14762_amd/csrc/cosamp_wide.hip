// CoSaMP (Alg. 5) when the merged support c = Theta U c^{i-1} can hold more
// atoms than there are measurements (3K > M).  Step 2's pseudo-inverse
// A(:, c)^+ y is then the least-squares solution while |c| <= M and the
// minimum-norm solution of A(:, c) s = y once |c| > M (A(:, c) has full row
// rank).  Both are solved from a symmetric positive definite system:
//   |c| <= M:  (A_c^T A_c) s = A_c^T y                 (d = |c|)
//   |c| >  M:  (A_c A_c^T) w = y,  s = A_c^T w         (d = M)
// In floating point both square the condition number of A_c, so this path
// computes in FP64 throughout (A and y are FP32 inputs; their products are
// exact in FP64).
//
// One pixel per workgroup of 256 threads (four waves), every step spread over
// the workgroup:
//   1. p = A^T r: thread j owns atom j (N <= 256), a coalesced read of row i
//      of A per step of the M-long dot product.  Theta = the 2K atoms of
//      largest |p| by rank (|p| descending, index ascending), each thread
//      counting the atoms ahead of its own, so no sequential selection.
//      c = Theta U c^{i-1} is compacted in ascending atom order with wave
//      ballots.
//   2. A_c is staged in LDS (FP32, the orientation of the system's inner
//      product, rows padded to 4 columns), the d x d system matrix is formed
//      by 4 x 4 register tiles of its lower triangle (packed in LDS, FP64),
//      then factored as L D L^T right-looking, one barrier per column, with
//      the right-hand side eliminated alongside.  The back substitution runs
//      on wave 0 with the right-hand side in registers.  Pivots are floored
//      at 2^-52 of the original diagonal, so a numerically dependent
//      column keeps the factor finite.
//   3. q = the K entries of largest |s| by rank (NaN-safe key, ties to the
//      lower atom index).
//   4. r = y - A(:, q) s_q from the staged A_c; Delta and ||r|| by
//      workgroup reductions; the stop tests of the on-chip kernels.
//
// LDS per workgroup (bytes): 8 (M(M+1)/2 + 3M + max(M, 3K) + 3K + N + 8)
// for the FP64 system, vectors and reductions, 4 ceil4(M) max(M, 3K) for
// A_c, and 4 (5K + N + 8) for index lists: about 76 KB at M = 90, N = 224,
// K = 33 (two workgroups, eight waves, per CU).
#include "common.hpp"

#include <cmath>

namespace csrec {
namespace {

constexpr int kWideThreads = 256;

struct WideArgs {
    const float* A;       // M x N row-major
    const float* Y;       // P x M
    float* X;             // P x N
    int32_t* support;     // P x K, nullable
    csrec_pixel_stats* stats;   // P, nullable
    int M, N, K, max_iter;
    double res_tol, eps;
    int64_t p0;
};

struct WideLds {
    double* C;       // packed lower triangle, d(d+1)/2
    double* y;       // M
    double* r;       // M
    double* w;       // max(M, 3K): right-hand side, then the solution
    double* dg;      // M: original diagonal (pivot floor), then the pivots D
    double* s;       // 3K: least-squares values on c
    double* p;       // N: |A^T r|
    double* red;     // 8
    float* Z;        // staged A_c, R rows of ceil4(d) columns
    int* T;          // 3K: the merged support c, ascending
    int* qpos;       // K: positions in T of the kept atoms
    int* qidx;       // K: their atom indices
    int* prev;       // N: 1 for atoms of c^{i-1}
    int* cnt;        // 8
};

__host__ __device__ inline int ceil4(int v) { return (v + 3) & ~3; }

// FP64 entries (an even count, so A_c's float4 rows stay 16-byte aligned)
__host__ __device__ inline int wide_doubles(int M, int N, int K) {
    const int wlen = M > 3 * K ? M : 3 * K;
    const int nd = M * (M + 1) / 2 + 3 * M + wlen + 3 * K + N + 8;
    return (nd + 1) & ~1;
}

// A_c staged: M rows of ceil4(|c|) (|c| <= M) or |c| <= 3K rows of ceil4(M)
__host__ __device__ inline int wide_floats(int M, int K) { return ceil4(M) * (M > 3 * K ? M : 3 * K); }

__host__ __device__ inline size_t wide_lds_bytes(int M, int N, int K) {
    return (size_t)wide_doubles(M, N, K) * 8 + (size_t)wide_floats(M, K) * 4 + (size_t)(3 * K + 2 * K + N + 8) * 4;
}

__device__ inline WideLds carve_wide(char* base, int M, int N, int K) {
    WideLds L;
    double* const d0 = reinterpret_cast<double*>(base);
    double* d = d0;
    const int wlen = M > 3 * K ? M : 3 * K;
    L.C = d;
    d += M * (M + 1) / 2;
    L.y = d;
    d += M;
    L.r = d;
    d += M;
    L.w = d;
    d += wlen;
    L.dg = d;
    d += M;
    L.s = d;
    d += 3 * K;
    L.p = d;
    d += N;
    L.red = d;
    float* f = reinterpret_cast<float*>(d0 + wide_doubles(M, N, K));
    L.Z = f;
    f += wide_floats(M, K);
    int* i = reinterpret_cast<int*>(f);
    L.T = i;
    i += 3 * K;
    L.qpos = i;
    i += K;
    L.qidx = i;
    i += K;
    L.prev = i;
    i += N;
    L.cnt = i;
    return L;
}

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum of v over the workgroup; every thread gets the total.  red must not be
// read by a thread still in an earlier reduction (a barrier separates them).
__device__ inline double block_sum(double v, double* red, int slot) {
    v = wave_sum(v);
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[slot * 4 + wid] = v;
    __syncthreads();
    return red[slot * 4 + 0] + red[slot * 4 + 1] + red[slot * 4 + 2] + red[slot * 4 + 3];
}

// Compacts the threads with pred set, in thread order: returns this thread's
// slot (valid when pred) and writes the total to *total.
__device__ inline int block_compact(bool pred, int* cnt, int* total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const unsigned long long m = __ballot(pred);
    const int below = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) cnt[wid] = __popcll(m);
    __syncthreads();
    int off = 0;
    for (int w = 0; w < wid; ++w) off += cnt[w];
    *total = cnt[0] + cnt[1] + cnt[2] + cnt[3];
    return off + below;
}

__global__ __launch_bounds__(kWideThreads) void cosamp_wide_kernel(WideArgs a) {
    extern __shared__ __align__(16) char lds_raw[];
    const int M = a.M, N = a.N, K = a.K;
    const int tid = threadIdx.x;
    const int64_t pix = a.p0 + blockIdx.x;
    WideLds L = carve_wide(lds_raw, M, N, K);

    // y, the finite check, ||y||
    double yy = 0.0;
    bool bad = false;
    for (int i = tid; i < M; i += kWideThreads) {
        const float v = a.Y[pix * M + i];
        bad |= !isfinite(v);
        L.y[i] = v;
        L.r[i] = v;
        yy += (double)v * v;
    }
    for (int j = tid; j < N; j += kWideThreads) L.prev[j] = 0;
    const int nbad = __syncthreads_or(bad);
    const double y2 = block_sum(yy, L.red, 0);
    const double ynorm = sqrt(y2);

    double rn2 = y2, last_d2 = __builtin_nan("");
    int iters = 0, nq = 0;
    bool converged = false;
    if (!nbad) {
        for (int it = 1; it <= a.max_iter; ++it) {
            // step 1: p = A^T r, Theta, c = Theta U c^{i-1}
            const int j = tid;
            double key = -1.0;
            if (j < N) {
                double acc = 0.0;
                for (int i = 0; i < M; ++i) acc = fma((double)a.A[(size_t)i * N + j], L.r[i], acc);
                key = fabs(acc);
                key = key == key ? key : -1.0;
                L.p[j] = key;
            }
            __syncthreads();
            bool inc = false;
            if (j < N) {
                int rank = 0;
                for (int k = 0; k < N; ++k) {
                    const double o = L.p[k];
                    rank += (o > key || (o == key && k < j)) ? 1 : 0;
                }
                inc = rank < 2 * K || L.prev[j] != 0;
            }
            int nT;
            const int slot = block_compact(inc, L.cnt, &nT);
            if (inc) L.T[slot] = j;
            __syncthreads();

            // step 2: stage A_c; the system, its L D L^T factor, the solve
            const bool wide = nT > M;
            const int d = wide ? M : nT;       // system order
            const int R = wide ? nT : M;       // inner dimension
            const int d4 = ceil4(d);
            for (int e = tid; e < R * d4; e += kWideThreads) {
                const int t = e / d4, u = e - t * d4;
                float v = 0.f;
                if (u < d) v = wide ? a.A[(size_t)u * N + L.T[t]] : a.A[(size_t)t * N + L.T[u]];
                L.Z[e] = v;
            }
            __syncthreads();
            {
                const int nb = d4 >> 2;
                for (int e = tid; e < nb * (nb + 1) / 2; e += kWideThreads) {
                    int bu = (int)((sqrtf(8.f * e + 1.f) - 1.f) * 0.5f);
                    while (bu * (bu + 1) / 2 > e) --bu;
                    while ((bu + 1) * (bu + 2) / 2 <= e) ++bu;
                    const int bv = e - bu * (bu + 1) / 2;
                    double acc[4][4] = {};
                    for (int t = 0; t < R; ++t) {
                        const float4 zu = *reinterpret_cast<const float4*>(L.Z + t * d4 + 4 * bu);
                        const float4 zv = *reinterpret_cast<const float4*>(L.Z + t * d4 + 4 * bv);
                        const double U[4] = {zu.x, zu.y, zu.z, zu.w};
                        const double V[4] = {zv.x, zv.y, zv.z, zv.w};
#pragma unroll
                        for (int x = 0; x < 4; ++x)
#pragma unroll
                            for (int y = 0; y < 4; ++y) acc[x][y] = fma(U[x], V[y], acc[x][y]);
                    }
#pragma unroll
                    for (int x = 0; x < 4; ++x) {
                        const int u = 4 * bu + x;
#pragma unroll
                        for (int y = 0; y < 4; ++y) {
                            const int v = 4 * bv + y;
                            if (u < d && v <= u) {
                                L.C[u * (u + 1) / 2 + v] = acc[x][y];
                                if (u == v) L.dg[u] = acc[x][y];
                            }
                        }
                    }
                }
                // right-hand side: A_c^T y (|c| <= M) or y
                for (int u = tid; u < d; u += kWideThreads) {
                    double acc = 0.0;
                    if (wide) {
                        acc = L.y[u];
                    } else {
                        for (int t = 0; t < R; ++t) acc = fma((double)L.Z[t * d4 + u], L.y[t], acc);
                    }
                    L.w[u] = acc;
                }
            }
            __syncthreads();
            // L D L^T, right-looking; the right-hand side is column d of the
            // augmented matrix and is eliminated with the rest
            const int tx = tid & 15, ty = tid >> 4;
            for (int k = 0; k < d; ++k) {
                const double floor_k = fmax(L.dg[k] * 0x1p-52, 1e-300);
                double Dk = L.C[k * (k + 1) / 2 + k];
                Dk = Dk > floor_k ? Dk : floor_k;
                const double iDk = 1.0 / Dk;
                const double wk = L.w[k];
                for (int u = k + 1 + ty; u < d; u += 16) {
                    const double cu = L.C[u * (u + 1) / 2 + k] * iDk;
                    for (int v = k + 1 + tx; v <= u; v += 16) L.C[u * (u + 1) / 2 + v] -= cu * L.C[v * (v + 1) / 2 + k];
                    if (tx == 0) L.w[u] -= cu * wk;
                }
                __syncthreads();
                if (tid == 0) L.dg[k] = Dk;    // dg[k] is not read again as a floor
            }
            __syncthreads();
            // back substitution L^T s = D^-1 w on wave 0, lane l holding
            // entries l and l + 64 (d <= 128)
            if (tid < 64) {
                const int l = tid;
                double z0 = 0.0, z1 = 0.0, id0 = 0.0, id1 = 0.0;
                if (l < d) {
                    id0 = 1.0 / L.dg[l];
                    z0 = L.w[l] * id0;
                }
                if (l + 64 < d) {
                    id1 = 1.0 / L.dg[l + 64];
                    z1 = L.w[l + 64] * id1;
                }
                for (int k = d - 1; k >= 0; --k) {
                    const double zk = __shfl(k < 64 ? z0 : z1, k & 63, 64);
                    const int row = k * (k + 1) / 2;
                    if (l < k) z0 -= L.C[row + l] * id0 * zk;
                    if (l + 64 < k) z1 -= L.C[row + l + 64] * id1 * zk;
                }
                if (l < d) L.w[l] = z0;
                if (l + 64 < d) L.w[l + 64] = z1;
            }
            __syncthreads();
            // s on c: the solution itself, or A_c^T w
            for (int t = tid; t < nT; t += kWideThreads) {
                double v;
                if (wide) {
                    v = 0.0;
                    for (int u = 0; u < M; ++u) v = fma((double)L.Z[t * d4 + u], L.w[u], v);
                } else {
                    v = L.w[t];
                }
                L.s[t] = v;
            }
            __syncthreads();

            // step 3: q = the K largest |s| on c
            bool keep = false;
            if (tid < nT) {
                double kv = fabs(L.s[tid]);
                kv = kv == kv ? kv : -1.0;
                int rank = 0;
                for (int b = 0; b < nT; ++b) {
                    double o = fabs(L.s[b]);
                    o = o == o ? o : -1.0;
                    rank += (o > kv || (o == kv && b < tid)) ? 1 : 0;
                }
                keep = rank < K;
            }
            for (int jj = tid; jj < N; jj += kWideThreads) L.prev[jj] = 0;
            int kept;
            const int ks = block_compact(keep, L.cnt + 4, &kept);
            if (keep) {
                L.qpos[ks] = tid;
                L.qidx[ks] = L.T[tid];
                L.prev[L.T[tid]] = 1;
            }
            nq = kept;
            __syncthreads();

            // step 4: r = y - A(:, q) s_q, Delta, ||r||
            double dd = 0.0, rr = 0.0;
            for (int i = tid; i < M; i += kWideThreads) {
                double v = L.y[i];
                for (int k = 0; k < nq; ++k) {
                    const int t = L.qpos[k];
                    const float aik = wide ? L.Z[t * d4 + i] : L.Z[i * d4 + t];
                    v = fma(-(double)aik, L.s[t], v);
                }
                const double df = v - L.r[i];
                dd = fma(df, df, dd);
                rr = fma(v, v, rr);
                L.r[i] = v;
            }
            const double d2 = block_sum(dd, L.red, 0);
            rn2 = block_sum(rr, L.red, 1);
            last_d2 = d2;
            iters = it;
            if (sqrt(d2) < a.eps || sqrt(rn2) <= a.res_tol * ynorm) {
                converged = true;
                break;
            }
        }
    }

    // x, support, stats
    float* xrow = a.X + pix * N;
    for (int j = tid; j < N; j += kWideThreads) {
        double v = 0.0;
        if (!nbad)
            for (int k = 0; k < nq; ++k) v = L.qidx[k] == j ? L.s[L.qpos[k]] : v;
        xrow[j] = (float)v;
    }
    if (a.support)
        for (int k = tid; k < K; k += kWideThreads) a.support[pix * K + k] = (!nbad && k < nq) ? L.qidx[k] : -1;
    if (a.stats && tid == 0) {
        csrec_pixel_stats st;
        st.iters = nbad ? 0 : iters;
        st.flags = nbad ? CSREC_FLAG_NONFINITE : (converged ? CSREC_FLAG_CONVERGED : CSREC_FLAG_ITER_CAP);
        st.resid = nbad ? 0.f : (float)sqrt(rn2);
        st.delta = (float)sqrt(last_d2);
        a.stats[pix] = st;
    }
}

}  // namespace

int cosamp_wide_supported(int M, int N, int K) {
    if (M < 1 || M > 96 || N < 1 || N > kWideThreads) return CSREC_E_UNSUPPORTED;
    if (K < 1 || 3 * K > N || 3 * K > 128) return CSREC_E_SHAPE;
    return CSREC_OK;
}

int cosamp_wide_launch(const GreedyLaunch& g) {
    if (g.P == 0) return CSREC_OK;
    const int e = cosamp_wide_supported(g.M, g.N, g.K);
    if (e) return e;
    WideArgs a;
    a.A = g.A;
    a.Y = g.Y;
    a.X = g.X;
    a.support = g.support;
    a.stats = g.stats;
    a.M = g.M;
    a.N = g.N;
    a.K = g.K;
    a.max_iter = g.max_iter;
    a.res_tol = g.res_tol;
    a.eps = g.eps;
    const size_t lds = wide_lds_bytes(g.M, g.N, g.K);
    CSREC_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(cosamp_wide_kernel),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    constexpr int64_t kChunk = int64_t(1) << 20;
    for (int64_t p0 = 0; p0 < g.P; p0 += kChunk) {
        const int64_t np = (g.P - p0) < kChunk ? (g.P - p0) : kChunk;
        a.p0 = p0;
        hipLaunchKernelGGL(cosamp_wide_kernel, dim3((unsigned)np), dim3(kWideThreads), lds, g.stream, a);
        CSREC_HIP_TRY(hipGetLastError());
    }
    return CSREC_OK;
}

}  // namespace csrec
