// gOMP (Alg. 3) with the least-squares state on chip.
//
// Work decomposition.  A workgroup is one wavefront holding 4 pixels; the
// 16 lanes t = 0..15 of lane row g cooperate on pixel g.  Every per-pixel
// quantity lives in LDS or in the lanes' registers for the whole solve, so
// the solve reads y and A^T and writes x, and nothing else leaves the CU.
//
// Least squares without triangular-solve chains.  With G[c,c] = L L^T the
// kernel keeps W = L^{-1} (lower triangular, packed rows in LDS) instead of
// L.  Appending atom j to c (a bordered Cholesky step) is then
//   l = W G[c, j],  d = G_jj - ||l||^2,  new row of W = [-l^T W, 1] / sqrt(d)
// and the least-squares solution of G[c,c] s = b_c is s = W^T (W b_c), with
// z = W b_c extended by one dot product per append.  Every one of these is a
// matrix-vector product whose rows (or columns) the 16 lanes split, so a step
// has constant depth instead of the |c| sequential steps of forward and back
// substitution.  d / G_jj is the pivot ratio (squared distance of a_j from
// span(A[:, c]) over ||a_j||^2); a pixel with a ratio below the threshold is
// marked for the FP64 pass of the scratch-based kernel.
//
// Per iteration (Alg. 3, steps 1-4), for each active pixel:
//   1. p = A^T r: lane t forms p_n for n = t + 16k from A^T rows (global,
//      L2-resident) and r (LDS); S rounds of a 16-lane argmax over the
//      non-members of c, ties to the lower index.
//   2. append the S atoms (above); s = W^T z.
//   3. if |c| > K: rank the |s_i| (ties to the lower index), keep the top K
//      as q, build the inverse factor of G[q, q] by K appends, s_q = W_q^T z_q.
//   4. r = y - A(:, q) s_q with lane t owning m = 4t + j + 64i; Delta, ||r||.
#include "common.hpp"

#include <cmath>

namespace csrec {
namespace {

constexpr int kGroups = 4;        // pixels per wavefront
constexpr int kMaxNT = 16;        // N <= 256

struct CoopArgs {
    const float* AT;      // N x MP, row n = column n of A (zero padded to MP)
    const float* Y;       // P x M
    const float* G32;     // N x N
    float* X;
    int32_t* support;
    csrec_pixel_stats* stats;
    uint32_t* fbflag;     // per pixel (chunk-local) FP64 hand-off, may be null
    int M, N, MP, K, S, Imax, prune;
    float res_tol, eps;
    double pivot_thr;
    int64_t P;            // pixels of this launch
    int64_t p0;           // first pixel (index into Y/X/support/stats)
    int CM;               // S * Imax
    int lds_floats;       // per pixel
};

__device__ __forceinline__ int tri(int k) { return k * (k + 1) / 2; }

// Atom indices read back from LDS are kept inside [0, N) before they address
// global memory.
__device__ __forceinline__ int clamp_atom(int j, int N) { return (unsigned)j < (unsigned)N ? j : 0; }

// Sum over the 16 lanes of a lane row.
__device__ __forceinline__ float row_sum(float v) {
    v += __shfl_xor(v, 8);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 1);
    return v;
}

// (value desc, index asc) argmax over a lane row; index -1 never wins.
__device__ __forceinline__ void row_argmax(float& v, int& i) {
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
        const float ov = __shfl_xor(v, o);
        const int oi = __shfl_xor(i, o);
        const bool take = (oi >= 0) && (i < 0 || ov > v || (ov == v && oi < i));
        v = take ? ov : v;
        i = take ? oi : i;
    }
}

// Per-pixel LDS carving (floats; index arrays stored as int bit patterns).
struct PixLds {
    float* rb;    // residual broadcast, MP
    float* W;     // inverse factor of G[c,c], tri(CM)
    float* z;     // W b_c, CM
    float* b;     // b_c, CM
    int* c;       // atoms, CM
    float* s;     // solution on c, CM
    float* g;     // temporary column, CM (also q-append temporaries)
    float* l;     // temporary, CM
    float* Wq;    // inverse factor of G[q,q], tri(K)
    float* zq;    // K
    float* bq;    // K
    int* q;       // K
    float* sq;    // K
};

__device__ __forceinline__ PixLds carve(float* base, const CoopArgs& a) {
    PixLds p;
    float* o = base;
    p.rb = o; o += a.MP;
    p.W = o; o += tri(a.CM);
    p.z = o; o += a.CM;
    p.b = o; o += a.CM;
    p.c = reinterpret_cast<int*>(o); o += a.CM;
    p.s = o; o += a.CM;
    p.g = o; o += a.CM;
    p.l = o; o += a.CM;
    p.Wq = o; o += tri(a.K);
    p.zq = o; o += a.K;
    p.bq = o; o += a.K;
    p.q = reinterpret_cast<int*>(o); o += a.K;
    p.sq = o;
    return p;
}

// One bordered step of the inverse factor: appends atom `atom` (rhs bj) to
// the factor (Wf, zf, bf, idx) of size n.  gcol[i] must hold G[idx[i], atom]
// for i < n (written by the caller before the barrier).  All 64 lanes call it;
// `on` masks the lane rows whose pixel takes part.  Returns d / G_jj.
__device__ float inv_append(bool on, int t, int n, float* Wf, float* zf, float* bf, int* idx, const float* gcol,
                            float* ltmp, int atom, float bj, float gjj) {
    // l = W g (rows i = t + 16u)
    float ll = 0.f;
    if (on) {
        for (int i = t; i < n; i += 16) {
            const float* wr = Wf + tri(i);
            float acc = 0.f;
            for (int k = 0; k <= i; ++k) acc += wr[k] * gcol[k];
            ltmp[i] = acc;
            ll += acc * acc;
        }
    }
    ll = row_sum(ll);
    __syncthreads();
    const float d = gjj - ll;
    const float ratio = d / gjj;
    // A pivot below FP32 resolution (the atom is numerically in the span) is
    // floored so the factor stays finite; such a pixel carries a ratio far
    // below any fallback threshold.
    const float floor_d = gjj * 5.9604645e-8f;
    const float dd = d > floor_d ? d : floor_d;
    const float inv = 1.f / sqrtf(dd);
    // new row: w[k] = -(sum_{i>=k} l_i W[i][k]) * inv, w[n] = inv; z_n = w . [b_c, bj]
    float zp = 0.f;
    if (on) {
        float* wn = Wf + tri(n);
        for (int k = t; k < n; k += 16) {
            float acc = 0.f;
            for (int i = k; i < n; ++i) acc += ltmp[i] * Wf[tri(i) + k];
            const float w = -acc * inv;
            wn[k] = w;
            zp += w * bf[k];
        }
        if (t == 0) {
            wn[n] = inv;
            zp += inv * bj;
        }
    }
    zp = row_sum(zp);
    if (on && t == 0) {
        zf[n] = zp;
        bf[n] = bj;
        idx[n] = atom;
    }
    __syncthreads();
    return ratio;
}

// s = W^T z on the first n entries (columns k = t + 16u).
__device__ void inv_solve(bool on, int t, int n, const float* Wf, const float* zf, float* sf) {
    if (on) {
        for (int k = t; k < n; k += 16) {
            float acc = 0.f;
            for (int i = k; i < n; ++i) acc += Wf[tri(i) + k] * zf[i];
            sf[k] = acc;
        }
    }
    __syncthreads();
}

__device__ __forceinline__ float rank_key(float v) {
    const float a = fabsf(v);
    return a <= 3.402823466e38f ? a : -1.f;   // NaN and inf rank last
}

// Step 3 of Alg. 3 for the lane rows with `on`: q = the K entries of c with
// largest |s| (ties to the lower index), then s_q = G[q,q]^{-1} b_q through
// a fresh inverse factor.  Called by every lane (it holds barriers).
__device__ void prune_to_q(bool on, int t, int nc, int K, int N, const float* G32, const PixLds& L) {
    if (on) {
        // the key maps non-finite |s| below every finite one, so (key desc,
        // index asc) is a strict total order over the distinct atoms of c and
        // the ranks are a permutation: q[0..K) is always fully written
        for (int k = t; k < nc; k += 16) {
            const float vk = rank_key(L.s[k]);
            const int ck = L.c[k];
            int rank = 0;
            for (int i = 0; i < nc; ++i) {
                const float vi = rank_key(L.s[i]);
                const int ci = L.c[i];
                rank += (vi > vk || (vi == vk && ci < ck)) ? 1 : 0;
            }
            if (rank < K) {
                L.q[rank] = ck;
                L.bq[rank] = L.b[k];
            }
        }
    }
    __syncthreads();
    for (int k = 0; k < K; ++k) {
        const int j = on ? clamp_atom(L.q[k], N) : 0;
        if (on)
            for (int i = t; i < k; i += 16) L.g[i] = G32[(size_t)clamp_atom(L.q[i], N) * N + j];
        const float gjj = on ? G32[(size_t)j * N + j] : 1.f;
        const float bj = on ? L.bq[k] : 0.f;
        __syncthreads();
        // the appended entry rewrites q[k] and bq[k] with their own values
        inv_append(on, t, k, L.Wq, L.zq, L.bq, L.q, L.g, L.l, j, bj, gjj);
    }
    inv_solve(on, t, K, L.Wq, L.zq, L.sq);
}

template <int MSLOT>
__device__ __forceinline__ void gomp_coop_body(const CoopArgs& a, int64_t block, float* lds) {
    const int lane = threadIdx.x;
    const int g = lane >> 4, t = lane & 15;
    const int64_t local = block * kGroups + g;
    const int64_t pix = a.p0 + local;
    const bool valid = local < a.P;
    const int M = a.M, N = a.N, K = a.K, MP = a.MP;
    PixLds L = carve(lds + g * a.lds_floats, a);

    // y and r: lane t owns m = 4t + j + 64i (i < MSLOT/4)
    float y[MSLOT], r[MSLOT];
    bool bad = false;
#pragma unroll
    for (int u = 0; u < MSLOT; ++u) {
        const int m = 4 * t + (u & 3) + 64 * (u >> 2);
        float v = 0.f;
        if (valid && m < M) {
            v = a.Y[pix * M + m];
            if (!isfinite(v)) bad = true;
        }
        y[u] = v;
    }
    int badi = bad ? 1 : 0;
    badi |= __shfl_xor(badi, 8);
    badi |= __shfl_xor(badi, 4);
    badi |= __shfl_xor(badi, 2);
    badi |= __shfl_xor(badi, 1);
    bad = badi != 0;
    float y2 = 0.f;
#pragma unroll
    for (int u = 0; u < MSLOT; ++u) {
        if (bad) y[u] = 0.f;
        r[u] = y[u];
        y2 += y[u] * y[u];
    }
    y2 = row_sum(y2);
    const float ynorm = sqrtf(y2);

    bool active = valid && !bad;
    bool converged = false, fallback = false;
    int iters = 0, nc = 0, nx = 0;
    bool x_on_q = false;
    float last_d2 = __builtin_nanf(""), rn2 = y2;
    uint32_t mask = 0u;   // bit k: atom n = t + 16k is in c

    for (int it = 1; it <= a.Imax; ++it) {
        // ---------------- step 1: correlation p = A^T r, top-S over the non-members
#pragma unroll
        for (int u = 0; u < MSLOT; ++u) {
            const int m = 4 * t + (u & 3) + 64 * (u >> 2);
            if (m < MP) L.rb[m] = r[u];
        }
        __syncthreads();
        float p[kMaxNT];
#pragma unroll
        for (int k = 0; k < kMaxNT; ++k) p[k] = 0.f;
        const int M4 = (M + 3) & ~3;
        if (active) {
            for (int m4 = 0; m4 < M4; m4 += 4) {
                const float4 rv = *reinterpret_cast<const float4*>(L.rb + m4);
#pragma unroll
                for (int k = 0; k < kMaxNT; ++k) {
                    const int n = t + 16 * k;
                    if (n < N) {
                        const float4 av = *reinterpret_cast<const float4*>(a.AT + (size_t)n * MP + m4);
                        p[k] += av.x * rv.x + av.y * rv.y + av.z * rv.z + av.w * rv.w;
                    }
                }
            }
        }
        // S rounds of argmax; the winners are appended in selection order
        int sel[8];
        for (int q = 0; q < a.S; ++q) {
            float bv = -1.f;
            int bi = -1;
#pragma unroll
            for (int k = 0; k < kMaxNT; ++k) {
                const int n = t + 16 * k;
                const float v = fabsf(p[k]);
                if (n < N && !((mask >> k) & 1u) && (bi < 0 || v > bv)) {
                    bv = v;
                    bi = n;
                }
            }
            row_argmax(bv, bi);
            sel[q] = bi;
            if (bi >= 0 && (bi & 15) == t) mask |= 1u << (bi >> 4);
        }

        // ---------------- step 2: append the atoms, s = W^T (W b_c)
        for (int q = 0; q < a.S; ++q) {
            const int j = sel[q];
            const bool on = active && j >= 0;
            // b_j = a_j^T y and G[c, j]
            float bpart = 0.f;
            if (on) {
#pragma unroll
                for (int u4 = 0; u4 < MSLOT / 4; ++u4) {
                    const int m = 4 * t + 64 * u4;
                    if (m < MP) {
                        const float4 av = *reinterpret_cast<const float4*>(a.AT + (size_t)j * MP + m);
                        bpart += av.x * y[4 * u4] + av.y * y[4 * u4 + 1] + av.z * y[4 * u4 + 2] + av.w * y[4 * u4 + 3];
                    }
                }
                for (int i = t; i < nc; i += 16) L.g[i] = a.G32[(size_t)L.c[i] * N + j];
            }
            const float bj = row_sum(bpart);
            const float gjj = on ? a.G32[(size_t)j * N + j] : 1.f;
            __syncthreads();
            const float ratio = inv_append(on, t, nc, L.W, L.z, L.b, L.c, L.g, L.l, j, bj, gjj);
            if (on && a.pivot_thr > 0.0 && (double)ratio < a.pivot_thr) fallback = true;
            if (on) ++nc;
        }
        inv_solve(active, t, nc, L.W, L.z, L.s);

        // ---------------- step 3: prune to K and re-solve on q
        const bool prune_g = active && a.prune == CSREC_PRUNE_EACH && nc > K;
        if (__any(prune_g)) {
            prune_to_q(prune_g, t, nc, K, N, a.G32, L);
        }
        // a pixel that stopped earlier keeps the x of its last iteration
        if (prune_g) {
            nx = K;
            x_on_q = true;
        } else if (active) {
            nx = nc;
            x_on_q = false;
        }

        // ---------------- step 4: residual r = y - A x, Delta, stop
        if (active) {
            const int* xi = x_on_q ? L.q : L.c;
            const float* xv = x_on_q ? L.sq : L.s;
            float rnew[MSLOT];
#pragma unroll
            for (int u = 0; u < MSLOT; ++u) rnew[u] = y[u];
            for (int k = 0; k < nx; ++k) {
                const float v = xv[k];
                const float* row = a.AT + (size_t)clamp_atom(xi[k], N) * MP;
#pragma unroll
                for (int u4 = 0; u4 < MSLOT / 4; ++u4) {
                    const int m = 4 * t + 64 * u4;
                    if (m < MP) {
                        const float4 av = *reinterpret_cast<const float4*>(row + m);
                        rnew[4 * u4] -= av.x * v;
                        rnew[4 * u4 + 1] -= av.y * v;
                        rnew[4 * u4 + 2] -= av.z * v;
                        rnew[4 * u4 + 3] -= av.w * v;
                    }
                }
            }
            float d2 = 0.f, n2 = 0.f;
#pragma unroll
            for (int u = 0; u < MSLOT; ++u) {
                const float dlt = rnew[u] - r[u];
                d2 += dlt * dlt;
                n2 += rnew[u] * rnew[u];
                r[u] = rnew[u];
            }
            d2 = row_sum(d2);
            n2 = row_sum(n2);
            iters = it;
            last_d2 = d2;
            rn2 = n2;
            if (sqrtf(n2) <= a.res_tol * ynorm || (a.eps > 0.f && sqrtf(d2) < a.eps)) {
                active = false;
                converged = true;
            }
        }
        __syncthreads();
        if (!__any(active)) break;
    }

    // ---------------- prune placed after the loop (textbook gOMP)
    const bool final_prune = a.prune == CSREC_PRUNE_FINAL && nc > K && valid && !bad;
    if (__any(final_prune)) {
        prune_to_q(final_prune, t, nc, K, N, a.G32, L);
        float n2 = 0.f;
        if (final_prune) {
            nx = K;
            x_on_q = true;
            float rnew[MSLOT];
#pragma unroll
            for (int u = 0; u < MSLOT; ++u) rnew[u] = y[u];
            for (int k = 0; k < nx; ++k) {
                const float v = L.sq[k];
                const float* row = a.AT + (size_t)clamp_atom(L.q[k], N) * MP;
#pragma unroll
                for (int u4 = 0; u4 < MSLOT / 4; ++u4) {
                    const int m = 4 * t + 64 * u4;
                    if (m < MP) {
                        const float4 av = *reinterpret_cast<const float4*>(row + m);
                        rnew[4 * u4] -= av.x * v;
                        rnew[4 * u4 + 1] -= av.y * v;
                        rnew[4 * u4 + 2] -= av.z * v;
                        rnew[4 * u4 + 3] -= av.w * v;
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < MSLOT; ++u) n2 += rnew[u] * rnew[u];
        }
        n2 = row_sum(n2);
        if (final_prune) rn2 = n2;
    }

    if (!valid) return;
    if (a.fbflag) {
        a.fbflag[local] = fallback ? 1u : 0u;
        if (fallback) return;   // the FP64 pass writes this pixel
    }
    // ---------------- outputs: x (dense row), support ascending, stats
    const int* xi = x_on_q ? L.q : L.c;
    const float* xv = x_on_q ? L.sq : L.s;
    float* xrow = a.X + pix * N;
    for (int n = t; n < N; n += 16) {
        float v = 0.f;
        for (int k = 0; k < nx; ++k) v = (xi[k] == n) ? xv[k] : v;
        xrow[n] = bad ? 0.f : v;
    }
    if (a.support) {
        int32_t* srow = a.support + pix * K;
        // ascending order by rank of the index among the nx support atoms
        for (int k = t; k < K; k += 16) {
            if (k >= nx || bad) {
                srow[k] = -1;
            }
        }
        for (int k = t; k < nx && !bad; k += 16) {
            const int ck = xi[k];
            int pos = 0;
            for (int i = 0; i < nx; ++i) pos += xi[i] < ck ? 1 : 0;
            if (pos < K) srow[pos] = ck;
        }
    }
    if (a.stats && t == 0) {
        csrec_pixel_stats st;
        st.iters = bad ? 0 : iters;
        st.flags = bad ? CSREC_FLAG_NONFINITE : (converged ? CSREC_FLAG_CONVERGED : CSREC_FLAG_ITER_CAP);
        st.resid = bad ? 0.f : sqrtf(rn2);
        st.delta = sqrtf(last_d2);
        a.stats[pix] = st;
    }
}

template <int MSLOT>
__global__ __launch_bounds__(64) void gomp_coop_kernel(CoopArgs a) {
    extern __shared__ float lds[];
    gomp_coop_body<MSLOT>(a, blockIdx.x, lds);
}

struct CoopItem {
    CoopArgs a;
    int64_t block0;
};

// Grouped launch: blocks [items[i].block0, items[i+1].block0) solve item i.
template <int MSLOT>
__global__ __launch_bounds__(64) void gomp_coop_grouped_kernel(const CoopItem* __restrict__ items, int nitems) {
    extern __shared__ float lds[];
    int it = 0;
    while (it + 1 < nitems && items[it + 1].block0 <= (int64_t)blockIdx.x) ++it;
    const CoopArgs a = items[it].a;
    gomp_coop_body<MSLOT>(a, (int64_t)blockIdx.x - items[it].block0, lds);
}

__global__ void transpose_pad_kernel(const float* __restrict__ A, int M, int N, int MP, float* __restrict__ AT) {
    const int n = blockIdx.x;
    for (int m = threadIdx.x; m < MP; m += blockDim.x) AT[(size_t)n * MP + m] = m < M ? A[(size_t)m * N + n] : 0.f;
}

}  // namespace

int gomp_coop_mp(int M) { return M <= 64 ? 64 : 128; }

// Rounded up to 4 floats so every pixel's region (and its float4-read
// residual at the front) is 16-byte aligned.
size_t gomp_coop_lds_floats(int MP, int CM, int K) {
    const size_t f = (size_t)MP + (size_t)CM * (CM + 1) / 2 + 6 * (size_t)CM + (size_t)K * (K + 1) / 2 + 4 * (size_t)K;
    return (f + 3) & ~(size_t)3;
}

int gomp_coop_supported(int M, int N, int K, int S, int Imax) {
    if (N > 16 * kMaxNT || M > 128) return CSREC_E_UNSUPPORTED;
    const int CM = S * Imax;
    const size_t lds = kGroups * gomp_coop_lds_floats(gomp_coop_mp(M), CM, K) * sizeof(float);
    return lds <= 160 * 1024 ? CSREC_OK : CSREC_E_UNSUPPORTED;
}

// AT (N x MP floats) must be in the workspace; fbflag (P entries) may be null.
int gomp_coop_launch(const float* A, const float* Y, float* X, int32_t* support, csrec_pixel_stats* stats,
                     const float* G32, float* AT, uint32_t* fbflag, int M, int N, int64_t p0, int64_t P, int K,
                     int S, int Imax, int prune, float res_tol, float eps, double pivot_thr, bool build_AT,
                     hipStream_t stream) {
    const int MP = gomp_coop_mp(M);
    if (build_AT) {
        hipLaunchKernelGGL(transpose_pad_kernel, dim3(N), dim3(128), 0, stream, A, M, N, MP, AT);
        CSREC_HIP_TRY(hipGetLastError());
    }
    if (P == 0) return CSREC_OK;
    CoopArgs a;
    a.AT = AT;
    a.Y = Y;
    a.G32 = G32;
    a.X = X;
    a.support = support;
    a.stats = stats;
    a.fbflag = fbflag;
    a.M = M;
    a.N = N;
    a.MP = MP;
    a.K = K;
    a.S = S;
    a.Imax = Imax;
    a.prune = prune;
    a.res_tol = res_tol;
    a.eps = eps;
    a.pivot_thr = pivot_thr;
    a.P = P;
    a.p0 = p0;
    a.CM = S * Imax;
    a.lds_floats = (int)gomp_coop_lds_floats(MP, a.CM, K);
    const size_t lds = (size_t)kGroups * a.lds_floats * sizeof(float);
    const int64_t blocks = ceil_div(P, kGroups);
    if (MP == 64) {
        CSREC_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(gomp_coop_kernel<4>),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(gomp_coop_kernel<4>, dim3((unsigned)blocks), dim3(64), lds, stream, a);
    } else {
        CSREC_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(gomp_coop_kernel<8>),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(gomp_coop_kernel<8>, dim3((unsigned)blocks), dim3(64), lds, stream, a);
    }
    CSREC_HIP_TRY(hipGetLastError());
    return CSREC_OK;
}

size_t gomp_coop_item_bytes() { return sizeof(CoopItem); }

void gomp_coop_transpose(const float* A, int M, int N, float* AT, hipStream_t stream) {
    hipLaunchKernelGGL(transpose_pad_kernel, dim3(N), dim3(128), 0, stream, A, M, N, gomp_coop_mp(M), AT);
}

// Items of one launch must share MP (64 or 128).
int gomp_coop_group_launch(const GompCoopItem* items, int nitems, void* table_host, void* table_dev, int K, int S,
                           int prune, float res_tol, float eps, double pivot_thr, hipStream_t stream) {
    if (nitems <= 0) return CSREC_OK;
    CoopItem* th = static_cast<CoopItem*>(table_host);
    int64_t blocks = 0;
    size_t lds = 0;
    const int MP = gomp_coop_mp(items[0].M);
    for (int i = 0; i < nitems; ++i) {
        const GompCoopItem& it = items[i];
        if (gomp_coop_mp(it.M) != MP) return CSREC_E_INVAL;
        CoopArgs& a = th[i].a;
        a.AT = it.AT;
        a.Y = it.Y;
        a.G32 = it.G32;
        a.X = it.X;
        a.support = it.support;
        a.stats = it.stats;
        a.fbflag = it.fbflag;
        a.M = it.M;
        a.N = it.N;
        a.MP = MP;
        a.K = K;
        a.S = S;
        a.Imax = it.max_iter;
        a.prune = prune;
        a.res_tol = res_tol;
        a.eps = eps;
        a.pivot_thr = pivot_thr;
        a.P = it.np;
        a.p0 = it.p0;
        a.CM = S * it.max_iter;
        a.lds_floats = (int)gomp_coop_lds_floats(MP, a.CM, K);
        th[i].block0 = blocks;
        blocks += ceil_div(it.np, kGroups);
        const size_t need = (size_t)kGroups * a.lds_floats * sizeof(float);
        lds = need > lds ? need : lds;
    }
    CSREC_HIP_TRY(hipMemcpyAsync(table_dev, th, (size_t)nitems * sizeof(CoopItem), hipMemcpyHostToDevice, stream));
    const CoopItem* td = static_cast<const CoopItem*>(table_dev);
    if (MP == 64) {
        CSREC_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(gomp_coop_grouped_kernel<4>),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(gomp_coop_grouped_kernel<4>, dim3((unsigned)blocks), dim3(64), lds, stream, td, nitems);
    } else {
        CSREC_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(gomp_coop_grouped_kernel<8>),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(gomp_coop_grouped_kernel<8>, dim3((unsigned)blocks), dim3(64), lds, stream, td, nitems);
    }
    CSREC_HIP_TRY(hipGetLastError());
    return CSREC_OK;
}

}  // namespace csrec
