// gOMP (Alg. 3) redone in FP64 for the pixels whose FP32 least squares met a
// pivot ratio below pivot_fallback, plus the launch logic of every greedy
// solver (gOMP, CoSaMP, BIHT).  The FP32 solves themselves run on the on-chip
// kernels of gomp_coop.hip; this file holds their workspace layout, the Gram
// matrix, the grouped (serving) launches and the FP64 redo.
//
// FP64 redo.  One lane owns one pixel and runs the algorithm's steps in the
// paper's order.  A^T sits in LDS (row n holds column n of A, padded to MMAX
// values) and is read two ways: the correlation A^T r loops over n with every
// lane reading the same row (an LDS broadcast), and the residual y - A x
// gathers the rows of the lane's own support.  The residual r stays in
// VGPRs.  The least-squares state -- the Cholesky factor of the Gram
// submatrix G[c, c] (G = A^T A), forward/back substitution vectors, supports
// -- lives in a per-pixel scratch region laid out [entry][pixel], so that
// every scratch access of a wavefront is one contiguous 256-byte
// transaction.  s = B^+ y with B = A(:, c) is solved through the normal
// equations G[c, c] s = A(:, c)^T y with a Cholesky factor L (G[c,c] = L L^T)
// to which the S new atoms of an iteration are appended column by column
// (bordered update), in FP64 throughout, right-hand sides included.
#include "common.hpp"

#include <cmath>
#include <vector>

namespace csrec {
namespace {

struct GArgs {
    const float* A;
    const float* Y;
    float* X;
    int32_t* support;
    csrec_pixel_stats* stats;
    const float* G32;      // N x N Gram, FP32
    const double* G64;     // N x N Gram, FP64 (fallback pass)
    int M, N, K, S, Imax, prune;
    float res_tol, eps;
    double pivot_thr;
    // scratch
    char* scr;             // base of the chunk scratch
    int64_t CH;            // pixels per chunk (scratch column count)
    int CM;                // largest support held by the factor
    int LM;                // candidate list length
    int64_t off_T;         // byte offset of the T-typed region
    int64_t off_i;         // byte offset of the 32-bit region
    int64_t off_r;         // byte offset of the per-lane residual rows
    uint32_t* fbflag;      // per chunk pixel: 1 = redo in FP64
};

struct GroupItem {
    GArgs g;            // the item's problem (dictionary, measurements, outputs) + batch scratch
    const float* dict;  // the dictionary copies of the on-chip gOMP kernel
    int64_t p0, np;     // pixels [p0, p0 + np) of the item's tile
    int64_t block0;     // first workgroup of the item in the grouped launch
    int64_t slot0;      // first batch scratch column of the item
};

// strided scratch view: element k of this lane's column.  The lane base is
// shared by every view of a region; offset and stride are wave-uniform.
template <typename E>
struct Col {
    E* base;
    int64_t off;
    int64_t s;
    __device__ __forceinline__ E& operator[](int k) const { return base[(off + k) * s]; }
};

template <typename T>
struct Scratch {
    Col<T> L, dinv, z, sv;   // factor (packed rows), 1/L_kk, L^{-1} b, solution
    Col<float> ball;         // b = A^T y, N entries
    float* rold;             // previous residual, MMAX contiguous entries of this lane
    Col<int> lidx;           // prune list (positions in c)
    Col<int> cidx;           // support c (CM)
    Col<int> xidx;           // support of x (CM)
    Col<float> xval;         // values of x (CM)
    Col<uint32_t> mask;      // bitmask over n (NW words)
    Col<uint32_t> keep;      // second bitmask (NW words)
};

__device__ __forceinline__ int tri(int k) { return k * (k + 1) / 2; }

// T-region layout (entries per pixel): L: CM(CM+1)/2, dinv: CM, z: CM, sv: CM
// 32-bit region: ball N, lidx LM, cidx CM, xidx CM, xval CM, mask NW, keep NW
template <typename T>
__device__ Scratch<T> make_scratch(const GArgs& g, int64_t local, int mmax) {
    Scratch<T> s;
    const int64_t CH = g.CH;
    T* tb = reinterpret_cast<T*>(g.scr + g.off_T) + local;
    int64_t o = 0;
    s.L = {tb, o, CH};    o += tri(g.CM);
    s.dinv = {tb, o, CH}; o += g.CM;
    s.z = {tb, o, CH};    o += g.CM;
    s.sv = {tb, o, CH};   o += g.CM;
    uint32_t* ib = reinterpret_cast<uint32_t*>(g.scr + g.off_i) + local;
    float* fb = reinterpret_cast<float*>(ib);
    int* nb = reinterpret_cast<int*>(ib);
    int64_t q = 0;
    s.ball = {fb, q, CH}; q += g.N;
    s.lidx = {nb, q, CH}; q += g.LM;
    s.cidx = {nb, q, CH}; q += g.CM;
    s.xidx = {nb, q, CH}; q += g.CM;
    s.xval = {fb, q, CH}; q += g.CM;
    const int NW = (g.N + 31) / 32;
    s.mask = {ib, q, CH}; q += NW;
    s.keep = {ib, q, CH};
    s.rold = reinterpret_cast<float*>(g.scr + g.off_r) + local * mmax;
    return s;
}

template <typename T>
__device__ __forceinline__ T gram(const GArgs& g, int a, int b);
template <>
__device__ __forceinline__ float gram<float>(const GArgs& g, int a, int b) { return g.G32[a * g.N + b]; }
template <>
__device__ __forceinline__ double gram<double>(const GArgs& g, int a, int b) { return g.G64[a * g.N + b]; }

// Right-hand side b_j = a_j^T y of the normal equations.  The FP32 pass
// reuses A^T y from its first correlation; the FP64 pass forms it in FP64,
// since an ill-conditioned G[c, c] amplifies any error of b as much as one
// of G.
template <typename T>
__device__ __forceinline__ T rhs(const GArgs& g, const Col<float>& ball, int64_t pix, int j);
template <>
__device__ __forceinline__ float rhs<float>(const GArgs&, const Col<float>& ball, int64_t, int j) {
    return ball[j];
}
template <>
__device__ __forceinline__ double rhs<double>(const GArgs& g, const Col<float>&, int64_t pix, int j) {
    double acc = 0.0;
    for (int m = 0; m < g.M; ++m) acc += (double)g.A[(size_t)m * g.N + j] * (double)g.Y[pix * g.M + m];
    return acc;
}

template <typename T>
__device__ __forceinline__ T tsqrt(T v);
template <>
__device__ __forceinline__ float tsqrt<float>(float v) { return sqrtf(v); }
template <>
__device__ __forceinline__ double tsqrt<double>(double v) { return sqrt(v); }

// Append atom j to the factor of G[c, c] (c = cidx[0 .. nc-1]):
//   l = L^{-1} G[c, j],  d = G_jj - ||l||^2,  L_new = [[L, 0], [l^T, sqrt(d)]]
// and extend z = L^{-1} b_c with b_j.  Returns the pivot ratio d / G_jj.
template <typename T>
__device__ T chol_append(const GArgs& g, const Scratch<T>& s, int nc, int j, T bj) {
    const int rn = tri(nc);
    T ll = 0, lz = 0;
    for (int k = 0; k < nc; ++k) {
        T acc = gram<T>(g, s.cidx[k], j);
        const int rk = tri(k);
        for (int t = 0; t < k; ++t) acc -= s.L[rk + t] * s.L[rn + t];
        const T lk = acc * s.dinv[k];
        s.L[rn + k] = lk;
        ll += lk * lk;
        lz += lk * s.z[k];
    }
    const T gjj = gram<T>(g, j, j);
    T d = gjj - ll;
    const T ratio = d / gjj;
    if (!(d > (T)0)) d = gjj * (T)1e-30 + (T)1e-38;
    const T lkk = tsqrt<T>(d);
    const T inv = (T)1 / lkk;
    s.L[rn + nc] = lkk;
    s.dinv[nc] = inv;
    s.z[nc] = (bj - lz) * inv;
    s.cidx[nc] = j;
    return ratio;
}

// Back substitution L^T s = z on the first nc entries.
template <typename T>
__device__ void chol_back(const Scratch<T>& s, int nc) {
    for (int k = nc - 1; k >= 0; --k) {
        T acc = s.z[k];
        for (int t = k + 1; t < nc; ++t) acc -= s.L[tri(t) + k] * s.sv[t];
        s.sv[k] = acc * s.dinv[k];
    }
}

// Fresh factorisation of G[c, c] for c = cidx[0 .. n-1], rhs b_c = ball[c];
// leaves s.sv = G[c,c]^{-1} b_c.  Returns the smallest pivot ratio.
template <typename T>
__device__ T chol_solve_fresh(const GArgs& g, const Scratch<T>& s, int n, int64_t pix) {
    T rmin = (T)1;
    for (int i = 0; i < n; ++i) {
        const T r = chol_append<T>(g, s, i, s.cidx[i], rhs<T>(g, s.ball, pix, s.cidx[i]));
        rmin = r < rmin ? r : rmin;
    }
    chol_back<T>(s, n);
    return rmin;
}

// keep = the k entries of cidx[0..n-1] with largest |sv| ((|sv| desc, index
// asc), compared in T): one pass inserting each position a into a sorted
// k-slot list (lidx), then the list's atoms as a bitmask.
template <typename T>
__device__ void mark_top_k(const GArgs& g, const Scratch<T>& s, int n, int k) {
    const int NW = (g.N + 31) / 32;
    int len = 0;
    T last = (T)-1;
    int last_i = 0x7fffffff;
    for (int a = 0; a < n; ++a) {
        const T sa = s.sv[a];
        const T va = sa < (T)0 ? -sa : sa;
        const int ia = s.cidx[a];
        if (len == k && !(va > last || (va == last && ia < last_i))) continue;
        int pos = len < k ? len : k - 1;
        while (pos > 0) {
            const int pa = s.lidx[pos - 1];
            const T ps = s.sv[pa];
            const T pv = ps < (T)0 ? -ps : ps;
            const int pi = s.cidx[pa];
            if (!(va > pv || (va == pv && ia < pi))) break;
            if (pos < k) s.lidx[pos] = pa;
            --pos;
        }
        s.lidx[pos] = a;
        if (len < k) ++len;
        const int la = s.lidx[len - 1];
        const T ls = s.sv[la];
        last = ls < (T)0 ? -ls : ls;
        last_i = s.cidx[la];
    }
    for (int w = 0; w < NW; ++w) s.keep[w] = 0u;
    for (int a = 0; a < len; ++a) {
        const int ia = s.cidx[s.lidx[a]];
        s.keep[ia >> 5] |= 1u << (ia & 31);
    }
}

// Writes the set bits of a bitmask (ascending) into dst; returns the count.
__device__ __forceinline__ int extract_bits(const Col<uint32_t>& bits, int NW, const Col<int>& dst) {
    int cnt = 0;
    for (int w = 0; w < NW; ++w) {
        uint32_t v = bits[w];
        while (v) {
            const int b = __builtin_ctz(v);
            v &= v - 1;
            dst[cnt++] = 32 * w + b;
        }
    }
    return cnt;
}

// A^T into LDS: row n holds column n of A, padded to MMAX + 4 values.
template <int MMAX>
__device__ __forceinline__ void load_at(const GArgs& g, float* sAT) {
    constexpr int PAT = MMAX + 4;
    const int M = g.M, N = g.N;
    for (int idx = threadIdx.x; idx < N * PAT; idx += blockDim.x) {
        const int n = idx / PAT;
        const int m = idx - n * PAT;
        sAT[idx] = (m < M) ? g.A[(size_t)m * N + n] : 0.f;
    }
    __syncthreads();
}

// One pixel: measurements Y[pix], FP64 hand-off flag fbflag[fidx], scratch
// column col (A^T already in sAT).
template <int MMAX, int SMAX, typename T>
__device__ __forceinline__ void greedy_pixel(const GArgs& g, int64_t pix, int64_t fidx, int64_t col, int pass,
                                             const float* sAT) {
    constexpr int PAT = MMAX + 4;
    const int M = g.M, N = g.N, K = g.K;
    if (pass == 1 && g.fbflag[fidx] == 0u) return;   // FP64 redo only for marked pixels
    const Scratch<T> s = make_scratch<T>(g, col, MMAX);
    const int NW = (N + 31) / 32;

    // ---- measurements
    float r[MMAX];
    bool bad = false;
    float ynorm2 = 0.f;
#pragma unroll
    for (int m = 0; m < MMAX; ++m) {
        float v = 0.f;
        if (m < M) {
            v = g.Y[pix * M + m];
            if (!isfinite(v)) bad = true;
        }
        r[m] = v;
    }
    if (bad) {
#pragma unroll
        for (int m = 0; m < MMAX; ++m) r[m] = 0.f;
    }
#pragma unroll
    for (int m = 0; m < MMAX; ++m) ynorm2 += r[m] * r[m];
    const float ynorm = sqrtf(ynorm2);
    for (int w = 0; w < NW; ++w) s.mask[w] = 0u;

    int nx = 0;          // entries in x (xidx/xval)
    int nc = 0;          // support size c
    int iters = 0;
    bool converged = false;
    bool fallback = false;
    float last_d2 = __builtin_nanf("");
    float rn2 = ynorm2;
    const int Imax = bad ? 0 : g.Imax;

    for (int it = 1; it <= Imax; ++it) {
        // ---------------- step 1: correlation with the residual, candidate selection
        float bv[SMAX];
        int bi[SMAX];
#pragma unroll
        for (int q = 0; q < SMAX; ++q) {
            bv[q] = -1.f;
            bi[q] = -1;
        }
        uint32_t mword = 0u;
        for (int n = 0; n < N; ++n) {
            const float4* row = reinterpret_cast<const float4*>(sAT + n * PAT);
            float acc = 0.f;
#pragma unroll
            for (int m4 = 0; m4 < MMAX / 4; ++m4) {
                const float4 a = row[m4];
                acc += a.x * r[4 * m4] + a.y * r[4 * m4 + 1] + a.z * r[4 * m4 + 2] + a.w * r[4 * m4 + 3];
            }
            if (it == 1) s.ball[n] = acc;   // A^T y
            {
                if ((n & 31) == 0) mword = s.mask[n >> 5];
                if ((mword >> (n & 31)) & 1u) continue;
                const float v = fabsf(acc);
                if (v > bv[SMAX - 1] || bi[SMAX - 1] < 0) {
                    // insertion into the register list (first S slots used)
                    float cv = v;
                    int ci = n;
#pragma unroll
                    for (int q = 0; q < SMAX; ++q) {
                        if (q < g.S && (bi[q] < 0 || cv > bv[q])) {
                            const float tv = bv[q];
                            const int ti = bi[q];
                            bv[q] = cv;
                            bi[q] = ci;
                            cv = tv;
                            ci = ti;
                        }
                    }
                }
            }
        }

        // ---------------- steps 2-3: support and least squares
        {
            for (int q = 0; q < g.S; ++q) {
                const int j = bi[q];
                if (j < 0) break;   // no admissible atom left (non-finite correlations)
                s.mask[j >> 5] |= 1u << (j & 31);
                const T ratio = chol_append<T>(g, s, nc, j, rhs<T>(g, s.ball, pix, j));
                if (g.pivot_thr > 0.0 && (double)ratio < g.pivot_thr) fallback = true;
                ++nc;
            }
            chol_back<T>(s, nc);
            if (g.prune == CSREC_PRUNE_EACH && nc > K) {
                mark_top_k<T>(g, s, nc, K);
                // re-solve on q: factor G[q, q] in the slots after c
                // (the factor of G[c, c] stays intact at rows 0 .. nc-1)
                int nq = 0;
                for (int w = 0; w < NW; ++w) {
                    uint32_t v = s.keep[w];
                    while (v) {
                        const int b = __builtin_ctz(v);
                        v &= v - 1;
                        s.xidx[nq++] = 32 * w + b;
                    }
                }
                // factor into a temporary region: rows nc .. nc+nq-1 of L would exceed CM,
                // so use a fresh solve on a copy of the indices placed after c.
                for (int a = 0; a < nq; ++a) s.cidx[nc + a] = s.xidx[a];
                // fresh factor of G[q, q] built in rows 0..nq-1 of a shifted view
                Scratch<T> sq = s;
                sq.L.off += tri(nc);
                sq.dinv.off += nc;
                sq.z.off += nc;
                sq.sv.off += nc;
                sq.cidx.off += nc;
                chol_solve_fresh<T>(g, sq, nq, pix);
                for (int a = 0; a < nq; ++a) s.xval[a] = (float)sq.sv[a];
                nx = nq;
            } else {
                for (int a = 0; a < NW; ++a) s.keep[a] = s.mask[a];
                nx = extract_bits(s.keep, NW, s.xidx);
                // values in the order of xidx: look them up in c
                for (int a = 0; a < nx; ++a) {
                    const int ia = s.xidx[a];
                    for (int b = 0; b < nc; ++b)
                        if (s.cidx[b] == ia) {
                            s.xval[a] = (float)s.sv[b];
                            break;
                        }
                }
            }
        }

        // ---------------- step 4: residual r = y - A x
#pragma unroll
        for (int m = 0; m < MMAX; ++m) {
            s.rold[m] = r[m];
            r[m] = (m >= M || bad) ? 0.f : g.Y[pix * M + m];
        }
        for (int a = 0; a < nx; ++a) {
            const float xv = s.xval[a];
            const float4* row = reinterpret_cast<const float4*>(sAT + s.xidx[a] * PAT);
#pragma unroll
            for (int m4 = 0; m4 < MMAX / 4; ++m4) {
                const float4 av = row[m4];
                r[4 * m4] -= av.x * xv;
                r[4 * m4 + 1] -= av.y * xv;
                r[4 * m4 + 2] -= av.z * xv;
                r[4 * m4 + 3] -= av.w * xv;
            }
        }
        float d2 = 0.f, n2 = 0.f;
#pragma unroll
        for (int m = 0; m < MMAX; ++m) {
            const float d = r[m] - s.rold[m];
            d2 += d * d;
            n2 += r[m] * r[m];
        }
        iters = it;
        last_d2 = d2;
        rn2 = n2;
        const bool stop = (sqrtf(n2) <= g.res_tol * ynorm) || (g.eps > 0.f && sqrtf(d2) < g.eps);
        if (stop) {
            converged = true;
            break;
        }
    }

    // gOMP with the prune placed after the loop
    if (g.prune == CSREC_PRUNE_FINAL && nc > K) {
        mark_top_k<T>(g, s, nc, K);
        int nq = 0;
        for (int w = 0; w < NW; ++w) {
            uint32_t v = s.keep[w];
            while (v) {
                const int b = __builtin_ctz(v);
                v &= v - 1;
                s.cidx[nc + nq] = 32 * w + b;
                s.xidx[nq++] = 32 * w + b;
            }
        }
        Scratch<T> sq = s;
        sq.L.off += tri(nc);
        sq.dinv.off += nc;
        sq.z.off += nc;
        sq.sv.off += nc;
        sq.cidx.off += nc;
        chol_solve_fresh<T>(g, sq, nq, pix);
        for (int a = 0; a < nq; ++a) s.xval[a] = (float)sq.sv[a];
        nx = nq;
        // residual of the pruned x
#pragma unroll
        for (int m = 0; m < MMAX; ++m) r[m] = (m < M) ? g.Y[pix * M + m] : 0.f;
        for (int a = 0; a < nx; ++a) {
            const float xv = s.xval[a];
            const float4* row = reinterpret_cast<const float4*>(sAT + s.xidx[a] * PAT);
#pragma unroll
            for (int m4 = 0; m4 < MMAX / 4; ++m4) {
                const float4 av = row[m4];
                r[4 * m4] -= av.x * xv;
                r[4 * m4 + 1] -= av.y * xv;
                r[4 * m4 + 2] -= av.z * xv;
                r[4 * m4 + 3] -= av.w * xv;
            }
        }
        float n2 = 0.f;
#pragma unroll
        for (int m = 0; m < MMAX; ++m) n2 += r[m] * r[m];
        rn2 = n2;
    }

    if (pass == 0 && g.fbflag) {
        g.fbflag[fidx] = fallback ? 1u : 0u;
        if (fallback) return;   // the FP64 pass writes this pixel's results
    }

    // ---------------- outputs
    float* xrow = g.X + pix * N;
    for (int n = 0; n < N; ++n) xrow[n] = 0.f;
    for (int a = 0; a < nx; ++a) xrow[s.xidx[a]] = s.xval[a];
    if (g.support) {
        int32_t* srow = g.support + pix * K;
        int a = 0;
        for (; a < nx && a < K; ++a) srow[a] = s.xidx[a];
        for (; a < K; ++a) srow[a] = -1;
    }
    if (g.stats) {
        csrec_pixel_stats st;
        st.iters = iters;
        uint32_t f = 0;
        if (bad) f = CSREC_FLAG_NONFINITE;
        else f = converged ? CSREC_FLAG_CONVERGED : CSREC_FLAG_ITER_CAP;
        if (pass == 1) f |= CSREC_FLAG_FP64_FALLBACK;
        st.flags = f;
        st.resid = bad ? 0.f : sqrtf(rn2);
        st.delta = sqrtf(last_d2);
        g.stats[pix] = st;
    }
}

// One workgroup of a solve: pixels p0 + block*blockDim + [0, blockDim) of the
// problem in g (at most np of them), using scratch columns slot0 + the same
// offsets.  Shared by the plain launch and the grouped (serving) launch.
template <int MMAX, int SMAX, typename T>
__device__ __forceinline__ void greedy_block(const GArgs& g, int64_t p0, int64_t np, int pass, int64_t block,
                                             int64_t slot0, float* sAT) {
    load_at<MMAX>(g, sAT);
    const int64_t within = block * blockDim.x + threadIdx.x;
    if (within >= np) return;
    greedy_pixel<MMAX, SMAX, T>(g, p0 + within, slot0 + within, slot0 + within, pass, sAT);
}

template <int MMAX, int SMAX, typename T>
__global__ __launch_bounds__(256, 2) void greedy_kernel(GArgs g, int64_t p0, int64_t np, int pass) {
    extern __shared__ float sAT[];
    greedy_block<MMAX, SMAX, T>(g, p0, np, pass, blockIdx.x, 0, sAT);
}

// The FP64 redo over pixels [p0, p0 + np) with g.CH scratch columns: thread
// c takes the flagged pixels c, c + CH, c + 2 CH, ... one after the other in
// column c, so a scratch smaller than the chunk serves it.  gridDim.x *
// blockDim.x == g.CH.
template <int MMAX, int SMAX, typename T>
__global__ __launch_bounds__(256, 2) void greedy_redo_strided_kernel(GArgs g, int64_t p0, int64_t np) {
    extern __shared__ float sAT[];
    load_at<MMAX>(g, sAT);
    const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t within = col; within < np; within += g.CH)
        greedy_pixel<MMAX, SMAX, T>(g, p0 + within, within, col, 1, sAT);
}

// Grouped launch: blocks [items[i].block0, items[i+1].block0) solve item i
// (its own dictionary, measurements and outputs); scratch columns are
// batch-wide slots.
template <int MMAX, int SMAX, typename T>
__global__ __launch_bounds__(256, 2) void greedy_grouped_kernel(const GroupItem* __restrict__ items, int nitems,
                                                                int pass) {
    extern __shared__ float sAT[];
    int it = 0;
    while (it + 1 < nitems && items[it + 1].block0 <= (int64_t)blockIdx.x) ++it;
    const GArgs g = items[it].g;
    greedy_block<MMAX, SMAX, T>(g, items[it].p0, items[it].np, pass, blockIdx.x - items[it].block0,
                                      items[it].slot0, sAT);
}

// Gram matrix G = A^T A in FP64, stored as FP32 and FP64.
__global__ void gram_kernel(const float* __restrict__ A, int M, int N, float* __restrict__ G32,
                            double* __restrict__ G64) {
    const int a = blockIdx.x;
    for (int b = threadIdx.x; b < N; b += blockDim.x) {
        double acc = 0.0;
        for (int m = 0; m < M; ++m) acc += (double)A[(size_t)m * N + a] * (double)A[(size_t)m * N + b];
        G32[a * N + b] = (float)acc;
        if (G64) G64[a * N + b] = acc;
    }
}

typedef void (*gk_t)(GArgs, int64_t, int64_t, int);

// The FP64 redo kernel for a dictionary with M rows and S atoms per iteration.
gk_t pick_kernel(int M, int S) {
    if (M <= 48) return S <= 2 ? greedy_kernel<48, 2, double> : greedy_kernel<48, 8, double>;
    if (M <= 80) return S <= 2 ? greedy_kernel<80, 2, double> : greedy_kernel<80, 8, double>;
    if (M <= 96) return S <= 2 ? greedy_kernel<96, 2, double> : greedy_kernel<96, 8, double>;
    return nullptr;
}

int mmax_for(int M) { return M <= 48 ? 48 : (M <= 80 ? 80 : 96); }

struct Layout {
    int CM, LM;
    int64_t CH;
    size_t gram32, gram64, off_AT, off_T, off_i, off_r, off_f, total;
};

constexpr int64_t kChunk = 65536;

Layout layout_for(const GreedyLaunch& a, int64_t ch_override = 0) {
    Layout L;
    // FP64 redo of gOMP: the factor holds c plus a q-sized tail
    const int CM = a.S * a.max_iter + a.K, LM = a.K;
    L.CM = CM;
    L.LM = LM;
    L.CH = a.P < kChunk ? ((a.P + 63) / 64) * 64 : kChunk;
    if (ch_override > 0) L.CH = ((ch_override + 63) / 64) * 64;
    if (L.CH == 0) L.CH = 64;
    const bool dbl = a.kind == GREEDY_GOMP && a.pivot_fallback > 0.0;
    const size_t tsz = dbl ? 8 : 4;
    const int NW = (a.N + 31) / 32;
    const int64_t tent = (int64_t)CM * (CM + 1) / 2 + 3 * (int64_t)CM;
    const int64_t ient = a.N + LM + 3 * CM + 2 * NW;
    L.gram32 = 0;
    L.gram64 = align_up((size_t)a.N * a.N * 4, 256);
    size_t o = L.gram64 + (dbl ? align_up((size_t)a.N * a.N * 8, 256) : 0);
    L.off_AT = o;
    o += align_up(gomp_coop_dict_floats(a.M, a.N) * 4, 256);
    L.off_f = o;
    o += align_up((size_t)L.CH * 4, 256);
    if (!dbl) {
        // the on-chip kernels need no per-pixel scratch
        L.off_T = L.off_i = L.off_r = o;
        L.total = o;
        return L;
    }
    L.off_T = o;
    o += align_up((size_t)tent * L.CH * tsz, 256);
    L.off_i = o;
    o += align_up((size_t)ient * L.CH * 4, 256);
    L.off_r = o;
    o += align_up((size_t)mmax_for(a.M) * L.CH * 4, 256);
    L.total = o;
    return L;
}

}  // namespace

size_t greedy_workspace(const GreedyLaunch& a) { return cosamp_is_wide(a) ? 0 : layout_for(a).total; }

// ---------------------------------------------------------------- grouped (serving) launches

namespace {
typedef void (*ggk_t)(const GroupItem*, int, int);

template <int MMAX>
ggk_t pick_grouped(int S) {
    return S <= 2 ? greedy_grouped_kernel<MMAX, 2, double> : greedy_grouped_kernel<MMAX, 8, double>;
}
ggk_t pick_grouped_m(int mmax, int S) {
    if (mmax == 48) return pick_grouped<48>(S);
    if (mmax == 80) return pick_grouped<80>(S);
    return pick_grouped<96>(S);
}
}  // namespace

int greedy_mmax_class(int M) { return mmax_for(M); }

size_t greedy_group_item_bytes() { return sizeof(GroupItem); }

size_t greedy_group_table_bytes(int nitems) {
    // the FP64 redo table, then up to four on-chip kernel tables (one per
    // kernel variant), each with its work cursor and padded to 256 bytes
    return align_up((size_t)nitems * sizeof(GroupItem), 256) + (size_t)nitems * gomp_coop_item_bytes() +
           4 * (gomp_coop_table_extra() + 256);
}

size_t greedy_group_workspace(const GreedyLaunch& proto_max, int64_t batch_pixels) {
    return layout_for(proto_max, batch_pixels).total;
}

int greedy_group_launch(const GreedyLaunch& proto_max, const GreedyTileItem* items, int nitems,
                        int64_t batch_pixels, void* ws, void* table_host, void* table_dev, hipStream_t stream) {
    if (nitems <= 0) return CSREC_OK;
    const GreedyLaunch& pm = proto_max;
    const Layout L = layout_for(pm, batch_pixels);
    const bool dbl = pm.pivot_fallback > 0.0;
    char* w = static_cast<char*>(ws);
    GroupItem* th = static_cast<GroupItem*>(table_host);
    GroupItem* td = static_cast<GroupItem*>(table_dev);
    // items of one MMAX class go to one launch; the table is laid out class by class
    int nt = 0;
    int64_t slot = 0;
    struct Range { int first, count; int64_t blocks; int mmax; size_t lds; };
    Range ranges[3];
    int nr = 0;
    const int classes[3] = {48, 80, 96};
    for (int c = 0; c < 3; ++c) {
        const int first = nt;
        int64_t blocks = 0;
        size_t lds = 0;
        for (int i = 0; i < nitems; ++i) {
            const GreedyTileItem& it = items[i];
            if (mmax_for(it.M) != classes[c]) continue;
            GroupItem gi{};
            GArgs& g = gi.g;
            g.A = it.A;
            g.Y = it.Y;
            g.X = it.X;
            g.support = it.support;
            g.stats = it.stats;
            g.G32 = it.G32;
            g.G64 = it.G64;
            g.M = it.M;
            g.N = it.N;
            g.K = pm.K;
            g.S = pm.S;
            g.Imax = it.max_iter;
            g.prune = pm.prune;
            g.res_tol = pm.res_tol;
            g.eps = pm.eps;
            g.pivot_thr = pm.pivot_fallback;
            g.scr = w;
            g.CH = L.CH;
            g.CM = pm.S * it.max_iter + pm.K;
            g.LM = pm.K;
            g.off_T = (int64_t)L.off_T;
            g.off_i = (int64_t)L.off_i;
            g.off_r = (int64_t)L.off_r;
            g.fbflag = dbl ? reinterpret_cast<uint32_t*>(w + L.off_f) : nullptr;
            gi.dict = it.dict;
            gi.p0 = it.p0;
            gi.np = it.np;
            gi.block0 = blocks;
            gi.slot0 = slot;
            if (slot + it.np > L.CH) return CSREC_E_SHAPE;
            slot += it.np;
            blocks += ceil_div(it.np, 256);
            const size_t need = (size_t)it.N * (classes[c] + 4) * sizeof(float);
            lds = need > lds ? need : lds;
            th[nt++] = gi;
        }
        if (nt > first) ranges[nr++] = Range{first, nt - first, blocks, classes[c], lds};
    }
    // pass 0: the on-chip gOMP kernel, items grouped by kernel variant
    char* chost = static_cast<char*>(table_host) + align_up((size_t)nitems * sizeof(GroupItem), 256);
    char* cdev = static_cast<char*>(table_dev) + align_up((size_t)nitems * sizeof(GroupItem), 256);
    size_t coff = 0;
    for (int cls = 0; cls < 4; ++cls) {
        std::vector<GompCoopItem> ci;
        for (int k = 0; k < nt; ++k) {
            const GroupItem& gi = th[k];
            if (gomp_coop_class(gi.g.M, gi.g.N) != cls) continue;
            GompCoopItem c{};
            c.dict = gi.dict;
            c.Y = gi.g.Y;
            c.G32 = gi.g.G32;
            c.X = gi.g.X;
            c.support = gi.g.support;
            c.stats = gi.g.stats;
            c.fbflag = gi.g.fbflag ? gi.g.fbflag + gi.slot0 : nullptr;
            c.M = gi.g.M;
            c.N = gi.g.N;
            c.max_iter = gi.g.Imax;
            c.p0 = gi.p0;
            c.np = gi.np;
            ci.push_back(c);
        }
        if (ci.empty()) continue;
        const int e = gomp_coop_group_launch(ci.data(), (int)ci.size(), chost + coff, cdev + coff, pm.K, pm.S,
                                             pm.prune, pm.res_tol, pm.eps, pm.pivot_fallback, (float)pm.redo_tol,
                                             pm.prec, stream);
        if (e) return e;
        coff += align_up(ci.size() * gomp_coop_item_bytes() + gomp_coop_table_extra(), 256);
    }
    if (!dbl) return CSREC_OK;
    // pass 1: FP64 redo of the marked pixels (scratch-based kernel)
    CSREC_HIP_TRY(hipMemcpyAsync(td, th, (size_t)nt * sizeof(GroupItem), hipMemcpyHostToDevice, stream));
    for (int pass = 1; pass < 2; ++pass) {
        for (int r = 0; r < nr; ++r) {
            ggk_t fn = pick_grouped_m(ranges[r].mmax, pm.S);
            CSREC_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)ranges[r].lds));
            hipLaunchKernelGGL(fn, dim3((unsigned)ranges[r].blocks), dim3(256), ranges[r].lds, stream,
                               td + ranges[r].first, ranges[r].count, pass);
            CSREC_HIP_TRY(hipGetLastError());
        }
    }
    return CSREC_OK;
}

int greedy_gram(const float* A, int M, int N, float* G32, double* G64, hipStream_t stream) {
    hipLaunchKernelGGL(gram_kernel, dim3(N), dim3(256), 0, stream, A, M, N, G32, G64);
    CSREC_HIP_TRY(hipGetLastError());
    return CSREC_OK;
}

int greedy_launch(const GreedyLaunch& a) {
    if (a.P == 0) return CSREC_OK;
    if (a.M > 96) return CSREC_E_UNSUPPORTED;
    if (cosamp_is_wide(a)) return cosamp_wide_launch(a);
    const Layout L = layout_for(a);
    if (!a.workspace || a.workspace_bytes < L.total) return CSREC_E_WORKSPACE;
    const bool dbl = a.kind == GREEDY_GOMP && a.pivot_fallback > 0.0;
    char* ws = static_cast<char*>(a.workspace);
    GArgs g;
    g.A = a.A;
    g.Y = a.Y;
    g.X = a.X;
    g.support = a.support;
    g.stats = a.stats;
    g.G32 = reinterpret_cast<const float*>(ws + L.gram32);
    g.G64 = dbl ? reinterpret_cast<const double*>(ws + L.gram64) : nullptr;
    g.M = a.M;
    g.N = a.N;
    g.K = a.K;
    g.S = a.S;
    g.Imax = a.max_iter;
    g.prune = a.prune;
    g.res_tol = a.res_tol;
    g.eps = a.eps;
    g.pivot_thr = a.pivot_fallback;
    g.scr = ws;
    g.CH = L.CH;
    g.CM = L.CM;
    g.LM = L.LM;
    g.off_T = (int64_t)L.off_T;
    g.off_i = (int64_t)L.off_i;
    g.off_r = (int64_t)L.off_r;
    g.fbflag = dbl ? reinterpret_cast<uint32_t*>(ws + L.off_f) : nullptr;

    if (a.kind != GREEDY_BIHT_ONE_BIT) {
        hipLaunchKernelGGL(gram_kernel, dim3(a.N), dim3(256), 0, a.stream, a.A, a.M, a.N,
                           reinterpret_cast<float*>(ws + L.gram32),
                           dbl ? reinterpret_cast<double*>(ws + L.gram64) : nullptr);
        CSREC_HIP_TRY(hipGetLastError());
    }
    float* dictbuf = reinterpret_cast<float*>(ws + L.off_AT);
    gomp_coop_prepare(a.A, a.M, a.N, dictbuf, a.stream);
    CSREC_HIP_TRY(hipGetLastError());
    if (a.kind != GREEDY_GOMP) {
        // CoSaMP and both BIHT forms: the on-chip kernel, in chunks
        if (coop_other_supported(a.kind, a.M, a.N, a.K) != CSREC_OK) return CSREC_E_UNSUPPORTED;
        for (int64_t p0 = 0; p0 < a.P; p0 += L.CH) {
            const int64_t np = (a.P - p0) < L.CH ? (a.P - p0) : L.CH;
            const int e = coop_other_launch(a.kind, a.Y, a.Ysign, a.X, a.support, a.stats, g.G32, dictbuf, a.M, a.N,
                                            p0, np, a.K, a.max_iter, a.mu, a.res_tol, a.eps, a.prec, a.stream);
            if (e) return e;
        }
        return CSREC_OK;
    }
    // gOMP: the on-chip FP32 pass, then (pivot_fallback > 0) the FP64 redo of
    // the pixels it flagged
    const int mmax = mmax_for(a.M);
    const size_t lds = (size_t)a.N * (mmax + 4) * sizeof(float);
    const int threads = 256;
    const gk_t redo = dbl ? pick_kernel(a.M, a.S) : nullptr;
    if (dbl) {
        if (!redo) return CSREC_E_UNSUPPORTED;
        CSREC_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(redo),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    }
    for (int64_t p0 = 0; p0 < a.P; p0 += L.CH) {
        const int64_t np = (a.P - p0) < L.CH ? (a.P - p0) : L.CH;
        const int e = gomp_coop_launch(a.Y, a.X, a.support, a.stats, g.G32, dictbuf, g.fbflag, a.M, a.N, p0, np,
                                       a.K, a.S, a.max_iter, a.prune, a.res_tol, a.eps, a.pivot_fallback,
                                       (float)a.redo_tol, a.prec, a.stream);
        if (e) return e;
        if (dbl) {
            hipLaunchKernelGGL(redo, dim3((unsigned)ceil_div(np, threads)), dim3(threads), lds, a.stream, g, p0,
                               np, 1);
            CSREC_HIP_TRY(hipGetLastError());
        }
    }
    return CSREC_OK;
}

}  // namespace csrec

namespace csrec {

namespace {
typedef void (*rk_t)(GArgs, int64_t, int64_t);
rk_t pick_redo_strided(int M, int S) {
    if (M <= 48) return S <= 2 ? greedy_redo_strided_kernel<48, 2, double> : greedy_redo_strided_kernel<48, 8, double>;
    if (M <= 80) return S <= 2 ? greedy_redo_strided_kernel<80, 2, double> : greedy_redo_strided_kernel<80, 8, double>;
    if (M <= 96) return S <= 2 ? greedy_redo_strided_kernel<96, 2, double> : greedy_redo_strided_kernel<96, 8, double>;
    return nullptr;
}
constexpr int kRedoThreads = 64;   // the strided redo's block; its column count is a multiple of it
}  // namespace

// Layout of gOMP on a fixed scratch of `cap` bytes: the Gram matrices, the
// dictionary copies and the FP64 hand-off flags of one chunk as in the
// workspace layout, then the FP64 redo's per-pixel state for as many
// columns (multiples of kRedoThreads, at most the chunk) as fit.  Returns
// the column count, 0 without an FP64 fallback, or -1 when it does not fit.
int64_t greedy_gomp_scratch_cols(const GreedyLaunch& a, size_t cap) {
    const Layout L = layout_for(a);
    const bool dbl = a.pivot_fallback > 0.0;
    if (L.off_T > cap) return -1;
    if (!dbl) return 0;
    const int NW = (a.N + 31) / 32;
    const int64_t tent = (int64_t)L.CM * (L.CM + 1) / 2 + 3 * (int64_t)L.CM;
    const int64_t ient = a.N + L.LM + 3 * L.CM + 2 * NW;
    const int64_t per_col = tent * 8 + ient * 4 + (int64_t)mmax_for(a.M) * 4;
    const int64_t room = (int64_t)cap - (int64_t)L.off_T - 3 * 256;
    int64_t cols = room > 0 ? room / per_col : 0;
    cols = cols / kRedoThreads * kRedoThreads;
    const int64_t chunk_cols = (L.CH + kRedoThreads - 1) / kRedoThreads * kRedoThreads;
    if (cols > chunk_cols) cols = chunk_cols;
    return cols >= kRedoThreads ? cols : -1;
}

int greedy_gomp_scratch_launch(const GreedyLaunch& a, char* scr, size_t cap) {
    if (a.P == 0) return CSREC_OK;
    if (a.M > 96 || a.kind != GREEDY_GOMP) return CSREC_E_UNSUPPORTED;
    const int64_t cols = greedy_gomp_scratch_cols(a, cap);
    if (cols < 0) return CSREC_E_WORKSPACE;
    const Layout L = layout_for(a);
    const bool dbl = a.pivot_fallback > 0.0;
    const int NW = (a.N + 31) / 32;
    const int64_t tent = (int64_t)L.CM * (L.CM + 1) / 2 + 3 * (int64_t)L.CM;
    const int64_t ient = a.N + L.LM + 3 * L.CM + 2 * NW;
    GArgs g;
    g.A = a.A;
    g.Y = a.Y;
    g.X = a.X;
    g.support = a.support;
    g.stats = a.stats;
    g.G32 = reinterpret_cast<const float*>(scr + L.gram32);
    g.G64 = dbl ? reinterpret_cast<const double*>(scr + L.gram64) : nullptr;
    g.M = a.M;
    g.N = a.N;
    g.K = a.K;
    g.S = a.S;
    g.Imax = a.max_iter;
    g.prune = a.prune;
    g.res_tol = a.res_tol;
    g.eps = a.eps;
    g.pivot_thr = a.pivot_fallback;
    g.scr = scr;
    g.CH = cols;
    g.CM = L.CM;
    g.LM = L.LM;
    g.off_T = (int64_t)L.off_T;
    g.off_i = g.off_T + (int64_t)align_up((size_t)(tent * cols * 8), 256);
    g.off_r = g.off_i + (int64_t)align_up((size_t)(ient * cols * 4), 256);
    g.fbflag = dbl ? reinterpret_cast<uint32_t*>(scr + L.off_f) : nullptr;
    if (dbl && (size_t)g.off_r + align_up((size_t)mmax_for(a.M) * cols * 4, 256) > cap) return CSREC_E_WORKSPACE;

    hipLaunchKernelGGL(gram_kernel, dim3(a.N), dim3(256), 0, a.stream, a.A, a.M, a.N,
                       reinterpret_cast<float*>(scr + L.gram32),
                       dbl ? reinterpret_cast<double*>(scr + L.gram64) : nullptr);
    CSREC_HIP_TRY(hipGetLastError());
    float* dictbuf = reinterpret_cast<float*>(scr + L.off_AT);
    gomp_coop_prepare(a.A, a.M, a.N, dictbuf, a.stream);
    CSREC_HIP_TRY(hipGetLastError());
    const size_t lds = (size_t)a.N * (mmax_for(a.M) + 4) * sizeof(float);
    const rk_t redo = dbl ? pick_redo_strided(a.M, a.S) : nullptr;
    if (dbl) {
        if (!redo) return CSREC_E_UNSUPPORTED;
        CSREC_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(redo),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    }
    for (int64_t p0 = 0; p0 < a.P; p0 += L.CH) {
        const int64_t np = (a.P - p0) < L.CH ? (a.P - p0) : L.CH;
        const int e = gomp_coop_launch(a.Y, a.X, a.support, a.stats, g.G32, dictbuf, g.fbflag, a.M, a.N, p0, np,
                                       a.K, a.S, a.max_iter, a.prune, a.res_tol, a.eps, a.pivot_fallback,
                                       (float)a.redo_tol, a.prec, a.stream);
        if (e) return e;
        if (dbl) {
            hipLaunchKernelGGL(redo, dim3((unsigned)(cols / kRedoThreads)), dim3(kRedoThreads), lds, a.stream, g,
                               p0, np);
            CSREC_HIP_TRY(hipGetLastError());
        }
    }
    return CSREC_OK;
}

}  // namespace csrec

namespace csrec {

namespace {
// The real M x NR dictionary of the conjugate-pair groups of a complex
// M x Nb matrix A (interleaved (re, im)) with conjugate-symmetric columns:
// column 2g holds 2 Re A[:, g] and column 2g + 1 holds -2 Im A[:, g] for a
// pair (0 < g < Nb / 2), so that A x = sum_g (col_2g Re x_g + col_2g+1 Im x_g)
// for a conjugate-symmetric x; a real bin (g = 0, g = Nb / 2 for even Nb)
// has Re A[:, g] in column 2g and a zero column 2g + 1.
__global__ void pair_dict_kernel(const float* __restrict__ A, int M, int Nb, int NR, float* __restrict__ C) {
    const int m = blockIdx.x;
    for (int j = threadIdx.x; j < NR; j += blockDim.x) {
        const int g = j >> 1;
        const bool single = g == 0 || ((Nb & 1) == 0 && g == Nb / 2);
        float v = 0.f;
        if (m < M && g <= Nb / 2) {
            const float re = A[((size_t)m * Nb + g) * 2], im = A[((size_t)m * Nb + g) * 2 + 1];
            v = (j & 1) ? (single ? 0.f : -2.f * im) : (single ? re : 2.f * re);
        }
        C[(size_t)m * NR + j] = v;
    }
}
}  // namespace

int pair_dict_atoms(int Nb) { return 2 * (Nb / 2 + 1); }

size_t greedy_hermitian_workspace(int M, int Nb) {
    const int NR = pair_dict_atoms(Nb);
    return align_up((size_t)M * NR * 4, 256) + align_up((size_t)NR * NR * 4, 256) +
           align_up(gomp_coop_dict_floats(M, NR) * 4, 256);
}

namespace {
// The group dictionary, its Gram matrix and the kernel's copies in the
// workspace, built on the stream.
struct PairDict {
    float* G32;
    float* dictbuf;
};
int build_pair_dict(const GreedyLaunch& a, PairDict* out) {
    const int Nb = a.N, NR = pair_dict_atoms(Nb), M = a.M;
    if (!a.workspace || a.workspace_bytes < greedy_hermitian_workspace(M, Nb)) return CSREC_E_WORKSPACE;
    char* ws = static_cast<char*>(a.workspace);
    float* C = reinterpret_cast<float*>(ws);
    out->G32 = reinterpret_cast<float*>(ws + align_up((size_t)M * NR * 4, 256));
    out->dictbuf = reinterpret_cast<float*>(ws + align_up((size_t)M * NR * 4, 256) +
                                            align_up((size_t)NR * NR * 4, 256));
    hipLaunchKernelGGL(pair_dict_kernel, dim3(M), dim3(256), 0, a.stream, a.A, M, Nb, NR, C);
    CSREC_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(gram_kernel, dim3(NR), dim3(256), 0, a.stream, C, M, NR, out->G32, nullptr);
    CSREC_HIP_TRY(hipGetLastError());
    gomp_coop_prepare(C, M, NR, out->dictbuf, a.stream);
    CSREC_HIP_TRY(hipGetLastError());
    return CSREC_OK;
}
}  // namespace

int other_hermitian_launch(const GreedyLaunch& a) {
    if (a.P == 0) return CSREC_OK;
    PairDict d;
    const int e0 = build_pair_dict(a, &d);
    if (e0) return e0;
    const int NR = pair_dict_atoms(a.N);
    constexpr int64_t kChunkH = 65536;
    for (int64_t p0 = 0; p0 < a.P; p0 += kChunkH) {
        const int64_t np = (a.P - p0) < kChunkH ? (a.P - p0) : kChunkH;
        const int e = coop_other_launch(a.kind, a.Y, nullptr, a.X, a.support, a.stats, d.G32, d.dictbuf, a.M, NR,
                                        p0, np, a.K, a.max_iter, a.mu, a.res_tol, a.eps, a.prec, a.stream, a.N);
        if (e) return e;
    }
    return CSREC_OK;
}

int gomp_hermitian_launch(const GreedyLaunch& a) {
    if (a.P == 0) return CSREC_OK;
    const int Nb = a.N, NR = pair_dict_atoms(Nb), M = a.M;
    if (!a.workspace || a.workspace_bytes < greedy_hermitian_workspace(M, Nb)) return CSREC_E_WORKSPACE;
    char* ws = static_cast<char*>(a.workspace);
    float* C = reinterpret_cast<float*>(ws);
    float* G32 = reinterpret_cast<float*>(ws + align_up((size_t)M * NR * 4, 256));
    float* dictbuf = reinterpret_cast<float*>(ws + align_up((size_t)M * NR * 4, 256) +
                                              align_up((size_t)NR * NR * 4, 256));
    hipLaunchKernelGGL(pair_dict_kernel, dim3(M), dim3(256), 0, a.stream, a.A, M, Nb, NR, C);
    CSREC_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(gram_kernel, dim3(NR), dim3(256), 0, a.stream, C, M, NR, G32, nullptr);
    CSREC_HIP_TRY(hipGetLastError());
    gomp_coop_prepare(C, M, NR, dictbuf, a.stream);
    CSREC_HIP_TRY(hipGetLastError());
    constexpr int64_t kChunkH = 65536;
    for (int64_t p0 = 0; p0 < a.P; p0 += kChunkH) {
        const int64_t np = (a.P - p0) < kChunkH ? (a.P - p0) : kChunkH;
        const int e = gomp_coop_launch(a.Y, a.X, a.support, a.stats, G32, dictbuf, nullptr, M, NR, p0, np, a.K,
                                       a.S, a.max_iter, a.prune, a.res_tol, a.eps, 0.0, 0.f, a.prec, a.stream, Nb);
        if (e) return e;
    }
    return CSREC_OK;
}

}  // namespace csrec
