// gOMP (Alg. 3) with the least-squares state on chip.
//
// Work decomposition.  A workgroup is one wavefront holding 4 pixels: lane l
// serves pixel x = l & 3 as sub-lane t = l >> 2 (0..15).  Every per-pixel
// quantity lives in LDS or in the lanes' registers for the whole solve, so
// the solve reads y and the dictionary copies and writes x, and nothing else
// leaves the CU.
//
// Correlation on the matrix cores.  p = A^T r for the wave's 4 pixels is a
// (N x M) by (M x 4) product: v_mfma_f32_4x4x1_16b_f32 forms 16 independent
// 4x4 outer products per instruction, lane 4b + i supplying A's entry for
// the block's row i and lane 4b + x pixel x's residual entry.  With NG
// instructions per row m, lane l loads the NG consecutive atoms NG l + g
// (g < NG) of row m in one vector load (fully coalesced over the wave) and
// feeds entry g to instruction g; lane 4b + x then holds p of pixel x for
// the 4 NG consecutive atoms from 4 NG b, which is where the top-S
// selection reads it.  A is read row-major from an L2-resident padded copy,
// eight rows ahead of the instructions that consume them.
//
// Least squares without triangular-solve chains.  With G[c,c] = L L^T the
// kernel keeps W = L^{-1} (lower triangular, packed rows in LDS) instead of
// L.  Appending atom j to c (a bordered Cholesky step) is then
//   l = W G[c, j],  d = G_jj - ||l||^2,  new row of W = [-l^T W, 1] / sqrt(d)
// and the least-squares solution of G[c,c] s = b_c is s = W^T (W b_c), with
// z = W b_c extended by one dot product per append.  Every one of these is a
// matrix-vector product whose rows (or columns) the 16 lanes split.  The
// atoms of an iteration are appended two at a time, with one pass over W's
// rows (both l) and one over its columns (both new rows) per pair.  The
// Gram entries an append needs are gathered from global memory beforehand,
// all at once, into the packed slot of the row the append then writes.
// d / G_jj is the pivot ratio (squared distance of a_j from span(A[:, c])
// over ||a_j||^2); a pixel with a ratio below the threshold is marked for
// the FP64 pass of the scratch-based kernel.
//
// Per iteration (Alg. 3, steps 1-4), for each active pixel:
//   1. p = A^T r on MFMA; S rounds of a 16-lane argmax over the non-members
//      of c, ties to the lower index.
//   2. append the S atoms; s = W^T z.
//   3. if |c| > K: rank the |s_i| (ties to the lower index), keep the top K
//      as q, solve G[q,q] s_q = b_q by LDL^T elimination (Gram entries
//      gathered in one batch).
//   4. r = y - A(:, q) s_q with lane t owning m = 4t + j + 64i; Delta, ||r||.
#include "common.hpp"

#include <cmath>

namespace csrec {
namespace {

constexpr int kGroups = 4;        // pixels per wavefront
constexpr int kMaxNG = 4;         // atoms per lane and row: N <= 64 NG
constexpr int kRowPad = 8;        // rows of the padded copy of A: multiple of 8
constexpr int kMaxS = 8;
constexpr int kMaxSel = 2 * kMaxS; // atoms selected per iteration (a conjugate pair is two)
constexpr int kGJ = 32;           // K up to this: the pruned system is solved in registers
constexpr float kFp32Limit = 9.5367432e-7f;   // 2^-20: CoSaMP's pivot-ratio limit of an FP32 solve
constexpr int kCU = 6;            // |c| <= 16 kCU entries: per-lane units of the rank and the Gram gather

typedef float v4f_t __attribute__((ext_vector_type(4)));

struct CoopArgs {
    const float* AT;      // N x MP: row n = column n of A (zero padded to MP)
    const float* Ap;      // M8 x NP: A with zero rows to M8 and zero columns to NP = 64 NG
    const float* Y;       // P x M
    const float* G32;     // N x N
    float* X;
    int32_t* support;
    csrec_pixel_stats* stats;
    uint32_t* fbflag;     // per pixel (launch-local) FP64 hand-off, may be null
    int M, N, MP, NP, K, S, Imax, prune;
    float res_tol, eps;
    double pivot_thr;
    float redo_tol;       // relative accuracy an FP32 least squares must keep, or the pixel is redone in FP64
    int64_t P;            // pixels of this launch
    int64_t p0;           // first pixel (index into Y/X/support/stats)
    int CM;               // S * Imax
    int lds_floats;       // per pixel
    float mu;             // BIHT step
    const int8_t* Ysign;  // one-bit BIHT: P x M signs
    const __bf16* Abf;    // (M8 / 4) x NP x 4: A in BF16, four consecutive rows of an atom together
    const _Float16* Ahf;  // the same in FP16
    int prec;             // precision of the correlation A^T v (CSREC_PREC_*)
    int grp;              // 1: conjugate-pair groups (the half-spectrum dictionary of a DFT basis)
    int Nb;               // grp: bins of the complex spectrum (N = 2 (Nb / 2 + 1) real atoms)
};

__host__ __device__ __forceinline__ int tri(int k) { return k * (k + 1) / 2; }

// Every kernel here is one wavefront per workgroup, and lanes exchange data
// only through LDS and cross-lane operations: the LDS executes a wave's
// instructions in issue order, so what lanes wrote is visible to a later
// read by any lane of the wave once the compiler keeps the order.  This
// orders LDS accesses across the point for the compiler without the
// workgroup barrier's waits on outstanding global loads.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__host__ __device__ __forceinline__ int up4(int k) { return (k + 3) & ~3; }

// Atom indices read back from LDS are kept inside [0, N) before they address
// global memory.
__device__ __forceinline__ int clamp_atom(int j, int N) { return (unsigned)j < (unsigned)N ? j : 0; }

// Largest value over the wave.
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int w = __shfl_xor(v, o);
        v = w > v ? w : v;
    }
    return v;
}

// Sum over the 16 lanes of a pixel (lanes x, x + 4, ..., x + 60).
__device__ __forceinline__ float pix_sum(float v) {
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

// (value desc, index asc) argmax over the 16 lanes of a pixel; index -1
// never wins.
__device__ __forceinline__ void pix_argmax(float& v, int& i) {
#pragma unroll
    for (int o = 4; o < 64; o <<= 1) {
        const float ov = __shfl_xor(v, o);
        const int oi = __shfl_xor(i, o);
        const bool take = (oi >= 0) && (i < 0 || ov > v || (ov == v && oi < i));
        v = take ? ov : v;
        i = take ? oi : i;
    }
}

// Per-pixel LDS carving (floats; index arrays stored as int bit patterns).
// Every array starts on a 16-byte boundary.
struct PixLds {
    float* rb;    // residual, MP (read as the MFMA B operand); aliases l, sel, bsel, Wq
    float* W;     // inverse factor of G[c,c], tri(CM); slot of row n holds G[c, j] before its append
    float* z;     // W b_c, CM
    float* b;     // b_c, CM
    float* s;     // solution on c, CM
    float* l;     // temporary, CM
    int* c;       // atoms, CM
    int* sel;     // this iteration's selected atoms, kMaxSel
    float* bsel;  // their a_j^T y, kMaxSel
    float* Wq;    // K > kGJ: LDL^T triangle of G[q,q], tri(K); K <= kGJ: pivot-row slots, 2 x 36
    float* bq;    // K
    float* sq;    // K
    int* q;       // K
    int* kp;      // CM: 1 where position k of c was kept by the last prune
};

struct LdsPlan {
    int rb, W, z, b, s, l, c, sel, bsel, Wq, bq, sq, q, kp, total;
};

// Offsets (floats) of one pixel's region; the stride is padded to 8 mod 64
// floats so that the 4 pixels' packed-row reads fall in distinct banks.  The
// residual (read by the correlation only) shares its space with the
// temporaries that are live only after the correlation: the selections, the
// append temporary l and the prune's scratch.
__host__ __device__ inline LdsPlan lds_plan(int MP, int CM, int K) {
    LdsPlan p;
    int o = 0;
    p.rb = o;
    p.l = o;
    p.sel = p.l + up4(CM);
    p.bsel = p.sel + kMaxSel;
    p.Wq = p.bsel + kMaxSel;
    const int tail = p.Wq + (K > kGJ ? up4(tri(K)) : 2 * (kGJ + 4));
    o = up4(MP) > tail ? up4(MP) : tail;
    p.W = o; o += up4(tri(CM));
    p.z = o; o += up4(CM);
    p.b = o; o += up4(CM);
    p.s = o; o += up4(CM);
    p.c = o; o += up4(CM);
    p.bq = o; o += up4(K);
    p.sq = o; o += up4(K);
    p.q = o; o += up4(K);
    p.kp = o; o += up4(CM);
    o += ((8 - o) % 64 + 64) % 64;
    p.total = o;
    return p;
}

__device__ __forceinline__ PixLds carve(float* base, const CoopArgs& a) {
    const LdsPlan pl = lds_plan(a.MP, a.CM, a.grp ? 2 * a.K : a.K);   // groups keep up to 2K atoms
    PixLds p;
    p.rb = base + pl.rb;
    p.W = base + pl.W;
    p.z = base + pl.z;
    p.b = base + pl.b;
    p.s = base + pl.s;
    p.l = base + pl.l;
    p.c = reinterpret_cast<int*>(base + pl.c);
    p.sel = reinterpret_cast<int*>(base + pl.sel);
    p.bsel = base + pl.bsel;
    p.Wq = base + pl.Wq;
    p.bq = base + pl.bq;
    p.sq = base + pl.sq;
    p.q = reinterpret_cast<int*>(base + pl.q);
    p.kp = reinterpret_cast<int*>(base + pl.kp);
    return p;
}

// sum_{k < len} u[k] v[k] over LDS operands with four independent partial sums.
__device__ __forceinline__ float dot4(const float* u, const float* v, int len) {
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    int k = 0;
    for (; k + 4 <= len; k += 4) {
        s0 += u[k] * v[k];
        s1 += u[k + 1] * v[k + 1];
        s2 += u[k + 2] * v[k + 2];
        s3 += u[k + 3] * v[k + 3];
    }
    for (; k < len; ++k) s0 += u[k] * v[k];
    return (s0 + s1) + (s2 + s3);
}

// sum_{k <= i < n} v[i] W[tri(i) + k]: column k of the packed factor below
// (and on) the diagonal against v, four independent partial sums.
__device__ __forceinline__ float coldot4(const float* Wf, const float* v, int k, int n) {
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    int i = k;
    int off = tri(k) + k;   // tri(i) + k, advanced by i + 1 per row
    for (; i + 4 <= n; i += 4) {
        const int o1 = off + i + 1, o2 = o1 + i + 2, o3 = o2 + i + 3;
        s0 += v[i] * Wf[off];
        s1 += v[i + 1] * Wf[o1];
        s2 += v[i + 2] * Wf[o2];
        s3 += v[i + 3] * Wf[o3];
        off = o3 + i + 4;
    }
    for (; i < n; ++i) {
        s0 += v[i] * Wf[off];
        off += i + 1;
    }
    return (s0 + s1) + (s2 + s3);
}

// dot4 of u against two vectors at once (u read once).
__device__ __forceinline__ void dot4x2(const float* u, const float* v0, const float* v1, int len, float& r0,
                                       float& r1) {
    float a0 = 0.f, a1 = 0.f, b0 = 0.f, b1 = 0.f;
    int k = 0;
    for (; k + 2 <= len; k += 2) {
        const float u0 = u[k], u1 = u[k + 1];
        a0 += u0 * v0[k];
        a1 += u1 * v0[k + 1];
        b0 += u0 * v1[k];
        b1 += u1 * v1[k + 1];
    }
    if (k < len) {
        a0 += u[k] * v0[k];
        b0 += u[k] * v1[k];
    }
    r0 = a0 + a1;
    r1 = b0 + b1;
}

// coldot4 against two vectors at once (the column of W read once).
__device__ __forceinline__ void coldot4x2(const float* Wf, const float* v0, const float* v1, int k, int n, float& r0,
                                          float& r1) {
    float a0 = 0.f, a1 = 0.f, b0 = 0.f, b1 = 0.f;
    int i = k;
    int off = tri(k) + k;
    for (; i + 2 <= n; i += 2) {
        const int o1 = off + i + 1;
        const float w0 = Wf[off], w1 = Wf[o1];
        a0 += v0[i] * w0;
        a1 += v0[i + 1] * w1;
        b0 += v1[i] * w0;
        b1 += v1[i + 1] * w1;
        off = o1 + i + 2;
    }
    if (i < n) {
        a0 += v0[i] * Wf[off];
        b0 += v1[i] * Wf[off];
    }
    r0 = a0 + a1;
    r1 = b0 + b1;
}

// Two bordered steps in one pass over W: appends atom j0 (the slot of row n
// holds G[idx, j0] and G_00) and, where on1, atom j1 (the slot of row n + 1
// holds G[idx, j1], G[j0, j1] and G_11) to the factor of size n.  With
// l0 = W g0 and l1 = W g1 (one pass over W's rows), the Schur complement of
// G[c,c] in the 2 x 2 block is [[G_00 - l0.l0, .], [G_01 - l0.l1,
// G_11 - l1.l1]]; its Cholesky factor gives the pivots d0 = G_00 - |l0|^2
// and d1 = G_11 - |l1|^2 - e^2 with e = (G_01 - l0.l1) / sqrt(d0), the
// last entry of atom j1's l once j0 is in the factor.  The new rows are
// then, with Q_u = W^T l_u (one pass over W's columns):
//   row n     = [-Q_0, 1] / sqrt(d0)
//   row n + 1 = [-(Q_1 + e row_n[:n]), -e / sqrt(d0), 1] / sqrt(d1)
// which is what two single steps compute.  l0 and l1 are LDS scratch of n
// floats each.  All 64 lanes call it; on0 masks the pixels that append,
// on1 (implies on0) those that append a second atom.  Returns the pivot
// ratios d / G_jj, the diagonal entries G_jj and, with want_sq, the squared
// norms of the new rows of W.
__device__ __forceinline__ void inv_append2(bool on0, bool on1, int t, int n, float* Wf, float* zf, float* bf,
                                            int* idx, float* l0, float* l1, int j0, int j1, float b0, float b1,
                                            bool want_sq, float& ratio0, float& ratio1, float& g00, float& g11,
                                            float& sq0, float& sq1) {
    float* w0 = Wf + tri(n);
    float* w1 = Wf + tri(n + 1);
    float a00 = 0.f, a01 = 0.f, a11 = 0.f;
    if (on1) {
        for (int i = t; i < n; i += 16) {
            float p0, p1;
            dot4x2(Wf + tri(i), w0, w1, i + 1, p0, p1);
            l0[i] = p0;
            l1[i] = p1;
            a00 += p0 * p0;
            a01 += p0 * p1;
            a11 += p1 * p1;
        }
    } else if (on0) {
        for (int i = t; i < n; i += 16) {
            const float p0 = dot4(Wf + tri(i), w0, i + 1);
            l0[i] = p0;
            a00 += p0 * p0;
        }
    }
    g00 = on0 ? w0[n] : 1.f;
    const float g01 = on1 ? w1[n] : 0.f;
    g11 = on1 ? w1[n + 1] : 1.f;
    a00 = pix_sum(a00);
    a01 = pix_sum(a01);
    a11 = pix_sum(a11);
    wave_sync();
    // A pivot below FP32 resolution (the atom is numerically in the span) is
    // floored so the factor stays finite; such a pixel carries a ratio far
    // below any fallback threshold.
    const float d0 = g00 - a00;
    ratio0 = d0 / g00;
    const float inv0 = 1.f / sqrtf(d0 > g00 * 5.9604645e-8f ? d0 : g00 * 5.9604645e-8f);
    const float e = (g01 - a01) * inv0;
    const float d1 = g11 - a11 - e * e;
    ratio1 = d1 / g11;
    const float inv1 = 1.f / sqrtf(d1 > g11 * 5.9604645e-8f ? d1 : g11 * 5.9604645e-8f);
    float z0 = 0.f, z1 = 0.f, s0 = 0.f, s1 = 0.f;
    if (on1) {
        for (int k = t; k < n; k += 16) {
            float q0, q1;
            coldot4x2(Wf, l0, l1, k, n, q0, q1);
            const float u0 = -q0 * inv0;
            const float u1 = -(q1 + e * u0) * inv1;
            w0[k] = u0;
            w1[k] = u1;
            z0 += u0 * bf[k];
            z1 += u1 * bf[k];
            s0 += u0 * u0;
            s1 += u1 * u1;
        }
    } else if (on0) {
        for (int k = t; k < n; k += 16) {
            const float u0 = -coldot4(Wf, l0, k, n) * inv0;
            w0[k] = u0;
            z0 += u0 * bf[k];
            s0 += u0 * u0;
        }
    }
    if (on0 && t == 0) {
        w0[n] = inv0;
        z0 += inv0 * b0;
        s0 += inv0 * inv0;
        if (on1) {
            const float u1n = -e * inv0 * inv1;
            w1[n] = u1n;
            w1[n + 1] = inv1;
            z1 += u1n * b0 + inv1 * b1;
            s1 += u1n * u1n + inv1 * inv1;
        }
    }
    z0 = pix_sum(z0);
    z1 = pix_sum(z1);
    if (want_sq) {
        sq0 = pix_sum(s0);
        sq1 = pix_sum(s1);
    }
    if (on0 && t == 0) {
        zf[n] = z0;
        bf[n] = b0;
        idx[n] = j0;
        if (on1) {
            zf[n + 1] = z1;
            bf[n + 1] = b1;
            idx[n + 1] = j1;
        }
    }
    wave_sync();
}

// s = W^T z on the first n entries (columns k = t + 16u).
__device__ __forceinline__ void inv_solve(bool on, int t, int n, const float* Wf, const float* zf, float* sf) {
    if (on)
        for (int k = t; k < n; k += 16) sf[k] = coldot4(Wf, zf, k, n);
    wave_sync();
}

__device__ __forceinline__ float rank_key(float v) {
    const float a = fabsf(v);
    return a <= 3.402823466e38f ? a : -1.f;   // NaN and inf rank last
}

// q[rank] = c[k] and qv[rank] = vals[k] for the K entries k < n with the
// largest |s[k]| (ties to the lower atom index).  The key maps non-finite
// |s| below every finite one, so (key desc, index asc) is a strict total
// order over distinct atoms and the ranks are a permutation: q[0..min(K, n))
// is always fully written.  No barrier inside; s, c, vals must be readable
// (their writes followed by a barrier).  s and c are read as 16-byte vectors
// up to n rounded to 4.  n <= 16 U.
template <int U>
__device__ __forceinline__ void rank_top(bool on, int t, int n, int K, const float* s, const int* c,
                                         const float* vals, int* q, float* qv) {
    if (!on) return;
    float vk[U];
    int ck[U], rk[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int k = t + 16 * u;
        vk[u] = k < n ? rank_key(s[k]) : 0.f;
        ck[u] = k < n ? c[k] : 0;
        rk[u] = 0;
    }
    for (int i0 = 0; i0 < n; i0 += 4) {
        const float4 sv = *reinterpret_cast<const float4*>(s + i0);
        const int4 cv = *reinterpret_cast<const int4*>(c + i0);
        const float v4[4] = {rank_key(sv.x), rank_key(sv.y), rank_key(sv.z), rank_key(sv.w)};
        const int c4[4] = {cv.x, cv.y, cv.z, cv.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (i0 + e < n) {
#pragma unroll
                for (int u = 0; u < U; ++u)
                    rk[u] += (v4[e] > vk[u] || (v4[e] == vk[u] && c4[e] < ck[u])) ? 1 : 0;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int k = t + 16 * u;
        if (k < n && rk[u] < K) {
            q[rk[u]] = ck[u];
            qv[rk[u]] = vals[k];
        }
    }
}

// sol = G[L,L]^{-1} rhs for the n atoms of the list L (n <= nmax, nmax
// uniform over the wave; a pixel with n < nmax is padded with identity rows
// and zero right-hand sides, so every pixel runs the same nmax barriered
// steps).  rhs (nmax entries) is destroyed.  Called by every lane.
//
// nmax <= GJ (GJ <= kGJ): Gauss-Jordan elimination on registers.  Lane t
// owns rows t and t + 16 of [G[L,L] | rhs], gathered in one batch.  Step k (fully
// unrolled, so every register index is static) publishes pivot row k
// through a double-buffered LDS slot in scr (2 x (kGJ + 4) floats; one
// barrier) and every other row subtracts its multiple of it over the columns
// j >= k still in play; all-zero padding columns are skipped.  After nmax
// steps row i reads d_i sol_i = rhs_i, with d_i the row's pivot.
//
// nmax > GJ: right-looking LDL^T elimination of the lower triangle C of
// G[L,L] in scr (tri(nmax) floats, gathered in one batch), the forward
// substitution of rhs riding along, then a column-oriented back
// substitution: 2 nmax steps, each one barrier and a set of independent
// element updates split over the 16 lanes.  C keeps the unscaled columns
// (C_ik = D_k Lt_ik), so no square roots.
//
// Every pivot is floored at 2^-24 of the original diagonal like the appends,
// so a numerically dependent atom keeps the solution finite.
// With RATIO, *rmin receives this lane's smallest pivot ratio d_k / G_kk
// (the Schur-complement pivot over the original diagonal, before the floor)
// over the pivots it saw: the Gauss-Jordan forms see their own rows', the
// LDL^T form every pivot of the pixel.
template <bool PAD, int GJ, bool RATIO = false>
__device__ __forceinline__ void solve_list_w(bool on, int t, int n, int nmax, int N, const float* __restrict__ G32,
                                           const int* L, float* rhs, float* sol, float* scr,
                                           float* rmin = nullptr) {
    float rl = 1.f;
    if (!PAD) n = nmax;   // every pixel solves a full list
    if (PAD) {
        if (on)
            for (int i = n + t; i < nmax; i += 16) rhs[i] = 0.f;
        wave_sync();
    }
    if (nmax <= GJ) {
        constexpr int W1 = GJ + 1;          // nmax columns (padded to GJ) + the right-hand side
        constexpr int SLOT = GJ + 4;
        float R0[W1], R1[W1];
        const bool h0 = on && t < n, h1 = on && t + 16 < n;
        const int q0 = clamp_atom(h0 ? L[t] : 0, N), q1 = clamp_atom(h1 ? L[t + 16] : 0, N);
#pragma unroll
        for (int j = 0; j < GJ; ++j) {
            const bool hj = on && j < n;
            const int qj = clamp_atom(hj ? L[j] : 0, N);
            R0[j] = (h0 && hj) ? G32[(size_t)q0 * N + qj] : ((PAD && j == t) ? 1.f : 0.f);
            R1[j] = (h1 && hj) ? G32[(size_t)q1 * N + qj] : ((PAD && j == t + 16) ? 1.f : 0.f);
        }
        R0[GJ] = (PAD ? on && t < nmax : h0) ? rhs[t] : 0.f;
        R1[GJ] = (PAD ? on && t + 16 < nmax : h1) ? rhs[t + 16] : 0.f;
        const float fl0 = (h0 ? G32[(size_t)q0 * N + q0] : 1.f) * 5.9604645e-8f;
        const float fl1 = (h1 ? G32[(size_t)q1 * N + q1] : 1.f) * 5.9604645e-8f;
        float dg0 = 1.f, dg1 = 1.f;
#pragma unroll
        for (int k = 0; k < GJ; ++k) {
            if (k < nmax) {   // uniform
                float* slot = scr + (k & 1) * SLOT;
                if (t == (k & 15)) {
                    float* R = k < 16 ? R0 : R1;
                    const float fl = k < 16 ? fl0 : fl1;
                    if constexpr (RATIO) rl = fminf(rl, R[k] / (fl * 16777216.f));
                    R[k] = R[k] > fl ? R[k] : fl;
                    if (k < 16) dg0 = R[k]; else dg1 = R[k];
                    if (on) {
#pragma unroll
                        for (int j = k & ~3; j < W1 + 3; j += 4) {
                            if (j >= nmax && j < GJ) continue;   // all-zero padding columns (uniform)
                            const float4 v = make_float4(R[j], j + 1 < W1 ? R[j + 1] : 0.f,
                                                         j + 2 < W1 ? R[j + 2] : 0.f, j + 3 < W1 ? R[j + 3] : 0.f);
                            *reinterpret_cast<float4*>(slot + j) = v;
                        }
                    }
                }
                wave_sync();
                if (on) {
                    const float rp = 1.f / slot[k];
                    const float f0 = (t == k) ? 0.f : R0[k] * rp;
                    const float f1 = (t + 16 == k) ? 0.f : R1[k] * rp;
#pragma unroll
                    for (int j = k & ~3; j < W1; j += 4) {
                        if (j >= nmax && j < GJ) continue;   // all-zero padding columns (uniform)
                        const float4 v = *reinterpret_cast<const float4*>(slot + j);
                        const float pv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            if (j + e > k && j + e < W1) {
                                R0[j + e] -= f0 * pv[e];
                                R1[j + e] -= f1 * pv[e];
                            }
                        }
                    }
                }
            }
        }
        if (on && t < n) sol[t] = R0[GJ] / dg0;
        if (on && t + 16 < n) sol[t + 16] = R1[GJ] / dg1;
        if constexpr (RATIO) *rmin = rl;
        wave_sync();
        return;
    }
    // all Gram entries of G[L,L] (lower triangle): lane t gathers rows
    // r = t + 16 m, entry (r, i), i <= r, to C[tri(r) + i] (identity beyond
    // n); the diagonal is also kept in sol (the pivot floors), which the back
    // substitution overwrites last
    float* C = scr;
    if (on) {
        for (int r = t; r < nmax; r += 16) {
            float* cr = C + tri(r);
            if (r < n) {
                const int qr = clamp_atom(L[r], N);
                int i = 0;
                for (; i + 4 <= r + 1; i += 4) {
                    const float g0 = G32[(size_t)clamp_atom(L[i], N) * N + qr];
                    const float g1 = G32[(size_t)clamp_atom(L[i + 1], N) * N + qr];
                    const float g2 = G32[(size_t)clamp_atom(L[i + 2], N) * N + qr];
                    const float g3 = G32[(size_t)clamp_atom(L[i + 3], N) * N + qr];
                    cr[i] = g0;
                    cr[i + 1] = g1;
                    cr[i + 2] = g2;
                    cr[i + 3] = g3;
                }
                for (; i <= r; ++i) cr[i] = G32[(size_t)clamp_atom(L[i], N) * N + qr];
            } else {
                for (int i = 0; i <= r; ++i) cr[i] = i == r ? 1.f : 0.f;
            }
            sol[r] = cr[r];
        }
    }
    wave_sync();
    // LDL^T elimination with the forward substitution of rhs, two pivots per
    // pass over the trailing rows: pivot k first updates column k + 1 and
    // rhs[k + 1] (barrier), then every row i >= k + 2 takes both pivots' terms
    // in one read and write per entry, in the order of two single steps (so
    // the factor is bit-identical to them).  Column k of rows j is read at
    // tri(j) + k, advanced by j + 1 per row; column k + 1 sits next to it.
    auto pivot = [&](int k) {
        float piv = C[tri(k) + k];
        const float fl = sol[k] * 5.9604645e-8f;
        if constexpr (RATIO) rl = fminf(rl, piv / sol[k]);
        return piv > fl ? piv : fl;
    };
    int k = 0;
    for (; k + 1 < nmax; k += 2) {
        float rp0 = 0.f;
        if (on) {
            const float piv = pivot(k);
            rp0 = 1.f / piv;
            const float c10 = C[tri(k + 1) + k];
            for (int i = k + 1 + t; i < nmax; i += 16) {
                float* ci = C + tri(i);
                const float f = ci[k] * rp0;
                ci[k + 1] -= f * c10;
            }
            if (t == 0) {
                const float f = c10 * rp0;
                rhs[k + 1] -= f * rhs[k];
                C[tri(k) + k] = piv;
            }
        }
        wave_sync();
        if (on) {
            const float piv1 = pivot(k + 1);
            const float rp1 = 1.f / piv1;
            const float bk = rhs[k], bk1 = rhs[k + 1];
            for (int i = k + 2 + t; i < nmax; i += 16) {
                float* ci = C + tri(i);
                const float f0 = ci[k] * rp0;
                const float f1 = ci[k + 1] * rp1;
                int off = tri(k + 2) + k;
                for (int j = k + 2; j <= i; ++j) {
                    float x = ci[j];
                    x -= f0 * C[off];
                    x -= f1 * C[off + 1];
                    ci[j] = x;
                    off += j + 1;
                }
                float r = rhs[i];
                r -= f0 * bk;
                r -= f1 * bk1;
                rhs[i] = r;
            }
            if (t == 0) C[tri(k + 1) + k + 1] = piv1;
        }
        wave_sync();
    }
    if (k < nmax) {   // the last pivot of an odd count (no rows below it)
        if (on && t == 0) C[tri(k) + k] = pivot(k);
        wave_sync();
    }
    // back substitution: sol_i = (bt_i - sum_{k>i} C_ki sol_k) / D_i, column-oriented
    for (int i = nmax - 1; i >= 0; --i) {
        if (on) {
            const float si = rhs[i] / C[tri(i) + i];
            for (int k = t; k < i; k += 16) rhs[k] -= C[tri(i) + k] * si;
            if (t == 0) sol[i] = si;
        }
        wave_sync();
    }
    if constexpr (RATIO) *rmin = rl;
}


// The register Gauss-Jordan elimination of solve_list_w for lists of 33 to
// 48 atoms (CoSaMP's merged supports up to 3K = 48): lane t owns rows t,
// t + 16 and t + 32 of [G[L,L] | rhs].  Step k publishes pivot row k through
// the double-buffered slot (one wave barrier) and every other row subtracts
// its multiple of it, so a solve is nmax steps with every row update in
// registers, against 2 nmax barriered steps of the LDS LDL^T form.  Same
// pivot floors, padding and arguments as solve_list_w; scr holds at least
// 2 (48 + 4) floats.  Called by every lane.
template <bool PAD, bool RATIO = false>
__device__ __forceinline__ void solve_gj48(bool on, int t, int n, int nmax, int N, const float* __restrict__ G32,
                                           const int* L, float* rhs, float* sol, float* scr,
                                           float* rmin = nullptr) {
    float rl = 1.f;
    constexpr int GJ = 48, RPL = 3;
    constexpr int W1 = GJ + 1;   // nmax columns (padded to GJ) + the right-hand side
    constexpr int SLOT = GJ + 4;
    if (!PAD) n = nmax;
    if (PAD) {
        if (on)
            for (int i = n + t; i < nmax; i += 16) rhs[i] = 0.f;
        wave_sync();
    }
    float R[RPL][W1];
    bool h[RPL];
    int qr[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        h[r] = on && t + 16 * r < n;
        qr[r] = clamp_atom(h[r] ? L[t + 16 * r] : 0, N);
    }
#pragma unroll
    for (int j = 0; j < GJ; ++j) {
        if ((j & 7) == 0) __builtin_amdgcn_sched_barrier(0);   // 24 gathers in flight at a time
        const bool hj = on && j < n;
        const int qj = clamp_atom(hj ? L[j] : 0, N);
#pragma unroll
        for (int r = 0; r < RPL; ++r)
            R[r][j] = (h[r] && hj) ? G32[(size_t)qr[r] * N + qj] : ((PAD && j == t + 16 * r) ? 1.f : 0.f);
    }
    float fl[RPL], dg[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        R[r][GJ] = (PAD ? on && t + 16 * r < nmax : h[r]) ? rhs[t + 16 * r] : 0.f;
        fl[r] = (h[r] ? G32[(size_t)qr[r] * N + qr[r]] : 1.f) * 5.9604645e-8f;
        dg[r] = 1.f;
    }
#pragma unroll
    for (int k = 0; k < GJ; ++k) {
        if (k < nmax) {   // uniform
            float* slot = scr + (k & 1) * SLOT;
            const int kr = k >> 4;
            if (t == (k & 15)) {
                if constexpr (RATIO) rl = fminf(rl, R[kr][k] / (fl[kr] * 16777216.f));
                R[kr][k] = R[kr][k] > fl[kr] ? R[kr][k] : fl[kr];
                dg[kr] = R[kr][k];
                if (on) {
#pragma unroll
                    for (int j = k & ~3; j < W1 + 3; j += 4) {
                        if (j >= nmax && j < GJ) continue;   // all-zero padding columns (uniform)
                        const float4 v = make_float4(R[kr][j], j + 1 < W1 ? R[kr][j + 1] : 0.f,
                                                     j + 2 < W1 ? R[kr][j + 2] : 0.f, j + 3 < W1 ? R[kr][j + 3] : 0.f);
                        *reinterpret_cast<float4*>(slot + j) = v;
                    }
                }
            }
            wave_sync();
            if (on) {
                const float rp = 1.f / slot[k];
                float f[RPL];
#pragma unroll
                for (int r = 0; r < RPL; ++r) f[r] = (t + 16 * r == k) ? 0.f : R[r][k] * rp;
#pragma unroll
                for (int j = k & ~3; j < W1; j += 4) {
                    if (j >= nmax && j < GJ) continue;   // all-zero padding columns (uniform)
                    // a few pivot-row reads in flight at a time: the rows
                    // already take 3 (GJ + 1) registers
                    if (((j - (k & ~3)) & 15) == 0) __builtin_amdgcn_sched_barrier(0);
                    const float4 v = *reinterpret_cast<const float4*>(slot + j);
                    const float pv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        if (j + e > k && j + e < W1) {
#pragma unroll
                            for (int r = 0; r < RPL; ++r) R[r][j + e] -= f[r] * pv[e];
                        }
                    }
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < RPL; ++r)
        if (on && t + 16 * r < n) sol[t + 16 * r] = R[r][GJ] / dg[r];
    if constexpr (RATIO) *rmin = rl;
    wave_sync();
}

// The register elimination is unrolled over its width, and its code is most
// of the kernel's: a list of at most kGJSmall atoms runs an instance of that
// width, so the loop's instructions stay within the instruction cache.
constexpr int kGJSmall = 20;
template <bool PAD, bool RATIO = false>
__device__ __forceinline__ void solve_list(bool on, int t, int n, int nmax, int N, const float* __restrict__ G32,
                                           const int* L, float* rhs, float* sol, float* scr,
                                           float* rmin = nullptr) {
    if (nmax <= kGJSmall)   // uniform over the wave
        solve_list_w<PAD, kGJSmall, RATIO>(on, t, n, nmax, N, G32, L, rhs, sol, scr, rmin);
    else
        solve_list_w<PAD, kGJ, RATIO>(on, t, n, nmax, N, G32, L, rhs, sol, scr, rmin);
}

// Step 3 of Alg. 3 for the pixels with `on`: q = the K entries of c with
// largest |s| (ties to the lower index), then s_q = G[q,q]^{-1} b_q.
// Called by every lane (it holds barriers).
// gOMP's prune: the K entries of largest |s| on c, ranked as rank_top, but
// written to q (atoms) and qv (their vals) in the order of their positions
// in c, so that the same kept set always gives the same list.  kp holds the
// kept flag of every position of c from the last prune (0 for positions
// appended since); it is updated here.  Returns, for a pixel with on, whether
// the kept set differs from the last prune's (the same on the pixel's 16
// lanes).  Called by every lane of the wave.
template <int U>
__device__ __forceinline__ bool rank_keep(bool on, int t, int n, int K, const float* s, const int* c,
                                          const float* vals, int* q, float* qv, int* kp) {
    int diff = 0;
    bool kept[U];
#pragma unroll
    for (int u = 0; u < U; ++u) kept[u] = false;
    if (on) {
        float vk[U];
        int ck[U], rk[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = t + 16 * u;
            vk[u] = k < n ? rank_key(s[k]) : 0.f;
            ck[u] = k < n ? c[k] : 0;
            rk[u] = 0;
        }
        for (int i0 = 0; i0 < n; i0 += 4) {
            const float4 sv = *reinterpret_cast<const float4*>(s + i0);
            const int4 cv = *reinterpret_cast<const int4*>(c + i0);
            const float v4[4] = {rank_key(sv.x), rank_key(sv.y), rank_key(sv.z), rank_key(sv.w)};
            const int c4[4] = {cv.x, cv.y, cv.z, cv.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (i0 + e < n) {
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        rk[u] += (v4[e] > vk[u] || (v4[e] == vk[u] && c4[e] < ck[u])) ? 1 : 0;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = t + 16 * u;
            if (k < n) {
                kept[u] = rk[u] < K;
                diff |= ((kp[k] != 0) != kept[u]) ? 1 : 0;
                kp[k] = kept[u] ? 1 : 0;
            }
        }
    }
    // the kept positions in order: position k = t + 16 u goes to the number
    // of kept positions before it, counted from one ballot per unit (the
    // pixel's 16 lanes are lanes x, x + 4, ..., x + 60 of the wave)
    const int lane = threadIdx.x & 63;
    const unsigned long long pix_bits = 0x1111111111111111ull << (lane & 3);
    const unsigned long long below = pix_bits & ((1ull << lane) - 1ull);
    int base = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const unsigned long long m = __ballot(kept[u]);
        if (kept[u]) {
            const int idx = base + __popcll(m & below);
            const int k = t + 16 * u;
            q[idx] = c[k];
            qv[idx] = vals[k];
        }
        base += __popcll(m & pix_bits);
    }
    diff |= __shfl_xor(diff, 4);
    diff |= __shfl_xor(diff, 8);
    diff |= __shfl_xor(diff, 16);
    diff |= __shfl_xor(diff, 32);
    return on && diff != 0;
}

// Returns, for a pixel with on, whether its kept set q changed since the
// last prune.  The solve on q is skipped when no pixel of the wave needs it:
// a pixel whose q did not change keeps the solution of its last prune, which
// the same list and right-hand side would reproduce exactly.
// BIG: K up to 48 solves q by the three-row register elimination (a kernel
// instance of its own, so the smaller K keep their register budget).
template <bool BIG = false>
__device__ __forceinline__ bool prune_to_q(bool on, int t, int nc, int nmax_c, int K, int N,
                                           const float* __restrict__ G32, const PixLds L) {
    // as many 16-atom rank units as the longest list in the wave needs
    const int nw = wave_max(on ? nc : 0);
    bool changed;
    if (nw <= 32)
        changed = rank_keep<2>(on, t, nc, K, L.s, L.c, L.b, L.q, L.bq, L.kp);
    else if (nw <= 48)
        changed = rank_keep<3>(on, t, nc, K, L.s, L.c, L.b, L.q, L.bq, L.kp);
    else if (nw <= 64)
        changed = rank_keep<4>(on, t, nc, K, L.s, L.c, L.b, L.q, L.bq, L.kp);
    else
        changed = rank_keep<kCU>(on, t, nc, K, L.s, L.c, L.b, L.q, L.bq, L.kp);
    (void)nmax_c;
    wave_sync();
    if (__any(changed)) {
        if (BIG && K > kGJ && K <= 48)   // uniform
            solve_gj48<false>(on, t, K, K, N, G32, L.q, L.bq, L.sq, L.Wq);
        else
            solve_list<false>(on, t, K, K, N, G32, L.q, L.bq, L.sq, L.Wq);
    }
    return changed;
}

// p = A^T v for the wave's 4 pixels, v in the pixel's LDS vector rb (MP
// entries, zero beyond M), on MFMA; lane 4b + x receives p of pixel x for
// atoms 4 NG b + NG i + g in acc[g][i].
//
// FP32: v_mfma_f32_4x4x1_16b_f32, one row m per instruction; lane l loads
// atoms NG l .. NG l + NG - 1 of row m of the padded copy Ap (coalesced over
// the wave), eight rows ahead of their use.
//
// BF16 / FP16: v_mfma_f32_4x4x4_16b_{bf16,f16}, four rows per instruction,
// FP32 accumulation: lane l loads the four rows of each of its NG atoms
// from the 16-bit copy (laid out (M8 / 4) x NP x 4, so that this is one
// contiguous 8 NG-byte load), and v is rounded to the same format.  Half the
// bytes and a quarter of the instructions of the FP32 form.
template <typename H>
__device__ __forceinline__ v4f_t mfma_4x4x4(const H __attribute__((ext_vector_type(4))) & a,
                                            const H __attribute__((ext_vector_type(4))) & b, v4f_t c);
template <>
__device__ __forceinline__ v4f_t mfma_4x4x4<__bf16>(const __bf16 __attribute__((ext_vector_type(4))) & a,
                                                    const __bf16 __attribute__((ext_vector_type(4))) & b, v4f_t c) {
    return __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(a, b, c, 0, 0, 0);
}
template <>
__device__ __forceinline__ v4f_t mfma_4x4x4<_Float16>(const _Float16 __attribute__((ext_vector_type(4))) & a,
                                                      const _Float16 __attribute__((ext_vector_type(4))) & b,
                                                      v4f_t c) {
    return __builtin_amdgcn_mfma_f32_4x4x4f16(a, b, c, 0, 0, 0);
}

template <int NG, typename H>
__device__ __forceinline__ void correlate16(const H* __restrict__ Ah, int NP, const float* rb, int lane, int M8,
                                            v4f_t (&acc)[NG]) {
    typedef H v4h __attribute__((ext_vector_type(4)));
    constexpr int AHEAD = 2;   // 4-row blocks loaded ahead of their use
    const v4h* ap = reinterpret_cast<const v4h*>(Ah) + NG * lane;   // block m4 starts at m4 * NP vectors
    const int nb = M8 / 4;
    v4h cur[AHEAD][NG];
#pragma unroll
    for (int d = 0; d < AHEAD; ++d)
#pragma unroll
        for (int g = 0; g < NG; ++g) cur[d][g] = d < nb ? ap[(size_t)d * NP + g] : v4h{};
    for (int m4 = 0; m4 < nb; m4 += AHEAD) {
        v4h nxt[AHEAD][NG];
#pragma unroll
        for (int d = 0; d < AHEAD; ++d)
#pragma unroll
            for (int g = 0; g < NG; ++g)
                nxt[d][g] = m4 + AHEAD + d < nb ? ap[(size_t)(m4 + AHEAD + d) * NP + g] : v4h{};
#pragma unroll
        for (int d = 0; d < AHEAD; ++d) {
            if (m4 + d < nb) {
                const float4 rr = *reinterpret_cast<const float4*>(rb + 4 * (m4 + d));
                const v4h bv = {(H)rr.x, (H)rr.y, (H)rr.z, (H)rr.w};
#pragma unroll
                for (int g = 0; g < NG; ++g) acc[g] = mfma_4x4x4<H>(cur[d][g], bv, acc[g]);
            }
        }
#pragma unroll
        for (int d = 0; d < AHEAD; ++d)
#pragma unroll
            for (int g = 0; g < NG; ++g) cur[d][g] = nxt[d][g];
    }
}

template <int NG>
__device__ __forceinline__ void correlate(const CoopArgs& a, const float* rb, int lane, int M8, int prec,
                                          v4f_t (&acc)[NG]) {
#pragma unroll
    for (int g = 0; g < NG; ++g) acc[g] = v4f_t{0.f, 0.f, 0.f, 0.f};
    if (prec == CSREC_PREC_BF16) {
        correlate16<NG, __bf16>(a.Abf, a.NP, rb, lane, M8, acc);
        return;
    }
    if (prec == CSREC_PREC_F16) {
        correlate16<NG, _Float16>(a.Ahf, a.NP, rb, lane, M8, acc);
        return;
    }
    typedef float vNG __attribute__((ext_vector_type(NG)));
    const vNG* ap = reinterpret_cast<const vNG*>(a.Ap) + lane;   // row m starts at m * 64 vectors
    vNG cur[kRowPad], nxt[kRowPad];
#pragma unroll
    for (int r8 = 0; r8 < kRowPad; ++r8) cur[r8] = ap[(size_t)r8 * 64];
    for (int m0 = 0; m0 < M8; m0 += kRowPad) {
        if (m0 + kRowPad < M8) {
#pragma unroll
            for (int r8 = 0; r8 < kRowPad; ++r8) nxt[r8] = ap[(size_t)(m0 + kRowPad + r8) * 64];
        }
        const float4 r0 = *reinterpret_cast<const float4*>(rb + m0);
        const float4 r1 = *reinterpret_cast<const float4*>(rb + m0 + 4);
        const float rv[kRowPad] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
#pragma unroll
        for (int r8 = 0; r8 < kRowPad; ++r8)
#pragma unroll
            for (int g = 0; g < NG; ++g)
                acc[g] = __builtin_amdgcn_mfma_f32_4x4x1f32(cur[r8][g], rv[r8], acc[g], 0, 0, 0);
#pragma unroll
        for (int r8 = 0; r8 < kRowPad; ++r8) cur[r8] = nxt[r8];
    }
}

// Conjugate-pair groups (half-spectrum dictionary of a DFT basis with real
// measurements): real atom 2g is the real part of bin g, atom 2g + 1 its
// imaginary part; the bins 0 and, for even Nb, Nb / 2 are real (singleton
// groups, whose odd atom is never selected).
__device__ __forceinline__ bool grp_singleton(int g, int Nb) { return g == 0 || ((Nb & 1) == 0 && g == Nb / 2); }

// |x_g|^2 of the group led by entry k of the list c (values s): a pair's
// atoms are next to each other, 2g then 2g + 1.  Every lane must get the
// same bits for the same group, so the products and the sum are rounded
// explicitly (no contraction that could differ between inlined copies).
// NaN-safe as rank_key.
__device__ __forceinline__ float grp_key(const float* s, const int* c, int k, int n) {
    const bool pair = k + 1 < n && c[k + 1] == c[k] + 1;
    const float a0 = __fmul_rn(s[k], s[k]);
    const float a = pair ? __fadd_rn(a0, __fmul_rn(s[k + 1], s[k + 1])) : a0;
    return a <= 3.402823466e38f ? a : -1.f;
}

// Step 3 over groups: of the groups in c (the n atoms c[0..n), pairs next
// to each other), the K with largest |x_g| (ties to the lower group), their
// atoms written to q and vals to qv in rank order.  Returns the number of
// kept atoms of the lane's pixel.  Called by every lane; no barrier inside.
template <int U>
__device__ __forceinline__ int rank_top_groups(bool on, int t, int n, int K, const float* s, const int* c,
                                               const float* vals, int* q, float* qv) {
    float vk[U];
    int ck[U], rk[U], pk[U], sz[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int k = t + 16 * u;
        const bool lead = on && k < n && (c[k] & 1) == 0;
        const bool pair = lead && k + 1 < n && c[k + 1] == c[k] + 1;
        vk[u] = lead ? grp_key(s, c, k, n) : 0.f;
        ck[u] = lead ? c[k] : 0;
        sz[u] = lead ? (pair ? 2 : 1) : 0;
        rk[u] = 0;
        pk[u] = 0;
    }
    if (on) {
        for (int i = 0; i < n; ++i) {
            const int ci = c[i];
            if (ci & 1) continue;
            const float key = grp_key(s, c, i, n);
            const int size = (i + 1 < n && c[i + 1] == ci + 1) ? 2 : 1;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool before = key > vk[u] || (key == vk[u] && ci < ck[u]);
                rk[u] += before ? 1 : 0;
                pk[u] += before ? size : 0;
            }
        }
    }
    float kept = 0.f;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int k = t + 16 * u;
        if (sz[u] > 0 && rk[u] < K) {
            q[pk[u]] = ck[u];
            qv[pk[u]] = vals[k];
            if (sz[u] == 2) {
                q[pk[u] + 1] = ck[u] + 1;
                qv[pk[u] + 1] = vals[k + 1];
            }
            kept += (float)sz[u];
        }
    }
    return (int)pix_sum(kept);
}

// Step 3 over groups for the pixels with `on`: keep the K groups of c with
// largest |x_g|, then s_q = G[q,q]^{-1} b_q on their atoms (pixels padded
// to the wave's longest list).  Returns the pixel's kept atoms.
__device__ __forceinline__ int prune_to_q_grp(bool on, int t, int nc, int K, int N, const float* __restrict__ G32,
                                              const PixLds L) {
    const int nw = wave_max(on ? nc : 0);
    int nq;
    if (nw <= 32)
        nq = rank_top_groups<2>(on, t, nc, K, L.s, L.c, L.b, L.q, L.bq);
    else if (nw <= 48)
        nq = rank_top_groups<3>(on, t, nc, K, L.s, L.c, L.b, L.q, L.bq);
    else if (nw <= 64)
        nq = rank_top_groups<4>(on, t, nc, K, L.s, L.c, L.b, L.q, L.bq);
    else
        nq = rank_top_groups<kCU>(on, t, nc, K, L.s, L.c, L.b, L.q, L.bq);
    wave_sync();
    const int nmax = wave_max(on ? nq : 0);
    solve_list<true>(on, t, nq, nmax, N, G32, L.q, L.bq, L.sq, L.Wq);
    return nq;
}

// r = y - sum_k xv[k] A[:, xi[k]] for the lane's m = 4t + j + 64i.
template <int MSLOT>
__device__ __forceinline__ void residual(const float* y, float* rnew, const int* xi, const float* xv, int nx,
                                         const float* __restrict__ AT, int MP, int N, int t) {
#pragma unroll
    for (int u = 0; u < MSLOT; ++u) rnew[u] = y[u];
    for (int k0 = 0; k0 < nx; k0 += 4) {
        float4 av[4][MSLOT / 4];
        float v[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            const int k = k0 + kk;
            v[kk] = k < nx ? xv[k] : 0.f;
            const float* row = AT + (size_t)clamp_atom(k < nx ? xi[k] : 0, N) * MP;
#pragma unroll
            for (int u4 = 0; u4 < MSLOT / 4; ++u4) {
                const int m = 4 * t + 64 * u4;
                av[kk][u4] = (m < MP) ? *reinterpret_cast<const float4*>(row + m) : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
            for (int u4 = 0; u4 < MSLOT / 4; ++u4) {
                rnew[4 * u4] -= av[kk][u4].x * v[kk];
                rnew[4 * u4 + 1] -= av[kk][u4].y * v[kk];
                rnew[4 * u4 + 2] -= av[kk][u4].z * v[kk];
                rnew[4 * u4 + 3] -= av[kk][u4].w * v[kk];
            }
    }
}

template <int MSLOT, int NG, bool GRP, bool BIG = false>
__device__ __forceinline__ void gomp_coop_body(const CoopArgs& a, int64_t block, float* lds) {
    const int lane = threadIdx.x;
    const int x = lane & 3, t = lane >> 2;
    const int64_t local = block * kGroups + x;
    const int64_t pix = a.p0 + local;
    const bool valid = local < a.P;
    const int M = a.M, N = a.N, K = a.K, MP = a.MP, NP = a.NP;
    PixLds L = carve(lds + x * a.lds_floats, a);

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
    badi |= __shfl_xor(badi, 4);
    badi |= __shfl_xor(badi, 8);
    badi |= __shfl_xor(badi, 16);
    badi |= __shfl_xor(badi, 32);
    bad = badi != 0;
    float y2 = 0.f;
#pragma unroll
    for (int u = 0; u < MSLOT; ++u) {
        if (bad) y[u] = 0.f;
        r[u] = y[u];
        y2 += y[u] * y[u];
    }
    y2 = pix_sum(y2);
    const float ynorm = sqrtf(y2);

    bool active = valid && !bad;
    bool converged = false, fallback = false;
    float trG = 0.f, trW = 0.f;   // trace(G[c,c]) and trace(G[c,c]^{-1}) (FP64 fallback test)
    int iters = 0, nc = 0, nx = 0;
    int ng = 0;           // groups in c (GRP: a pair is one group of two atoms)
    bool x_on_q = false;
    float last_d2 = __builtin_nanf(""), rn2 = y2;
    uint32_t mask = 0u;   // bit k: atom 4 NG t + k is in c
    const int M8 = (M + kRowPad - 1) / kRowPad * kRowPad;
    for (int k = t; k < a.CM; k += 16) L.kp[k] = 0;
    v4f_t acc[NG];
    bool same_r = false;   // every active pixel of the wave kept r last iteration: p = A^T r is unchanged

    for (int it = 1; it <= a.Imax; ++it) {
        // ---------------- step 1: p = A^T r on MFMA, top-S over the non-members
        if (!same_r) {
#pragma unroll
            for (int u = 0; u < MSLOT; ++u) {
                const int m = 4 * t + (u & 3) + 64 * (u >> 2);
                if (m < MP) L.rb[m] = r[u];
            }
            wave_sync();
            correlate<NG>(a, L.rb, lane, M8, a.prec, acc);
        }
        // S rounds of argmax; the winners are appended in selection order.
        // Lane t holds atoms 4 NG t + NG i + g (entry i of accumulator g).
        int nsel = 0;
        if (!GRP) {
            for (int q = 0; q < a.S; ++q) {
                float bv = -1.f;
                int bi = -1;
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int g = 0; g < NG; ++g) {
                        const int k = NG * i + g;
                        const int n = 4 * NG * t + k;
                        const float v = fabsf(acc[g][i]);
                        const bool member = (mask >> k) & 1u;
                        if (n < N && !member && (bi < 0 || v > bv)) {
                            bv = v;
                            bi = n;
                        }
                    }
                pix_argmax(bv, bi);
                if (bi >= 0 && bi / (4 * NG) == t) mask |= 1u << (bi % (4 * NG));
                if (t == 0) L.sel[q] = bi;
                nsel += (bi >= 0) ? 1 : 0;   // the valid selections form a prefix
            }
        } else {
            // groups: the score of bin g is |p_g| = |(A^* r)_g|, from its two
            // real correlations: (1/2) sqrt(p_2g^2 + p_2g+1^2) for a pair (its
            // atoms carry 2 Re a_g and -2 Im a_g), |p_2g| for a real bin
            for (int q = 0; q < a.S; ++q) {
                float bv = -1.f;
                int bi = -1;
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int g = 0; g < NG; g += 2) {
                        const int k = NG * i + g;
                        const int n = 4 * NG * t + k;
                        const int gb = n >> 1;
                        const float p0 = acc[g][i], p1 = acc[g + 1][i];
                        const float v = grp_singleton(gb, a.Nb) ? fabsf(p0) : 0.5f * sqrtf(p0 * p0 + p1 * p1);
                        const bool member = (mask >> k) & 1u;
                        if (n < N && !member && (bi < 0 || v > bv)) {
                            bv = v;
                            bi = gb;
                        }
                    }
                pix_argmax(bv, bi);
                if (bi >= 0 && (2 * bi) / (4 * NG) == t) mask |= 3u << ((2 * bi) % (4 * NG));
                if (bi >= 0) {
                    const bool single = grp_singleton(bi, a.Nb);
                    if (t == 0) {
                        L.sel[nsel] = 2 * bi;
                        if (!single) L.sel[nsel + 1] = 2 * bi + 1;
                    }
                    nsel += single ? 1 : 2;
                    ng += active ? 1 : 0;
                }
            }
        }
        wave_sync();

        // ---------------- step 2: append the atoms, s = W^T (W b_c)
        // gather G[c + earlier selections, j] into the slot of row nc + q and
        // form b_j = a_j^T y, all loads of the iteration in one batch
        const int nq = active ? nsel : 0;
        const int SA = GRP ? 2 * a.S : a.S;   // atoms appended per iteration at most (uniform)
        for (int q = 0; q < SA; ++q) {
            const int j = q < nq ? L.sel[q] : -1;
            float bpart = 0.f;
            if (j >= 0) {
                const int n = nc + q;
                float v[kCU];
#pragma unroll
                for (int u = 0; u < kCU; ++u) {
                    const int i = t + 16 * u;
                    v[u] = 0.f;
                    if (i <= n) {
                        const int ci = i < nc ? L.c[i] : (i < n ? L.sel[i - nc] : j);
                        v[u] = a.G32[(size_t)clamp_atom(ci, N) * N + j];
                    }
                }
                float4 av[MSLOT / 4];
#pragma unroll
                for (int u4 = 0; u4 < MSLOT / 4; ++u4) {
                    const int m = 4 * t + 64 * u4;
                    av[u4] = (m < MP) ? *reinterpret_cast<const float4*>(a.AT + (size_t)j * MP + m)
                                      : make_float4(0.f, 0.f, 0.f, 0.f);
                }
#pragma unroll
                for (int u = 0; u < kCU; ++u) {
                    const int i = t + 16 * u;
                    if (i <= n) L.W[tri(n) + i] = v[u];
                }
#pragma unroll
                for (int u4 = 0; u4 < MSLOT / 4; ++u4)
                    bpart += av[u4].x * y[4 * u4] + av[u4].y * y[4 * u4 + 1] + av[u4].z * y[4 * u4 + 2] +
                             av[u4].w * y[4 * u4 + 3];
            }
            const float bj = pix_sum(bpart);
            if (t == 0) L.bsel[q] = bj;
        }
        wave_sync();
        // appended two at a time (one pass over W per pair); L.s is free
        // until the solve below and holds the second atom's l
        for (int q = 0; q < SA; q += 2) {
            const bool on0 = q < nq, on1 = q + 1 < nq;
            const int j0 = on0 ? L.sel[q] : 0, j1 = on1 ? L.sel[q + 1] : 0;
            const float b0 = on0 ? L.bsel[q] : 0.f, b1 = on1 ? L.bsel[q + 1] : 0.f;
            float ratio0, ratio1, g00, g11, sq0 = 0.f, sq1 = 0.f;
            const bool want = a.pivot_thr > 0.0;
            inv_append2(on0, on1, t, nc, L.W, L.z, L.b, L.c, L.l, L.s, j0, j1, b0, b1, want, ratio0, ratio1, g00,
                        g11, sq0, sq1);
            // a small pivot, or an FP32 error estimate of the normal
            // equations on c above the FP32 result tolerance redo_tol:
            // 2^-24 kappa(G[c,c]), kappa estimated as trace(G[c,c])
            // trace(G[c,c]^{-1}) / |c| (between the lower bound, that over
            // |c|^2, and the upper bound, the product itself).  Pruned
            // supports q are subsets of c, and the estimate of c bounds
            // theirs.
            if (on0 && want) {
                trG += g00;
                trW += sq0;
                if ((double)ratio0 < a.pivot_thr || trG * trW * 5.9604645e-8f > a.redo_tol * (float)(nc + 1))
                    fallback = true;
            }
            if (on0) ++nc;
            if (on1 && want) {
                trG += g11;
                trW += sq1;
                if ((double)ratio1 < a.pivot_thr || trG * trW * 5.9604645e-8f > a.redo_tol * (float)(nc + 1))
                    fallback = true;
            }
            if (on1) ++nc;
        }
        inv_solve(active, t, nc, L.W, L.z, L.s);

        // ---------------- step 3: prune to K and re-solve on q
        if (!GRP) ng = nc;
        const bool prune_g = active && a.prune == CSREC_PRUNE_EACH && ng > K;
        int nqa = K;
        bool q_same = false;   // q (and so x and r) as after the last prune
        if (__any(prune_g)) {
            if (GRP)
                nqa = prune_to_q_grp(prune_g, t, nc, K, N, a.G32, L);
            else {
                // called by every lane (it synchronises the wave); not short-circuited
                const bool changed = prune_to_q<BIG>(prune_g, t, nc, a.CM, K, N, a.G32, L);
                q_same = prune_g && !changed;
            }
        }
        // a pixel that stopped earlier keeps the x of its last iteration
        if (prune_g) {
            nx = nqa;
            x_on_q = true;
        } else if (active) {
            nx = nc;
            x_on_q = false;
        }

        // ---------------- step 4: residual r = y - A x, Delta, stop
        // (when every active pixel of the wave kept its q, r is unchanged:
        // Delta = 0, the norm as before)
        const bool keep_r = __all(!active || q_same);
        same_r = keep_r;
        if (active) {
            float d2 = 0.f, n2 = rn2;
            if (!keep_r) {
                float rnew[MSLOT];
                residual<MSLOT>(y, rnew, x_on_q ? L.q : L.c, x_on_q ? L.sq : L.s, nx, a.AT, MP, N, t);
                n2 = 0.f;
#pragma unroll
                for (int u = 0; u < MSLOT; ++u) {
                    const float dlt = rnew[u] - r[u];
                    d2 += dlt * dlt;
                    n2 += rnew[u] * rnew[u];
                    r[u] = rnew[u];
                }
                d2 = pix_sum(d2);
                n2 = pix_sum(n2);
            }
            iters = it;
            last_d2 = d2;
            rn2 = n2;
            if (sqrtf(n2) <= a.res_tol * ynorm || (a.eps > 0.f && sqrtf(d2) < a.eps)) {
                active = false;
                converged = true;
            }
        }
        wave_sync();
        if (!__any(active)) break;
    }

    // ---------------- prune placed after the loop (textbook gOMP)
    if (!GRP) ng = nc;
    const bool final_prune = a.prune == CSREC_PRUNE_FINAL && ng > K && valid && !bad;
    if (__any(final_prune)) {
        int nqa = K;
        if (GRP)
            nqa = prune_to_q_grp(final_prune, t, nc, K, N, a.G32, L);
        else
            prune_to_q<BIG>(final_prune, t, nc, a.CM, K, N, a.G32, L);
        float n2 = 0.f;
        if (final_prune) {
            nx = nqa;
            x_on_q = true;
            float rnew[MSLOT];
            residual<MSLOT>(y, rnew, L.q, L.sq, nx, a.AT, MP, N, t);
#pragma unroll
            for (int u = 0; u < MSLOT; ++u) n2 += rnew[u] * rnew[u];
        }
        n2 = pix_sum(n2);
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
    if (!GRP) {
        float* xrow = a.X + pix * N;
        for (int n = t; n < N; n += 16) {
            float v = 0.f;
            for (int k = 0; k < nx; ++k) v = (xi[k] == n) ? xv[k] : v;
            xrow[n] = bad ? 0.f : v;
        }
    } else {
        // the complex spectrum, interleaved (re, im): bin n of group
        // g = min(n, Nb - n) is (v_2g, +-v_2g+1), conjugated above Nb / 2
        const int Nb = a.Nb;
        float* xrow = a.X + pix * 2 * Nb;
        for (int n = t; n < Nb; n += 16) {
            const int g = (2 * n <= Nb) ? n : Nb - n;
            float re = 0.f, im = 0.f;
            for (int k = 0; k < nx; ++k) {
                re = (xi[k] == 2 * g) ? xv[k] : re;
                im = (xi[k] == 2 * g + 1) ? xv[k] : im;
            }
            if (2 * n > Nb) im = -im;
            xrow[2 * n] = bad ? 0.f : re;
            xrow[2 * n + 1] = bad ? 0.f : im;
        }
    }
    if (a.support) {
        // ascending order by rank of the index among the nx support atoms
        // (GRP: atom 2g is bin g, atom 2g + 1 bin Nb - g; KS = 2 K bins)
        const int KS = GRP ? 2 * K : K;
        int32_t* srow = a.support + pix * KS;
        for (int k = t; k < KS; k += 16)
            if (k >= nx || bad) srow[k] = -1;
        for (int k = t; k < nx && !bad; k += 16) {
            const int ck = GRP ? ((xi[k] & 1) ? a.Nb - (xi[k] >> 1) : (xi[k] >> 1)) : xi[k];
            int pos = 0;
            for (int i = 0; i < nx; ++i) {
                const int ci = GRP ? ((xi[i] & 1) ? a.Nb - (xi[i] >> 1) : (xi[i] >> 1)) : xi[i];
                pos += ci < ck ? 1 : 0;
            }
            if (pos < KS) srow[pos] = ck;
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

// ------------------------------------------------------------ CoSaMP and BIHT on chip
//
// The same wave / lane / LDS organisation as gOMP.  Per iteration, for each
// active pixel (Alg. 5, Alg. 4 and the one-bit variant):
//   1. p = A^T v on MFMA, with v = r (CoSaMP, BIHT) or v = y - sgn(A x)
//      (one-bit); u = p (CoSaMP) or u = x + mu p (BIHT, one-bit); the first
//      iteration's p = A^T y is kept in LDS as the least-squares right-hand
//      side of every atom.
//   2. Theta = the 2K (CoSaMP) or K (BIHT) largest |u|, ties to the lower
//      index, by rounds of a 16-lane argmax.
//   3. c = Theta U (previous kept support: CoSaMP all of it, BIHT its nonzero
//      entries); s = G[c,c]^{-1} (A^T y)_c (solve_list, list lengths padded
//      to the wave's largest); keep the K largest |s| with their values and
//      no second solve.  One-bit: x = u on Theta.
//   4. r = y - A x, Delta, stop (CoSaMP, BIHT); one-bit: v = y - sgn(A x).

struct OtherPlan {
    int rb, ball, c, b, s, scr, sel, selv, q, sq, total;
};

__host__ __device__ inline int other_nc(int kind, int K) {
    return kind == GREEDY_COSAMP ? 3 * K : (kind == GREEDY_BIHT ? 2 * K : 0);
}

__host__ __device__ inline OtherPlan other_plan(int kind, int MP, int N, int K) {
    const int nc = other_nc(kind, K);
    const int nsel = kind == GREEDY_COSAMP ? 2 * K : K;
    OtherPlan p;
    int o = 0;
    // the residual (read by the correlation only) shares its space with the
    // selections and the solve scratch, live only after the correlation
    p.rb = o;
    p.sel = o;
    p.selv = p.sel + up4(nsel);
    p.scr = p.selv + up4(nsel);
    const int tail = p.scr + (nc == 0 ? 0 : (nc > kGJ ? up4(tri(nc)) : 2 * (kGJ + 4)));
    o = up4(MP) > tail ? up4(MP) : tail;
    p.ball = o; o += nc > 0 ? up4(N) : 0;
    p.c = o; o += up4(nc);
    p.b = o; o += up4(nc);
    p.s = o; o += up4(nc);
    p.q = o; o += up4(K);
    p.sq = o; o += up4(K);
    o += ((8 - o) % 64 + 64) % 64;
    p.total = o;
    return p;
}

template <int KIND, int MSLOT, int NG, bool GRP>
__device__ __forceinline__ void other_body(const CoopArgs& a, int64_t block, float* lds) {
    constexpr int NV = 4 * NG;   // atoms per lane: 4 NG t + k, k < NV
    const int lane = threadIdx.x;
    const int x = lane & 3, t = lane >> 2;
    const int64_t local = block * kGroups + x;
    const int64_t pix = a.p0 + local;
    const bool valid = local < a.P;
    const int M = a.M, N = a.N, K = a.K, MP = a.MP;
    // GRP: conjugate-pair groups, K and the selections counted in groups of
    // up to two atoms, so every list holds twice as many atoms
    const OtherPlan pl = other_plan(KIND, MP, N, GRP ? 2 * K : K);
    float* base = lds + x * a.lds_floats;
    float* rb = base + pl.rb;
    float* ball = base + pl.ball;
    int* c = reinterpret_cast<int*>(base + pl.c);
    float* b = base + pl.b;
    float* sv = base + pl.s;
    float* scr = base + pl.scr;
    int* sel = reinterpret_cast<int*>(base + pl.sel);
    float* selv = base + pl.selv;
    int* q = reinterpret_cast<int*>(base + pl.q);
    float* sq = base + pl.sq;
    const int nsel = KIND == GREEDY_COSAMP ? 2 * K : K;

    // y (one-bit: the signs) and the vector v that is correlated
    float y[MSLOT], v[MSLOT];
    bool bad = false;
#pragma unroll
    for (int u = 0; u < MSLOT; ++u) {
        const int m = 4 * t + (u & 3) + 64 * (u >> 2);
        float w = 0.f;
        if (valid && m < M) {
            w = KIND == GREEDY_BIHT_ONE_BIT ? (float)a.Ysign[pix * M + m] : a.Y[pix * M + m];
            if (!isfinite(w)) bad = true;
        }
        y[u] = w;
    }
    int badi = bad ? 1 : 0;
    badi |= __shfl_xor(badi, 4);
    badi |= __shfl_xor(badi, 8);
    badi |= __shfl_xor(badi, 16);
    badi |= __shfl_xor(badi, 32);
    bad = badi != 0;
    float y2 = 0.f;
#pragma unroll
    for (int u = 0; u < MSLOT; ++u) {
        if (bad) y[u] = 0.f;
        v[u] = y[u];
        y2 += y[u] * y[u];
    }
    y2 = pix_sum(y2);
    const float ynorm = sqrtf(y2);

    bool active = valid && !bad;
    bool converged = false, limited = false;
    int iters = 0, nq = 0;
    float last_d2 = __builtin_nanf(""), rn2 = y2;
    const int M8 = (M + kRowPad - 1) / kRowPad * kRowPad;

    for (int it = 1; it <= a.Imax; ++it) {
        // ---------------- step 1: p = A^T v on MFMA, u
#pragma unroll
        for (int u = 0; u < MSLOT; ++u) {
            const int m = 4 * t + (u & 3) + 64 * (u >> 2);
            if (m < MP) rb[m] = v[u];
        }
        wave_sync();
        v4f_t acc[NG];
        // the first correlation of CoSaMP and BIHT is A^T y, the right-hand
        // sides of every least-squares solve: always in FP32
        correlate<NG>(a, rb, lane, M8, (it == 1 && KIND != GREEDY_BIHT_ONE_BIT) ? CSREC_PREC_F32 : a.prec, acc);
        float u[NV];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const float p = acc[g][i];
                // GRP: the complex correlation of a pair is half its two real
                // ones (atoms 2 Re a_g and -2 Im a_g), of a real bin the one
                const float w = (GRP && !grp_singleton((NV * t + NG * i + g) >> 1, a.Nb)) ? 0.5f : 1.f;
                u[NG * i + g] = KIND == GREEDY_COSAMP ? w * p : (a.mu * w) * p;
            }
        if (KIND != GREEDY_COSAMP && nq > 0) {
            // u = x + mu p: add the kept values to the lanes holding their atoms
            for (int kk = 0; kk < nq; ++kk) {
                const int j = q[kk] - NV * t;
                const float xv = sq[kk];
#pragma unroll
                for (int k = 0; k < NV; ++k) u[k] += (j == k) ? xv : 0.f;
            }
        }
        if (it == 1 && KIND != GREEDY_BIHT_ONE_BIT) {
            // r = y in the first iteration, so p = A^T y: the right-hand sides
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    const int n = NV * t + NG * i + g;
                    if (n < N) ball[n] = acc[g][i];
                }
        }
        // ---------------- step 2: the nsel largest |u| (no membership mask)
        uint32_t taken = 0u;
        int nsl = 0;
        if (GRP) {
            // over groups: |u_g| = sqrt(u_2g^2 + u_2g+1^2), the atoms of the
            // winners appended in selection order, pairs next to each other
            for (int qq = 0; qq < nsel; ++qq) {
                float bv = -1.f;
                int bi = -1;
#pragma unroll
                for (int k = 0; k < NV; k += 2) {
                    const int n = NV * t + k;
                    const float w = sqrtf(u[k] * u[k] + u[k + 1] * u[k + 1]);
                    if (n < N && !((taken >> k) & 1u) && (bi < 0 || w > bv)) {
                        bv = w;
                        bi = n >> 1;
                    }
                }
                pix_argmax(bv, bi);
                if (bi >= 0 && (2 * bi) / NV == t) taken |= 3u << (2 * bi - NV * t);
                if (bi >= 0) {
                    const bool single = grp_singleton(bi, a.Nb);
                    if (t == 0) {
                        sel[nsl] = 2 * bi;
                        if (!single) sel[nsl + 1] = 2 * bi + 1;
                    }
                    nsl += single ? 1 : 2;
                }
            }
        }
        for (int qq = 0; qq < (GRP ? 0 : nsel); ++qq) {
            float bv = -1.f;
            int bi = -1;
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                const int n = NV * t + k;
                const float w = fabsf(u[k]);
                if (n < N && !((taken >> k) & 1u) && (bi < 0 || w > bv)) {
                    bv = w;
                    bi = n;
                }
            }
            pix_argmax(bv, bi);
            if (bi >= 0 && bi / NV == t) {
                const int k0 = bi - NV * t;
                taken |= 1u << k0;
                float uv = 0.f;
#pragma unroll
                for (int k = 0; k < NV; ++k) uv = (k == k0) ? u[k] : uv;
                selv[qq] = uv;
            }
            if (t == 0) sel[qq] = bi;
            nsl += (bi >= 0) ? 1 : 0;
        }
        wave_sync();
        if (KIND == GREEDY_BIHT_ONE_BIT) {
            // x = H_K(u), then v = y - sgn(A x)
            if (active) {
                for (int k = t; k < nsl; k += 16) {
                    q[k] = sel[k];
                    sq[k] = selv[k];
                }
                nq = nsl;
            }
            wave_sync();
            if (active) {
                const float zero[MSLOT] = {};
                float ax[MSLOT];
                residual<MSLOT>(zero, ax, q, sq, nq, a.AT, MP, N, t);   // ax = -A x
                float d2 = 0.f, n2 = 0.f;
#pragma unroll
                for (int uu = 0; uu < MSLOT; ++uu) {
                    const int m = 4 * t + (uu & 3) + 64 * (uu >> 2);
                    const float sg = ax[uu] < 0.f ? 1.f : (ax[uu] > 0.f ? -1.f : 0.f);   // sgn(A x)
                    const float vn = m < M ? y[uu] - sg : 0.f;
                    const float dl = vn - v[uu];
                    d2 += dl * dl;
                    n2 += vn * vn;
                    v[uu] = vn;
                }
                d2 = pix_sum(d2);
                n2 = pix_sum(n2);
                iters = it;
                last_d2 = d2;
                rn2 = n2;
            }
            wave_sync();
            continue;
        }
        // ---------------- step 3: c = Theta U previous support; least squares; keep K
        int nc = 0;
        if (active) {
            for (int k = t; k < nsl; k += 16) c[k] = sel[k];
            // previous support entries not in Theta, appended in their order
            bool keep[4];
#pragma unroll
            for (int u2 = 0; u2 < 4; ++u2) {
                const int kk = t + 16 * u2;
                bool nz = kk < nq && sq[kk] != 0.f;
                if (GRP && kk < nq) {
                    // a group stays when either of its atoms is nonzero
                    const int pr = (q[kk] & 1) ? kk - 1 : kk + 1;
                    const bool partner = pr >= 0 && pr < nq && (q[pr] >> 1) == (q[kk] >> 1);
                    nz = nz || (partner && sq[pr] != 0.f);
                }
                bool kp = kk < nq && (KIND == GREEDY_COSAMP || nz);
                if (kp) {
                    const int j = q[kk];
                    for (int i = 0; i < nsl; ++i) kp = kp && (sel[i] != j);
                }
                keep[u2] = kp;
            }
            int total = 0;
#pragma unroll
            for (int u2 = 0; u2 < 4; ++u2) {
                const uint64_t bal = __ballot(keep[u2]);
                uint64_t mine = 0;   // this pixel's lanes (x, x + 4, ...), compacted to bit t
#pragma unroll
                for (int tt = 0; tt < 16; ++tt) mine |= ((bal >> (4 * tt + x)) & 1ull) << tt;
                const int below = __builtin_popcountll(mine & ((1ull << t) - 1ull));
                if (keep[u2]) c[nsl + total + below] = q[t + 16 * u2];
                total += __builtin_popcountll(mine);
            }
            nc = nsl + total;
        }
        wave_sync();
        if (active)
            for (int k = t; k < nc; k += 16) b[k] = ball[clamp_atom(c[k], N)];
        int nmax = nc;
        nmax = max(nmax, __shfl_xor(nmax, 1));
        nmax = max(nmax, __shfl_xor(nmax, 2));
        if (KIND == GREEDY_COSAMP) {
            // A pivot ratio below kFp32Limit leaves the FP32 solution of the
            // normal equations on c without a correct digit (its error bound
            // is about 2^-24 over the ratio): the pixel stops with its
            // previous iterate instead of pruning it (CSREC_FLAG_FP32_LIMIT).
            // It happens where FP32 cannot reach the residual stop and the
            // further iterations select rounding-level atoms into c.
            float rl = 1.f;
            if (nmax > kGJ && nmax <= 48)   // uniform over the wave
                solve_gj48<true, true>(active, t, nc, nmax, N, a.G32, c, b, sv, scr, &rl);
            else
                solve_list<true, true>(active, t, nc, nmax, N, a.G32, c, b, sv, scr, &rl);
            rl = fminf(rl, __shfl_xor(rl, 4));
            rl = fminf(rl, __shfl_xor(rl, 8));
            rl = fminf(rl, __shfl_xor(rl, 16));
            rl = fminf(rl, __shfl_xor(rl, 32));
            if (active && !(rl >= kFp32Limit)) {
                active = false;
                limited = true;
            }
        } else {
            solve_list<true>(active, t, nc, nmax, N, a.G32, c, b, sv, scr);
        }
        // as many 16-atom rank units as the longest list in the wave needs
        if (GRP) {
            int nk;
            if (nmax <= 32)
                nk = rank_top_groups<2>(active, t, nc, K, sv, c, sv, q, sq);
            else if (nmax <= 48)
                nk = rank_top_groups<3>(active, t, nc, K, sv, c, sv, q, sq);
            else if (nmax <= 64)
                nk = rank_top_groups<4>(active, t, nc, K, sv, c, sv, q, sq);
            else
                nk = rank_top_groups<kCU>(active, t, nc, K, sv, c, sv, q, sq);
            if (active) nq = nk;
        } else {
            if (nmax <= 32)
                rank_top<2>(active, t, nc, K, sv, c, sv, q, sq);
            else if (nmax <= 48)
                rank_top<3>(active, t, nc, K, sv, c, sv, q, sq);
            else if (nmax <= 64)
                rank_top<4>(active, t, nc, K, sv, c, sv, q, sq);
            else
                rank_top<kCU>(active, t, nc, K, sv, c, sv, q, sq);
            if (active) nq = nc < K ? nc : K;
        }
        wave_sync();

        // ---------------- step 4: residual r = y - A x, Delta, stop
        if (active) {
            float rnew[MSLOT];
            residual<MSLOT>(y, rnew, q, sq, nq, a.AT, MP, N, t);
            float d2 = 0.f, n2 = 0.f;
#pragma unroll
            for (int uu = 0; uu < MSLOT; ++uu) {
                const float dl = rnew[uu] - v[uu];
                d2 += dl * dl;
                n2 += rnew[uu] * rnew[uu];
                v[uu] = rnew[uu];
            }
            d2 = pix_sum(d2);
            n2 = pix_sum(n2);
            iters = it;
            last_d2 = d2;
            rn2 = n2;
            if (sqrtf(n2) <= a.res_tol * ynorm || (a.eps > 0.f && sqrtf(d2) < a.eps)) {
                active = false;
                converged = true;
            }
        }
        wave_sync();
        if (!__any(active)) break;
    }

    if (!valid) return;
    // ---------------- outputs: x (dense row; one-bit scaled to unit norm), support ascending, stats
    float scale = 1.f;
    if (KIND == GREEDY_BIHT_ONE_BIT) {
        float x2 = 0.f;
        for (int k = 0; k < nq; ++k) x2 += sq[k] * sq[k];
        scale = x2 > 0.f ? 1.f / sqrtf(x2) : 0.f;
    }
    if (GRP) {
        // the complex spectrum (re, im), as gOMP's; the support lists the
        // bins whose value is nonzero
        const int Nb = a.Nb;
        float* xrow = a.X + pix * 2 * Nb;
        for (int n = t; n < Nb; n += 16) {
            const int g = (2 * n <= Nb) ? n : Nb - n;
            float re = 0.f, im = 0.f;
            for (int k = 0; k < nq; ++k) {
                re = (q[k] == 2 * g) ? sq[k] : re;
                im = (q[k] == 2 * g + 1) ? sq[k] : im;
            }
            if (2 * n > Nb) im = -im;
            xrow[2 * n] = bad ? 0.f : re;
            xrow[2 * n + 1] = bad ? 0.f : im;
        }
        if (a.support) {
            int32_t* srow = a.support + pix * 2 * K;
            auto bin_of = [&](int j) { return (j & 1) ? Nb - (j >> 1) : (j >> 1); };
            // atom k stands for a nonzero bin when its group has a nonzero value
            auto live = [&](int k) {
                if (KIND == GREEDY_COSAMP) return true;
                const int pr = (q[k] & 1) ? k - 1 : k + 1;
                const bool partner = pr >= 0 && pr < nq && (q[pr] >> 1) == (q[k] >> 1);
                return sq[k] != 0.f || (partner && sq[pr] != 0.f);
            };
            int cnt = 0;
            for (int k = 0; k < nq; ++k) cnt += live(k) ? 1 : 0;
            for (int k = t; k < 2 * K; k += 16)
                if (k >= cnt || bad) srow[k] = -1;
            for (int k = t; k < nq && !bad; k += 16) {
                if (!live(k)) continue;
                const int ck = bin_of(q[k]);
                int pos = 0;
                for (int i = 0; i < nq; ++i) pos += (live(i) && bin_of(q[i]) < ck) ? 1 : 0;
                if (pos < 2 * K) srow[pos] = ck;
            }
        }
    } else {
    float* xrow = a.X + pix * N;
    for (int n = t; n < N; n += 16) {
        float w = 0.f;
        for (int k = 0; k < nq; ++k) w = (q[k] == n) ? sq[k] : w;
        xrow[n] = bad ? 0.f : w * scale;
    }
    if (a.support) {
        int32_t* srow = a.support + pix * K;
        // CoSaMP lists its kept atoms; BIHT the nonzero entries of x
        const bool all = KIND == GREEDY_COSAMP;
        int cnt = 0;
        for (int k = 0; k < nq; ++k) cnt += (all || sq[k] != 0.f) ? 1 : 0;
        for (int k = t; k < K; k += 16)
            if (k >= cnt || bad) srow[k] = -1;
        for (int k = t; k < nq && !bad; k += 16) {
            if (!(all || sq[k] != 0.f)) continue;
            const int ck = q[k];
            int pos = 0;
            for (int i = 0; i < nq; ++i) pos += ((all || sq[i] != 0.f) && q[i] < ck) ? 1 : 0;
            if (pos < K) srow[pos] = ck;
        }
    }
    }
    if (a.stats && t == 0) {
        csrec_pixel_stats st;
        st.iters = bad ? 0 : iters;
        st.flags = bad ? CSREC_FLAG_NONFINITE : (limited ? CSREC_FLAG_FP32_LIMIT : (converged ? CSREC_FLAG_CONVERGED : CSREC_FLAG_ITER_CAP));
        st.resid = bad ? 0.f : sqrtf(rn2);
        st.delta = sqrtf(last_d2);
        a.stats[pix] = st;
    }
}

template <int KIND, int MSLOT, int NG, bool GRP>
__global__ __launch_bounds__(64, 2) void other_coop_kernel(CoopArgs a) {
    extern __shared__ float lds[];
    other_body<KIND, MSLOT, NG, GRP>(a, blockIdx.x, lds);
}

template <int MSLOT, int NG, bool GRP, bool BIG = false>
__global__ __launch_bounds__(64, 2) void gomp_coop_kernel(CoopArgs a) {
    extern __shared__ float lds[];
    gomp_coop_body<MSLOT, NG, GRP, BIG>(a, blockIdx.x, lds);
}

struct CoopItem {
    CoopArgs a;
    int64_t block0;
};

// Grouped launch with persistent workgroups: the grid holds at most as many
// single-wave workgroups as the CUs keep resident, and each of them claims
// 4-pixel units in order from the cursor behind the item table (zeroed by
// the table's copy) until every unit of every item is taken; unit u belongs
// to the last item i with items[i].block0 <= u.  Units of the items of all
// tiles in the batch are claimed in admission order, so a wave that finishes
// a unit of early-stopping pixels takes the next unit at once.
template <int MSLOT, int NG>
__global__ __launch_bounds__(64, 2) void gomp_coop_persistent_kernel(const CoopItem* __restrict__ items, int nitems,
                                                                     int64_t units,
                                                                     unsigned long long* __restrict__ cursor) {
    extern __shared__ float lds[];
    while (true) {
        unsigned long long c = 0;
        if (threadIdx.x == 0) c = atomicAdd(cursor, 1ull);
        // lane 0's claim, made wave-uniform so that the item lookup and its
        // arguments live in scalar registers
        const int64_t u = (int64_t)(((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(c >> 32)) << 32) |
                                    (unsigned)__builtin_amdgcn_readfirstlane((int)(c & 0xffffffffull)));
        if (u >= units) break;
        int lo = 0, hi = nitems - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (items[mid].block0 <= u) lo = mid; else hi = mid - 1;
        }
        const CoopArgs a = items[lo].a;
        gomp_coop_body<MSLOT, NG, false>(a, u - items[lo].block0, lds);
        wave_sync();
    }
}

typedef void (*coop_kernel_t)(CoopArgs);
typedef void (*coop_grouped_t)(const CoopItem*, int, int64_t, unsigned long long*);

coop_kernel_t pick_coop(int MP, int NG, bool grp, bool big = false) {
    if (grp) {
        if (MP == 64) return NG == 2 ? gomp_coop_kernel<4, 2, true> : gomp_coop_kernel<4, 4, true>;
        return NG == 2 ? gomp_coop_kernel<8, 2, true> : gomp_coop_kernel<8, 4, true>;
    }
    if (big) {   // K from 33 to 48
        if (MP == 64) return NG == 2 ? gomp_coop_kernel<4, 2, false, true> : gomp_coop_kernel<4, 4, false, true>;
        return NG == 2 ? gomp_coop_kernel<8, 2, false, true> : gomp_coop_kernel<8, 4, false, true>;
    }
    if (MP == 64) return NG == 2 ? gomp_coop_kernel<4, 2, false> : gomp_coop_kernel<4, 4, false>;
    return NG == 2 ? gomp_coop_kernel<8, 2, false> : gomp_coop_kernel<8, 4, false>;
}

coop_grouped_t pick_coop_grouped(int MP, int NG) {
    if (MP == 64) return NG == 2 ? gomp_coop_persistent_kernel<4, 2> : gomp_coop_persistent_kernel<4, 4>;
    return NG == 2 ? gomp_coop_persistent_kernel<8, 2> : gomp_coop_persistent_kernel<8, 4>;
}

// The two dictionary copies: AT (N x MP, rows zero padded) and Ap (M8 x NP,
// zero rows and columns).  Block n < N writes row n of AT; block N + m
// (m < M8) writes row m of Ap.
// The dictionary copies: AT (N x MP, rows zero padded), Ap (M8 x NP, zero
// rows and columns) and Ap in BF16 and FP16 laid out (M8 / 4) x NP x 4
// (entry (m, n) at ((m / 4) NP + n) 4 + m % 4).  Block n < N writes row n of
// AT; block N + m (m < M8) writes row m of Ap and of the 16-bit copies.
__global__ void prepare_kernel(const float* __restrict__ A, int M, int N, int MP, int M8, int NP,
                               float* __restrict__ AT, float* __restrict__ Ap, __bf16* __restrict__ Abf,
                               _Float16* __restrict__ Ahf) {
    const int bidx = blockIdx.x;
    if (bidx < N) {
        for (int m = threadIdx.x; m < MP; m += blockDim.x)
            AT[(size_t)bidx * MP + m] = m < M ? A[(size_t)m * N + bidx] : 0.f;
    } else {
        const int m = bidx - N;
        for (int n = threadIdx.x; n < NP; n += blockDim.x) {
            const float v = (m < M && n < N) ? A[(size_t)m * N + n] : 0.f;
            Ap[(size_t)m * NP + n] = v;
            const size_t o = ((size_t)(m / 4) * NP + n) * 4 + (m % 4);
            Abf[o] = (__bf16)v;
            Ahf[o] = (_Float16)v;
        }
    }
}

int coop_ng(int N) { return N <= 128 ? 2 : 4; }
int coop_np(int N) { return 64 * coop_ng(N); }
int coop_m8(int M) { return (M + kRowPad - 1) / kRowPad * kRowPad; }

void fill_args(CoopArgs& a, const float* dictbuf, int M, int N, int K, int S, int Imax, int prune, float res_tol,
               float eps, double pivot_thr, float redo_tol, int prec) {
    a.M = M;
    a.N = N;
    a.MP = gomp_coop_mp(M);
    a.NP = coop_np(N);
    a.AT = dictbuf;
    a.Ap = dictbuf + (size_t)N * a.MP;
    const size_t n16 = (size_t)coop_m8(M) * a.NP;   // entries of each 16-bit copy
    a.Abf = reinterpret_cast<const __bf16*>(a.Ap + n16);
    a.Ahf = reinterpret_cast<const _Float16*>(a.Ap + n16 + n16 / 2);
    a.prec = prec;
    a.grp = 0;
    a.Nb = N;
    a.K = K;
    a.S = S;
    a.Imax = Imax;
    a.prune = prune;
    a.res_tol = res_tol;
    a.eps = eps;
    a.pivot_thr = pivot_thr;
    a.redo_tol = redo_tol;
    a.CM = S * Imax;
    a.lds_floats = (int)gomp_coop_lds_floats(a.MP, a.CM, K);
    a.mu = 0.f;
    a.Ysign = nullptr;
}

}  // namespace

int gomp_coop_mp(int M) { return M <= 64 ? 64 : 128; }

size_t gomp_coop_lds_floats(int MP, int CM, int K) { return (size_t)lds_plan(MP, CM, K).total; }

size_t gomp_coop_dict_floats(int M, int N) {
    // AT, Ap, and the BF16 and FP16 copies of Ap (half a float per entry each)
    return (size_t)N * gomp_coop_mp(M) + 2 * (size_t)coop_m8(M) * coop_np(N);
}

int gomp_coop_supported_grp(int M, int N, int K, int S, int Imax) {
    if (N > 64 * kMaxNG || M > 128 || S > kMaxS) return CSREC_E_UNSUPPORTED;
    const int CM = 2 * S * Imax;
    if (CM > 16 * kCU || 2 * K > 16 * kCU) return CSREC_E_UNSUPPORTED;
    const size_t lds = kGroups * gomp_coop_lds_floats(gomp_coop_mp(M), CM, 2 * K) * sizeof(float);
    return lds <= 160 * 1024 ? CSREC_OK : CSREC_E_UNSUPPORTED;
}

int gomp_coop_supported(int M, int N, int K, int S, int Imax) {
    if (N > 64 * kMaxNG || M > 128 || S > kMaxS) return CSREC_E_UNSUPPORTED;   // M8 <= MP holds for M <= 128
    const int CM = S * Imax;
    if (CM > 16 * kCU || K > 16 * kCU) return CSREC_E_UNSUPPORTED;
    const size_t lds = kGroups * gomp_coop_lds_floats(gomp_coop_mp(M), CM, K) * sizeof(float);
    return lds <= 160 * 1024 ? CSREC_OK : CSREC_E_UNSUPPORTED;
}

void gomp_coop_prepare(const float* A, int M, int N, float* dictbuf, hipStream_t stream) {
    const int MP = gomp_coop_mp(M), M8 = coop_m8(M), NP = coop_np(N);
    float* Ap = dictbuf + (size_t)N * MP;
    const size_t n16 = (size_t)M8 * NP;
    hipLaunchKernelGGL(prepare_kernel, dim3(N + M8), dim3(128), 0, stream, A, M, N, MP, M8, NP, dictbuf, Ap,
                       reinterpret_cast<__bf16*>(Ap + n16), reinterpret_cast<_Float16*>(Ap + n16 + n16 / 2));
}

// dictbuf (gomp_coop_dict_floats(M, N) floats, built by gomp_coop_prepare);
// fbflag (P entries) may be null.
int gomp_coop_launch(const float* Y, float* X, int32_t* support, csrec_pixel_stats* stats, const float* G32,
                     const float* dictbuf, uint32_t* fbflag, int M, int N, int64_t p0, int64_t P, int K, int S,
                     int Imax, int prune, float res_tol, float eps, double pivot_thr, float redo_tol, int prec, hipStream_t stream,
                     int Nb) {
    if (P == 0) return CSREC_OK;
    CoopArgs a;
    fill_args(a, dictbuf, M, N, K, S, Imax, prune, res_tol, eps, pivot_thr, redo_tol, prec);
    if (Nb > 0) {
        // conjugate-pair groups: up to 2 S atoms per iteration and 2 K kept
        a.grp = 1;
        a.Nb = Nb;
        a.CM = 2 * S * Imax;
        a.lds_floats = (int)gomp_coop_lds_floats(a.MP, a.CM, 2 * K);
    }
    a.Y = Y;
    a.G32 = G32;
    a.X = X;
    a.support = support;
    a.stats = stats;
    a.fbflag = fbflag;
    a.P = P;
    a.p0 = p0;
    const size_t lds = (size_t)kGroups * a.lds_floats * sizeof(float);
    const int64_t blocks = ceil_div(P, kGroups);
    const coop_kernel_t fn = pick_coop(a.MP, a.NP / 64, a.grp != 0, K > kGJ && K <= 48);
    CSREC_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)lds));
    hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(64), lds, stream, a);
    CSREC_HIP_TRY(hipGetLastError());
    return CSREC_OK;
}

typedef void (*other_kernel_t)(CoopArgs);

template <int KIND, bool GRP>
other_kernel_t pick_other_k(int MP, int NG) {
    if (MP == 64) return NG == 2 ? other_coop_kernel<KIND, 4, 2, GRP> : other_coop_kernel<KIND, 4, 4, GRP>;
    return NG == 2 ? other_coop_kernel<KIND, 8, 2, GRP> : other_coop_kernel<KIND, 8, 4, GRP>;
}

size_t coop_other_lds_floats(int kind, int M, int N, int K) {
    return (size_t)other_plan(kind, gomp_coop_mp(M), N, K).total;
}

int coop_other_supported_grp(int kind, int M, int N, int K) {
    // the lists hold the atoms of K groups (up to 2K), as an atom-level
    // solve with 2K would
    if (kind == GREEDY_BIHT_ONE_BIT) return CSREC_E_UNSUPPORTED;
    return coop_other_supported(kind, M, N, 2 * K);
}

int coop_other_supported(int kind, int M, int N, int K) {
    if (N > 64 * kMaxNG || M > 128) return CSREC_E_UNSUPPORTED;
    // the previous support is read by 4 units of 16 lanes (K <= 64); the
    // merged support is ranked by up to kCU units
    if (K > 64 || other_nc(kind, K) > 16 * kCU) return CSREC_E_UNSUPPORTED;
    const size_t lds = kGroups * coop_other_lds_floats(kind, M, N, K) * sizeof(float);
    return lds <= 160 * 1024 ? CSREC_OK : CSREC_E_UNSUPPORTED;
}

int coop_other_launch(int kind, const float* Y, const int8_t* Ysign, float* X, int32_t* support,
                      csrec_pixel_stats* stats, const float* G32, const float* dictbuf, int M, int N, int64_t p0,
                      int64_t P, int K, int Imax, float mu, float res_tol, float eps, int prec, hipStream_t stream,
                      int Nb) {
    if (P == 0) return CSREC_OK;
    CoopArgs a;
    fill_args(a, dictbuf, M, N, K, 1, Imax, 0, res_tol, eps, 0.0, 0.f, prec);
    a.lds_floats = (int)coop_other_lds_floats(kind, M, N, Nb > 0 ? 2 * K : K);
    if (Nb > 0) {
        a.grp = 1;
        a.Nb = Nb;
    }
    a.Y = Y;
    a.Ysign = Ysign;
    a.mu = mu;
    a.G32 = G32;
    a.X = X;
    a.support = support;
    a.stats = stats;
    a.fbflag = nullptr;
    a.P = P;
    a.p0 = p0;
    const size_t lds = (size_t)kGroups * a.lds_floats * sizeof(float);
    const int64_t blocks = ceil_div(P, kGroups);
    const int NG = a.NP / 64;
    other_kernel_t fn;
    if (a.grp)
        fn = kind == GREEDY_COSAMP ? pick_other_k<GREEDY_COSAMP, true>(a.MP, NG)
                                   : pick_other_k<GREEDY_BIHT, true>(a.MP, NG);
    else
        fn = kind == GREEDY_COSAMP ? pick_other_k<GREEDY_COSAMP, false>(a.MP, NG)
             : kind == GREEDY_BIHT ? pick_other_k<GREEDY_BIHT, false>(a.MP, NG)
                                   : pick_other_k<GREEDY_BIHT_ONE_BIT, false>(a.MP, NG);
    CSREC_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)lds));
    hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(64), lds, stream, a);
    CSREC_HIP_TRY(hipGetLastError());
    return CSREC_OK;
}

size_t gomp_coop_item_bytes() { return sizeof(CoopItem); }
size_t gomp_coop_table_extra() { return 64; }

// Items of one launch must share MP (64 or 128) and the atom grouping NG
// (gomp_coop_class tells them apart).
int gomp_coop_class(int M, int N) { return (gomp_coop_mp(M) == 64 ? 0 : 2) + (coop_ng(N) == 2 ? 0 : 1); }

namespace {
// Workgroups of `fn` that the device keeps resident at `lds` bytes each.
int64_t resident_groups(const void* fn, size_t lds) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64, lds) != hipSuccess) return 0;
    return (int64_t)cus * (per_cu > 0 ? per_cu : 1);
}
}  // namespace

// table_host / table_dev: nitems items and gomp_coop_table_extra() bytes
// behind them (the work cursor).
int gomp_coop_group_launch(const GompCoopItem* items, int nitems, void* table_host, void* table_dev, int K, int S,
                           int prune, float res_tol, float eps, double pivot_thr, float redo_tol, int prec,
                           hipStream_t stream) {
    if (nitems <= 0) return CSREC_OK;
    CoopItem* th = static_cast<CoopItem*>(table_host);
    int64_t blocks = 0;
    size_t lds = 0;
    const int cls = gomp_coop_class(items[0].M, items[0].N);
    for (int i = 0; i < nitems; ++i) {
        const GompCoopItem& it = items[i];
        if (gomp_coop_class(it.M, it.N) != cls) return CSREC_E_INVAL;
        CoopArgs& a = th[i].a;
        fill_args(a, it.dict, it.M, it.N, K, S, it.max_iter, prune, res_tol, eps, pivot_thr, redo_tol, prec);
        a.Y = it.Y;
        a.G32 = it.G32;
        a.X = it.X;
        a.support = it.support;
        a.stats = it.stats;
        a.fbflag = it.fbflag;
        a.P = it.np;
        a.p0 = it.p0;
        th[i].block0 = blocks;
        blocks += ceil_div(it.np, kGroups);
        const size_t need = (size_t)kGroups * a.lds_floats * sizeof(float);
        lds = need > lds ? need : lds;
    }
    const size_t tbytes = (size_t)nitems * sizeof(CoopItem);
    unsigned long long* cur_h = reinterpret_cast<unsigned long long*>(static_cast<char*>(table_host) + tbytes);
    *cur_h = 0ull;
    CSREC_HIP_TRY(hipMemcpyAsync(table_dev, th, tbytes + sizeof(unsigned long long), hipMemcpyHostToDevice,
                                 stream));
    const CoopItem* td = static_cast<const CoopItem*>(table_dev);
    unsigned long long* cur_d = reinterpret_cast<unsigned long long*>(static_cast<char*>(table_dev) + tbytes);
    const coop_grouped_t fn = pick_coop_grouped(th[0].a.MP, th[0].a.NP / 64);
    CSREC_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)lds));
    int64_t grid = resident_groups(reinterpret_cast<const void*>(fn), lds);
    if (grid <= 0 || grid > blocks) grid = blocks;
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(64), lds, stream, td, nitems, blocks, cur_d);
    CSREC_HIP_TRY(hipGetLastError());
    return CSREC_OK;
}

}  // namespace csrec
