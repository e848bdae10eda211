// GSVD step of arXiv 2504.03373 eq.4: SVD of A = K^{-1} R per frequency bin and the noise subspace
// E_n = [e_{Ns+1} .. e_M] of its left singular vectors (the definition following eq.4).
//
// Method: one-sided (Hestenes) Jacobi -- the paper's "category 1" solver of Sec. III-B -- with two
// Householder QR preconditioners (the paper's own building block, Sec. III-B category 2):
//   1. A P = Q R         Householder QR with column pivoting (largest remaining column first),
//                        stopped at the numerical rank rk (R: rk x M);
//   2. R^H = Q1 R1       Householder QR without pivoting (Q1 is never formed);
//   3. X = R1^H          one-sided Jacobi from the right, X V = W with orthogonal columns;
//   4. U = Q [W S^-1, 0; 0, I]   normalised columns, reflectors applied back.
// Since R = R1^H Q1^H = X Q1^H, R's left singular vectors are X's, i.e. W S^-1 (S = diag |w_i|),
// and A = Q R P^T gives U as above; sigma_i = |w_i|, the columns rk..M-1 of U are Q's and span the
// numerical null space.  The Jacobi iteration works on X^H X = R1 R1^H, the Gram matrix of a
// twice-triangularised pivoted factor, which is close to diagonal: about 6 sweeps on the
// 60-channel workload (about 17 on A itself), and no rotation has to be accumulated.
//
// Stopping at the noise subspace (sub_full >= 0, the p = 2 localization): eq.5 with p = 2 reads
// only E_n E_n^H.  After sub_full full sweeps the Ns columns of largest norm form the signal set S
// and only the pairs with a member in S are visited (the larger result kept in S) until such a
// sweep changes nothing; if then min_S |x|^2 exceeds the sum of |x|^2 over the other columns (a
// bound on their largest squared singular value), X_S spans the Ns dominant singular vectors and
// E_n is built as the orthogonal complement of X_S (Householder vectors of X_S) instead of from
// the rotations that would still run inside the noise cluster (or, for the signal-subspace form
// of eq.5, only X_S's vectors are formed).  The localization paths switch before any full sweep
// (sub_full = 0: the pivoted QR already grades X's column norms); on the 60-channel workload the
// projector has then converged after about 2.4 such sweeps, against about 6 full sweeps for the
// singular vectors; the noise vectors then are not singular vectors (sigma is not produced).
//
// Signal vectors only (eq.5 through the signal subspace; no E_n wanted): neither the second QR
// nor Q is used.  With A = Q R~ (R~ = R P^T), Z = R~^H has the singular values of A and its left
// singular vectors are A's right ones, so the (subspace) sweeps run on Z itself (M x rk: the
// pivoted QR grades its columns as it grades R's rows, about 3 subspace sweeps per bin on the
// 60-channel workload), and A W_S -- the input A, untouched, times the signal columns of W = Z V
// -- spans the Ns dominant left singular vectors of A, each direction scaled by its singular
// value (a power step: the other directions that the rotation tolerance leaves in W_S shrink
// relative to the signal).  The reflectors are then never parked, reloaded or applied.
//
// GPU mapping (gfx950):
//  * one workgroup per bin; one complex64 MP x MP column-major matrix in LDS (32 KB at MP = 64,
//    four bins per CU) holds A -> its QR -> R^H -> R1 -> X -> W -> U in turn (the two
//    transposes in place, each thread exchanging the pair of entries it owns);
//  * pivoted QR step k (one barrier): every group reads the pivot (a 64-bit LDS max over
//    norm/column keys posted by the previous step), forms the reflector itself, applies it to its
//    remaining columns and posts their new trailing norms; columns are never moved;
//  * parallel (round-robin) ordering: each sweep is rk'-1 rounds of rk'/2 disjoint column pairs
//    (rk' = rk rounded up to even), one pair per group of G lanes, each lane owning MP/G rows;
//  * alpha = |x_i|^2, beta = |x_j|^2 and gamma = x_i^H x_j are reduced across the G lanes with DPP
//    butterflies (every lane ends with the same bits, so the rotation decision is uniform in the
//    group);
//  * convergence test in FP64: rotate iff |gamma|^2 > tol^2 alpha beta with tol = 2 sqrt(M) 2^-24;
//    a sweep without any rotation ends the solve (a fixed point: a converged bin is never changed
//    again), and the columns of W S^-1 are then orthonormal to tol.  The inner products are
//    accumulated in FP32 (at most R = MP/G products per lane, then log2 G butterfly levels), so
//    their rounding error is below (R + log2 G) 2^-24 |x_i| |x_j|: 11 2^-24 for the default
//    8-lane variant at MP = 64, under the threshold 2 sqrt(M) 2^-24 (15.5 2^-24 at M = 60), and
//    below it at every M for the 8-lane variants; the test is not decided by rounding;
//  * the sweeps run on a permuted layout (swx) that spreads the reads of a round over the LDS
//    banks, switched in place before and after them;
//  * epilogue: sigma from the column norms, stable descending rank sort (ties: lower column
//    first), U = Q U_R with each group taking its columns through all reflectors in registers,
//    E_n = sorted columns Ns..M-1 of U, written column-major per bin.
#include "ssl_internal.h"

#include <atomic>

namespace {

template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Sum over aligned groups of G lanes (G = 4, 8 or 16); all lanes of a group get identical bits.
template <int G>
__device__ __forceinline__ float group_sum(float v)
{
    v += dpp<0xB1>(v);                    // quad_perm [1,0,3,2]
    v += dpp<0x4E>(v);                    // quad_perm [2,3,0,1]
    if (G >= 8) v += dpp<0x141>(v);       // row_half_mirror
    if (G >= 16) v += dpp<0x140>(v);      // row_mirror
    return v;
}

// The same in FP64 (cross-lane moves of both halves through __shfl_xor).
template <int G>
__device__ __forceinline__ double group_sum_f64(double v)
{
#pragma unroll
    for (int o = 1; o < G; o <<= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ bool finite2(float2 v) { return isfinite(v.x) && isfinite(v.y); }

// 1/sqrt(x) for normal x > 0: hardware estimate plus one Newton-Raphson step.
__device__ __forceinline__ float rsqrt_refined(float x)
{
    const float y = __builtin_amdgcn_rsqf(x);
    return y * fmaf(-0.5f * x * y, y, 1.5f);
}
__device__ __forceinline__ float2 conj2(float2 v) { return make_float2(v.x, -v.y); }

// Index of (row r, column c) in a bin's LDS matrix: column-major.
template <int MP>
__device__ __forceinline__ int at(int c, int r)
{
    return c * MP + r;
}

// Layout of the Jacobi sweeps: column c's 8-row (64-byte) chunks permuted by the low bits of c
// (row r stored at r XOR 8 (c mod MP/8)).  The lane groups of a round read the same rows of
// different columns; with a column stride of 512 bytes those reads would all fall on the same LDS
// banks, here they spread over all of them.  The permutation is an involution within each column
// (r <-> r XOR s), so the layout is switched in place by swapping those row pairs.
template <int MP>
__device__ __forceinline__ int swz_mask(int c)
{
    constexpr int mask = MP >= 16 ? MP / 8 - 1 : 0;
    return (c & mask) << 3;
}
template <int MP>
__device__ __forceinline__ int swx(int c, int r)
{
    return c * MP + (r ^ swz_mask<MP>(c));
}

template <int MP, int G>
struct JacobiCfg {
    static constexpr int R = MP / G;                       // rows per lane
    static constexpr int NG = MP / 2;                      // lane groups
    static constexpr int THREADS = ((NG * G + 63) / 64) * 64;
    // register budget of the persistent variant: at MP = 64 the LDS admits 4 bins per CU; aim
    // for 3 (16 lanes, <= 80 VGPRs) or 4 (8 lanes, <= 128) resident workgroups
    static constexpr int WAVES_PER_EU = (MP == 64) ? (G == 16 ? 6 : G == 8 ? 4 : 2) : 1;
};

// Applies the reflector H = I - tau v v^H to column c of X, rows k..M-1, by one lane group:
// v_k = vk, v_r = Vk[r] for r > k.  Rows >= M hold zeros in every column (so v_r = 0 there and
// those rows stay zero), rows < k are left as they are (v_r = 0; rewritten unchanged).  Returns
// the group-summed |x_r|^2 over rows > k of the result (the column's trailing norm for the next
// step).  A lane's rows are q + G j; the slots j < k / G lie above row k and are skipped, so the
// loop runs over the slots from k / G on, numbered from 0: only the first of them holds rows <= k
// and needs masks, and every access is an immediate offset from one base address per column.
template <int MP, int G>
__device__ __forceinline__ float apply_reflector(int pc, float2 vk, int k, float tau,
                                                 float2 *X, int c, int M, int q)
{
    constexpr int R = MP / G;
    (void)M;
    const int js = k / G, r0 = G * js + q;        // slot js holds row k; this lane's first row
    const float2 *vp = X + at<MP>(pc, r0);
    float2 *xp = X + at<MP>(c, r0);
    float wr = 0.f, wi = 0.f;
    float2 x[R], v[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        if (js + j >= R) {                        // uniform, and so for every later j
            if constexpr (R <= 8) break;          // (R = 16 stays unrolled only with continue)
            else continue;
        }
        const float2 raw = vp[G * j];
        if (j == 0) v[j] = (r0 > k) ? raw : ((r0 == k) ? vk : make_float2(0.f, 0.f));
        else v[j] = raw;                          // rows > k
        x[j] = xp[G * j];
        // conj(v) x
        wr = fmaf(v[j].x, x[j].x, fmaf(v[j].y, x[j].y, wr));
        wi = fmaf(v[j].x, x[j].y, fmaf(-v[j].y, x[j].x, wi));
    }
    wr = group_sum<G>(wr) * tau;
    wi = group_sum<G>(wi) * tau;
    float tn = 0.f;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        if (js + j >= R) {
            if constexpr (R <= 8) break;
            else continue;
        }
        // x -= v * (tau w)
        x[j].x = fmaf(-v[j].x, wr, fmaf(v[j].y, wi, x[j].x));
        x[j].y = fmaf(-v[j].x, wi, fmaf(-v[j].y, wr, x[j].y));
        xp[G * j] = x[j];
        const float n2 = fmaf(x[j].x, x[j].x, x[j].y * x[j].y);
        if (j == 0) tn += (r0 > k) ? n2 : 0.0f;
        else tn += n2;
    }
    return group_sum<G>(tn);
}

// The same reflector applied to two columns c0, c1 of X at once (one read of v, the two
// dependency chains interleaved); the results for c1 are stored only if two.  tn0, tn1: their
// trailing norms as in apply_reflector.
template <int MP, int G>
__device__ __forceinline__ void apply_reflector2(int pc, float2 vk, int k, float tau,
                                                 float2 *X, int c0, int c1, bool two, int q,
                                                 float &tn0, float &tn1)
{
    constexpr int R = MP / G;
    const int js = k / G, r0 = G * js + q;
    const float2 *vp = X + at<MP>(pc, r0);
    float2 *xp0 = X + at<MP>(c0, r0);
    float2 *xp1 = X + at<MP>(c1, r0);
    float wr0 = 0.f, wi0 = 0.f, wr1 = 0.f, wi1 = 0.f;
    float2 x0[R], x1[R], v[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        if (js + j >= R) {
            if constexpr (R <= 8) break;
            else continue;
        }
        const float2 raw = vp[G * j];
        if (j == 0) v[j] = (r0 > k) ? raw : ((r0 == k) ? vk : make_float2(0.f, 0.f));
        else v[j] = raw;
        x0[j] = xp0[G * j];
        x1[j] = xp1[G * j];
        wr0 = fmaf(v[j].x, x0[j].x, fmaf(v[j].y, x0[j].y, wr0));
        wi0 = fmaf(v[j].x, x0[j].y, fmaf(-v[j].y, x0[j].x, wi0));
        wr1 = fmaf(v[j].x, x1[j].x, fmaf(v[j].y, x1[j].y, wr1));
        wi1 = fmaf(v[j].x, x1[j].y, fmaf(-v[j].y, x1[j].x, wi1));
    }
    wr0 = group_sum<G>(wr0) * tau;
    wi0 = group_sum<G>(wi0) * tau;
    wr1 = group_sum<G>(wr1) * tau;
    wi1 = group_sum<G>(wi1) * tau;
    float s0 = 0.f, s1 = 0.f;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        if (js + j >= R) {
            if constexpr (R <= 8) break;
            else continue;
        }
        x0[j].x = fmaf(-v[j].x, wr0, fmaf(v[j].y, wi0, x0[j].x));
        x0[j].y = fmaf(-v[j].x, wi0, fmaf(-v[j].y, wr0, x0[j].y));
        x1[j].x = fmaf(-v[j].x, wr1, fmaf(v[j].y, wi1, x1[j].x));
        x1[j].y = fmaf(-v[j].x, wi1, fmaf(-v[j].y, wr1, x1[j].y));
        xp0[G * j] = x0[j];
        if (two) xp1[G * j] = x1[j];
        const float n0 = fmaf(x0[j].x, x0[j].x, x0[j].y * x0[j].y);
        const float n1 = fmaf(x1[j].x, x1[j].x, x1[j].y * x1[j].y);
        if (j == 0) {
            s0 += (r0 > k) ? n0 : 0.0f;
            s1 += (r0 > k) ? n1 : 0.0f;
        } else {
            s0 += n0;
            s1 += n1;
        }
    }
    tn0 = group_sum<G>(s0);
    tn1 = group_sum<G>(s1);
}

// Pivot key: larger squared norm first, then the lower column index (norms are >= 0, so the
// float bits order like the values).
__device__ __forceinline__ unsigned long long pivot_key(float nrm2, int c)
{
    return ((unsigned long long)__float_as_uint(nrm2) << 32) | (unsigned int)(0x7fffffff - c);
}

// One pair visit of a Jacobi sweep on columns ci < cj (sweep layout): NR row slots q + G k per
// lane, enough to cover the numerical rank (rows >= rk are zero), all loaded before the first
// product.  alpha = |x_i|^2, beta = |x_j|^2 and gamma = x_i^H x_j are reduced across the G lanes
// with DPP butterflies (every lane ends with the same bits, so the decision is uniform in the
// group); the pair is rotated iff |gamma|^2 > tol^2 alpha beta, tested in FP64.  Returns whether
// it was rotated.
template <int MP, int G, int NR>
__device__ __forceinline__ bool jacobi_pair(float2 *Bs, int ci, int cj, int q, double tol2)
{
    float2 bi[NR], bj[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const int r = q + G * k;
        bi[k] = Bs[swx<MP>(ci, r)];
        bj[k] = Bs[swx<MP>(cj, r)];
    }
    __builtin_amdgcn_sched_barrier(0);            // every read in flight before the products
    float al = 0.f, be = 0.f, gr = 0.f, gi = 0.f;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        al = fmaf(bi[k].x, bi[k].x, fmaf(bi[k].y, bi[k].y, al));
        be = fmaf(bj[k].x, bj[k].x, fmaf(bj[k].y, bj[k].y, be));
        gr = fmaf(bi[k].x, bj[k].x, fmaf(bi[k].y, bj[k].y, gr));
        gi = fmaf(bi[k].x, bj[k].y, fmaf(-bi[k].y, bj[k].x, gi));
    }
    al = group_sum<G>(al);
    be = group_sum<G>(be);
    gr = group_sum<G>(gr);
    gi = group_sum<G>(gi);
    const double g2 = (double)gr * gr + (double)gi * gi;
    const double ab = (double)al * be;
    if (!(g2 > tol2 * ab && ab > 0.0)) return false;
    // 2x2 Hermitian Gram [[al, gamma], [conj gamma, be]]: the real Jacobi angle after removing the
    // phase of gamma, in FP32: t = tan from the smaller root of t^2 + 2 zeta t - 1 = 0, c =
    // 1/sqrt(1 + t^2) refined by one Newton step, s = c t.  c and s come from the same t, so the
    // rotation is unitary to rounding whatever t's last-bit error (hardware sqrt and reciprocal).
    // 1/|gamma| from |gamma|^2 when that is a normal FP32 number; otherwise (columns of a
    // numerically rank-deficient bin) without squaring.  gamma != 0 here.
    const float g2f = (float)g2;
    float rg;
    if (g2f >= 1e-36f) {
        rg = __builtin_amdgcn_rsqf(g2f);
    } else {
        const float ax = fabsf(gr), ay = fabsf(gi);
        const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
        const float rt = mn * __builtin_amdgcn_rcpf(mx);
        rg = __builtin_amdgcn_rcpf(mx * __builtin_amdgcn_sqrtf(fmaf(rt, rt, 1.0f)));
    }
    const float zeta = (be - al) * 0.5f * rg;
    // |zeta| > 1e18 would need |x_i|^2 / |x_j|^2 > 1e24 for the pair to be rotated at all; the
    // clamp only keeps zeta^2 finite
    const float az = fminf(fabsf(zeta), 1e18f);
    float t = __builtin_amdgcn_rcpf(az + __builtin_amdgcn_sqrtf(fmaf(az, az, 1.0f)));
    t = copysignf(t, zeta);
    const float c = rsqrt_refined(fmaf(t, t, 1.0f));
    const float s = c * t;
    // w = s e^{-i arg gamma}:  x_i' = c x_i - w x_j,  x_j' = conj(w) x_i + c x_j
    const float wr = s * gr * rg;
    const float wi = -s * gi * rg;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const int r = q + G * k;
        float2 x = bi[k], y = bj[k];
        float2 ni, nj;
        ni.x = fmaf(c, x.x, -fmaf(wr, y.x, -wi * y.y));
        ni.y = fmaf(c, x.y, -fmaf(wr, y.y, wi * y.x));
        nj.x = fmaf(c, y.x, fmaf(wr, x.x, wi * x.y));
        nj.y = fmaf(c, y.y, fmaf(wr, x.y, -wi * x.x));
        Bs[swx<MP>(ci, r)] = ni;
        Bs[swx<MP>(cj, r)] = nj;
    }
    return true;
}

// Subspace phase limits: signal sets of at most kSubMaxNs columns (their complement's reflectors
// take three LDS arrays that are free by then), at most kSubMaxSweeps sweeps over their pairs
// before the solve returns to full sweeps.
constexpr int kSubMaxNs = 3;
constexpr int kSubMaxSweeps = 6;

// |x_c|^2 of the columns c < rk (sweep layout) into nrm[c], one lane group per column.
template <int MP, int G>
__device__ __forceinline__ void sub_norms(const float2 *Bs, int rk, int g, int q, float *nrm)
{
    constexpr int R = MP / G, NG = MP / 2;
    for (int c = g; c < rk && g < NG; c += NG) {
        float s = 0.f;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const float2 v = Bs[swx<MP>(c, q + G * k)];
            s = fmaf(v.x, v.x, fmaf(v.y, v.y, s));
        }
        s = group_sum<G>(s);
        if (q == 0) nrm[c] = s;
    }
}

// Whether a subspace-phase sweep would change nothing: every pair with a member in S tested at
// once (no rotation in between, so a sweep over them in any order would see the same columns),
// a lane group per pair.  A signal / noise pair fails if it would be rotated (the jacobi_pair
// test, same sums: rows >= rk are zero) or exchanged (noise column longer); a signal / signal
// pair if it would be rotated.  slist = S's columns, nlist = the others (< rk).  Uniform result.
template <int MP, int G>
__device__ __forceinline__ bool sub_settled(const float2 *Bs, const int *slist, const int *nlist,
                                            int Ns, int rk, int g, int q, double tol2)
{
    constexpr int R = MP / G, NG = MP / 2;
    const int nn = rk - Ns, ncross = Ns * nn, npairs = ncross + Ns * (Ns - 1) / 2;
    int bad = 0;
    for (int p = g; p < npairs && g < NG; p += NG) {
        int ci, cj;
        if (p < ncross) {
            ci = slist[p / nn];
            cj = nlist[p % nn];
        } else {                                     // (a, b), a < b < Ns, enumerated by b
            int t = p - ncross, b = 1;
            while (t >= b) {
                t -= b;
                ++b;
            }
            ci = slist[t];
            cj = slist[b];
        }
        float al = 0.f, be = 0.f, gr = 0.f, gi = 0.f;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int r = q + G * k;
            const float2 x = Bs[swx<MP>(ci, r)], y = Bs[swx<MP>(cj, r)];
            al = fmaf(x.x, x.x, fmaf(x.y, x.y, al));
            be = fmaf(y.x, y.x, fmaf(y.y, y.y, be));
            gr = fmaf(x.x, y.x, fmaf(x.y, y.y, gr));
            gi = fmaf(x.x, y.y, fmaf(-x.y, y.x, gi));
        }
        al = group_sum<G>(al);
        be = group_sum<G>(be);
        gr = group_sum<G>(gr);
        gi = group_sum<G>(gi);
        const double g2 = (double)gr * gr + (double)gi * gi;
        const double ab = (double)al * be;
        if ((g2 > tol2 * ab && ab > 0.0) || (p < ncross && be > al)) bad = 1;
    }
    return __syncthreads_count(bad) == 0;
}

// A pair visit of the subspace phase: column cs of the signal set S, column cn outside it.  The
// pair is rotated as in jacobi_pair, and the result of larger norm is kept in the signal slot:
// the minimal rotation keeps the order of the two norms (|x_s'|^2 = alpha - t |gamma|,
// |x_n'|^2 = beta + t |gamma|, t of the sign of beta - alpha), so the two results trade places
// iff beta > alpha; an orthogonal pair with beta > alpha is exchanged.  |X_S|_F^2 never
// decreases.  Returns whether the columns changed.
template <int MP, int G, int NR>
__device__ __forceinline__ bool jacobi_pair_sorted(float2 *Bs, int cs, int cn, int q, double tol2)
{
    float2 bi[NR], bj[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const int r = q + G * k;
        bi[k] = Bs[swx<MP>(cs, r)];
        bj[k] = Bs[swx<MP>(cn, r)];
    }
    __builtin_amdgcn_sched_barrier(0);
    float al = 0.f, be = 0.f, gr = 0.f, gi = 0.f;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        al = fmaf(bi[k].x, bi[k].x, fmaf(bi[k].y, bi[k].y, al));
        be = fmaf(bj[k].x, bj[k].x, fmaf(bj[k].y, bj[k].y, be));
        gr = fmaf(bi[k].x, bj[k].x, fmaf(bi[k].y, bj[k].y, gr));
        gi = fmaf(bi[k].x, bj[k].y, fmaf(-bi[k].y, bj[k].x, gi));
    }
    al = group_sum<G>(al);
    be = group_sum<G>(be);
    gr = group_sum<G>(gr);
    gi = group_sum<G>(gi);
    const bool swap = be > al;
    const double g2 = (double)gr * gr + (double)gi * gi;
    const double ab = (double)al * be;
    if (!(g2 > tol2 * ab && ab > 0.0)) {
        if (!swap) return false;
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const int r = q + G * k;
            Bs[swx<MP>(cs, r)] = bj[k];
            Bs[swx<MP>(cn, r)] = bi[k];
        }
        return true;
    }
    const float g2f = (float)g2;
    float rg;
    if (g2f >= 1e-36f) {
        rg = __builtin_amdgcn_rsqf(g2f);
    } else {
        const float ax = fabsf(gr), ay = fabsf(gi);
        const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
        const float rt = mn * __builtin_amdgcn_rcpf(mx);
        rg = __builtin_amdgcn_rcpf(mx * __builtin_amdgcn_sqrtf(fmaf(rt, rt, 1.0f)));
    }
    const float zeta = (be - al) * 0.5f * rg;
    const float az = fminf(fabsf(zeta), 1e18f);
    float t = __builtin_amdgcn_rcpf(az + __builtin_amdgcn_sqrtf(fmaf(az, az, 1.0f)));
    t = copysignf(t, zeta);
    const float c = rsqrt_refined(fmaf(t, t, 1.0f));
    const float sn = c * t;
    const float wr = sn * gr * rg;
    const float wi = -sn * gi * rg;
    const int ds = swap ? cn : cs, dn = swap ? cs : cn;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const int r = q + G * k;
        float2 x = bi[k], y = bj[k];
        float2 ni, nj;
        ni.x = fmaf(c, x.x, -fmaf(wr, y.x, -wi * y.y));
        ni.y = fmaf(c, x.y, -fmaf(wr, y.y, wi * y.x));
        nj.x = fmaf(c, y.x, fmaf(wr, x.x, wi * x.y));
        nj.y = fmaf(c, y.y, fmaf(wr, x.y, -wi * x.x));
        Bs[swx<MP>(ds, r)] = ni;
        Bs[swx<MP>(dn, r)] = nj;
    }
    return true;
}

// Orders a wave's LDS writes before its later LDS reads: the hardware completes one wave's LDS
// instructions in issue order, so only the compiler has to be kept from moving accesses across.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Sum over aligned groups of GS lanes (GS = 4, 8, 16, 32 or 64); all lanes of a group get
// identical bits (the cross-row steps add a lane's value to its partner's, which commutes).
template <int GS>
__device__ __forceinline__ float lane_sum(float v)
{
    v = group_sum<(GS < 16 ? GS : 16)>(v);
    if (GS >= 32) v += __shfl_xor(v, 16);
    if (GS >= 64) v += __shfl_xor(v, 32);
    return v;
}

// One signal column's part of a subspace sweep, by one group of GS lanes (qs = lane in group,
// MP / GS rows each): column cs against the non-signal columns nlist[j0], nlist[j0 + 1], ..
// (cyclically, nn of them), each visit as jacobi_pair_sorted.  The signal column stays in
// registers for the whole pass; each partner is loaded, rotated and written back.  The other
// groups of the same wave run the same pass for the other signal columns from starting slots at
// least two apart (cyclically), so that no two groups visit a column in the same visit step, and
// every write reaches the LDS before the wave's later reads (issue order; see wave_lds_sync).
// A group spans 16 to 64 lanes (one wave holds all Ns <= 3 passes), so a visit costs few
// instructions per lane.  Returns the number of visits that changed the columns.
template <int MP, int GS>
__device__ __forceinline__ int sub_pass(float2 *Bs, int cs, const int *nlist, int nn, int j0,
                                        int qs, double tol2)
{
    constexpr int NR = MP / GS;
    float2 xs[NR], y[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) xs[k] = Bs[swx<MP>(cs, qs + GS * k)];
    int j = j0;
    int changed = 0;
    for (int t = 0; t < nn; ++t) {
        const int cn = nlist[j];
        if (++j == nn) j = 0;
#pragma unroll
        for (int k = 0; k < NR; ++k) y[k] = Bs[swx<MP>(cn, qs + GS * k)];
        float al = 0.f, be = 0.f, gr = 0.f, gi = 0.f;
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            al = fmaf(xs[k].x, xs[k].x, fmaf(xs[k].y, xs[k].y, al));
            be = fmaf(y[k].x, y[k].x, fmaf(y[k].y, y[k].y, be));
            gr = fmaf(xs[k].x, y[k].x, fmaf(xs[k].y, y[k].y, gr));
            gi = fmaf(xs[k].x, y[k].y, fmaf(-xs[k].y, y[k].x, gi));
        }
        al = lane_sum<GS>(al);
        be = lane_sum<GS>(be);
        gr = lane_sum<GS>(gr);
        gi = lane_sum<GS>(gi);
        const bool swap = be > al;
        const double g2 = (double)gr * gr + (double)gi * gi;
        const double ab = (double)al * be;
        if (g2 > tol2 * ab && ab > 0.0) {
            const float g2f = (float)g2;
            float rg;
            if (g2f >= 1e-36f) {
                rg = __builtin_amdgcn_rsqf(g2f);
            } else {
                const float ax = fabsf(gr), ay = fabsf(gi);
                const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
                const float rt = mn * __builtin_amdgcn_rcpf(mx);
                rg = __builtin_amdgcn_rcpf(mx * __builtin_amdgcn_sqrtf(fmaf(rt, rt, 1.0f)));
            }
            const float zeta = (be - al) * 0.5f * rg;
            const float az = fminf(fabsf(zeta), 1e18f);
            float tt = __builtin_amdgcn_rcpf(az + __builtin_amdgcn_sqrtf(fmaf(az, az, 1.0f)));
            tt = copysignf(tt, zeta);
            const float c = rsqrt_refined(fmaf(tt, tt, 1.0f));
            const float sn = c * tt;
            const float wr = sn * gr * rg;
            const float wi = -sn * gi * rg;
#pragma unroll
            for (int k = 0; k < NR; ++k) {
                const float2 x = xs[k], v = y[k];
                float2 ni, nj;
                ni.x = fmaf(c, x.x, -fmaf(wr, v.x, -wi * v.y));
                ni.y = fmaf(c, x.y, -fmaf(wr, v.y, wi * v.x));
                nj.x = fmaf(c, v.x, fmaf(wr, x.x, wi * x.y));
                nj.y = fmaf(c, v.y, fmaf(wr, x.y, -wi * x.x));
                xs[k] = swap ? nj : ni;
                Bs[swx<MP>(cn, qs + GS * k)] = swap ? ni : nj;
            }
            ++changed;
        } else if (swap) {
#pragma unroll
            for (int k = 0; k < NR; ++k) {
                Bs[swx<MP>(cn, qs + GS * k)] = xs[k];
                xs[k] = y[k];
            }
            ++changed;
        }
        wave_lds_sync();
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) Bs[swx<MP>(cs, qs + GS * k)] = xs[k];
    return changed;
}

// Sum over the 64 lanes of a wave; every lane gets the same bits.
__device__ __forceinline__ float wave_sum(float v)
{
    v = group_sum<16>(v);
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

// One bin: Af = its A (row-major M x M, overwritten), kst = upstream status of the bin (noise
// factorisation), Enf = [M-Ns][M] output (null: only the signal vectors are formed, see Esf),
// sigf = [M] or null, stf = status or null,
// convf = (sweeps, rotations, numerical rank) or null.  sub_full >= 0 (only with sigf and Uf
// null, 1 <= Ns <= kSubMaxNs) asks for the noise subspace alone: E_n is then an orthonormal basis
// of the span of the M - Ns smallest left singular vectors (what eq.5 with p = 2 depends on), not
// the singular vectors themselves; see the subspace phase below.  Esf ([Ns][M], or null) receives
// the signal vectors: the Ns leading sorted singular vectors, or with the subspace stop a basis of
// their span of unit vectors (orthogonal to the rotation tolerance); with Enf null (then Esf is
// set and 1 <= Ns <= 3) unit vectors A w_s spanning that subspace, not orthogonal (see the
// signal vectors without Q below).  Lf ([6], with Esf, Ns <= 3,
// or null): the inverse L^{-1} of the Cholesky factor of their Gram matrix E_s^H E_s, computed in
// FP64 from the stored complex64 values, lower triangle by rows (00, 10, 11, 20, 21, 22), zero if
// the bin failed: the projector onto span E_s is E_s (E_s^H E_s)^{-1} E_s^H exactly.
template <int MP, int G>
__device__ __forceinline__ void jacobi_bin(float2 *__restrict__ Af, int kst, int M, int Ns,
                                           int max_sweeps, float2 *__restrict__ Enf,
                                           float *__restrict__ sigf, int32_t *__restrict__ stf,
                                           int32_t *__restrict__ convf,
                                           float2 *__restrict__ Uf = nullptr, int sub_full = -1,
                                           float2 *__restrict__ Esf = nullptr,
                                           double2 *__restrict__ Lf = nullptr)
{
    typedef JacobiCfg<MP, G> C;
    constexpr int R = C::R;
    constexpr int NT = C::THREADS;
    constexpr int NG = C::NG;
    // column c at c*MP: A -> QR (R above, reflectors below) -> Z = R^H -> R1 -> X = R1^H -> W ->
    // U_R (-> registers while the reflectors of Q pass through) -> U
    __shared__ float2 X[MP * MP];
    __shared__ float2 diag[MP];         // diagonal of R (step order)
    __shared__ float2 vhead[MP];        // leading element v_k of reflector k
    __shared__ float tau[MP];
    __shared__ int colmap[MP];          // step k's pivot: physical column colmap[k]
    __shared__ int pos[MP];             // step at which physical column c was chosen (M: never)
    __shared__ int clist[MP];           // unused columns of the pivoted QR, packed
    __shared__ int cinv[MP];            // slot of column c in clist
    __shared__ float sig[MP];
    __shared__ int perm[MP];
    __shared__ unsigned long long pkey[3];   // pivot keys of steps k, k+1 (k+2 being cleared)
    __shared__ int flag;                // upstream failure / non-finite input
    __shared__ float amax_s;
    __shared__ int rot_total;
    __shared__ int rank_s;              // numerical rank found by the pivoted QR
    __shared__ float2 diag1[MP];        // diagonal of R1 (second QR)
    __shared__ float nrm1[MP];          // trailing norm of the next column (second QR)
    __shared__ int degen;               // a column of W vanished

    const int tid = threadIdx.x;
    const int g = tid / G;              // lane group
    const int q = tid % G;              // lane in group
    const int Nn = M - Ns;
    // only the signal vectors are wanted (eq.5 evaluated through them): no complement basis, and
    // only their Ns columns pass through Q
    const bool sig_only = Enf == nullptr;

    __syncthreads();                    // the previous bin of a persistent workgroup is done
    if (tid == 0) {
        flag = kst;
        amax_s = 0.0f;
        rot_total = 0;
        rank_s = M;
        degen = 0;
        pkey[0] = pkey[1] = pkey[2] = 0ull;
    }
    if (tid < MP) {
        pos[tid] = M;
        clist[tid] = tid;
        cinv[tid] = tid;
    }
    __syncthreads();

    // ---- load A column-major into X (padding zero) ---------------------------------------------
    float amax = 0.0f;
    bool nonfinite = false;
    for (int e = tid; e < MP * MP; e += NT) {
        const int r = e / MP, c = e - r * MP;            // read row-major A: coalesced
        float2 a = make_float2(0.f, 0.f);
        if (r < M && c < M) {
            a = Af[(size_t)r * M + c];
            if (!finite2(a)) nonfinite = true;
            amax = fmaxf(amax, fmaxf(fabsf(a.x), fabsf(a.y)));
        }
        X[at<MP>(c, r)] = a;
    }
    const int nf_count = __syncthreads_count(nonfinite ? 1 : 0);
    if (!nonfinite && amax > 0.0f) atomicMax((int *)&amax_s, __float_as_int(amax));
    __syncthreads();
    if (tid == 0 && nf_count > 0 && flag == SSL_BIN_OK) flag = SSL_BIN_NONFINITE;
    __syncthreads();

    int sweeps = 0;
    bool converged = false;
    bool sub_done = false;              // stopped by the subspace phase
    int ex = 0;
    if (flag == SSL_BIN_OK) {
        // scale by a power of two so that max |A_ij| lies in [0.5, 1): exact, keeps every Gram
        // entry far from FP32 overflow; singular values are scaled back at the end.
        const float am = amax_s;
        if (am > 0.0f) frexpf(am, &ex);
        const float sc = ldexpf(1.0f, -ex);
        for (int e = tid; e < MP * MP; e += NT) {
            const float2 b = X[e];
            X[e] = make_float2(b.x * sc, b.y * sc);
        }
        __syncthreads();

        // ---- 1. Householder QR with column pivoting: A P = Q R ----------------------------------
        // Columns stay where they are; step k picks the unused column of largest trailing norm
        // (rows k..M-1; ties: lower column), known from a 64-bit LDS max over (norm, column) keys
        // that the previous step's update pass posts, so a step costs one barrier.  The reflector
        // v = x - alpha e_k, alpha = -e^{i arg x_k}|x|, is formed redundantly by every group; its
        // head v_k goes to vhead (x_k itself stays in place, R's diagonal is kept in diag).
        // Once the pivot norm drops to M 2^-24 times the first one, the remaining rows of R are
        // FP32 noise: the numerical rank is k.  The unused columns are kept packed in clist
        // (the pivot leaves by swapping in the last entry), so the update pass of step k occupies
        // only ceil((M - k - 1) / groups-per-wave) waves' worth of groups.
        for (int c = g; c < M && g < NG; c += NG) {
            float s = 0.f;
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const float2 v = X[at<MP>(c, q + G * j)];
                s = fmaf(v.x, v.x, fmaf(v.y, v.y, s));
            }
            s = group_sum<G>(s);
            if (q == 0) atomicMax(&pkey[0], pivot_key(s, c));
        }
        __syncthreads();
        int rk = M;
        float thr = 0.0f;
        int nrem = M;                      // unused columns: clist[0 .. nrem)
        int kc = 0, kn = 1, kz = 2;        // pkey slots of steps k, k+1, k+2
        for (int k = 0; k < M; ++k) {
            const unsigned long long key = pkey[kc];
            const int p = 0x7fffffff - (int)(unsigned int)(key & 0xffffffffull);
            const float nx = sqrtf(__uint_as_float((unsigned int)(key >> 32)));
            if (nx <= thr) {               // uniform: every thread read the same key
                rk = k;
                break;
            }
            if (k == 0) thr = (float)M * 5.9604644775390625e-08f * nx;
            const float2 xk = X[at<MP>(p, k)];
            const float axk = sqrtf(fmaf(xk.x, xk.x, xk.y * xk.y));
            const float rax = __builtin_amdgcn_rcpf(axk);
            const float2 ph = axk > 0.f ? make_float2(xk.x * rax, xk.y * rax) : make_float2(1.f, 0.f);
            const float tk = __builtin_amdgcn_rcpf(nx * (nx + axk));
            const float2 vk = make_float2(ph.x * (axk + nx), ph.y * (axk + nx));
            // p leaves the list: slot idx takes the last entry.  Every thread applies the swap
            // virtually in this step (slot idx reads `last`), thread 0 writes it for the next;
            // nothing else reads clist[idx] or cinv[last] in this step.
            const int idx = cinv[p];
            const int last = clist[nrem - 1];
            --nrem;
            if (tid == 0) {
                diag[k] = make_float2(-ph.x * nx, -ph.y * nx);
                vhead[k] = vk;
                tau[k] = tk;
                colmap[k] = p;
                pos[p] = k;
                pkey[kz] = 0ull;           // read by everyone in step k-1, posted in step k+1
                clist[idx] = last;
                cinv[last] = idx;
            }
            // slots g and g + NG (nrem <= 2 NG); a wave with any second slot takes the two-column
            // path for all its groups
            if (g < NG && g < nrem) {
                const int c0 = (g == idx) ? last : clist[g];
                const int s1 = g + NG;
                const bool two = s1 < nrem;
                if (__any(two)) {
                    const int c1 = two ? ((s1 == idx) ? last : clist[s1]) : c0;
                    float tn0, tn1;
                    apply_reflector2<MP, G>(p, vk, k, tk, X, c0, c1, two, q, tn0, tn1);
                    if (q == 0) {
                        atomicMax(&pkey[kn], pivot_key(tn0, c0));
                        if (two) atomicMax(&pkey[kn], pivot_key(tn1, c1));
                    }
                } else {
                    const float tn = apply_reflector<MP, G>(p, vk, k, tk, X, c0, M, q);
                    if (q == 0) atomicMax(&pkey[kn], pivot_key(tn, c0));
                }
            }
            __syncthreads();
            const int t = kc;
            kc = kn;
            kn = kz;
            kz = t;
        }

        // ---- 2. park the reflectors in A's rows (workspace); Z = R^H in place ------------------
        // Only the leading rk rows of R are kept (R: rk x M); the columns rk..M-1 of U are Q's,
        // spanning the null space.  Z's rows follow the physical column order (a row permutation
        // of R^H changes neither the Gram matrix of its columns nor the triangular factor below):
        // Z[x][c] = conj(R[c][pos x]).  R[c][pos x] sits at (column x, row c), so Z is a masked
        // conjugate transpose: each thread exchanges the pair (c, x), (x, c) it owns.
        if (tid == 0) rank_s = rk;
        for (int e = tid; e < rk * MP && !sig_only; e += NT) {   // reflector k = e / MP, row e % MP
            const int k = e / MP, r = e % MP;
            if (r >= k && r < M) Af[k * M + r] = (r == k) ? vhead[k] : X[at<MP>(colmap[k], r)];
        }
        __syncthreads();
        for (int e = tid; e < MP * MP; e += NT) {
            const int c = e / MP, x = e - c * MP;
            if (c > x) continue;
            const float2 o1 = X[at<MP>(x, c)], o2 = X[at<MP>(c, x)];
            float2 n1 = make_float2(0.f, 0.f), n2 = make_float2(0.f, 0.f);
            if (c < rk && x < M) {                       // Z[x][c]
                const int px = pos[x];
                if (px > c) n1 = conj2(o1);
                else if (px == c) n1 = conj2(diag[c]);
            }
            if (x < rk && c < M) {                       // Z[c][x]
                const int pc = pos[c];
                if (pc > x) n2 = conj2(o2);
                else if (pc == x) n2 = conj2(diag[x]);
            }
            X[at<MP>(c, x)] = n1;
            X[at<MP>(x, c)] = n2;
        }
        __syncthreads();

        // ---- 3. Z = Q1 R1 (Householder, no pivoting; Q1 is not needed), then X = R1^H --------
        // R = R1^H Q1^H, so R's left singular vectors are X's; X's column Gram X^H X = R1 R1^H
        // is closer still to diagonal than R R^H.  The trailing norm of the next column comes out
        // of each update pass.  With sig_only none of this: the sweeps run on Z itself (see the
        // signal vectors below).
        if (!sig_only) {
            if (g == 0) {
                float s = 0.f;
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const float2 v = X[at<MP>(0, q + G * j)];
                    s = fmaf(v.x, v.x, fmaf(v.y, v.y, s));
                }
                s = group_sum<G>(s);
                if (q == 0) nrm1[0] = s;
            }
            __syncthreads();
            for (int k = 0; k < rk; ++k) {
                const float nx = sqrtf(nrm1[k]);
                const float2 xk = X[at<MP>(k, k)];
                const float axk = sqrtf(fmaf(xk.x, xk.x, xk.y * xk.y));
                const float rax = __builtin_amdgcn_rcpf(axk);
                const float2 ph = axk > 0.f ? make_float2(xk.x * rax, xk.y * rax)
                                            : make_float2(1.f, 0.f);
                const float tk = nx > 0.f ? __builtin_amdgcn_rcpf(nx * (nx + axk)) : 0.0f;
                const float2 vk = make_float2(ph.x * (axk + nx), ph.y * (axk + nx));
                if (tid == 0) diag1[k] = make_float2(-ph.x * nx, -ph.y * nx);
                // columns k + 1 + g and k + 1 + g + NG, as in the pivoted QR
                const int c0 = k + 1 + g;
                if (g < NG && c0 < rk) {
                    const int c1 = c0 + NG;
                    const bool two = c1 < rk;
                    if (__any(two)) {
                        float tn0, tn1;
                        apply_reflector2<MP, G>(k, vk, k, tk, X, c0, two ? c1 : c0, two, q,
                                                tn0, tn1);
                        if (c0 == k + 1 && q == 0) nrm1[c0] = tn0;
                    } else {
                        const float tn = apply_reflector<MP, G>(k, vk, k, tk, X, c0, M, q);
                        if (c0 == k + 1 && q == 0) nrm1[c0] = tn;
                    }
                }
                __syncthreads();
            }
            // X[i][c] = conj(R1[c][i]), R1[c][i] at (column i, row c) for i > c: masked transpose
            for (int e = tid; e < MP * MP; e += NT) {
                const int c = e / MP, i = e - c * MP;
                if (c > i) continue;
                const float2 o1 = X[at<MP>(i, c)], o2 = X[at<MP>(c, i)];
                float2 n1 = make_float2(0.f, 0.f), n2 = make_float2(0.f, 0.f);
                if (i < rk) {
                    if (i > c) n1 = conj2(o1);               // X[i][c], below the diagonal
                    else n1 = conj2(diag1[c]);               // i == c
                }
                (void)o2;                                    // X[c][i] (c < i) is above: zero
                X[at<MP>(c, i)] = n1;
                if (c != i) X[at<MP>(i, c)] = n2;
            }
            __syncthreads();
        }

        // ---- 4. one-sided Jacobi on X: X V = W, columns orthogonalised in place ----------------
        // The sweeps work on a swizzled copy of the layout (swx): each column's 8-row chunks are
        // permuted by its index, so that the lane groups of a round, which read the same rows of
        // different columns, fall on different LDS banks.
        float2 *Bs = X;
        // to the sweep layout (row pairs r, r XOR s of each column exchanged)
        for (int e = tid; e < MP * MP; e += NT) {
            const int c = e / MP, r = e - c * MP, rr = r ^ swz_mask<MP>(c);
            if (r < rr) {
                const float2 u = X[c * MP + r], v = X[c * MP + rr];
                X[c * MP + r] = v;
                X[c * MP + rr] = u;
            }
        }
        __syncthreads();
        const int Me = rk + (rk & 1);                // players of the round-robin tournament
        // rotate iff |cos| > 2 sqrt(M) 2^-24 (twice the usual FP32 one-sided Jacobi threshold)
        const double tol = 2.0 * sqrt((double)M) * 5.9604644775390625e-08;
        const double tol2 = tol * tol;
        int my_rot = 0;
        // A partly active wave costs as much as a full one.  When the Me/2 pairs of a round fill
        // whole waves but one pair (Me/2 = 1 mod pairs-per-wave), that pair (group Me/2 - 1) is
        // left out of every round: over the Me - 1 rounds the left-out pairs are (c - 1, c) for
        // every c mod Me - 1, a single odd cycle, played after the regular rounds as the
        // matchings {(0,1), (2,3), ..}, {(1,2), (3,4), ..} and {(Me-2, 0)}.  Every pair is still
        // rotated once per sweep.
        constexpr int kPairsPerWave = 64 / G;
        const int P = Me / 2;
        const bool defer = P > 1 && P % kPairsPerWave == 1;
        const int Pr = defer ? P - 1 : P;
        const int n_rounds = Me - 1 + (defer ? 3 : 0);
        // row slots per lane: R - 1 when they cover the rank (the 60-channel rank-50 case), else R
        constexpr int RLO = R > 1 ? R - 1 : 1;
        const bool nr_lo = (sig_only ? M : rk) <= G * RLO;   // rows of X: rk, or M for Z
        // Subspace phase (sub_full >= 0): after sub_full full sweeps, S = the Ns columns of
        // largest norm; then only the pairs with a member in S are visited (jacobi_pair_sorted
        // for a signal / noise pair, so that S keeps the larger results), until such a sweep
        // changes nothing: X_S is then orthogonal to the other columns and within itself to the
        // rotation tolerance, and X's singular values split into those of X_S and of the rest.
        // X_S spans the Ns dominant left singular vectors when min_S |x|^2 > sum of |x|^2 over
        // the rest (that sum bounds the square of the largest singular value of the rest),
        // checked on the column norms; the noise subspace is then the orthogonal complement of
        // X_S, and the rotations inside it that the full solve would still make change nothing
        // eq.5 with p = 2 reads.  A failed check, or kSubMaxSweeps subspace sweeps without
        // convergence, returns to full sweeps (the full solve); so does a bin whose weakest
        // signal column holds less than the other columns' energy at the switch.
        // A subspace sweep runs in wave 0 alone: its lane group i < Ns (64 / 32 / 16 lanes for
        // Ns = 1 / 2 / 3) takes signal column i against the non-signal columns from slot
        // i floor((rk - Ns) / Ns) on (sub_pass; the starting slots are at least two apart when
        // rk >= 3 Ns), then the pairs inside S one at a time; a wave's LDS accesses complete in
        // issue order, so no workgroup barrier is needed.
        const bool sub = sub_full >= 0 && sigf == nullptr && Uf == nullptr && Ns >= 1 &&
                         Ns <= kSubMaxNs && 3 * Ns <= rk;
        int phase = 0;                               // 0 full, 1 subspace, 2 full after a fallback
        int sub_sweeps = 0;
        unsigned long long smask = 0ull;
        for (int sw = 0; sw < max_sweeps; ++sw) {
            if (sub && phase == 0 && sw == sub_full) {
                sub_norms<MP, G>(Bs, rk, g, q, nrm1);
                __syncthreads();
                if (tid == 0) {
                    unsigned long long m = 0ull;
                    float tot = 0.0f;
                    for (int c = 0; c < rk; ++c) tot += nrm1[c];
                    for (int k = 0; k < Ns; ++k) {
                        int best = -1;
                        float bv = -1.0f;
                        for (int c = 0; c < rk; ++c)
                            if (!((m >> c) & 1ull) && (best < 0 || nrm1[c] > bv)) {
                                bv = nrm1[c];
                                best = c;
                            }
                        m |= 1ull << best;              // rk > Ns: a column is always left
                    }
                    // a bin whose weakest signal column holds less than the rest's energy
                    // will hardly pass the dominance check: it stays with full sweeps (this
                    // decides speed only, not the result's accuracy)
                    float mins = 3.4e38f, sums = 0.0f;
                    for (int c = 0; c < rk; ++c)
                        if ((m >> c) & 1ull) {
                            mins = fminf(mins, nrm1[c]);
                            sums += nrm1[c];
                        }
                    pkey[0] = (mins > tot - sums) ? m : 0ull;
                    int ks = 0, kn = 0;              // S and the other columns, ascending
                    for (int c = 0; c < rk; ++c) {
                        if ((m >> c) & 1ull) cinv[ks++] = c;
                        else clist[kn++] = c;
                    }
                }
                __syncthreads();
                smask = pkey[0];
                phase = smask ? 1 : 2;
            }
            // a subspace sweep that would change nothing is replaced by one parallel test
            bool settled = false;
            if (phase == 1) {
                settled = sub_settled<MP, G>(Bs, cinv, clist, Ns, rk, g, q, tol2);
                if (!settled && sub_sweeps >= kSubMaxSweeps) phase = 2;
            }
            if (!settled) {
                int rotated = 0;
                if (phase == 1) {
                    if (tid < 64) {
                        // GS lanes per signal column: 64, 32 or 16 for Ns = 1, 2, 3 (at most MP)
                        constexpr int G1 = MP < 64 ? MP : 64, G2 = MP < 32 ? MP : 32,
                                      G3 = MP < 16 ? MP : 16;
                        const int nn = rk - Ns;
                        const int gs = Ns == 1 ? G1 : (Ns == 2 ? G2 : G3);
                        const int i = tid / gs, qs = tid % gs;
                        if (i < Ns) {
                            const int cs = cinv[i], j0 = i * (nn / Ns);
                            const int ch =
                                Ns == 1 ? sub_pass<MP, G1>(Bs, cs, clist, nn, j0, qs, tol2)
                                : Ns == 2 ? sub_pass<MP, G2>(Bs, cs, clist, nn, j0, qs, tol2)
                                          : sub_pass<MP, G3>(Bs, cs, clist, nn, j0, qs, tol2);
                            if (ch) {
                                rotated = 1;
                                if (qs == 0) my_rot += ch;
                            }
                        }
                        wave_lds_sync();
                        for (int a = 0; a + 1 < Ns; ++a)
                            for (int b = a + 1; b < Ns; ++b) {
                                if (g == 0) {
                                    const bool rot =
                                        nr_lo ? jacobi_pair<MP, G, RLO>(Bs, cinv[a], cinv[b], q, tol2)
                                              : jacobi_pair<MP, G, R>(Bs, cinv[a], cinv[b], q, tol2);
                                    if (rot) {
                                        rotated = 1;
                                        if (q == 0) ++my_rot;
                                    }
                                }
                                wave_lds_sync();
                            }
                    }
                }
                for (int rd = 0; rd < n_rounds && phase != 1; ++rd) {
                    int a = 0, b = 0;
                    bool play;
                    if (rd < Me - 1) {
                        play = g < Pr;
                        if (g == 0) {
                            a = Me - 1;
                            b = rd;
                        } else {                         // (rd +- g) mod (Me - 1), 0 < g < Me/2
                            a = rd + g;
                            if (a >= Me - 1) a -= Me - 1;
                            b = rd - g;
                            if (b < 0) b += Me - 1;
                        }
                    } else if (rd < Me + 1) {            // (2g + e, 2g + e + 1), e = 0, 1
                        play = g < (Me - 2) / 2;
                        a = 2 * g + (rd - (Me - 1));
                        b = a + 1;
                    } else {
                        play = g == 0;
                        a = Me - 2;
                        b = 0;
                    }
                    if (play) {
                        const int ci = min(a, b), cj = max(a, b);
                        if (cj < rk) {
                            const bool rot =
                                nr_lo ? jacobi_pair<MP, G, RLO>(Bs, ci, cj, q, tol2)
                                      : jacobi_pair<MP, G, R>(Bs, ci, cj, q, tol2);
                            if (rot) {
                                rotated = 1;
                                if (q == 0) ++my_rot;
                            }
                        }
                    }
                    __syncthreads();
                }
                ++sweeps;
                const bool none = __syncthreads_count(rotated) == 0;
                if (phase != 1) {
                    if (none) {
                        converged = true;
                        break;
                    }
                    continue;
                }
                ++sub_sweeps;
                if (!none) continue;
            }
            // the split has converged: dominance check on the column norms (fixed-order sum)
            sub_norms<MP, G>(Bs, rk, g, q, nrm1);
            __syncthreads();
            if (tid == 0) {
                float mins = 3.4e38f, sumn = 0.0f;
                for (int c = 0; c < rk; ++c) {
                    if ((smask >> c) & 1ull) mins = fminf(mins, nrm1[c]);
                    else sumn += nrm1[c];
                }
                pkey[1] = mins > sumn ? 1ull : 0ull;
            }
            __syncthreads();
            if (pkey[1] != 0ull) {
                converged = true;
                sub_done = true;
                break;
            }
            phase = 2;
        }
        if (my_rot) atomicAdd(&rot_total, my_rot);
        // back to the plain layout
        for (int e = tid; e < MP * MP; e += NT) {
            const int c = e / MP, r = e - c * MP, rr = r ^ swz_mask<MP>(c);
            if (r < rr) {
                const float2 u = X[c * MP + r], v = X[c * MP + rr];
                X[c * MP + r] = v;
                X[c * MP + rr] = u;
            }
        }
        __syncthreads();

        if (!sub_done) {
            // ---- 5. sigma_c = |w_c| (scaled back); U_R = W Sigma^-1 extended by the identity on the
            // null-space columns rk..M-1; stable descending rank of sigma ------------------------------
            for (int c = g; c < MP && g < NG; c += NG) {
                float2 x[R];
                float s = 0.f;
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    x[k] = Bs[at<MP>(c, q + G * k)];
                    s = fmaf(x[k].x, x[k].x, fmaf(x[k].y, x[k].y, s));
                }
                s = group_sum<G>(s);
                if (c < rk) {
                    // X is nonsingular (rank rk), so a zero column means a numerical breakdown
                    const float inv = s > 0.f ? rsqrt_refined(s) : 0.0f;
#pragma unroll
                    for (int k = 0; k < R; ++k)
                        Bs[at<MP>(c, q + G * k)] = make_float2(x[k].x * inv, x[k].y * inv);
                    if (q == 0 && !(s > 0.f)) degen = 1;
                } else {
#pragma unroll
                    for (int k = 0; k < R; ++k)
                        Bs[at<MP>(c, q + G * k)] = make_float2((q + G * k == c && c < M) ? 1.f : 0.f, 0.f);
                }
                if (q == 0) sig[c] = (c < M) ? ldexpf(sqrtf(s), ex) : -1.0f;
            }
            for (int c = tid; c < MP; c += NT) perm[c] = c;
            __syncthreads();
            if (degen) converged = false;
            for (int c = tid; c < M; c += NT) {
                const float sc_ = sig[c];
                int rank = 0;
                for (int k = 0; k < M; ++k) {
                    const float sk = sig[k];
                    rank += (sk > sc_ || (sk == sc_ && k < c)) ? 1 : 0;
                }
                if (rank < M) perm[rank] = c;
            }
        } else {
            // ---- 5'. noise subspace: the orthogonal complement of X_S -------------------------
            // Householder QR of the Ns columns of S (wave 0, one row per lane; S in ascending
            // column order, listed in cinv): reflector k (rows k..rk-1) goes to the k-th of the
            // arrays diag, vhead, diag1 (free since the transposes) and its tau to sig[k]; the S
            // columns themselves are normalised in place (the signal vectors).  Every other
            // column c < rk takes the complement vector H_0 .. H_{Ns-1} e_kc (kc = Ns + its
            // position among the non-S columns), an orthonormal basis of the complement of
            // span X_S; columns rk.. stay the identity (null space).
            float2 *refl[kSubMaxNs] = {diag, vhead, diag1};
            if (tid < 64) {
                const int r = tid;
                float2 col[kSubMaxNs];
                int sl[kSubMaxNs];
#pragma unroll
                for (int j = 0; j < kSubMaxNs; ++j) sl[j] = 0;
                {
                    int k = 0;
                    for (int c = 0; c < rk; ++c)
                        if ((smask >> c) & 1ull) {
#pragma unroll
                            for (int j = 0; j < kSubMaxNs; ++j)
                                if (j == k) sl[j] = c;
                            ++k;
                        }
                }
#pragma unroll
                for (int k = 0; k < kSubMaxNs; ++k)
                    col[k] = (k < Ns && r < MP) ? Bs[at<MP>(sl[k], r)] : make_float2(0.f, 0.f);
#pragma unroll
                for (int k = 0; k < kSubMaxNs; ++k) {
                    if (k >= Ns) break;
                    const float2 x = col[k];
                    const float n2 = wave_sum(fmaf(x.x, x.x, x.y * x.y));
                    const float inv = n2 > 0.f ? rsqrt_refined(n2) : 0.0f;
                    if (r < MP) Bs[at<MP>(sl[k], r)] = make_float2(x.x * inv, x.y * inv);
                }
#pragma unroll
                for (int k = 0; k < kSubMaxNs; ++k) {
                    if (k >= Ns || sig_only) break;
                    const float2 x = col[k];
                    const float a2 = wave_sum((r >= k && r < rk) ? fmaf(x.x, x.x, x.y * x.y) : 0.f);
                    const float xr = __shfl(x.x, k), xi = __shfl(x.y, k);
                    const float nx = sqrtf(a2);
                    const float axk = sqrtf(fmaf(xr, xr, xi * xi));
                    const float rax = axk > 0.f ? __builtin_amdgcn_rcpf(axk) : 0.f;
                    const float2 ph = axk > 0.f ? make_float2(xr * rax, xi * rax) : make_float2(1.f, 0.f);
                    const float tk = nx > 0.f ? __builtin_amdgcn_rcpf(nx * (nx + axk)) : 0.0f;
                    const float2 vk = make_float2(ph.x * (axk + nx), ph.y * (axk + nx));
                    const float2 v = (r > k && r < rk) ? x : ((r == k) ? vk : make_float2(0.f, 0.f));
                    if (r < MP) refl[k][r] = v;
                    if (r == 0) {
                        sig[k] = tk;
                        cinv[k] = sl[k];
                    }
#pragma unroll
                    for (int j = 0; j < kSubMaxNs; ++j) {
                        if (j <= k || j >= Ns) continue;
                        const float2 y = col[j];
                        float wr = wave_sum(fmaf(v.x, y.x, v.y * y.y));       // conj(v) y
                        float wi = wave_sum(fmaf(v.x, y.y, -v.y * y.x));
                        wr *= tk;
                        wi *= tk;
                        col[j] = make_float2(y.x - fmaf(v.x, wr, -v.y * wi),
                                             y.y - fmaf(v.x, wi, v.y * wr));
                    }
                }
            }
            __syncthreads();
            for (int c = g; c < MP && g < NG && !sig_only; c += NG) {
                if (c < rk && ((smask >> c) & 1ull)) continue;
                float2 z[R];
                if (c < rk) {
                    const int kc = Ns + c - __popcll(smask & ((1ull << c) - 1ull));
#pragma unroll
                    for (int j = 0; j < R; ++j)
                        z[j] = make_float2(q + G * j == kc ? 1.f : 0.f, 0.f);
#pragma unroll
                    for (int k = kSubMaxNs - 1; k >= 0; --k) {
                        if (k >= Ns) continue;
                        const float2 *vk = refl[k];
                        const float tk = sig[k];
                        float2 v[R];
                        float wr = 0.f, wi = 0.f;
#pragma unroll
                        for (int j = 0; j < R; ++j) {
                            v[j] = vk[q + G * j];
                            wr = fmaf(v[j].x, z[j].x, fmaf(v[j].y, z[j].y, wr));
                            wi = fmaf(v[j].x, z[j].y, fmaf(-v[j].y, z[j].x, wi));
                        }
                        wr = group_sum<G>(wr) * tk;
                        wi = group_sum<G>(wi) * tk;
#pragma unroll
                        for (int j = 0; j < R; ++j) {
                            z[j].x = fmaf(-v[j].x, wr, fmaf(v[j].y, wi, z[j].x));
                            z[j].y = fmaf(-v[j].x, wi, fmaf(-v[j].y, wr, z[j].y));
                        }
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < R; ++j)
                        z[j] = make_float2((q + G * j == c && c < M) ? 1.f : 0.f, 0.f);
                }
#pragma unroll
                for (int j = 0; j < R; ++j) Bs[at<MP>(c, q + G * j)] = z[j];
            }
            for (int c = tid; c < M; c += NT) {
                const int below = __popcll(smask & ((1ull << c) - 1ull));
                if (c < rk && ((smask >> c) & 1ull)) perm[below] = c;
                else perm[Ns + c - below] = c;
            }
            __syncthreads();
        }
        // ---- 6. U = Q U_R, reflectors applied last to first ----------------------------------
        // U's columns move to registers (a group owns at most two: c = g, g + NG), the reflectors
        // take the buffer (stored with zeros outside rows k..M-1, so their loads need no row
        // test), and each group takes its columns through every reflector with no barrier.
        if (!sig_only) {
            const int c0 = g, c1 = g + NG;
            const bool h0 = g < NG && c0 < M, h1 = g < NG && c1 < M;
            float2 x0[R], x1[R];
#pragma unroll
            for (int j = 0; j < R; ++j) {
                x0[j] = h0 ? X[at<MP>(c0, q + G * j)] : make_float2(0.f, 0.f);
                x1[j] = h1 ? X[at<MP>(c1, q + G * j)] : make_float2(0.f, 0.f);
            }
            __syncthreads();
            for (int e = tid; e < rk * MP; e += NT) {
                const int k = e / MP, r = e - k * MP;
                X[at<MP>(k, r)] = (r >= k && r < M) ? Af[k * M + r] : make_float2(0.f, 0.f);
            }
            __syncthreads();
            for (int k = rk - 1; k >= 0; --k) {
                const float tk = tau[k];
                float2 v[R];
                float ar = 0.f, ai = 0.f, br = 0.f, bi = 0.f;
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    if (G * (j + 1) <= k) continue;      // slot entirely above the reflector
                    v[j] = X[at<MP>(k, q + G * j)];
                    ar = fmaf(v[j].x, x0[j].x, fmaf(v[j].y, x0[j].y, ar));
                    ai = fmaf(v[j].x, x0[j].y, fmaf(-v[j].y, x0[j].x, ai));
                    br = fmaf(v[j].x, x1[j].x, fmaf(v[j].y, x1[j].y, br));
                    bi = fmaf(v[j].x, x1[j].y, fmaf(-v[j].y, x1[j].x, bi));
                }
                ar = group_sum<G>(ar) * tk;
                ai = group_sum<G>(ai) * tk;
                br = group_sum<G>(br) * tk;
                bi = group_sum<G>(bi) * tk;
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    if (G * (j + 1) <= k) continue;
                    x0[j].x = fmaf(-v[j].x, ar, fmaf(v[j].y, ai, x0[j].x));
                    x0[j].y = fmaf(-v[j].x, ai, fmaf(-v[j].y, ar, x0[j].y));
                    x1[j].x = fmaf(-v[j].x, br, fmaf(v[j].y, bi, x1[j].x));
                    x1[j].y = fmaf(-v[j].x, bi, fmaf(-v[j].y, br, x1[j].y));
                }
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < R; ++j) {
                if (h0) X[at<MP>(c0, q + G * j)] = x0[j];
                if (h1) X[at<MP>(c1, q + G * j)] = x1[j];
            }
            __syncthreads();
        }
        // ---- 6'. signal vectors without Q: E_s = A W_S --------------------------------------
        // With sig_only the sweeps ran on Z = R~^H (R~ = R P^T: R's columns in physical order,
        // A = Q R~): Z V = W makes W_S span the dominant right singular subspace of R~, A's (Q is
        // unitary), so A W_S spans the Ns dominant left singular vectors of A (W_S's columns are
        // unit vectors here, so each direction comes out scaled by its singular value: a step of
        // power iteration, in which what the rotation tolerance leaves of the other directions
        // is damped by their smaller singular values).  A is the input, still intact (nothing was
        // parked in it), read row by row by groups of G lanes, scaled by 2^-ex as X was.  The
        // sums run in FP64: A w_s for a weaker signal cancels the stronger ones' share of A, and
        // FP32 sums would lose sigma_1 / sigma_s times the rounding of the result.  Each vector
        // is normalised in FP32 (Lf below makes the projector exact); they go to diag, vhead,
        // diag1, free by now.
        if (sig_only) {
            __syncthreads();                            // perm is complete
            auto sv = [&](int k) -> float2 * { return k == 0 ? diag : (k == 1 ? vhead : diag1); };
            const float sc = ldexpf(1.0f, -ex);
            for (int r = g; r < M && g < NG; r += NG) {
                double2 acc[kSubMaxNs];
#pragma unroll
                for (int k = 0; k < kSubMaxNs; ++k) acc[k] = make_double2(0.0, 0.0);
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const int x = q + G * j;
                    const float2 a = x < M ? Af[(size_t)r * M + x] : make_float2(0.f, 0.f);
#pragma unroll
                    for (int k = 0; k < kSubMaxNs; ++k) {
                        if (k >= Ns) break;
                        const float2 w = X[at<MP>(perm[k], x)];
                        acc[k].x = fma((double)a.x, w.x, fma(-(double)a.y, w.y, acc[k].x));
                        acc[k].y = fma((double)a.x, w.y, fma((double)a.y, w.x, acc[k].y));
                    }
                }
#pragma unroll
                for (int k = 0; k < kSubMaxNs; ++k) {
                    if (k >= Ns) break;
                    const double ar = group_sum_f64<G>(acc[k].x), ai = group_sum_f64<G>(acc[k].y);
                    if (q == 0) sv(k)[r] = make_float2((float)(ar * sc), (float)(ai * sc));
                }
            }
            __syncthreads();
            if (tid < 64) {                             // wave 0: normalise, one row per lane
                const int r = tid;
#pragma unroll
                for (int k = 0; k < kSubMaxNs; ++k) {
                    if (k >= Ns) break;
                    const float2 v = r < M ? sv(k)[r] : make_float2(0.f, 0.f);
                    const float n2 = wave_sum(fmaf(v.x, v.x, v.y * v.y));
                    const float inv = n2 > 0.f ? rsqrt_refined(n2) : 0.0f;
                    if (r < MP) sv(k)[r] = make_float2(v.x * inv, v.y * inv);
                }
            }
            __syncthreads();
        }
    }

    // ---- outputs ------------------------------------------------------------------------------
    const bool ok = (flag == SSL_BIN_OK) && converged;
    const int st = (flag != SSL_BIN_OK) ? flag : (converged ? SSL_BIN_OK : SSL_BIN_NO_CONV);
    for (int e = tid; e < Nn * MP && !sig_only; e += NT) { // noise vector c = e / MP, row e % MP
        const int c = e / MP, r = e % MP;
        if (r < M) Enf[c * M + r] = ok ? X[at<MP>(perm[Ns + c], r)] : make_float2(0.f, 0.f);
    }
    // the signal vectors: diag, vhead, diag1 with sig_only, else columns perm[0 .. Ns) of U
    auto sigvec = [&](int c, int r) -> float2 {
        if (!sig_only) return X[at<MP>(perm[c], r)];
        return c == 0 ? diag[r] : (c == 1 ? vhead[r] : diag1[r]);
    };
    if (Esf != nullptr)                                    // [Ns][M]
        for (int e = tid; e < Ns * MP; e += NT) {
            const int c = e / MP, r = e % MP;
            if (r < M) Esf[c * M + r] = ok ? sigvec(c, r) : make_float2(0.f, 0.f);
        }
    if (Esf != nullptr && Lf != nullptr && Ns <= 3 && tid < 64) {
        // Gram matrix of the stored signal vectors in FP64 (wave 0, one row per lane), then the
        // inverse of its Cholesky factor on lane 0
        const int r = tid;
        double2 e[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float2 v = (ok && k < Ns && r < M) ? sigvec(k, r) : make_float2(0.f, 0.f);
            e[k] = make_double2(v.x, v.y);
        }
        double gr[6], gi[6];                       // Gamma_st = e_s^H e_t, index t (t + 1) / 2 + s
#pragma unroll
        for (int t = 0; t < 3; ++t)
#pragma unroll
            for (int s2 = 0; s2 <= t; ++s2) {
                const int i = t * (t + 1) / 2 + s2;
                double a = fma(e[s2].x, e[t].x, e[s2].y * e[t].y);
                double b = fma(e[s2].x, e[t].y, -e[s2].y * e[t].x);
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    a += __shfl_xor(a, o);
                    b += __shfl_xor(b, o);
                }
                gr[i] = a;
                gi[i] = b;
            }
        if (r == 0) {
            double2 out[6];
#pragma unroll
            for (int i = 0; i < 6; ++i) out[i] = make_double2(0.0, 0.0);
            // Gamma = L L^H: L_t0 = conj(Gamma_0t) / L00, ... (lower rows t, columns s)
            const double l00 = sqrt(gr[0]);
            bool pd = ok && gr[0] > 0.0;
            double2 l10 = make_double2(0.0, 0.0), l20 = l10, l21 = l10;
            double l11 = 1.0, l22 = 1.0;
            if (Ns >= 2 && pd) {
                l10 = make_double2(gr[1] / l00, -gi[1] / l00);
                const double d = gr[2] - (l10.x * l10.x + l10.y * l10.y);
                pd = d > 0.0;
                l11 = sqrt(fmax(d, 0.0));
            }
            if (Ns >= 3 && pd) {
                l20 = make_double2(gr[3] / l00, -gi[3] / l00);
                // Gamma_21 = conj(Gamma_12) minus L20 conj(L10), over L11
                const double2 g21 = make_double2(gr[4], -gi[4]);
                const double2 t21 = make_double2(g21.x - (l20.x * l10.x + l20.y * l10.y),
                                                 g21.y - (l20.y * l10.x - l20.x * l10.y));
                l21 = make_double2(t21.x / l11, t21.y / l11);
                const double d = gr[5] - (l20.x * l20.x + l20.y * l20.y) -
                                 (l21.x * l21.x + l21.y * l21.y);
                pd = d > 0.0;
                l22 = sqrt(fmax(d, 0.0));
            }
            if (pd) {
                const double i00 = 1.0 / l00, i11 = 1.0 / l11, i22 = 1.0 / l22;
                // inverse of the lower triangular L, column by column
                const double2 i10 = make_double2(-l10.x * i00 * i11, -l10.y * i00 * i11);
                const double2 i21 = make_double2(-l21.x * i11 * i22, -l21.y * i11 * i22);
                const double2 s20 = make_double2(l20.x * i00 + (l21.x * i10.x - l21.y * i10.y),
                                                 l20.y * i00 + (l21.x * i10.y + l21.y * i10.x));
                const double2 i20 = make_double2(-s20.x * i22, -s20.y * i22);
                out[0] = make_double2(i00, 0.0);
                out[1] = i10;
                out[2] = make_double2(i11, 0.0);
                out[3] = i20;
                out[4] = i21;
                out[5] = make_double2(i22, 0.0);
            }
#pragma unroll
            for (int i = 0; i < 6; ++i) Lf[i] = out[i];
        }
    }
    if (sigf != nullptr)
        for (int k = tid; k < M; k += NT) sigf[k] = ok ? sig[perm[k]] : 0.0f;
    if (Uf != nullptr)                                     // all M sorted columns (identity if failed)
        for (int e = tid; e < M * MP; e += NT) {
            const int c = e / MP, r = e % MP;
            if (r < M)
                Uf[c * M + r] = ok ? X[at<MP>(perm[c], r)] : make_float2(r == c ? 1.f : 0.f, 0.f);
        }
    if (tid == 0) {
        if (stf != nullptr) *stf = st;
        if (convf != nullptr) {
            convf[0] = sweeps;
            convf[1] = rot_total;
            convf[2] = rank_s;
        }
    }
}

// one workgroup per bin of one block
template <int MP, int G>
__global__ __launch_bounds__((JacobiCfg<MP, G>::THREADS)) void jacobi_svd(
    float2 *__restrict__ A, const int32_t *__restrict__ kstatus, int M, int Ns, int max_sweeps,
    float2 *__restrict__ En, float *__restrict__ sigma, int32_t *__restrict__ bin_status,
    int32_t *__restrict__ conv, float2 *__restrict__ U, int sub_full, float2 *__restrict__ Es,
    double2 *__restrict__ Esl)
{
    const int f = blockIdx.x;
    jacobi_bin<MP, G>(A + (size_t)f * M * M, kstatus ? kstatus[f] : SSL_BIN_OK, M, Ns, max_sweeps,
                      En ? En + (size_t)f * (M - Ns) * M : nullptr,
                      sigma ? sigma + (size_t)f * M : nullptr,
                      bin_status ? bin_status + f : nullptr, conv ? conv + 3 * f : nullptr,
                      U ? U + (size_t)f * M * M : nullptr, sub_full,
                      Es ? Es + (size_t)f * Ns * M : nullptr, Esl ? Esl + 6 * (size_t)f : nullptr);
}

// Persistent: a fixed grid of workgroups draws (block, bin) items from a device counter until the
// list is exhausted, so bins that converge in fewer sweeps free their CU for the next item.  Every
// workgroup draws exactly one ticket >= n_items; the one drawing the last ticket re-arms the
// counter to 0 for the next launch.
template <int MP, int G>
__global__ __launch_bounds__((JacobiCfg<MP, G>::THREADS))
__attribute__((amdgpu_waves_per_eu(JacobiCfg<MP, G>::WAVES_PER_EU))) void jacobi_persistent(
    const BlockDev *__restrict__ blk, const int2 *__restrict__ items, int n_items,
    int max_sweeps, unsigned int *__restrict__ queue, int sub_full)
{
    __shared__ int item_s;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned int t = atomicAdd(queue, 1u);
            item_s = (int)t;
            if (t == (unsigned int)n_items + gridDim.x - 1u) atomicExch(queue, 0u);
        }
        __syncthreads();
        const int it = item_s;
        if (it >= n_items) break;
        const int2 w = items[it];
        const BlockDev &B = blk[w.x];
        const int f = w.y, M = B.M, Ns = B.Ns;
        jacobi_bin<MP, G>(B.A + (size_t)f * M * M, B.kstatus ? B.kstatus[f] : SSL_BIN_OK, M, Ns,
                          max_sweeps, B.En ? B.En + (size_t)f * (M - Ns) * M : nullptr,
                          nullptr, B.status + f, B.conv ? B.conv + 3 * (size_t)f : nullptr,
                          nullptr, B.p == 2 ? sub_full : -1,
                          B.Es ? B.Es + (size_t)f * Ns * M : nullptr,
                          B.Esl ? B.Esl + 6 * (size_t)f : nullptr);
    }
}

// Warm-started solve for a stream of windows whose A changes little from one call to the next
// (the sliding correlation of eq.3, one frame in and one out): U0 = the previous solve's sorted
// left singular vectors.  Y = A^H U0 has nearly orthogonal columns when U0 is close to A's left
// singular vectors; one-sided Jacobi on Y from the right, Y V = Z with orthogonal columns,
// applying the same rotations to U = U0 V, gives A^H U = Z: U's columns are left singular vectors
// of A with sigma_k = |z_k|.  A few sweeps replace the two preconditioning QRs and the cold
// sweeps.  No rank truncation: columns of Y in A's null space are rounding-level and are only
// rotated among themselves or by negligible angles, so they stay inside the noise subspace.
// LDS: Y and U, both MP x MP complex64 column-major (64 KB at MP = 64).  Same pair test and
// rotation as the cold sweeps (jacobi_pair), on both matrices.
template <int MP, int G, int NR>
__device__ __forceinline__ bool warm_pair(float2 *Ys, float2 *Us, int ci, int cj, int q,
                                          double tol2)
{
    float2 bi[NR], bj[NR], ui[NR], uj[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const int r = q + G * k;
        bi[k] = Ys[at<MP>(ci, r)];
        bj[k] = Ys[at<MP>(cj, r)];
        ui[k] = Us[at<MP>(ci, r)];
        uj[k] = Us[at<MP>(cj, r)];
    }
    __builtin_amdgcn_sched_barrier(0);            // every read in flight before the products
    float al = 0.f, be = 0.f, gr = 0.f, gi = 0.f;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        al = fmaf(bi[k].x, bi[k].x, fmaf(bi[k].y, bi[k].y, al));
        be = fmaf(bj[k].x, bj[k].x, fmaf(bj[k].y, bj[k].y, be));
        gr = fmaf(bi[k].x, bj[k].x, fmaf(bi[k].y, bj[k].y, gr));
        gi = fmaf(bi[k].x, bj[k].y, fmaf(-bi[k].y, bj[k].x, gi));
    }
    al = group_sum<G>(al);
    be = group_sum<G>(be);
    gr = group_sum<G>(gr);
    gi = group_sum<G>(gi);
    const double g2 = (double)gr * gr + (double)gi * gi;
    const double ab = (double)al * be;
    if (!(g2 > tol2 * ab && ab > 0.0)) return false;
    const float g2f = (float)g2;
    float rg;
    if (g2f >= 1e-36f) {
        rg = __builtin_amdgcn_rsqf(g2f);
    } else {
        const float ax = fabsf(gr), ay = fabsf(gi);
        const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
        const float rt = mn * __builtin_amdgcn_rcpf(mx);
        rg = __builtin_amdgcn_rcpf(mx * __builtin_amdgcn_sqrtf(fmaf(rt, rt, 1.0f)));
    }
    const float zeta = (be - al) * 0.5f * rg;
    const float az = fminf(fabsf(zeta), 1e18f);
    float t = __builtin_amdgcn_rcpf(az + __builtin_amdgcn_sqrtf(fmaf(az, az, 1.0f)));
    t = copysignf(t, zeta);
    const float c = rsqrt_refined(fmaf(t, t, 1.0f));
    const float s = c * t;
    const float wr = s * gr * rg;
    const float wi = -s * gi * rg;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const int r = q + G * k;
        float2 x = bi[k], y = bj[k];
        Ys[at<MP>(ci, r)] = make_float2(fmaf(c, x.x, -fmaf(wr, y.x, -wi * y.y)),
                                        fmaf(c, x.y, -fmaf(wr, y.y, wi * y.x)));
        Ys[at<MP>(cj, r)] = make_float2(fmaf(c, y.x, fmaf(wr, x.x, wi * x.y)),
                                        fmaf(c, y.y, fmaf(wr, x.y, -wi * x.x)));
        x = ui[k];
        y = uj[k];
        Us[at<MP>(ci, r)] = make_float2(fmaf(c, x.x, -fmaf(wr, y.x, -wi * y.y)),
                                        fmaf(c, x.y, -fmaf(wr, y.y, wi * y.x)));
        Us[at<MP>(cj, r)] = make_float2(fmaf(c, y.x, fmaf(wr, x.x, wi * x.y)),
                                        fmaf(c, y.y, fmaf(wr, x.y, -wi * x.x)));
    }
    return true;
}

template <int MP, int G>
__global__ __launch_bounds__((JacobiCfg<MP, G>::THREADS)) void jacobi_warm(
    const float2 *__restrict__ Aall, const int32_t *__restrict__ kstatus, int M, int Ns,
    int max_sweeps, float2 *__restrict__ Uall, float2 *__restrict__ Enall,
    int32_t *__restrict__ status, int32_t *__restrict__ conv)
{
    typedef JacobiCfg<MP, G> C;
    constexpr int R = C::R;
    constexpr int NT = C::THREADS;
    constexpr int NG = C::NG;
    static_assert((MP / 4) * (MP / 4) <= NT, "one 4 x 4 tile of Y per thread");
    __shared__ float2 Ys[MP * MP];      // A (column-major), then Y = A^H U0, then Z
    __shared__ float2 Us[MP * MP];      // U0, then U = U0 V
    __shared__ float sig[MP];
    __shared__ int perm[MP];
    __shared__ int flag;
    __shared__ float amax_s;
    __shared__ int rot_total;

    const int f = blockIdx.x;
    const float2 *Af = Aall + (size_t)f * M * M;
    float2 *Uf = Uall + (size_t)f * M * M;
    float2 *Enf = Enall + (size_t)f * (M - Ns) * M;
    const int tid = threadIdx.x;
    const int g = tid / G;
    const int q = tid % G;
    const int Nn = M - Ns;

    if (tid == 0) {
        flag = kstatus ? kstatus[f] : SSL_BIN_OK;
        amax_s = 0.0f;
        rot_total = 0;
    }
    // A column-major (entry (i, j) at column j, row i) and U0; zero padding
    float amax = 0.0f;
    bool nonfinite = false;
    for (int e = tid; e < MP * MP; e += NT) {
        const int i = e / MP, j = e - i * MP;           // read row-major A: coalesced
        float2 a = make_float2(0.f, 0.f);
        if (i < M && j < M) {
            a = Af[(size_t)i * M + j];
            if (!finite2(a)) nonfinite = true;
            amax = fmaxf(amax, fmaxf(fabsf(a.x), fabsf(a.y)));
        }
        Ys[at<MP>(j, i)] = a;
        const int c = e / MP, r = e - c * MP;           // U0 column-major: coalesced
        Us[at<MP>(c, r)] = (c < M && r < M) ? Uf[(size_t)c * M + r] : make_float2(0.f, 0.f);
    }
    const int nf_count = __syncthreads_count(nonfinite ? 1 : 0);
    if (!nonfinite && amax > 0.0f) atomicMax((int *)&amax_s, __float_as_int(amax));
    __syncthreads();
    if (tid == 0 && nf_count > 0 && flag == SSL_BIN_OK) flag = SSL_BIN_NONFINITE;
    __syncthreads();

    int sweeps = 0;
    bool converged = false;
    if (flag == SSL_BIN_OK) {
        // Y = 2^-ex A^H U0 (the power of two keeps every Gram entry far from FP32 overflow); one
        // 4 x 4 tile of Y per thread, kept in registers until every thread has read A
        int ex = 0;
        if (amax_s > 0.0f) frexpf(amax_s, &ex);
        const float sc = ldexpf(1.0f, -ex);
        constexpr int TB = MP / 4;
        const int ti = tid / TB, tk = tid - ti * TB;   // rows 4 ti.., columns 4 tk..
        float2 acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = make_float2(0.f, 0.f);
        if (tid < TB * TB) {
            for (int j = 0; j < M; ++j) {
                float2 av[4], uv[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) av[a] = Ys[at<MP>(4 * ti + a, j)];   // A[j][i]
#pragma unroll
                for (int b = 0; b < 4; ++b) uv[b] = Us[at<MP>(4 * tk + b, j)];   // U0[j][k]
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) {     // conj(A[j][i]) U0[j][k]
                        acc[a][b].x = fmaf(av[a].x, uv[b].x, fmaf(av[a].y, uv[b].y, acc[a][b].x));
                        acc[a][b].y = fmaf(av[a].x, uv[b].y, fmaf(-av[a].y, uv[b].x, acc[a][b].y));
                    }
            }
        }
        __syncthreads();
        if (tid < TB * TB) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    Ys[at<MP>(4 * tk + b, 4 * ti + a)] =
                        make_float2(acc[a][b].x * sc, acc[a][b].y * sc);
        }
        __syncthreads();

        const int Me = M + (M & 1);
        const double tol = 2.0 * sqrt((double)M) * 5.9604644775390625e-08;
        const double tol2 = tol * tol;
        const int P = Me / 2;
        int my_rot = 0;
        for (int sw = 0; sw < max_sweeps; ++sw) {
            int rotated = 0;
            for (int rd = 0; rd < Me - 1; ++rd) {
                if (g < P && g < NG) {
                    int a, b;
                    if (g == 0) {
                        a = Me - 1;
                        b = rd;
                    } else {
                        a = rd + g;
                        if (a >= Me - 1) a -= Me - 1;
                        b = rd - g;
                        if (b < 0) b += Me - 1;
                    }
                    const int ci = min(a, b), cj = max(a, b);
                    if (cj < M && warm_pair<MP, G, R>(Ys, Us, ci, cj, q, tol2)) {
                        rotated = 1;
                        if (q == 0) ++my_rot;
                    }
                }
                __syncthreads();
            }
            ++sweeps;
            if (__syncthreads_count(rotated) == 0) {
                converged = true;
                break;
            }
        }
        if (my_rot) atomicAdd(&rot_total, my_rot);
        // sigma_c = |z_c| and the stable descending rank (ties: lower column first)
        for (int c = g; c < M && g < NG; c += NG) {
            float s2 = 0.f;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const float2 v = Ys[at<MP>(c, q + G * k)];
                s2 = fmaf(v.x, v.x, fmaf(v.y, v.y, s2));
            }
            s2 = group_sum<G>(s2);
            if (q == 0) sig[c] = sqrtf(s2);
        }
        __syncthreads();
        for (int c = tid; c < M; c += NT) {
            const float sc_ = sig[c];
            int rank = 0;
            for (int k = 0; k < M; ++k) {
                const float sk = sig[k];
                rank += (sk > sc_ || (sk == sc_ && k < c)) ? 1 : 0;
            }
            perm[rank] = c;
        }
        __syncthreads();
    }
    const bool ok = (flag == SSL_BIN_OK) && converged;
    const int st = (flag != SSL_BIN_OK) ? flag : (converged ? SSL_BIN_OK : SSL_BIN_NO_CONV);
    for (int e = tid; e < Nn * MP; e += NT) {
        const int c = e / MP, r = e % MP;
        if (r < M) Enf[c * M + r] = ok ? Us[at<MP>(perm[Ns + c], r)] : make_float2(0.f, 0.f);
    }
    for (int e = tid; e < M * MP; e += NT) {          // next start: sorted U (identity if failed)
        const int c = e / MP, r = e % MP;
        if (r < M)
            Uf[c * M + r] = ok ? Us[at<MP>(perm[c], r)] : make_float2(r == c ? 1.f : 0.f, 0.f);
    }
    if (tid == 0) {
        if (status) status[f] = st;
        if (conv) {
            conv[3 * f] = sweeps;
            conv[3 * f + 1] = rot_total;
            conv[3 * f + 2] = M;
        }
    }
}

template <int MP, int G>
hipError_t launch_cfg(ssl_c64 *A, const int32_t *kstatus, int F, int M, int Ns, int max_sweeps,
                      ssl_c64 *En, float *sigma, int32_t *bin_status, int32_t *conv, ssl_c64 *U,
                      int sub_full, ssl_c64 *Es, ssl_c128 *Esl, hipStream_t st)
{
    hipLaunchKernelGGL((jacobi_svd<MP, G>), dim3(F), dim3(JacobiCfg<MP, G>::THREADS), 0, st,
                       reinterpret_cast<float2 *>(A), kstatus, M, Ns, max_sweeps,
                       reinterpret_cast<float2 *>(En), sigma, bin_status, conv,
                       reinterpret_cast<float2 *>(U), sub_full, reinterpret_cast<float2 *>(Es),
                       reinterpret_cast<double2 *>(Esl));
    return hipGetLastError();
}

template <int MP, int G>
hipError_t launch_persistent(const BlockDev *blk, const int2 *items, int n_items, int max_sweeps,
                             unsigned int *queue, int grid, int sub_full, hipStream_t st)
{
    hipLaunchKernelGGL((jacobi_persistent<MP, G>), dim3(grid), dim3(JacobiCfg<MP, G>::THREADS), 0,
                       st, blk, items, n_items, max_sweeps, queue, sub_full);
    return hipGetLastError();
}

// Calls fn.template operator()<MP, G>() for the (class, lanes) variant; false if not compiled.
template <class Fn>
bool dispatch(int cls, int lanes, Fn &&fn)
{
    switch (cls) {
    case 8:
        if (lanes == 4) return fn.template operator()<8, 4>(), true;
        if (lanes == 8) return fn.template operator()<8, 8>(), true;
        return false;
    case 16:
        if (lanes == 4) return fn.template operator()<16, 4>(), true;
        if (lanes == 8) return fn.template operator()<16, 8>(), true;
        if (lanes == 16) return fn.template operator()<16, 16>(), true;
        return false;
    case 32:
        if (lanes == 8) return fn.template operator()<32, 8>(), true;
        if (lanes == 16) return fn.template operator()<32, 16>(), true;
        return false;
    default:
        if (lanes == 4) return fn.template operator()<64, 4>(), true;
        if (lanes == 8) return fn.template operator()<64, 8>(), true;
        if (lanes == 16) return fn.template operator()<64, 16>(), true;
        return false;
    }
}

}  // namespace

bool jacobi_variant_ok(int cls, int lanes)
{
    return dispatch(cls, lanes, [&]<int MP, int G>() {});
}

int jacobi_threads(int cls, int lanes)
{
    int t = 0;
    dispatch(cls, lanes, [&]<int MP, int G>() { t = JacobiCfg<MP, G>::THREADS; });
    return t;
}

int jacobi_persistent_wg_per_cu(int cls, int lanes)
{
    // resident workgroups per CU of the persistent variant (LDS and registers decide), cached
    static std::atomic<int> cache[4][3];
    const int ci = cls == 8 ? 0 : cls == 16 ? 1 : cls == 32 ? 2 : 3;
    const int li = lanes == 4 ? 0 : lanes == 8 ? 1 : 2;
    int n = cache[ci][li].load(std::memory_order_relaxed);
    if (n > 0) return n;
    dispatch(cls, lanes, [&]<int MP, int G>() {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, jacobi_persistent<MP, G>,
                                                         JacobiCfg<MP, G>::THREADS, 0) != hipSuccess)
            n = 0;
    });
    if (n <= 0) return 1;
    cache[ci][li].store(n, std::memory_order_relaxed);
    return n;
}

hipError_t launch_jacobi(ssl_c64 *A, const int32_t *kstatus, int F, int M, int Ns, int max_sweeps,
                         int lanes, ssl_c64 *En, float *sigma, int32_t *bin_status, int32_t *conv,
                         hipStream_t st, ssl_c64 *U, int sub_full, ssl_c64 *Es, ssl_c128 *Esl)
{
    hipError_t e = hipErrorInvalidValue;
    dispatch(jacobi_class(M), lanes, [&]<int MP, int G>() {
        e = launch_cfg<MP, G>(A, kstatus, F, M, Ns, max_sweeps, En, sigma, bin_status, conv, U,
                              sub_full, Es, Esl, st);
    });
    return e;
}

hipError_t launch_jacobi_warm(const ssl_c64 *A, const int32_t *kstatus, int F, int M, int Ns,
                              int max_sweeps, ssl_c64 *U, ssl_c64 *En, int32_t *bin_status,
                              int32_t *conv, hipStream_t st)
{
    const float2 *a = reinterpret_cast<const float2 *>(A);
    float2 *u = reinterpret_cast<float2 *>(U), *en = reinterpret_cast<float2 *>(En);
    switch (jacobi_class(M)) {
    case 8:
        hipLaunchKernelGGL((jacobi_warm<8, 8>), dim3(F), dim3(JacobiCfg<8, 8>::THREADS), 0, st, a,
                           kstatus, M, Ns, max_sweeps, u, en, bin_status, conv);
        break;
    case 16:
        hipLaunchKernelGGL((jacobi_warm<16, 8>), dim3(F), dim3(JacobiCfg<16, 8>::THREADS), 0, st,
                           a, kstatus, M, Ns, max_sweeps, u, en, bin_status, conv);
        break;
    case 32:
        hipLaunchKernelGGL((jacobi_warm<32, 8>), dim3(F), dim3(JacobiCfg<32, 8>::THREADS), 0, st,
                           a, kstatus, M, Ns, max_sweeps, u, en, bin_status, conv);
        break;
    default:
        hipLaunchKernelGGL((jacobi_warm<64, 8>), dim3(F), dim3(JacobiCfg<64, 8>::THREADS), 0, st,
                           a, kstatus, M, Ns, max_sweeps, u, en, bin_status, conv);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_jacobi_batch(const BlockDev *blk, const int2 *items, int n_items, int cls,
                               int lanes, int max_sweeps, unsigned int *queue, int grid,
                               hipStream_t st, int sub_full)
{
    if (n_items <= 0) return hipSuccess;
    hipError_t e = hipErrorInvalidValue;
    dispatch(cls, lanes, [&]<int MP, int G>() {
        e = launch_persistent<MP, G>(blk, items, n_items, max_sweeps, queue, grid, sub_full, st);
    });
    return e;
}
