// The SVD of A = K^{-1} R (eq.4) by the paper's own method (Sec. III-B, the Householder / QR
// category; its steps SVD1..SVD6), as a second backend beside the one-sided Jacobi:
//   SVD1  A = Q_L B Q_R^H by alternating Householder reflectors (left ones zero a column below
//         the diagonal, right ones a row right of the superdiagonal), then the phase transform
//         B = D_L B' D_R^H with D_L, D_R diagonal unitary and B' real, non-negative bidiagonal;
//   SVD2  tolerance from the largest |d_k| + |e_k| over the columns of B';
//   SVD3  left singular vectors of B' start as the identity;
//   SVD4  implicit-shift QR iterations (Golub-Kahan steps with a Wilkinson shift from the trailing
//         2 x 2 of B'^T B', and the zero-diagonal chase) until every superdiagonal entry is below
//         the tolerance, the left rotations accumulated into U';
//   SVD5  singular values |d_k| sorted descending (ties: lower index first);
//   SVD6  back-transformation E = Q_L D_L U' of the sorted columns; E_n = columns Ns..M-1.
// Only left singular vectors are needed, so the right reflectors and rotations are applied to A
// and B' but never accumulated.
//
// GPU mapping (gfx950): one workgroup per bin, A column-major in LDS (32 KB at MP = 64, the left
// reflectors stay below its diagonal).  Reflector steps: a left reflector is applied by lane
// groups of G lanes owning one column each (DPP reductions), a right reflector by lane groups
// owning one row each; two barriers per k.  QR iterations: thread 0 runs the scalar bulge chase
// of one step and posts its left rotations; every thread then applies them to its row of U'
// (one barrier per step).  Back-transformation: lane groups own output columns and take them
// through every reflector in registers.  FP32 throughout, as the Jacobi backend.
#include "ssl_internal.h"

namespace {

template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Sum over aligned groups of G lanes (G = 4 or 8); every lane of a group gets the same bits.
template <int G>
__device__ __forceinline__ float gsum(float v)
{
    v += dpp<0xB1>(v);                    // quad_perm [1,0,3,2]
    v += dpp<0x4E>(v);                    // quad_perm [2,3,0,1]
    if (G >= 8) v += dpp<0x141>(v);       // row_half_mirror
    return v;
}

__device__ __forceinline__ bool finite2(float2 v) { return isfinite(v.x) && isfinite(v.y); }

// sqrt(a^2 + b^2) without overflow or underflow of the squares
__device__ __forceinline__ float hyp(float a, float b)
{
    a = fabsf(a);
    b = fabsf(b);
    const float m = fmaxf(a, b), n = fminf(a, b);
    if (m == 0.0f) return 0.0f;
    const float r = n / m;
    return m * sqrtf(fmaf(r, r, 1.0f));
}

template <int MP>
struct GkCfg {
    static constexpr int G = MP >= 16 ? 4 : 8;           // lanes per column (or row)
    static constexpr int R = (MP + G - 1) / G;           // rows (or columns) per lane
    static constexpr int THREADS = MP * G < 64 ? 64 : MP * G;
};

// Householder vector of x (length n, x_0 = x0, |x|^2 = nrm2): H = I - tau v v^H (tau real, H
// Hermitian and unitary) with H x = alpha e_1, alpha = -e^{i arg x0} |x|; v = x - alpha e_1, so
// v_0 = e^{i arg x0} (|x0| + |x|) and v_r = x_r beyond.  A zero x gives tau = 0 (H = I).
__device__ __forceinline__ void householder(float2 x0, float nrm2, float2 &alpha, float2 &v0,
                                            float &tau)
{
    const float nx = sqrtf(nrm2);
    const float ax = hyp(x0.x, x0.y);
    const float2 ph = ax > 0.f ? make_float2(x0.x / ax, x0.y / ax) : make_float2(1.f, 0.f);
    alpha = make_float2(-ph.x * nx, -ph.y * nx);
    v0 = make_float2(ph.x * (ax + nx), ph.y * (ax + nx));
    tau = nx > 0.f ? 1.0f / (nx * (nx + ax)) : 0.0f;
}

// One bin.  Af: A row-major M x M (read only); Enf: [M-Ns][M] out; sigf [M] / stf / convf
// (iterations, QR steps, zero-diagonal chases) or null.
template <int MP>
__device__ __forceinline__ void gk_bin(const float2 *__restrict__ Af, int kst, int M, int Ns,
                                       int max_steps, float2 *__restrict__ Enf,
                                       float *__restrict__ sigf, int32_t *__restrict__ stf,
                                       int32_t *__restrict__ convf)
{
    typedef GkCfg<MP> C;
    constexpr int G = C::G, R = C::R, NT = C::THREADS;
    __shared__ float2 X[MP * MP];          // A column-major; left reflector k below X[k][k]
    __shared__ float Ut[MP * MP];          // U' row-major: row t at t*MP (thread t's row)
    __shared__ float2 dcx[MP], ecx[MP];    // complex bidiagonal: d_k, e_k = B[k][k+1]
    __shared__ float2 vhead[MP];           // v_0 of left reflector k
    __shared__ float tau[MP];
    __shared__ float2 lph[MP];             // D_L
    __shared__ float d[MP], e[MP];         // real bidiagonal B'
    __shared__ float rc[MP], rs[MP];       // rotations of one step: columns (ri[k], rj[k])
    __shared__ int ri[MP], rj[MP];
    __shared__ int nrot, done, flag;
    __shared__ float amax_s, sig[MP];
    __shared__ int perm[MP];
    __shared__ int steps_s, chases_s;

    const int tid = threadIdx.x;
    const int g = tid / G, q = tid % G;
    const int Nn = M - Ns;
    if (tid == 0) {
        flag = kst;
        amax_s = 0.0f;
        steps_s = 0;
        chases_s = 0;
    }
    float amax = 0.0f;
    bool nonfinite = false;
    for (int el = tid; el < MP * MP; el += NT) {
        const int r = el / MP, c = el - r * MP;          // row-major read: coalesced
        float2 a = make_float2(0.f, 0.f);
        if (r < M && c < M) {
            a = Af[(size_t)r * M + c];
            if (!finite2(a)) nonfinite = true;
            amax = fmaxf(amax, fmaxf(fabsf(a.x), fabsf(a.y)));
        }
        X[c * MP + r] = a;
        Ut[el] = (r == c) ? 1.0f : 0.0f;
    }
    const int nf = __syncthreads_count(nonfinite ? 1 : 0);
    if (!nonfinite && amax > 0.0f) atomicMax((int *)&amax_s, __float_as_int(amax));
    __syncthreads();
    if (tid == 0 && nf > 0 && flag == SSL_BIN_OK) flag = SSL_BIN_NONFINITE;
    __syncthreads();
    bool converged = false;
    int ex = 0;
    if (flag == SSL_BIN_OK) {
        if (amax_s > 0.0f) frexpf(amax_s, &ex);
        const float sc = ldexpf(1.0f, -ex);             // exact: max |A_ij| in [0.5, 1)
        for (int el = tid; el < MP * MP; el += NT) {
            const float2 b = X[el];
            X[el] = make_float2(b.x * sc, b.y * sc);
        }
        __syncthreads();

        // ---- SVD1: bidiagonalisation ------------------------------------------------------------
        for (int k = 0; k < M; ++k) {
            // left reflector from column k, rows k..M-1 (every group forms it from the same reads)
            float2 alpha, v0;
            float tk;
            {
                float s2 = 0.f;
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const int r = q + G * j;
                    if (r >= k && r < M) {
                        const float2 x = X[k * MP + r];
                        s2 = fmaf(x.x, x.x, fmaf(x.y, x.y, s2));
                    }
                }
                s2 = gsum<G>(s2);
                householder(X[k * MP + k], s2, alpha, v0, tk);
            }
            if (k == M - 1) tk = 0.0f;                    // 1 x 1: keep the complex entry
            const int c = g;                              // this group's column
            if (tk > 0.0f && c > k && c < M) {
                float wr = 0.f, wi = 0.f;
                float2 xs[R], vs[R];
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const int r = q + G * j;
                    vs[j] = (r > k && r < M) ? X[k * MP + r] : (r == k ? v0 : make_float2(0.f, 0.f));
                    xs[j] = (r < M) ? X[c * MP + r] : make_float2(0.f, 0.f);
                    wr = fmaf(vs[j].x, xs[j].x, fmaf(vs[j].y, xs[j].y, wr));   // v^H x
                    wi = fmaf(vs[j].x, xs[j].y, fmaf(-vs[j].y, xs[j].x, wi));
                }
                wr = gsum<G>(wr) * tk;
                wi = gsum<G>(wi) * tk;
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const int r = q + G * j;
                    if (r >= k && r < M)                  // x -= v (tau w)
                        X[c * MP + r] = make_float2(fmaf(-vs[j].x, wr, fmaf(vs[j].y, wi, xs[j].x)),
                                                    fmaf(-vs[j].x, wi, fmaf(-vs[j].y, wr, xs[j].y)));
                }
            }
            if (tid == 0) {
                dcx[k] = (k == M - 1) ? X[k * MP + k] : alpha;
                vhead[k] = v0;
                tau[k] = tk;
            }
            __syncthreads();
            if (k >= M - 1) break;
            if (k == M - 2) {                             // e_{M-2}: nothing right of it to zero
                if (tid == 0) ecx[k] = X[(k + 1) * MP + k];
                __syncthreads();
                continue;
            }
            // right reflector from row k, columns k+1..M-1: H z = beta e_1 for z = conj(row), so
            // row H = conj(beta) e_1^T; applied to rows k+1..M-1 (one group per row)
            float2 beta, w0;
            float tr;
            {
                float s2 = 0.f;
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const int cc = q + G * j;
                    if (cc > k && cc < M) {
                        const float2 x = X[cc * MP + k];
                        s2 = fmaf(x.x, x.x, fmaf(x.y, x.y, s2));
                    }
                }
                s2 = gsum<G>(s2);
                const float2 z0 = X[(k + 1) * MP + k];
                householder(make_float2(z0.x, -z0.y), s2, beta, w0, tr);
            }
            const int rrow = g;                           // this group's row
            if (tr > 0.0f && rrow > k && rrow < M) {
                // s = sum_c A[row][c] w_c, w_c = conj(A[k][c]) (c > k+1), w_{k+1} = w0
                float sr = 0.f, si = 0.f;
                float2 as[R], ws[R];
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const int cc = q + G * j;
                    float2 wv = make_float2(0.f, 0.f);
                    if (cc == k + 1) {
                        wv = w0;
                    } else if (cc > k + 1 && cc < M) {
                        const float2 t = X[cc * MP + k];
                        wv = make_float2(t.x, -t.y);
                    }
                    ws[j] = wv;
                    as[j] = (cc > k && cc < M) ? X[cc * MP + rrow] : make_float2(0.f, 0.f);
                    sr = fmaf(as[j].x, wv.x, fmaf(-as[j].y, wv.y, sr));        // a w
                    si = fmaf(as[j].x, wv.y, fmaf(as[j].y, wv.x, si));
                }
                sr = gsum<G>(sr) * tr;
                si = gsum<G>(si) * tr;
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const int cc = q + G * j;
                    if (cc > k && cc < M)                 // a -= (tau s) conj(w)
                        X[cc * MP + rrow] =
                            make_float2(as[j].x - fmaf(sr, ws[j].x, si * ws[j].y),
                                        as[j].y - fmaf(si, ws[j].x, -sr * ws[j].y));
                }
            }
            if (tid == 0) ecx[k] = make_float2(beta.x, -beta.y);
            __syncthreads();
        }

        // ---- phase transform: B' = D_L^H B D_R real and non-negative --------------------------
        if (tid == 0) {
            float2 rk = make_float2(1.f, 0.f);           // D_R[k]
            for (int k = 0; k < M; ++k) {
                const float2 dk = dcx[k];
                const float2 t = make_float2(dk.x * rk.x - dk.y * rk.y, dk.x * rk.y + dk.y * rk.x);
                const float at = hyp(t.x, t.y);
                const float2 l = at > 0.f ? make_float2(t.x / at, t.y / at) : make_float2(1.f, 0.f);
                lph[k] = l;
                d[k] = at;
                if (k < M - 1) {
                    const float2 ek = ecx[k];            // u = conj(l) e_k r_{k+1}; r_{k+1} = conj(u0)/|u0|
                    const float2 u0 = make_float2(l.x * ek.x + l.y * ek.y, l.x * ek.y - l.y * ek.x);
                    const float au = hyp(u0.x, u0.y);
                    rk = au > 0.f ? make_float2(u0.x / au, -u0.y / au) : make_float2(1.f, 0.f);
                    e[k] = au;
                }
            }
            e[M - 1] = 0.0f;
            done = 0;
        }
        __syncthreads();

        // ---- SVD2..SVD4: implicit-shift QR on B', left rotations into U' -----------------------
        float anorm = 0.f;
        for (int k = 0; k < M; ++k) anorm = fmaxf(anorm, d[k] + e[k]);
        const float tol = (float)M * 5.9604644775390625e-08f * anorm;
        int steps = 0;
        for (;;) {
            if (tid == 0) {
                nrot = 0;
                for (int k = 0; k + 1 < M; ++k)
                    if (fabsf(e[k]) <= tol) e[k] = 0.0f;
                int hi = M - 1;
                while (hi > 0 && e[hi - 1] == 0.0f) --hi;
                if (hi == 0) {
                    done = 1;
                } else if (steps >= max_steps) {
                    done = 2;
                } else {
                    int lo = hi - 1;
                    while (lo > 0 && e[lo - 1] != 0.0f) --lo;
                    int zi = -1;                          // a negligible diagonal entry above hi
                    for (int k = lo; k < hi; ++k)
                        if (fabsf(d[k]) <= tol) {
                            zi = k;
                            break;
                        }
                    if (fabsf(d[hi]) <= tol) {
                        // zero column hi: chase e_{hi-1} up with right rotations on columns
                        // (j, hi), j = hi-1..lo (right rotations: nothing to accumulate)
                        d[hi] = 0.0f;
                        float x = e[hi - 1];
                        e[hi - 1] = 0.0f;
                        for (int j = hi - 1; j >= lo && x != 0.0f; --j) {
                            const float rr = hyp(d[j], x);
                            const float cs = d[j] / rr, sn = x / rr;
                            d[j] = rr;
                            if (j > lo) {
                                x = -sn * e[j - 1];
                                e[j - 1] = cs * e[j - 1];
                            }
                        }
                        ++chases_s;
                    } else if (zi >= 0) {
                        // zero row zi: chase its superdiagonal entry right with left rotations
                        // (rows zi, j), j = zi+1..hi, each fixing d_j
                        d[zi] = 0.0f;
                        float x = e[zi];
                        e[zi] = 0.0f;
                        int n = 0;
                        for (int j = zi + 1; j <= hi && x != 0.0f; ++j) {
                            const float rr = hyp(d[j], x);
                            const float cs = d[j] / rr, sn = x / rr;
                            d[j] = rr;
                            ri[n] = zi;
                            rj[n] = j;
                            rc[n] = cs;                   // row zi <- c row zi - s row j
                            rs[n] = -sn;                  // row j  <- s row zi + c row j
                            ++n;
                            if (j < hi) {
                                x = -sn * e[j];
                                e[j] = cs * e[j];
                            }
                        }
                        nrot = n;
                        ++chases_s;
                    } else {
                        // Golub-Kahan step on [lo, hi], Wilkinson shift from the trailing 2 x 2
                        // of B'^T B'
                        const float dm = d[hi - 1], dn = d[hi], em = e[hi - 1];
                        const float ep = hi - 1 > lo ? e[hi - 2] : 0.0f;
                        const float t11 = fmaf(dm, dm, ep * ep), t22 = fmaf(dn, dn, em * em);
                        const float t12 = dm * em;
                        const float dl = 0.5f * (t11 - t22);
                        const float den = dl + copysignf(hyp(dl, t12), dl);
                        const float mu = den != 0.0f ? t22 - t12 * t12 / den : t22;
                        float y = fmaf(d[lo], d[lo], -mu), z = d[lo] * e[lo];
                        int n = 0;
                        for (int k = lo; k < hi; ++k) {
                            // right rotation on columns k, k+1 (not accumulated)
                            float rr = hyp(y, z);
                            float cs = rr > 0.f ? y / rr : 1.0f, sn = rr > 0.f ? z / rr : 0.0f;
                            if (k > lo) e[k - 1] = rr;
                            const float dk = d[k], ek = e[k], dk1 = d[k + 1];
                            y = fmaf(cs, dk, sn * ek);
                            e[k] = fmaf(-sn, dk, cs * ek);
                            z = sn * dk1;
                            d[k + 1] = cs * dk1;
                            // left rotation on rows k, k+1, zeroing the bulge z
                            rr = hyp(y, z);
                            cs = rr > 0.f ? y / rr : 1.0f;
                            sn = rr > 0.f ? z / rr : 0.0f;
                            d[k] = rr;
                            const float ek2 = e[k], dk2 = d[k + 1];
                            e[k] = fmaf(cs, ek2, sn * dk2);
                            d[k + 1] = fmaf(-sn, ek2, cs * dk2);
                            if (k + 1 < hi) {
                                y = e[k];
                                z = sn * e[k + 1];
                                e[k + 1] = cs * e[k + 1];
                            }
                            ri[n] = k;
                            rj[n] = k + 1;
                            rc[n] = cs;                   // U_k <- c U_k + s U_k+1
                            rs[n] = sn;                   // U_k+1 <- -s U_k + c U_k+1
                            ++n;
                        }
                        nrot = n;
                    }
                }
            }
            __syncthreads();
            if (done) break;
            ++steps;
            // U' <- U' G^T: thread t updates row t (columns ri, rj of each rotation, in order)
            const int n = nrot;
            if (tid < M) {
                float *u = Ut + tid * MP;
                for (int k = 0; k < n; ++k) {
                    const int a = ri[k], b = rj[k];
                    const float cs = rc[k], sn = rs[k];
                    const float ua = u[a], ub = u[b];
                    u[a] = fmaf(cs, ua, sn * ub);
                    u[b] = fmaf(-sn, ua, cs * ub);
                }
            }
            __syncthreads();
        }
        converged = done == 1;
        if (tid == 0) steps_s = steps;

        // ---- SVD5: sigma = |d_k| (a negative d_k flips its column of U'), sorted ---------------
        for (int k = tid; k < M; k += NT) sig[k] = fabsf(d[k]);
        if (tid < M)
            for (int k = 0; k < M; ++k)
                if (d[k] < 0.0f) Ut[tid * MP + k] = -Ut[tid * MP + k];
        __syncthreads();
        for (int c = tid; c < M; c += NT) {
            const float s0 = sig[c];
            int rank = 0;
            for (int k = 0; k < M; ++k) {
                const float sk = sig[k];
                rank += (sk > s0 || (sk == s0 && k < c)) ? 1 : 0;
            }
            perm[rank] = c;
        }
        __syncthreads();
    }

    // ---- SVD6: E_n columns = Q_L D_L U'[:, perm[Ns + c]], reflectors M-1 .. 0 -----------------
    const bool ok = flag == SSL_BIN_OK && converged;
    for (int c = g; c < Nn && g < MP; c += NT / G) {
        float2 x[R];
        const int src = ok ? perm[Ns + c] : 0;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int r = q + G * j;
            if (ok && r < M) {
                const float u = Ut[r * MP + src];
                x[j] = make_float2(lph[r].x * u, lph[r].y * u);
            } else {
                x[j] = make_float2(0.f, 0.f);
            }
        }
        if (ok)
            for (int k = M - 2; k >= 0; --k) {
                const float tk = tau[k];
                if (tk == 0.0f) continue;                 // uniform: read from LDS by all
                float wr = 0.f, wi = 0.f;
                float2 vs[R];
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const int r = q + G * j;
                    vs[j] = (r > k && r < M) ? X[k * MP + r] : (r == k ? vhead[k] : make_float2(0.f, 0.f));
                    wr = fmaf(vs[j].x, x[j].x, fmaf(vs[j].y, x[j].y, wr));
                    wi = fmaf(vs[j].x, x[j].y, fmaf(-vs[j].y, x[j].x, wi));
                }
                wr = gsum<G>(wr) * tk;
                wi = gsum<G>(wi) * tk;
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    x[j].x = fmaf(-vs[j].x, wr, fmaf(vs[j].y, wi, x[j].x));
                    x[j].y = fmaf(-vs[j].x, wi, fmaf(-vs[j].y, wr, x[j].y));
                }
            }
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int r = q + G * j;
            if (r < M) Enf[(size_t)c * M + r] = x[j];
        }
    }
    if (sigf)
        for (int k = tid; k < M; k += NT) sigf[k] = ok ? ldexpf(sig[perm[k]], ex) : 0.0f;
    if (tid == 0) {
        if (stf) *stf = flag != SSL_BIN_OK ? flag : (converged ? SSL_BIN_OK : SSL_BIN_NO_CONV);
        if (convf) {
            convf[0] = steps_s;
            convf[1] = chases_s;
            convf[2] = M;
        }
    }
}

template <int MP>
__global__ __launch_bounds__(GkCfg<MP>::THREADS) void gk_svd(const float2 *__restrict__ A,
                                                             const int32_t *__restrict__ kstatus,
                                                             int M, int Ns, int max_steps,
                                                             float2 *__restrict__ En,
                                                             float *__restrict__ sigma,
                                                             int32_t *__restrict__ status,
                                                             int32_t *__restrict__ conv)
{
    const int f = blockIdx.x;
    gk_bin<MP>(A + (size_t)f * M * M, kstatus ? kstatus[f] : SSL_BIN_OK, M, Ns, max_steps,
               En + (size_t)f * (M - Ns) * M, sigma ? sigma + (size_t)f * M : nullptr,
               status ? status + f : nullptr, conv ? conv + 3 * f : nullptr);
}

// batched: one workgroup per (block, bin) item of one size class
template <int MP>
__global__ __launch_bounds__(GkCfg<MP>::THREADS) void gk_svd_batch(const BlockDev *__restrict__ blk,
                                                                   const int2 *__restrict__ items,
                                                                   int max_steps)
{
    const int2 w = items[blockIdx.x];
    const BlockDev &B = blk[w.x];
    const int f = w.y, M = B.M, Ns = B.Ns;
    gk_bin<MP>(B.A + (size_t)f * M * M, B.kstatus ? B.kstatus[f] : SSL_BIN_OK, M, Ns, max_steps,
               B.En + (size_t)f * (M - Ns) * M, nullptr, B.status + f, nullptr);
}

}  // namespace

hipError_t launch_gk_svd(const ssl_c64 *A, const int32_t *kstatus, int F, int M, int Ns,
                         int max_steps, ssl_c64 *En, float *sigma, int32_t *bin_status,
                         int32_t *conv, hipStream_t st)
{
    const float2 *a = reinterpret_cast<const float2 *>(A);
    float2 *en = reinterpret_cast<float2 *>(En);
    switch (jacobi_class(M)) {
    case 8:
        hipLaunchKernelGGL((gk_svd<8>), dim3(F), dim3(GkCfg<8>::THREADS), 0, st, a, kstatus, M, Ns,
                           max_steps, en, sigma, bin_status, conv);
        break;
    case 16:
        hipLaunchKernelGGL((gk_svd<16>), dim3(F), dim3(GkCfg<16>::THREADS), 0, st, a, kstatus, M,
                           Ns, max_steps, en, sigma, bin_status, conv);
        break;
    case 32:
        hipLaunchKernelGGL((gk_svd<32>), dim3(F), dim3(GkCfg<32>::THREADS), 0, st, a, kstatus, M,
                           Ns, max_steps, en, sigma, bin_status, conv);
        break;
    default:
        hipLaunchKernelGGL((gk_svd<64>), dim3(F), dim3(GkCfg<64>::THREADS), 0, st, a, kstatus, M,
                           Ns, max_steps, en, sigma, bin_status, conv);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_gk_svd_batch(const BlockDev *blk, const int2 *items, int n_items, int cls,
                               int max_steps, hipStream_t st)
{
    if (n_items <= 0) return hipSuccess;
    switch (cls) {
    case 8:
        hipLaunchKernelGGL((gk_svd_batch<8>), dim3(n_items), dim3(GkCfg<8>::THREADS), 0, st, blk,
                           items, max_steps);
        break;
    case 16:
        hipLaunchKernelGGL((gk_svd_batch<16>), dim3(n_items), dim3(GkCfg<16>::THREADS), 0, st,
                           blk, items, max_steps);
        break;
    case 32:
        hipLaunchKernelGGL((gk_svd_batch<32>), dim3(n_items), dim3(GkCfg<32>::THREADS), 0, st,
                           blk, items, max_steps);
        break;
    default:
        hipLaunchKernelGGL((gk_svd_batch<64>), dim3(n_items), dim3(GkCfg<64>::THREADS), 0, st,
                           blk, items, max_steps);
        break;
    }
    return hipGetLastError();
}
