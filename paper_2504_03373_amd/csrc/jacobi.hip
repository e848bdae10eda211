// GSVD step of arXiv 2504.03373 eq.4: SVD of A = K^{-1} R per frequency bin and the noise subspace
// E_n = [e_{Ns+1} .. e_M] of its left singular vectors (the definition following eq.4).
//
// Method: one-sided (Hestenes) Jacobi -- the paper's "category 1" solver of Sec. III-B -- applied
// from the right to B = A^H with the rotations accumulated in J (J = I initially).  When the
// columns of B J are mutually orthogonal, A^H J = W with orthogonal columns, so A = J W^H: the
// left singular vectors of A are the columns of J (exactly unitary even for zero singular values)
// and sigma_i = |w_i|.
//
// GPU mapping (gfx950):
//  * one workgroup per bin; B and J (complex64, MP x MP, column-major) stay in LDS for the whole
//    solve -- 64 KB at MP = 64, two bins per CU;
//  * parallel (round-robin) ordering: each sweep is M'-1 rounds of M'/2 disjoint column pairs
//    (M' = M rounded up to even), one pair per group of G lanes, each lane owning MP/G rows;
//  * the pair's alpha = |b_i|^2, beta = |b_j|^2 and gamma = b_i^H b_j are reduced across the G
//    lanes with DPP butterflies (every lane ends with the same bits, so the rotation decision is
//    uniform in the group);
//  * convergence test in FP64: rotate iff |gamma|^2 > tol^2 alpha beta with tol = M 2^-24; a sweep
//    without any rotation ends the solve (a fixed point: a converged bin is never changed again);
//  * epilogue: sigma from the column norms, stable descending rank sort (ties: lower column
//    first), E_n = sorted columns Ns..M-1 of J, written column-major per bin.
#include "ssl_internal.h"

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

__device__ __forceinline__ bool finite2(float2 v) { return isfinite(v.x) && isfinite(v.y); }

template <int MP, int G>
struct JacobiCfg {
    static constexpr int R = MP / G;                       // rows per lane
    static constexpr int NG = MP / 2;                      // pair groups
    static constexpr int THREADS = ((NG * G + 63) / 64) * 64;
};

template <int MP, int G>
__global__ __launch_bounds__((JacobiCfg<MP, G>::THREADS)) void jacobi_svd(
    const float2 *__restrict__ A, const int32_t *__restrict__ kstatus, int M, int Ns,
    int max_sweeps, float2 *__restrict__ En, float *__restrict__ sigma,
    int32_t *__restrict__ bin_status, int32_t *__restrict__ conv)
{
    typedef JacobiCfg<MP, G> C;
    constexpr int R = C::R;
    constexpr int NT = C::THREADS;
    __shared__ float2 Bs[MP * MP];      // column c at c*MP
    __shared__ float2 Js[MP * MP];
    __shared__ float sig[MP];
    __shared__ int perm[MP];
    __shared__ int flag;                // non-finite input / upstream failure
    __shared__ float amax_s;
    __shared__ int rot_total;

    const int f = blockIdx.x;
    const int tid = threadIdx.x;
    const int g = tid / G;              // pair group
    const int q = tid % G;              // lane in group
    const int Nn = M - Ns;
    const float2 *Af = A + (size_t)f * M * M;

    if (tid == 0) {
        flag = (kstatus != nullptr && kstatus[f] != SSL_BIN_OK) ? kstatus[f] : SSL_BIN_OK;
        amax_s = 0.0f;
        rot_total = 0;
    }
    __syncthreads();

    // ---- load B = A^H (column c of B = conj of row c of A), J = I; padding stays zero --------
    float amax = 0.0f;
    bool nonfinite = false;
    for (int e = tid; e < MP * MP; e += NT) {
        const int c = e / MP, r = e - c * MP;
        float2 b = make_float2(0.f, 0.f);
        if (c < M && r < M) {
            const float2 a = Af[(size_t)c * M + r];
            if (!finite2(a)) nonfinite = true;
            b = make_float2(a.x, -a.y);
            amax = fmaxf(amax, fmaxf(fabsf(a.x), fabsf(a.y)));
        }
        Bs[e] = b;
        Js[e] = make_float2((c == r && c < M) ? 1.f : 0.f, 0.f);
    }
    // reduce the non-finite flag and the max magnitude over the block
    const int nf_count = __syncthreads_count(nonfinite ? 1 : 0);
    if (nonfinite == false && amax > 0.0f) atomicMax((int *)&amax_s, __float_as_int(amax));
    __syncthreads();
    if (tid == 0 && nf_count > 0 && flag == SSL_BIN_OK) flag = SSL_BIN_NONFINITE;
    __syncthreads();

    int sweeps = 0;
    bool converged = false;
    if (flag == SSL_BIN_OK) {
        // scale by a power of two so that max |A_ij| lies in [0.5, 1): exact, avoids FP32 overflow
        // of the Gram entries; singular values are scaled back at the end.
        const float am = amax_s;
        int ex = 0;
        if (am > 0.0f) frexpf(am, &ex);
        const float sc = ldexpf(1.0f, -ex);
        if (ex != 0) {
            for (int e = tid; e < MP * MP; e += NT) {
                float2 b = Bs[e];
                Bs[e] = make_float2(b.x * sc, b.y * sc);
            }
        }
        __syncthreads();

        const int Me = M + (M & 1);                  // players of the round-robin tournament
        const double tol = (double)M * 5.9604644775390625e-08;   // M * 2^-24
        const double tol2 = tol * tol;
        int my_rot = 0;
        for (int sw = 0; sw < max_sweeps; ++sw) {
            int rotated = 0;
            for (int rd = 0; rd < Me - 1; ++rd) {
                if (g < Me / 2) {
                    int a, b;
                    if (g == 0) {
                        a = Me - 1;
                        b = rd;
                    } else {
                        a = (rd + g) % (Me - 1);
                        b = (rd - g + (Me - 1)) % (Me - 1);
                    }
                    const int ci = min(a, b), cj = max(a, b);
                    if (cj < M) {
                        float2 bi[R], bj[R];
                        float al = 0.f, be = 0.f, gr = 0.f, gi = 0.f;
#pragma unroll
                        for (int k = 0; k < R; ++k) {
                            const int r = q + G * k;
                            bi[k] = Bs[ci * MP + r];
                            bj[k] = Bs[cj * MP + r];
                            al = fmaf(bi[k].x, bi[k].x, fmaf(bi[k].y, bi[k].y, al));
                            be = fmaf(bj[k].x, bj[k].x, fmaf(bj[k].y, bj[k].y, be));
                            // conj(b_i) * b_j
                            gr = fmaf(bi[k].x, bj[k].x, fmaf(bi[k].y, bj[k].y, gr));
                            gi = fmaf(bi[k].x, bj[k].y, fmaf(-bi[k].y, bj[k].x, gi));
                        }
                        al = group_sum<G>(al);
                        be = group_sum<G>(be);
                        gr = group_sum<G>(gr);
                        gi = group_sum<G>(gi);
                        const double g2 = (double)gr * gr + (double)gi * gi;
                        const double ab = (double)al * be;
                        if (g2 > tol2 * ab && ab > 0.0) {
                            rotated = 1;
                            // 2x2 Hermitian Gram [[al, gamma], [conj gamma, be]]: real Jacobi angle
                            // after removing the phase of gamma
                            const double gm = sqrt(g2);
                            const double zeta = ((double)be - (double)al) / (2.0 * gm);
                            const double az = fabs(zeta);
                            double t = (az > 1e150) ? 0.5 / az : 1.0 / (az + sqrt(1.0 + az * az));
                            if (zeta < 0.0) t = -t;
                            const double cd = 1.0 / sqrt(1.0 + t * t);
                            const double sd = cd * t;
                            const float c = (float)cd;
                            // w = s e^{-i arg gamma}:  b_i' = c b_i - w b_j,  b_j' = conj(w) b_i + c b_j
                            const float wr = (float)(sd * gr / gm);
                            const float wi = (float)(-sd * gi / gm);
                            float2 ui[R], uj[R];
#pragma unroll
                            for (int k = 0; k < R; ++k) {
                                const int r = q + G * k;
                                ui[k] = Js[ci * MP + r];
                                uj[k] = Js[cj * MP + r];
                            }
#pragma unroll
                            for (int k = 0; k < R; ++k) {
                                const int r = q + G * k;
                                float2 x = bi[k], y = bj[k];
                                float2 ni, nj;
                                ni.x = fmaf(c, x.x, -fmaf(wr, y.x, -wi * y.y));
                                ni.y = fmaf(c, x.y, -fmaf(wr, y.y, wi * y.x));
                                nj.x = fmaf(c, y.x, fmaf(wr, x.x, wi * x.y));
                                nj.y = fmaf(c, y.y, fmaf(wr, x.y, -wi * x.x));
                                Bs[ci * MP + r] = ni;
                                Bs[cj * MP + r] = nj;
                                x = ui[k];
                                y = uj[k];
                                ni.x = fmaf(c, x.x, -fmaf(wr, y.x, -wi * y.y));
                                ni.y = fmaf(c, x.y, -fmaf(wr, y.y, wi * y.x));
                                nj.x = fmaf(c, y.x, fmaf(wr, x.x, wi * x.y));
                                nj.y = fmaf(c, y.y, fmaf(wr, x.y, -wi * x.x));
                                Js[ci * MP + r] = ni;
                                Js[cj * MP + r] = nj;
                            }
                            if (q == 0) ++my_rot;
                        }
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

        // ---- singular values: sigma_c = |b_c| (scaled back) ----------------------------------
        for (int c = g; c < MP && g < C::NG; c += C::NG) {
            float s = 0.f;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const float2 v = Bs[c * MP + q + G * k];
                s = fmaf(v.x, v.x, fmaf(v.y, v.y, s));
            }
            s = group_sum<G>(s);
            if (q == 0) sig[c] = (c < M) ? ldexpf(sqrtf(s), ex) : -1.0f;
        }
        for (int c = tid; c < MP; c += NT) perm[c] = c;
        __syncthreads();
        // stable descending rank: rank_c = #{k : s_k > s_c or (s_k == s_c and k < c)}
        for (int c = tid; c < M; c += NT) {
            const float sc_ = sig[c];
            int rank = 0;
            for (int k = 0; k < M; ++k) {
                const float sk = sig[k];
                rank += (sk > sc_ || (sk == sc_ && k < c)) ? 1 : 0;
            }
            if (rank < M) perm[rank] = c;
        }
        __syncthreads();
    }

    // ---- outputs ------------------------------------------------------------------------------
    const bool ok = (flag == SSL_BIN_OK) && converged;
    const int st = (flag != SSL_BIN_OK) ? flag : (converged ? SSL_BIN_OK : SSL_BIN_NO_CONV);
    float2 *Enf = En + (size_t)f * Nn * M;
    for (int e = tid; e < Nn * M; e += NT) {
        const int c = e / M, r = e - c * M;
        Enf[e] = ok ? Js[perm[Ns + c] * MP + r] : make_float2(0.f, 0.f);
    }
    if (sigma != nullptr)
        for (int k = tid; k < M; k += NT) sigma[(size_t)f * M + k] = ok ? sig[perm[k]] : 0.0f;
    if (tid == 0) {
        if (bin_status != nullptr) bin_status[f] = st;
        if (conv != nullptr) {
            conv[2 * f] = sweeps;
            conv[2 * f + 1] = rot_total;
        }
    }
}

template <int MP, int G>
hipError_t launch_cfg(const ssl_c64 *A, const int32_t *kstatus, int F, int M, int Ns,
                      int max_sweeps, ssl_c64 *En, float *sigma, int32_t *bin_status,
                      int32_t *conv, hipStream_t st)
{
    hipLaunchKernelGGL((jacobi_svd<MP, G>), dim3(F), dim3(JacobiCfg<MP, G>::THREADS), 0, st,
                       reinterpret_cast<const float2 *>(A), kstatus, M, Ns, max_sweeps,
                       reinterpret_cast<float2 *>(En), sigma, bin_status, conv);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_jacobi(const ssl_c64 *A, const int32_t *kstatus, int F, int M, int Ns,
                         int max_sweeps, ssl_c64 *En, float *sigma, int32_t *bin_status,
                         int32_t *conv, hipStream_t st)
{
    if (M <= 8) return launch_cfg<8, 8>(A, kstatus, F, M, Ns, max_sweeps, En, sigma, bin_status, conv, st);
    if (M <= 16) return launch_cfg<16, 16>(A, kstatus, F, M, Ns, max_sweeps, En, sigma, bin_status, conv, st);
    if (M <= 32) return launch_cfg<32, 16>(A, kstatus, F, M, Ns, max_sweeps, En, sigma, bin_status, conv, st);
    return launch_cfg<64, 16>(A, kstatus, F, M, Ns, max_sweeps, En, sigma, bin_status, conv, st);
}
