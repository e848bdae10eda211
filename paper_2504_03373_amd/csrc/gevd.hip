// GEVD-MUSIC, the generalized-eigenvalue alternative to GSVD-MUSIC (Sec. II): the noise vectors
// are the generalized eigenvectors R e = lambda K e of the M - Ns smallest lambda.  With
// W = K^{-1/2} (Hermitian inverse square root of the noise correlation):
//   C = W R W,   C y = lambda y (C Hermitian positive semi-definite),   e = W y,
// so the path whitens with W on both sides, decomposes C with the same SVD kernels (C's left
// singular vectors are its eigenvectors), and maps the noise vectors back through W.  The e are
// K-orthonormal, and h^H e = (W h)^H y vanishes at noise-free sources.
//
// Kernels (all FP64, one workgroup per bin):
//   noise_isqrt  once per noise set: one-sided Jacobi on K from the right with the rotations
//                accumulated (K V = Z, K Hermitian positive definite: K = V diag(|z_k|) V^H),
//                round-robin pairs, 8 lanes per pair with shuffle reductions, rotate iff
//                |gamma| > M 2^-53 sqrt(ab); then W = V diag(|z_k|^{-1/2}) V^H (plain VALU loops);
//   gevd_whiten  per block: C = W R W on the matrix cores, T = W R kept in LDS in FP64 and
//                C = W T^H (R and W Hermitian), rounded once to complex64 for the SVD;
//   gevd_back    per block: E_n <- W E_n on the matrix cores (the SVD's noise vectors mapped to
//                generalized eigenvectors).
#include "ssl_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int MPX = SSL_MAX_M;                 // LDS matrices sized for the largest M
constexpr int G = 8;                           // lanes per column pair
constexpr int RW = MPX / G;                    // rows per lane

__device__ __forceinline__ double gsum8(double v)
{
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    return v;
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b)      // a conj(b)
{
    return make_double2(fma(a.x, b.x, a.y * b.y), fma(a.y, b.x, -a.x * b.y));
}

__global__ __launch_bounds__(kThreads) void noise_isqrt(const double2 *__restrict__ Kall,
                                                        const int32_t *__restrict__ kstatus,
                                                        int M, int max_sweeps,
                                                        double2 *__restrict__ Wall,
                                                        int32_t *__restrict__ wstatus)
{
    __shared__ double2 Z[MPX * MPX];           // column-major: K, then K V
    __shared__ double2 V[MPX * MPX];           // column-major
    __shared__ double inv_rt[MPX];
    __shared__ int flag;
    const int f = blockIdx.x, tid = threadIdx.x, g = tid / G, q = tid % G;
    const double2 *Kf = Kall + (size_t)f * M * M;
    double2 *Wf = Wall + (size_t)f * M * M;
    if (tid == 0) flag = kstatus ? kstatus[f] : SSL_BIN_OK;
    for (int e = tid; e < MPX * MPX; e += kThreads) {
        const int r = e / MPX, c = e - r * MPX;          // K row-major: coalesced; K = K^H
        Z[c * MPX + r] = (r < M && c < M) ? Kf[(size_t)r * M + c] : make_double2(0.0, 0.0);
        V[c * MPX + r] = make_double2(r == c ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    bool converged = false;
    if (flag == SSL_BIN_OK) {
        const int Me = M + (M & 1);
        const double tol = (double)M * 1.1102230246251565e-16;
        for (int sw = 0; sw < max_sweeps; ++sw) {
            int rotated = 0;
            for (int rd = 0; rd < Me - 1; ++rd) {
                if (g < Me / 2) {
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
                    if (cj < M) {
                        double2 zi[RW], zj[RW];
                        double al = 0.0, be = 0.0, gr = 0.0, gi = 0.0;
#pragma unroll
                        for (int k = 0; k < RW; ++k) {
                            const int r = q + G * k;
                            zi[k] = Z[ci * MPX + r];
                            zj[k] = Z[cj * MPX + r];
                            al = fma(zi[k].x, zi[k].x, fma(zi[k].y, zi[k].y, al));
                            be = fma(zj[k].x, zj[k].x, fma(zj[k].y, zj[k].y, be));
                            gr = fma(zi[k].x, zj[k].x, fma(zi[k].y, zj[k].y, gr));
                            gi = fma(zi[k].x, zj[k].y, fma(-zi[k].y, zj[k].x, gi));
                        }
                        al = gsum8(al);
                        be = gsum8(be);
                        gr = gsum8(gr);
                        gi = gsum8(gi);
                        const double ag = sqrt(fma(gr, gr, gi * gi));
                        if (ag > tol * sqrt(al * be) && al * be > 0.0) {
                            rotated = 1;
                            const double zeta = (be - al) / (2.0 * ag);
                            const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(fma(zeta, zeta, 1.0)));
                            const double c = 1.0 / sqrt(fma(t, t, 1.0)), s = c * t;
                            const double2 w = make_double2(s * gr / ag, -s * gi / ag);   // s e^{-i arg}
#pragma unroll
                            for (int k = 0; k < RW; ++k) {
                                const int r = q + G * k;
                                const double2 x = zi[k], y = zj[k];
                                const double2 wy = cmul(w, y), wx = cmulc(x, w);      // w y, x conj(w)
                                Z[ci * MPX + r] = make_double2(c * x.x - wy.x, c * x.y - wy.y);
                                Z[cj * MPX + r] = make_double2(wx.x + c * y.x, wx.y + c * y.y);
                                const double2 u = V[ci * MPX + r], v = V[cj * MPX + r];
                                const double2 wv = cmul(w, v), uw = cmulc(u, w);
                                V[ci * MPX + r] = make_double2(c * u.x - wv.x, c * u.y - wv.y);
                                V[cj * MPX + r] = make_double2(uw.x + c * v.x, uw.y + c * v.y);
                            }
                        }
                    }
                }
                __syncthreads();
            }
            if (__syncthreads_count(rotated) == 0) {
                converged = true;
                break;
            }
        }
        // eigenvalues |z_k| (K positive definite: K V = V diag(lambda)), lambda^{-1/2}
        for (int c = g; c < M; c += kThreads / G) {
            double s2 = 0.0;
#pragma unroll
            for (int k = 0; k < RW; ++k) {
                const double2 z = Z[c * MPX + q + G * k];
                s2 = fma(z.x, z.x, fma(z.y, z.y, s2));
            }
            s2 = gsum8(s2);
            if (q == 0) inv_rt[c] = s2 > 0.0 ? 1.0 / sqrt(sqrt(s2)) : 0.0;
        }
        __syncthreads();
        if (tid == 0 && !converged) flag = SSL_BIN_NO_CONV;
        __syncthreads();
    }
    const bool ok = flag == SSL_BIN_OK;
    // W = V diag(lambda^{-1/2}) V^H, row-major
    for (int e = tid; e < M * M; e += kThreads) {
        const int i = e / M, j = e - i * M;
        double2 acc = make_double2(0.0, 0.0);
        if (ok)
            for (int k = 0; k < M; ++k) {
                const double2 t = cmulc(V[k * MPX + i], V[k * MPX + j]);       // V_ik conj(V_jk)
                acc.x = fma(inv_rt[k], t.x, acc.x);
                acc.y = fma(inv_rt[k], t.y, acc.y);
            }
        Wf[e] = acc;
    }
    if (tid == 0 && wstatus) wstatus[f] = flag;
}

// The two per-block products on the matrix cores in FP64 (v_mfma_f64_16x16x4f64), as the GSVD
// whitening: complex products split into real ones over k-steps of 4; NT = MP / 16 waves, wave w
// owning rows 16 w .. 16 w + 15 of the result and all its column tiles, its A operands (W's rows)
// in registers.  Padding rows, columns and k-steps (beyond M) are zero on both operands.
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <int MP> struct GvCfg {
    static constexpr int NT = MP / 16;
    static constexpr int THREADS = 64 * NT;
    static constexpr int KQ = MP / 4;
    static constexpr int TS = MP + 1;          // complex128 row stride of T in LDS
    static constexpr int RS = MP + 16;         // complex64 row stride of the R stage (aliases T)
    static constexpr int ES = MP + 4;          // complex64 row stride of the E_n stage
    static constexpr size_t LDS = sizeof(double2) * MP * TS;
};

// w[q] = W[16 wave + (lane & 15)][4 q + (lane >> 4)]: the A operand of k-step q
template <int MP>
__device__ __forceinline__ void load_w_rows(const double2 *__restrict__ Wf, int M,
                                            double2 (&w)[GvCfg<MP>::KQ])
{
    const int lane = threadIdx.x & 63, row = 16 * (threadIdx.x >> 6) + (lane & 15), kl = lane >> 4;
#pragma unroll
    for (int q = 0; q < GvCfg<MP>::KQ; ++q) {
        const int k = 4 * q + kl;
        w[q] = (row < M && k < M) ? gload(Wf + (size_t)row * M + k) : make_double2(0.0, 0.0);
    }
}

// (ar, ai) = W B over the k-steps below M and the first nct column tiles; bop(q, ct) returns
// (Re, Im) of B[4 q + kl][16 ct + (lane & 15)], kl = lane / 16
template <int MP, class BOp>
__device__ __forceinline__ void wmul(const double2 (&w)[GvCfg<MP>::KQ], int M, doublex4 (&ar)[GvCfg<MP>::NT],
                                     doublex4 (&ai)[GvCfg<MP>::NT], int nct, BOp &&bop)
{
    const int KQ = (M + 3) >> 2;
#pragma unroll
    for (int ct = 0; ct < GvCfg<MP>::NT; ++ct) {
        ar[ct] = doublex4{0.0, 0.0, 0.0, 0.0};
        ai[ct] = doublex4{0.0, 0.0, 0.0, 0.0};
    }
#pragma unroll
    for (int q = 0; q < GvCfg<MP>::KQ; ++q) {
        if (q < KQ) {                              // uniform; w[] stays register-indexed
#pragma unroll
            for (int ct = 0; ct < GvCfg<MP>::NT; ++ct) {
                if (ct < nct) {
                    const double2 b = bop(q, ct);
                    ar[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(w[q].x, b.x, ar[ct], 0, 0, 0);
                    ar[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(w[q].y, -b.y, ar[ct], 0, 0, 0);
                    ai[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(w[q].x, b.y, ai[ct], 0, 0, 0);
                    ai[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(w[q].y, b.x, ai[ct], 0, 0, 0);
                }
            }
        }
    }
}

// C = W R W for one bin: T = W R on the matrix cores, T kept in LDS in FP64, then C = W T^H (= W R W
// for the Hermitian R and W of the method), rounded once to complex64.  W [M][M] complex128,
// R and C [M][M] complex64, row-major.  FP64 accumulator element e of lane l is row
// l / 16 + 4 e, column l % 16 of its 16 x 16 tile.
template <int MP>
__device__ __forceinline__ void gevd_whiten_bin(const double2 *__restrict__ Wf,
                                                const float2 *__restrict__ Rf, int M,
                                                float2 *__restrict__ Cf, double2 *Ts)
{
    typedef GvCfg<MP> C;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, kl = lane >> 4, lc = lane & 15;
    float2 *Rs = reinterpret_cast<float2 *>(Ts);
    double2 w[C::KQ];
    load_w_rows<MP>(Wf, M, w);
    for (int e = tid; e < MP * MP; e += C::THREADS) {
        const int k = e / MP, j = e % MP;
        Rs[k * C::RS + j] = (k < M && j < M) ? gload(Rf + (size_t)k * M + j) : make_float2(0.f, 0.f);
    }
    __syncthreads();
    doublex4 ar[C::NT], ai[C::NT];
    wmul<MP>(w, M, ar, ai, C::NT, [&](int q, int ct) {
        const float2 r = Rs[(4 * q + kl) * C::RS + 16 * ct + lc];
        return make_double2((double)r.x, (double)r.y);
    });
    __syncthreads();                               // every wave has read the R stage
#pragma unroll
    for (int ct = 0; ct < C::NT; ++ct)
#pragma unroll
        for (int e = 0; e < 4; ++e)
            Ts[(16 * wave + kl + 4 * e) * C::TS + 16 * ct + lc] = make_double2(ar[ct][e], ai[ct][e]);
    __syncthreads();
    wmul<MP>(w, M, ar, ai, C::NT, [&](int q, int ct) {
        const double2 t = Ts[(16 * ct + lc) * C::TS + 4 * q + kl];      // T^H[k][j] = conj T[j][k]
        return make_double2(t.x, -t.y);
    });
#pragma unroll
    for (int ct = 0; ct < C::NT; ++ct) {
        const int j = 16 * ct + lc;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r = 16 * wave + kl + 4 * e;
            if (r < M && j < M)
                gstore(Cf + (size_t)r * M + j, make_float2((float)ar[ct][e], (float)ai[ct][e]));
        }
    }
    __syncthreads();                               // LDS reused by the next bin
}

// E_n <- W E_n for one bin; E_n [Nn][M] complex64 (noise vector c at c M), staged in LDS, the
// product written back through the stage so that the stores are row-contiguous
template <int MP>
__device__ __forceinline__ void gevd_back_bin(const double2 *__restrict__ Wf,
                                              float2 *__restrict__ Ef, int M, int Nn, float2 *Es)
{
    typedef GvCfg<MP> C;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, kl = lane >> 4, lc = lane & 15;
    double2 w[C::KQ];
    load_w_rows<MP>(Wf, M, w);
    const int nct = (Nn + 15) >> 4;
    for (int e = tid; e < MP * MP; e += C::THREADS) {
        const int j = e / MP, k = e % MP;
        Es[j * C::ES + k] = (j < Nn && k < M) ? gload(Ef + (size_t)j * M + k) : make_float2(0.f, 0.f);
    }
    __syncthreads();
    doublex4 ar[C::NT], ai[C::NT];
    wmul<MP>(w, M, ar, ai, nct, [&](int q, int ct) {
        const float2 v = Es[(16 * ct + lc) * C::ES + 4 * q + kl];      // E[k][j] = E_n[j][k]
        return make_double2((double)v.x, (double)v.y);
    });
    __syncthreads();
#pragma unroll
    for (int ct = 0; ct < C::NT; ++ct)
        if (ct < nct)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                Es[(16 * ct + lc) * C::ES + 16 * wave + kl + 4 * e] =
                    make_float2((float)ar[ct][e], (float)ai[ct][e]);
    __syncthreads();
    for (int e = tid; e < Nn * M; e += C::THREADS) {
        const int j = e / M, k = e - j * M;
        gstore(Ef + e, Es[j * C::ES + k]);
    }
    __syncthreads();
}

template <int MP>
__global__ __launch_bounds__(GvCfg<MP>::THREADS) void gevd_whiten(const double2 *__restrict__ W,
                                                                  const float2 *__restrict__ R,
                                                                  int M, float2 *__restrict__ Cm)
{
    __shared__ double2 Ts[MP * GvCfg<MP>::TS];
    const size_t o = (size_t)blockIdx.x * M * M;
    gevd_whiten_bin<MP>(W + o, R + o, M, Cm + o, Ts);
}

template <int MP>
__global__ __launch_bounds__(GvCfg<MP>::THREADS) void gevd_back(const double2 *__restrict__ W,
                                                                float2 *__restrict__ En, int M,
                                                                int Ns)
{
    __shared__ float2 Es[MP * GvCfg<MP>::ES];
    const int f = blockIdx.x;
    gevd_back_bin<MP>(W + (size_t)f * M * M, En + (size_t)f * (M - Ns) * M, M, M - Ns, Es);
}

// batched forms over (block, bin) items of one size class; the blocks' Kisq hold W
template <int MP>
__global__ __launch_bounds__(GvCfg<MP>::THREADS) void gevd_whiten_batch(
    const BlockDev *__restrict__ blk, const int2 *__restrict__ items)
{
    __shared__ double2 Ts[MP * GvCfg<MP>::TS];
    const int2 it = items[blockIdx.x];
    const BlockDev &B = blk[it.x];
    const size_t o = (size_t)it.y * B.M * B.M;
    gevd_whiten_bin<MP>(B.Kisq + o, B.R + o, B.M, B.A + o, Ts);
}

template <int MP>
__global__ __launch_bounds__(GvCfg<MP>::THREADS) void gevd_back_batch(
    const BlockDev *__restrict__ blk, const int2 *__restrict__ items)
{
    __shared__ float2 Es[MP * GvCfg<MP>::ES];
    const int2 it = items[blockIdx.x];
    const BlockDev &B = blk[it.x];
    gevd_back_bin<MP>(B.Kisq + (size_t)it.y * B.M * B.M, B.En + (size_t)it.y * (B.M - B.Ns) * B.M,
                      B.M, B.M - B.Ns, Es);
}

}  // namespace

hipError_t launch_noise_isqrt(const ssl_c128 *K, const int32_t *kstatus, int F, int M,
                              ssl_c128 *W, int32_t *wstatus, hipStream_t st)
{
    hipLaunchKernelGGL(noise_isqrt, dim3(F), dim3(kThreads), 0, st,
                       reinterpret_cast<const double2 *>(K), kstatus, M, 40,
                       reinterpret_cast<double2 *>(W), wstatus);
    return hipGetLastError();
}

#define GEVD_DISPATCH(MPV, ...)                                                            \
    switch (MPV) {                                                                         \
    case 16: { constexpr int MP = 16; __VA_ARGS__; } break;                                \
    case 32: { constexpr int MP = 32; __VA_ARGS__; } break;                                \
    default: { constexpr int MP = 64; __VA_ARGS__; } break;                                \
    }

hipError_t launch_gevd_whiten(const ssl_c128 *W, const ssl_c64 *R, ssl_c64 *C, int F, int M,
                              hipStream_t st)
{
    const double2 *Wp = reinterpret_cast<const double2 *>(W);
    const float2 *Rp = reinterpret_cast<const float2 *>(R);
    float2 *Cp = reinterpret_cast<float2 *>(C);
    GEVD_DISPATCH(whiten_class(M), hipLaunchKernelGGL(gevd_whiten<MP>, dim3(F),
                                                      dim3(GvCfg<MP>::THREADS), 0, st, Wp, Rp, M, Cp))
    return hipGetLastError();
}

hipError_t launch_gevd_back(const ssl_c128 *W, ssl_c64 *En, int F, int M, int Ns, hipStream_t st)
{
    const double2 *Wp = reinterpret_cast<const double2 *>(W);
    float2 *Ep = reinterpret_cast<float2 *>(En);
    GEVD_DISPATCH(whiten_class(M), hipLaunchKernelGGL(gevd_back<MP>, dim3(F),
                                                      dim3(GvCfg<MP>::THREADS), 0, st, Wp, Ep, M, Ns))
    return hipGetLastError();
}

hipError_t launch_gevd_whiten_batch(const BlockDev *blk, const int2 *items, int n_items, int cls,
                                    hipStream_t st)
{
    if (n_items <= 0) return hipSuccess;
    GEVD_DISPATCH(cls, hipLaunchKernelGGL(gevd_whiten_batch<MP>, dim3(n_items),
                                          dim3(GvCfg<MP>::THREADS), 0, st, blk, items))
    return hipGetLastError();
}

hipError_t launch_gevd_back_batch(const BlockDev *blk, const int2 *items, int n_items, int cls,
                                  hipStream_t st)
{
    if (n_items <= 0) return hipSuccess;
    GEVD_DISPATCH(cls, hipLaunchKernelGGL(gevd_back_batch<MP>, dim3(n_items),
                                          dim3(GvCfg<MP>::THREADS), 0, st, blk, items))
    return hipGetLastError();
}
