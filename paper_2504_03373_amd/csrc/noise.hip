// Noise whitening for eq.4 of arXiv 2504.03373 (GSVD of K^{-1} R), all in FP64.
//
// The paper inverts the preset noise correlation K by Gaussian elimination and then forms
// A = K^{-1} R with a matrix product (Sec. III-B).  K is Hermitian positive definite and fixed per
// stream (or slowly updated), so here K^{-1} is computed once per noise set by in-place
// Gauss-Jordan elimination in FP64 and kept resident; each block then needs only the FP64 product
// A = K^{-1} R, rounded to complex64 for the FP32 Jacobi SVD.  Without pivoting on a Hermitian
// positive definite matrix the elimination pivots are the Schur-complement diagonals, i.e. the
// squared diagonal of the Cholesky factor, so they double as the positive-definiteness test.
#include "ssl_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kFactorThreads = 512;
constexpr double kPdRel = 9.094947017729282e-13;   // 2^-40: pivot floor relative to max_i K_ii

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// One workgroup per bin; the whole MP x MP complex128 matrix in LDS (64 KB at MP = 64).
// Step k with pivot p = W_kk (real for Hermitian input):
//   W_ij -= W_ik W_kj / p (i, j != k);  W_kj /= p;  W_ik = -W_ik / p;  W_kk = 1 / p.
// After M steps W = K^{-1}.  A pivot p <= 2^-40 max_i K_ii (or non-finite) marks the bin NOT_PD.
template <int MP>
__global__ __launch_bounds__(kFactorThreads) void noise_factor(const double2 *__restrict__ K,
                                                               double2 *__restrict__ Kinv,
                                                               int32_t *__restrict__ status,
                                                               int M)
{
    __shared__ double2 W[MP * MP];
    __shared__ double thr_s;
    __shared__ int bad_s;
    const int f = blockIdx.x;
    const int tid = threadIdx.x;
    const double2 *Kf = K + (size_t)f * M * M;
    double2 *Wf = Kinv + (size_t)f * M * M;

    for (int e = tid; e < M * MP; e += kFactorThreads) {
        const int i = e / MP, j = e % MP;
        if (j < M) W[i * MP + j] = Kf[i * M + j];
    }
    __syncthreads();
    if (tid == 0) {
        double dm = 0.0;
        bool fin = true;
        for (int i = 0; i < M; ++i) {
            const double d = W[i * MP + i].x;
            fin = fin && isfinite(d);
            dm = fmax(dm, d);
        }
        bad_s = (!(dm > 0.0) || !isfinite(dm) || !fin) ? 1 : 0;
        thr_s = kPdRel * dm;
    }
    __syncthreads();
    bool bad = bad_s != 0;
    const double thr = thr_s;
    for (int k = 0; k < M && !bad; ++k) {
        const double p = W[k * MP + k].x;             // every thread reads the same pivot
        if (!isfinite(p) || p <= thr) {
            bad = true;
            break;
        }
        const double ip = 1.0 / p;
        for (int e = tid; e < MP * MP; e += kFactorThreads) {
            const int i = e / MP, j = e % MP;             // MP is a power of two: shifts
            if (i >= M || j >= M || i == k || j == k) continue;
            const double2 t = cmul(W[i * MP + k], W[k * MP + j]);
            double2 w = W[i * MP + j];
            w.x = fma(-t.x, ip, w.x);
            w.y = fma(-t.y, ip, w.y);
            W[i * MP + j] = w;
        }
        __syncthreads();
        for (int e = tid; e < M; e += kFactorThreads) {
            if (e == k) {
                W[k * MP + k] = make_double2(ip, 0.0);
            } else {
                const double2 r = W[k * MP + e], c = W[e * MP + k];
                W[k * MP + e] = make_double2(r.x * ip, r.y * ip);
                W[e * MP + k] = make_double2(-c.x * ip, -c.y * ip);
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < M * MP; e += kFactorThreads) {
        const int i = e / MP, j = e % MP;
        if (j < M) Wf[i * M + j] = bad ? make_double2(0.0, 0.0) : W[i * MP + j];
    }
    if (tid == 0) status[f] = bad ? SSL_BIN_NOT_PD : SSL_BIN_OK;
}

// K <- alpha K + (1 - alpha) Khat
__global__ void noise_blend_c128(double2 *__restrict__ K, const double2 *__restrict__ Kh,
                                 double alpha, size_t n)
{
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x) {
        const double2 a = K[e], b = Kh[e];
        K[e] = make_double2(alpha * a.x + (1.0 - alpha) * b.x, alpha * a.y + (1.0 - alpha) * b.y);
    }
}
__global__ void noise_blend_c64(double2 *__restrict__ K, const float2 *__restrict__ Kh,
                                double alpha, size_t n)
{
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x) {
        const double2 a = K[e];
        const float2 b = Kh[e];
        K[e] = make_double2(alpha * a.x + (1.0 - alpha) * (double)b.x,
                            alpha * a.y + (1.0 - alpha) * (double)b.y);
    }
}

// K <- Kin (complex128 copy or complex64 widened)
__global__ void noise_load_c128(double2 *__restrict__ K, const double2 *__restrict__ Kin, size_t n)
{
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x)
        K[e] = Kin[e];
}
__global__ void noise_load_c64(double2 *__restrict__ K, const float2 *__restrict__ Kin, size_t n)
{
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x) {
        const float2 v = Kin[e];
        K[e] = make_double2((double)v.x, (double)v.y);
    }
}

// A = K^{-1} R per bin in FP64.  One workgroup per bin, each thread a 4x4 register tile of A.
// LDS: K^{-1} transposed (KT[k][i]) so a thread's 4 rows are contiguous, R upcast to FP64.
template <int MP>
__device__ __forceinline__ void whiten_bin(const double2 *__restrict__ Wf,
                                           const float2 *__restrict__ Rf,
                                           float2 *__restrict__ Af, int M)
{
    static_assert(MP % 4 == 0 && (MP / 4) * (MP / 4) <= kThreads, "tile grid must fit");
    __shared__ double2 KT[MP * MP];
    __shared__ double2 Rs[MP * MP];
    const int tid = threadIdx.x;
    for (int e = tid; e < MP * MP; e += kThreads) {
        const int i = e / MP, j = e - i * MP;
        double2 w = make_double2(0.0, 0.0), r = make_double2(0.0, 0.0);
        if (i < M && j < M) {
            w = Wf[(size_t)i * M + j];
            const float2 rv = Rf[(size_t)i * M + j];
            r = make_double2((double)rv.x, (double)rv.y);
        }
        KT[j * MP + i] = w;
        Rs[i * MP + j] = r;
    }
    __syncthreads();
    constexpr int NB = MP / 4;
    if (tid >= NB * NB) return;
    const int i0 = 4 * (tid / NB), j0 = 4 * (tid % NB);
    if (i0 >= M || j0 >= M) return;
    double2 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = make_double2(0.0, 0.0);
    for (int k = 0; k < M; ++k) {
        double2 w[4], r[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) w[a] = KT[k * MP + i0 + a];
#pragma unroll
        for (int b = 0; b < 4; ++b) r[b] = Rs[k * MP + j0 + b];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                acc[a][b].x = fma(w[a].x, r[b].x, acc[a][b].x);
                acc[a][b].x = fma(-w[a].y, r[b].y, acc[a][b].x);
                acc[a][b].y = fma(w[a].x, r[b].y, acc[a][b].y);
                acc[a][b].y = fma(w[a].y, r[b].x, acc[a][b].y);
            }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = i0 + a, j = j0 + b;
            if (i < M && j < M)
                Af[(size_t)i * M + j] = make_float2((float)acc[a][b].x, (float)acc[a][b].y);
        }
}

template <int MP>
__global__ __launch_bounds__(kThreads) void whiten(const double2 *__restrict__ Kinv,
                                                   const float2 *__restrict__ R,
                                                   float2 *__restrict__ A, int M)
{
    const size_t o = (size_t)blockIdx.x * M * M;
    whiten_bin<MP>(Kinv + o, R + o, A + o, M);
}

template <int MP>
__global__ __launch_bounds__(kThreads) void whiten_batch(const BlockDev *__restrict__ blk,
                                                         const int2 *__restrict__ items)
{
    const int2 it = items[blockIdx.x];
    const BlockDev &B = blk[it.x];
    const size_t o = (size_t)it.y * B.M * B.M;
    whiten_bin<MP>(B.Kinv + o, B.R + o, B.A + o, B.M);
}

int grid_for(size_t n) { return (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096); }

}  // namespace

hipError_t launch_noise_factor(ssl_c128 *K, ssl_c128 *Kinv, int32_t *status, int F, int M,
                               hipStream_t st)
{
    const double2 *Kp = reinterpret_cast<const double2 *>(K);
    double2 *Wp = reinterpret_cast<double2 *>(Kinv);
    if (M <= 16)
        hipLaunchKernelGGL(noise_factor<16>, dim3(F), dim3(kFactorThreads), 0, st, Kp, Wp, status, M);
    else if (M <= 32)
        hipLaunchKernelGGL(noise_factor<32>, dim3(F), dim3(kFactorThreads), 0, st, Kp, Wp, status, M);
    else
        hipLaunchKernelGGL(noise_factor<64>, dim3(F), dim3(kFactorThreads), 0, st, Kp, Wp, status, M);
    return hipGetLastError();
}

hipError_t launch_noise_load(ssl_c128 *K, const void *Kin, ssl_prec kprec, int F, int M,
                             hipStream_t st)
{
    const size_t n = (size_t)F * M * M;
    if (kprec == SSL_FP64)
        hipLaunchKernelGGL(noise_load_c128, dim3(grid_for(n)), dim3(256), 0, st,
                           reinterpret_cast<double2 *>(K), static_cast<const double2 *>(Kin), n);
    else
        hipLaunchKernelGGL(noise_load_c64, dim3(grid_for(n)), dim3(256), 0, st,
                           reinterpret_cast<double2 *>(K), static_cast<const float2 *>(Kin), n);
    return hipGetLastError();
}

hipError_t launch_noise_blend(ssl_c128 *K, const void *Khat, ssl_prec kprec, double alpha, int F,
                              int M, hipStream_t st)
{
    const size_t n = (size_t)F * M * M;
    if (kprec == SSL_FP64)
        hipLaunchKernelGGL(noise_blend_c128, dim3(grid_for(n)), dim3(256), 0, st,
                           reinterpret_cast<double2 *>(K), static_cast<const double2 *>(Khat),
                           alpha, n);
    else
        hipLaunchKernelGGL(noise_blend_c64, dim3(grid_for(n)), dim3(256), 0, st,
                           reinterpret_cast<double2 *>(K), static_cast<const float2 *>(Khat),
                           alpha, n);
    return hipGetLastError();
}

hipError_t launch_whiten(const ssl_c128 *Kinv, const ssl_c64 *R, ssl_c64 *A, int F, int M,
                         hipStream_t st)
{
    const double2 *Wp = reinterpret_cast<const double2 *>(Kinv);
    const float2 *Rp = reinterpret_cast<const float2 *>(R);
    float2 *Ap = reinterpret_cast<float2 *>(A);
    switch (whiten_class(M)) {
    case 16: hipLaunchKernelGGL(whiten<16>, dim3(F), dim3(kThreads), 0, st, Wp, Rp, Ap, M); break;
    case 32: hipLaunchKernelGGL(whiten<32>, dim3(F), dim3(kThreads), 0, st, Wp, Rp, Ap, M); break;
    default: hipLaunchKernelGGL(whiten<64>, dim3(F), dim3(kThreads), 0, st, Wp, Rp, Ap, M); break;
    }
    return hipGetLastError();
}

hipError_t launch_whiten_batch(const BlockDev *blk, const int2 *items, int n_items, int cls,
                               hipStream_t st)
{
    if (n_items <= 0) return hipSuccess;
    switch (cls) {
    case 16: hipLaunchKernelGGL(whiten_batch<16>, dim3(n_items), dim3(kThreads), 0, st, blk, items); break;
    case 32: hipLaunchKernelGGL(whiten_batch<32>, dim3(n_items), dim3(kThreads), 0, st, blk, items); break;
    default: hipLaunchKernelGGL(whiten_batch<64>, dim3(n_items), dim3(kThreads), 0, st, blk, items); break;
    }
    return hipGetLastError();
}
