// Noise whitening for eq.4 of arXiv 2504.03373 (GSVD of K^{-1} R), all in FP64.
//
// The paper inverts the preset noise correlation K by Gaussian elimination and then forms
// A = K^{-1} R with a matrix product (Sec. III-B).  K is Hermitian positive definite and fixed per
// stream, so here it is factored once per noise set with a complex Cholesky K = L L^H (the
// pivots double as the positive-definiteness test), inverted as K^{-1} = L^{-H} L^{-1}, and kept
// resident; each block then needs only the FP64 product A = K^{-1} R, rounded to complex64 for the
// FP32 Jacobi SVD.
#include "ssl_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr double kPdRel = 9.094947017729282e-13;   // 2^-40: pivot floor relative to max_i K_ii

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ double2 cmulc(double2 a, double2 b)
{
    return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

// One workgroup per bin.  L (then L^{-1}) lives in LDS; both use MP x MP complex128 slots.
template <int MP>
__global__ __launch_bounds__(kThreads) void noise_factor(const double2 *__restrict__ K,
                                                         double2 *__restrict__ Kinv,
                                                         int32_t *__restrict__ status, int M)
{
    __shared__ double2 L[MP * MP];
    __shared__ double2 Y[MP * MP];
    __shared__ int bad;
    __shared__ double dmax_s;
    const int f = blockIdx.x;
    const int tid = threadIdx.x;
    const double2 *Kf = K + (size_t)f * M * M;
    double2 *Wf = Kinv + (size_t)f * M * M;

    for (int e = tid; e < M * M; e += kThreads) {
        const int i = e / M, j = e - i * M;
        L[i * MP + j] = Kf[e];
        Y[i * MP + j] = make_double2(0.0, 0.0);
    }
    if (tid == 0) bad = 0;
    __syncthreads();
    if (tid == 0) {
        double dm = 0.0;
        for (int i = 0; i < M; ++i) dm = fmax(dm, L[i * MP + i].x);
        dmax_s = dm;
        if (!(dm > 0.0) || !isfinite(dm)) bad = 1;
    }
    __syncthreads();
    // right-looking Cholesky on the lower triangle
    for (int k = 0; k < M && !bad; ++k) {
        if (tid == 0) {
            const double d = L[k * MP + k].x;
            if (!isfinite(d) || d <= kPdRel * dmax_s) {
                bad = 1;
            } else {
                L[k * MP + k] = make_double2(sqrt(d), 0.0);
            }
        }
        __syncthreads();
        if (bad) break;
        const double inv = 1.0 / L[k * MP + k].x;
        for (int i = k + 1 + tid; i < M; i += kThreads) {
            double2 v = L[i * MP + k];
            L[i * MP + k] = make_double2(v.x * inv, v.y * inv);
        }
        __syncthreads();
        // trailing update of the lower triangle: L_ij -= L_ik conj(L_jk), k < j <= i
        const int n = M - k - 1;
        for (int e = tid; e < n * n; e += kThreads) {
            const int i = k + 1 + e / n, j = k + 1 + e % n;
            if (j > i) continue;
            const double2 p = cmulc(L[i * MP + k], L[j * MP + k]);
            double2 v = L[i * MP + j];
            L[i * MP + j] = make_double2(v.x - p.x, v.y - p.y);
        }
        __syncthreads();
    }
    if (bad) {
        for (int e = tid; e < M * M; e += kThreads) Wf[e] = make_double2(0.0, 0.0);
        if (tid == 0) status[f] = SSL_BIN_NOT_PD;
        return;
    }
    // Y = L^{-1}: row by row, Y_ic = (delta_ic - sum_{c<=k<i} L_ik Y_kc) / L_ii, columns in parallel
    for (int i = 0; i < M; ++i) {
        const double linv = 1.0 / L[i * MP + i].x;
        for (int c = tid; c <= i; c += kThreads) {
            double2 s = make_double2(c == i ? 1.0 : 0.0, 0.0);
            for (int k = c; k < i; ++k) {
                const double2 p = cmul(L[i * MP + k], Y[k * MP + c]);
                s.x -= p.x;
                s.y -= p.y;
            }
            Y[i * MP + c] = make_double2(s.x * linv, s.y * linv);
        }
        __syncthreads();
    }
    // K^{-1} = Y^H Y: W_ij = sum_{k >= max(i,j)} conj(Y_ki) Y_kj; upper triangle computed once,
    // the lower written as its conjugate (exactly Hermitian, real diagonal)
    const int nent = M * (M + 1) / 2;
    for (int e0 = tid; e0 < nent; e0 += kThreads) {
        int e = e0, i = 0;
        while (e >= M - i) { e -= M - i; ++i; }
        const int j = i + e;
        double2 s = make_double2(0.0, 0.0);
        for (int k = j; k < M; ++k) {
            const double2 p = cmulc(Y[k * MP + j], Y[k * MP + i]);   // Y_kj conj(Y_ki)
            s.x += p.x;
            s.y += p.y;
        }
        if (i == j) {
            Wf[(size_t)i * M + i] = make_double2(s.x, 0.0);
        } else {
            Wf[(size_t)i * M + j] = s;
            Wf[(size_t)j * M + i] = make_double2(s.x, -s.y);
        }
    }
    if (tid == 0) status[f] = SSL_BIN_OK;
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

}  // namespace

hipError_t launch_noise_factor(ssl_c128 *K, ssl_c128 *Kinv, int32_t *status, int F, int M,
                               hipStream_t st)
{
    const double2 *Kp = reinterpret_cast<const double2 *>(K);
    double2 *Wp = reinterpret_cast<double2 *>(Kinv);
    if (M <= 16)
        hipLaunchKernelGGL(noise_factor<16>, dim3(F), dim3(kThreads), 0, st, Kp, Wp, status, M);
    else if (M <= 32)
        hipLaunchKernelGGL(noise_factor<32>, dim3(F), dim3(kThreads), 0, st, Kp, Wp, status, M);
    else
        hipLaunchKernelGGL(noise_factor<64>, dim3(F), dim3(kThreads), 0, st, Kp, Wp, status, M);
    return hipGetLastError();
}

hipError_t launch_noise_load(ssl_c128 *K, const void *Kin, ssl_prec kprec, int F, int M,
                             hipStream_t st)
{
    const size_t n = (size_t)F * M * M;
    const int blocks = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
    if (kprec == SSL_FP64)
        hipLaunchKernelGGL(noise_load_c128, dim3(blocks), dim3(256), 0, st,
                           reinterpret_cast<double2 *>(K), static_cast<const double2 *>(Kin), n);
    else
        hipLaunchKernelGGL(noise_load_c64, dim3(blocks), dim3(256), 0, st,
                           reinterpret_cast<double2 *>(K), static_cast<const float2 *>(Kin), n);
    return hipGetLastError();
}

hipError_t launch_noise_blend(ssl_c128 *K, const void *Khat, ssl_prec kprec, double alpha, int F,
                              int M, hipStream_t st)
{
    const size_t n = (size_t)F * M * M;
    const int blocks = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
    if (kprec == SSL_FP64)
        hipLaunchKernelGGL(noise_blend_c128, dim3(blocks), dim3(256), 0, st,
                           reinterpret_cast<double2 *>(K), static_cast<const double2 *>(Khat),
                           alpha, n);
    else
        hipLaunchKernelGGL(noise_blend_c64, dim3(blocks), dim3(256), 0, st,
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
