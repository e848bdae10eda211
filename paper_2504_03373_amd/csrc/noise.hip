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

#include <atomic>

namespace {

constexpr double kPdRel = 9.094947017729282e-13;   // 2^-40: pivot floor relative to max_i K_ii

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// One workgroup per bin, the MP x MP complex128 matrix in registers: thread t owns column
// j = t % MP of rows t / MP + (MP / 8) u, u < 8.  Step k with pivot p = W_kk (real for Hermitian
// input):
//   W_ij -= W_ik W_kj / p (i, j != k);  W_kj /= p;  W_ik = -W_ik / p;  W_kk = 1 / p.
// Only the pivot row and column travel, through two LDS buffers alternating by step: the owners
// post row and column k + 1 after their update, so a step costs one barrier.  After M steps
// W = K^{-1}.  A pivot p <= 2^-40 max_i K_ii (or non-finite) marks the bin NOT_PD.
template <int MP> constexpr int kFactorThreads = MP * MP / 8;

template <int MP>
__device__ __forceinline__ void noise_factor_bin(const double2 *__restrict__ Kf,
                                                 double2 *__restrict__ Wf,
                                                 int32_t *__restrict__ stf, int M)
{
    constexpr int RG = MP / 8;                     // row groups: rows of thread t are t / MP + RG u
    __shared__ double2 colb[2][MP], rowb[2][MP];
    __shared__ double diag_s[MP];
    __shared__ double thr_s;
    __shared__ int bad_s;
    const int t = threadIdx.x;
    const int j = t % MP, i0 = t / MP;

    double2 w[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {                      // every load in flight first
        const int i = i0 + RG * u;
        w[u] = (i < M && j < M) ? gload(Kf + (size_t)i * M + j) : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int i = i0 + RG * u;
        if (i == j) diag_s[i] = w[u].x;
        if (j == 0) colb[0][i] = w[u];
        if (i == 0) rowb[0][j] = w[u];
    }
    __syncthreads();
    if (t == 0) {
        double dm = 0.0;
        bool fin = true;
        for (int i = 0; i < M; ++i) {
            const double d = diag_s[i];
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
        const int b = k & 1;
        const double p = rowb[b][k].x;                // every thread reads the same pivot
        if (!isfinite(p) || p <= thr) {
            bad = true;
            break;
        }
        const double ip = 1.0 / p;
        const double2 wkj = rowb[b][j];
        double2 wik[8];                                // every pivot-column read in flight first
#pragma unroll
        for (int u = 0; u < 8; ++u) wik[u] = colb[b][i0 + RG * u];
        // row i is the same for every lane of a wave (uniform branch); column j == k is one lane
        // (a select).  Padding rows and columns hold zeros and stay zero: their w_kj / w_ik are 0.
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + RG * u;
            if (i == k) {
                const double2 row = make_double2(w[u].x * ip, w[u].y * ip);
                w[u] = (j == k) ? make_double2(ip, 0.0) : row;
            } else {
                const double2 tt = cmul(wik[u], wkj);
                const double2 gen = make_double2(fma(-tt.x, ip, w[u].x), fma(-tt.y, ip, w[u].y));
                const double2 col = make_double2(-w[u].x * ip, -w[u].y * ip);
                w[u] = (j == k) ? col : gen;
            }
        }
        if (k + 1 < M) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = i0 + RG * u;
                if (j == k + 1) colb[b ^ 1][i] = w[u];
                if (i == k + 1) rowb[b ^ 1][j] = w[u];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const int i = i0 + RG * u;
        if (i < M && j < M) gstore(Wf + (size_t)i * M + j, bad ? make_double2(0.0, 0.0) : w[u]);
    }
    if (t == 0) gstore(stf, (int32_t)(bad ? SSL_BIN_NOT_PD : SSL_BIN_OK));
}

template <int MP>
__global__ __launch_bounds__(kFactorThreads<MP>) void noise_factor(const double2 *__restrict__ K,
                                                                    double2 *__restrict__ Kinv,
                                                                    int32_t *__restrict__ status,
                                                                    int M)
{
    const int f = blockIdx.x;
    noise_factor_bin<MP>(K + (size_t)f * M * M, Kinv + (size_t)f * M * M, status + f, M);
}

// Item (handle, bin) of a batched noise update.
template <int MP>
__global__ __launch_bounds__(kFactorThreads<MP>) void noise_factor_batch(
    const NoiseUpdDev *__restrict__ h, const int2 *__restrict__ items)
{
    const int2 it = items[blockIdx.x];
    const NoiseUpdDev &H = h[it.x];
    const int M = H.M, f = it.y;
    noise_factor_bin<MP>(H.K + (size_t)f * M * M, H.Kinv + (size_t)f * M * M, H.status + f, M);
}

// K <- alpha K + (1 - alpha) Khat
__global__ void noise_blend_c128(double2 *__restrict__ K, const double2 *__restrict__ Kh,
                                 double alpha, size_t n)
{
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x) {
        const double2 a = K[e], b = Kh[e];
        K[e] = make_double2(fma(alpha, a.x, (1.0 - alpha) * b.x), fma(alpha, a.y, (1.0 - alpha) * b.y));
    }
}
__global__ void noise_blend_c64(double2 *__restrict__ K, const float2 *__restrict__ Kh,
                                double alpha, size_t n)
{
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x) {
        const double2 a = K[e];
        const float2 b = Kh[e];
        K[e] = make_double2(fma(alpha, a.x, (1.0 - alpha) * (double)b.x),
                            fma(alpha, a.y, (1.0 - alpha) * (double)b.y));
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

// A = K^{-1} R per bin in FP64 on the matrix cores (v_mfma_f64_16x16x4f64: FP64 inputs, FP64
// accumulation).  The complex product takes three real ones (Gauss's trick), W = K^{-1}:
//   P1 = Wr Rr,  P2 = Wi Ri,  P3 = (Wr + Wi)(Rr + Ri);   Re A = P1 - P2,  Im A = P3 - P1 - P2,
// over k-steps of 4: a quarter fewer matrix-core cycles than the four-product form, for an FP64
// rounding error at most a small constant times larger (the sums it rounds are bounded by
// (|Wr| + |Wi|)(|Rr| + |Ri|) instead of |Wr||Ri| + |Wi||Rr|).  A workgroup takes one bin of a noise set for a run of blocks that share it:
// NT = MP / 16 waves, wave w owning rows 16 w .. 16 w + 15 and all NT column tiles.  Its A
// operands (W's rows, FP64) are loaded into registers once and reused for every block of the
// run; each block's R (complex64) is staged in LDS -- the next block's R is loaded into
// registers under the current block's products -- and read as B operands, widened to FP64.
// Padding rows, columns and k-steps (beyond M) are zero on both operands and never stored.
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <int MP> struct WhCfg {
    static constexpr int NT = MP / 16;          // row tiles = column tiles = waves
    static constexpr int THREADS = 64 * NT;
    static constexpr int KQ = MP / 4;           // k-steps at M = MP
    static constexpr int RS = MP + 16;          // LDS row stride (complex64 elements)
    static constexpr int NIT = MP * MP / THREADS;
};

// Thread t stages R elements (k0 + 4u, j), k0 = t / MP, j = t % MP, u < NIT (THREADS = 4 MP).
template <int MP>
__device__ __forceinline__ void load_r(const float2 *__restrict__ Rf, int M, int tid,
                                       float2 (&v)[WhCfg<MP>::NIT])
{
    const int k0 = tid / MP, j = tid % MP;
    const float2 *src = Rf + (size_t)k0 * M + j;
#pragma unroll
    for (int u = 0; u < WhCfg<MP>::NIT; ++u)
        v[u] = (j < M && k0 + 4 * u < M) ? gload(src + (size_t)u * 4 * M) : make_float2(0.f, 0.f);
}

template <int MP>
__device__ __forceinline__ void store_r(const float2 (&v)[WhCfg<MP>::NIT], float2 *Rs, int tid)
{
    const int k0 = tid / MP, j = tid % MP;
#pragma unroll
    for (int u = 0; u < WhCfg<MP>::NIT; ++u) Rs[(k0 + 4 * u) * WhCfg<MP>::RS + j] = v[u];
}

// One workgroup: bin `Wf` (K^{-1} of the bin, [M][M] FP64) for nb blocks; blk(i, Rf, Af) gives
// block i's R and A of the bin.
template <int MP, class BlockAt>
__device__ __forceinline__ void whiten_run(const double2 *__restrict__ Wf, int M, int nb,
                                           BlockAt &&blk)
{
    typedef WhCfg<MP> C;
    __shared__ float2 Rs[MP * C::RS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int KQ = (M + 3) >> 2;
    const int row = 16 * wave + (lane & 15);     // A-operand row of this lane
    const int kl = lane >> 4;                    // k within a k-step (A and B operands)

    double2 w[C::KQ];
#pragma unroll
    for (int q = 0; q < C::KQ; ++q) {
        const int k = 4 * q + kl;
        w[q] = (row < M && k < M) ? gload(Wf + (size_t)row * M + k) : make_double2(0.0, 0.0);
    }

    const float2 *Rf;
    float2 *Af;
    blk(0, Rf, Af);
    {
        float2 v[C::NIT];
        load_r<MP>(Rf, M, tid, v);
        store_r<MP>(v, Rs, tid);
    }
    __syncthreads();
    for (int i = 0; i < nb; ++i) {
        float2 *const cur_A = Af;
        const bool more = i + 1 < nb;
        float2 v[C::NIT];
        if (more) {
            blk(i + 1, Rf, Af);
            load_r<MP>(Rf, M, tid, v);
        }
        doublex4 p1[C::NT], p2[C::NT], p3[C::NT];
#pragma unroll
        for (int ct = 0; ct < C::NT; ++ct) {
            p1[ct] = doublex4{0.0, 0.0, 0.0, 0.0};
            p2[ct] = doublex4{0.0, 0.0, 0.0, 0.0};
            p3[ct] = doublex4{0.0, 0.0, 0.0, 0.0};
        }
#pragma unroll
        for (int q = 0; q < C::KQ; ++q) {
            if (q < KQ) {                        // uniform; w[] stays register-indexed
                const float2 *rrow = Rs + (4 * q + kl) * C::RS + (lane & 15);
                const double ws = w[q].x + w[q].y;
#pragma unroll
                for (int ct = 0; ct < C::NT; ++ct) {
                    const float2 r = rrow[16 * ct];
                    const double br = (double)r.x, bi = (double)r.y;
                    p1[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(w[q].x, br, p1[ct], 0, 0, 0);
                    p2[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(w[q].y, bi, p2[ct], 0, 0, 0);
                    p3[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(ws, br + bi, p3[ct], 0, 0, 0);
                }
            }
        }
        doublex4 ar[C::NT], ai[C::NT];
#pragma unroll
        for (int ct = 0; ct < C::NT; ++ct) {
            ar[ct] = p1[ct] - p2[ct];
            ai[ct] = p3[ct] - p1[ct] - p2[ct];
        }
        // FP64 result layout: accumulator element e of lane l is row l / 16 + 4 e, column l % 16
        // of the 16 x 16 tile (rows interleaved, unlike the FP32 16x16x4 layout)
#pragma unroll
        for (int ct = 0; ct < C::NT; ++ct) {
            const int j = 16 * ct + (lane & 15);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = 16 * wave + kl + 4 * e;
                if (r < M && j < M)
                    gstore(cur_A + (size_t)r * M + j, make_float2((float)ar[ct][e], (float)ai[ct][e]));
            }
        }
        __syncthreads();                         // every wave has read Rs
        if (more) store_r<MP>(v, Rs, tid);
        __syncthreads();
    }
}

template <int MP>
__global__ __launch_bounds__(WhCfg<MP>::THREADS) __attribute__((amdgpu_waves_per_eu(2))) void whiten(const double2 *__restrict__ Kinv,
                                                              const float2 *__restrict__ R,
                                                              float2 *__restrict__ A, int M)
{
    const size_t o = (size_t)blockIdx.x * M * M;
    whiten_run<MP>(Kinv + o, M, 1, [&](int, const float2 *&Rf, float2 *&Af) {
        Rf = R + o;
        Af = A + o;
    });
}

// Batched: item = (chunk, bin); chunks[c] = (first, count) into cblocks, a run of blocks that
// share one noise set (the same K^{-1}).
template <int MP>
__global__ __launch_bounds__(WhCfg<MP>::THREADS) __attribute__((amdgpu_waves_per_eu(2))) void whiten_batch(const BlockDev *__restrict__ blk,
                                                                    const int2 *__restrict__ items,
                                                                    const int2 *__restrict__ chunks,
                                                                    const int *__restrict__ cblocks)
{
    const int2 it = items[blockIdx.x];
    const int2 ch = chunks[it.x];
    const BlockDev &B0 = blk[cblocks[ch.x]];
    const int M = B0.M;
    const size_t o = (size_t)it.y * M * M;
    whiten_run<MP>(B0.Kinv + o, M, ch.y, [&](int i, const float2 *&Rf, float2 *&Af) {
        const BlockDev &B = blk[cblocks[ch.x + i]];
        Rf = B.R + o;
        Af = B.A + o;
    });
}

int grid_for(size_t n) { return (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096); }

}  // namespace

hipError_t launch_noise_factor(ssl_c128 *K, ssl_c128 *Kinv, int32_t *status, int F, int M,
                               hipStream_t st)
{
    const double2 *Kp = reinterpret_cast<const double2 *>(K);
    double2 *Wp = reinterpret_cast<double2 *>(Kinv);
    if (M <= 16)
        hipLaunchKernelGGL(noise_factor<16>, dim3(F), dim3(kFactorThreads<16>), 0, st, Kp, Wp,
                           status, M);
    else if (M <= 32)
        hipLaunchKernelGGL(noise_factor<32>, dim3(F), dim3(kFactorThreads<32>), 0, st, Kp, Wp,
                           status, M);
    else
        hipLaunchKernelGGL(noise_factor<64>, dim3(F), dim3(kFactorThreads<64>), 0, st, Kp, Wp,
                           status, M);
    return hipGetLastError();
}

hipError_t launch_noise_factor_batch(const NoiseUpdDev *h, const int2 *items, int n_items,
                                     int cls, hipStream_t st)
{
    if (n_items <= 0) return hipSuccess;
    if (cls == 16)
        hipLaunchKernelGGL(noise_factor_batch<16>, dim3(n_items), dim3(kFactorThreads<16>), 0, st,
                           h, items);
    else if (cls == 32)
        hipLaunchKernelGGL(noise_factor_batch<32>, dim3(n_items), dim3(kFactorThreads<32>), 0, st,
                           h, items);
    else
        hipLaunchKernelGGL(noise_factor_batch<64>, dim3(n_items), dim3(kFactorThreads<64>), 0, st,
                           h, items);
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
    case 16:
        hipLaunchKernelGGL(whiten<16>, dim3(F), dim3(WhCfg<16>::THREADS), 0, st, Wp, Rp, Ap, M);
        break;
    case 32:
        hipLaunchKernelGGL(whiten<32>, dim3(F), dim3(WhCfg<32>::THREADS), 0, st, Wp, Rp, Ap, M);
        break;
    default:
        hipLaunchKernelGGL(whiten<64>, dim3(F), dim3(WhCfg<64>::THREADS), 0, st, Wp, Rp, Ap, M);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_whiten_batch(const BlockDev *blk, const int2 *items, int n_items,
                               const int2 *chunks, const int *cblocks, int cls, hipStream_t st)
{
    if (n_items <= 0) return hipSuccess;
    switch (cls) {
    case 16:
        hipLaunchKernelGGL(whiten_batch<16>, dim3(n_items), dim3(WhCfg<16>::THREADS), 0, st, blk,
                           items, chunks, cblocks);
        break;
    case 32:
        hipLaunchKernelGGL(whiten_batch<32>, dim3(n_items), dim3(WhCfg<32>::THREADS), 0, st, blk,
                           items, chunks, cblocks);
        break;
    default:
        hipLaunchKernelGGL(whiten_batch<64>, dim3(n_items), dim3(WhCfg<64>::THREADS), 0, st, blk,
                           items, chunks, cblocks);
        break;
    }
    return hipGetLastError();
}

int whiten_wg_per_cu(int cls)
{
    // resident workgroups per CU of the batched kernel (registers and LDS decide), cached
    static std::atomic<int> cache[3];
    const int i = cls == 16 ? 0 : cls == 32 ? 1 : 2;
    int n = cache[i].load(std::memory_order_relaxed);
    if (n > 0) return n;
    hipError_t e;
    if (cls == 16)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, whiten_batch<16>, WhCfg<16>::THREADS, 0);
    else if (cls == 32)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, whiten_batch<32>, WhCfg<32>::THREADS, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, whiten_batch<64>, WhCfg<64>::THREADS, 0);
    if (e != hipSuccess || n < 1) return 1;
    cache[i].store(n, std::memory_order_relaxed);
    return n;
}
