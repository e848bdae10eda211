// Correlation accumulation, eq.2-3 of arXiv 2504.03373 (AddCorrelation + NormalizeCorrelation):
//   R[f] = scale * sum_t x_t x_t^H,   x_t = X[f, t, :] in C^M.
//
// MFMA path (FP32, and bf16/fp16 inputs with FP32 accumulation).  With x = a + i b,
//   Re R_ij = sum_t a_i a_j + b_i b_j,     Im R_ij = sum_t b_i a_j - a_i b_j,
// i.e. four real rank-T products of the [T][M] panels a and b.  One workgroup per bin stages the
// bin's frames in LDS (chunks of 64 frames, real and imaginary planes split) and each wave owns
// 16x16 tiles of the upper block triangle (I <= J) of the MP x MP padded result; the lower
// triangle is written as the conjugate of the same registers, so R is Hermitian to the bit.
//
// FP64 path (for the noise correlation K): same staging and tiling on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64), FP64 products of the exactly widened frames, FP64 accumulation.
#include "ssl_internal.h"

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int kChunk = 64;      // frames staged per LDS pass
constexpr int kThreads = 256;   // 4 waves

// Tile (I, J), I <= J, of an NT x NT block grid, enumerated row by row.
__device__ __forceinline__ void tile_coords(int t, int NT, int &I, int &J)
{
    I = 0;
    while (t >= NT - I) { t -= NT - I; ++I; }
    J = I + t;
}

// The bin's result goes through LDS (row stride MP + 1 complex, no bank conflicts on the mirrored
// writes) and leaves in coalesced rows.  Lane l, register r of a tile holds element
// (4*(l/16) + r, l%16); the lower triangle is the conjugate of the same registers.
__device__ __forceinline__ void tile_to_lds(float2 *Rs, int RS, int I, int J, const floatx4 &re,
                                            const floatx4 &im, float scale, int lane)
{
    const int j = 16 * J + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = 16 * I + 4 * (lane >> 4) + r;
        if (I == J && i > j) continue;      // mirrored from the (j, i) lane
        const float vr = re[r] * scale;
        const float vi = (i == j) ? 0.0f : im[r] * scale;
        Rs[i * RS + j] = make_float2(vr, vi);
        if (i != j) Rs[j * RS + i] = make_float2(vr, -vi);
    }
}

__device__ __forceinline__ void lds_to_out(const float2 *Rs, int RS, int M, int accumulate,
                                           float2 *__restrict__ Rf, int tid)
{
    // row i by wave, column j by lane (M <= 64): coalesced rows, no index division
    for (int i = tid >> 6; i < M; i += kThreads / 64) {
        const int j = tid & 63;
        if (j >= M) continue;
        float2 v = Rs[i * RS + j];
        if (accumulate) {
            const float2 a = gload(Rf + (size_t)i * M + j);
            v.x += a.x;
            v.y += a.y;
        }
        gstore(Rf + (size_t)i * M + j, v);
    }
}

// Frames t0 .. t0 + nf - 1 of a bin into registers, every load in flight at once; element
// e = tid + u * kThreads of the kChunk x MP grid is frame e / MP, channel e % MP (zero beyond nf
// frames or M channels).
template <int MP> constexpr int kChunkRegs = kChunk * MP / kThreads;
template <int MP>
__device__ __forceinline__ void load_chunk(const float2 *__restrict__ Xf, int t0, int nf, int M,
                                           int64_t sT, int tid, float2 (&v)[kChunkRegs<MP>])
{
    // opaque copy of the thread index: the addresses are recomputed at each call rather than
    // hoisted out of the bin loop and held in registers
    int t = tid;
    asm volatile("" : "+v"(t));
#pragma unroll
    for (int u = 0; u < kChunkRegs<MP>; ++u) {
        const int e = t + u * kThreads;
        const int tt = e / MP, m = e - tt * MP;
        v[u] = (tt < nf && m < M) ? gload(Xf + (size_t)(t0 + tt) * sT + m) : make_float2(0.f, 0.f);
    }
}

// ---------------------------------------------------------------------------------------------
// Both bin kernels take the bin's first chunk already in registers (v) and call next(v) once
// the last chunk is staged in LDS: the next bin's first chunk is then loaded while this bin's
// products and result stores run.
//
// FP32 inputs, v_mfma_f32_16x16x4f32: per 4-frame step, A[i][k] = plane[t0+k][16I+i] from lane
// i + 16k, B[k][j] = plane[t0+k][16J+j] from lane j + 16k.
template <int MP, class Next>
__device__ __forceinline__ void corr_f32_bin(const float2 *__restrict__ Xf, int T, int M,
                                             int64_t sT, float scale, int accumulate,
                                             float2 *__restrict__ Rf,
                                             float2 (&v)[kChunkRegs<MP>], Next &&next)
{
    constexpr int S = MP + 16;                 // row stride: 4 frame rows of a step hit other banks
    constexpr int NT = MP / 16;
    constexpr int NTILE = NT * (NT + 1) / 2;
    constexpr int TPW = (NTILE + 3) / 4;       // tiles per wave
    constexpr int RS = MP + 1;
    static_assert(2 * kChunk * S * 4 >= MP * RS * 8, "result staging exceeds the frame buffer");
    __shared__ __attribute__((aligned(16))) float Z[2 * kChunk * S];
    float *Zr = Z, *Zi = Z + kChunk * S;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;

    floatx4 acc_re[TPW], acc_im[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        acc_re[q] = floatx4{0.f, 0.f, 0.f, 0.f};
        acc_im[q] = floatx4{0.f, 0.f, 0.f, 0.f};
    }

    for (int t0 = 0; t0 < T; t0 += kChunk) {
        const int nf = min(kChunk, T - t0);
        if (t0 > 0) load_chunk<MP>(Xf, t0, nf, M, sT, tid, v);
        __syncthreads();
        constexpr int NIT = kChunkRegs<MP>;
#pragma unroll
        for (int u = 0; u < NIT; ++u) {
            const int e = tid + u * kThreads;
            const int tt = e / MP, m = e - tt * MP;
            Zr[tt * S + m] = v[u].x;
            Zi[tt * S + m] = v[u].y;
        }
        __syncthreads();
        if (t0 + kChunk >= T) next(v);
        const int nsteps = (nf + 3) >> 2;
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            const int tile = wave + 4 * q;
            if (tile < NTILE) {
                int I, J;
                tile_coords(tile, NT, I, J);
                const int ca = 16 * I + (lane & 15), cb = 16 * J + (lane & 15);
                for (int s = 0; s < nsteps; ++s) {
                    const int row = (4 * s + (lane >> 4)) * S;
                    const float ar = Zr[row + ca], ai = Zi[row + ca];
                    const float br = Zr[row + cb], bi = Zi[row + cb];
                    acc_re[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, br, acc_re[q], 0, 0, 0);
                    acc_re[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, bi, acc_re[q], 0, 0, 0);
                    acc_im[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, br, acc_im[q], 0, 0, 0);
                    acc_im[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ar, bi, acc_im[q], 0, 0, 0);
                }
            }
        }
    }
    __syncthreads();                           // frames no longer needed: Z holds the result
    float2 *Rs = reinterpret_cast<float2 *>(Z);
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        const int tile = wave + 4 * q;
        if (tile < NTILE) {
            int I, J;
            tile_coords(tile, NT, I, J);
            tile_to_lds(Rs, RS, I, J, acc_re[q], acc_im[q], scale, lane);
        }
    }
    __syncthreads();
    lds_to_out(Rs, RS, M, accumulate, Rf, tid);
}

// ---------------------------------------------------------------------------------------------
// bf16 / fp16 inputs, v_mfma_f32_16x16x32_{bf16,f16}: lane l holds 8 consecutive k (frames)
// k = 8*(l/16) .. +7 of row (A) / column (B) l%16.  Planes are stored transposed in LDS,
// [m][t] with t contiguous, so each operand is one 16-byte read.
template <typename E> struct Mfma32;
template <> struct Mfma32<__bf16> {
    typedef bf16x8 vec;
    static __device__ __forceinline__ floatx4 run(vec a, vec b, floatx4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma32<_Float16> {
    typedef halfx8 vec;
    static __device__ __forceinline__ floatx4 run(vec a, vec b, floatx4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

template <int MP, typename E, class Next>
__device__ __forceinline__ void corr_lp_bin(const float2 *__restrict__ Xf, int T, int M,
                                            int64_t sT, float scale, int accumulate,
                                            float2 *__restrict__ Rf,
                                            float2 (&v)[kChunkRegs<MP>], Next &&next)
{
    typedef typename Mfma32<E>::vec vec;
    constexpr int S = kChunk + 8;              // elements per transposed row (16 B pad)
    constexpr int NT = MP / 16;
    constexpr int NTILE = NT * (NT + 1) / 2;
    constexpr int TPW = (NTILE + 3) / 4;
    constexpr int RS = MP + 1;
    constexpr int PLANES = 3 * MP * S * (int)sizeof(E), RESULT = MP * RS * 8;
    __shared__ __attribute__((aligned(16))) float Z[(PLANES > RESULT ? PLANES : RESULT) / 4];
    E *Pr = reinterpret_cast<E *>(Z);
    E *Pi = Pr + MP * S;
    E *Pn = Pi + MP * S;                                     // -Re, for the Im product

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;

    floatx4 acc_re[TPW], acc_im[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        acc_re[q] = floatx4{0.f, 0.f, 0.f, 0.f};
        acc_im[q] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
    for (int t0 = 0; t0 < T; t0 += kChunk) {
        const int nf = min(kChunk, T - t0);
        if (t0 > 0) load_chunk<MP>(Xf, t0, nf, M, sT, tid, v);
        __syncthreads();
        constexpr int NIT = kChunkRegs<MP>;
#pragma unroll
        for (int u = 0; u < NIT; ++u) {
            const int e = tid + u * kThreads;
            const int tt = e / MP, m = e - tt * MP;
            const E r = (E)v[u].x, im = (E)v[u].y;
            Pr[m * S + tt] = r;
            Pi[m * S + tt] = im;
            Pn[m * S + tt] = -r;
        }
        __syncthreads();
        if (t0 + kChunk >= T) next(v);
        const int nsteps = (nf + 31) >> 5;
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            const int tile = wave + 4 * q;
            if (tile < NTILE) {
                int I, J;
                tile_coords(tile, NT, I, J);
                const int ca = (16 * I + (lane & 15)) * S, cb = (16 * J + (lane & 15)) * S;
                for (int s = 0; s < nsteps; ++s) {
                    const int k0 = 32 * s + 8 * (lane >> 4);
                    const vec ar = *(const vec *)&Pr[ca + k0];
                    const vec ai = *(const vec *)&Pi[ca + k0];
                    const vec an = *(const vec *)&Pn[ca + k0];
                    const vec br = *(const vec *)&Pr[cb + k0];
                    const vec bi = *(const vec *)&Pi[cb + k0];
                    acc_re[q] = Mfma32<E>::run(ar, br, acc_re[q]);
                    acc_re[q] = Mfma32<E>::run(ai, bi, acc_re[q]);
                    acc_im[q] = Mfma32<E>::run(ai, br, acc_im[q]);
                    acc_im[q] = Mfma32<E>::run(an, bi, acc_im[q]);
                }
            }
        }
    }
    __syncthreads();                           // frames no longer needed: Z holds the result
    float2 *Rs = reinterpret_cast<float2 *>(Z);
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        const int tile = wave + 4 * q;
        if (tile < NTILE) {
            int I, J;
            tile_coords(tile, NT, I, J);
            tile_to_lds(Rs, RS, I, J, acc_re[q], acc_im[q], scale, lane);
        }
    }
    __syncthreads();
    lds_to_out(Rs, RS, M, accumulate, Rf, tid);
}

// ---------------------------------------------------------------------------------------------
// Launch wrappers: one workgroup per bin, either bin f of one block or item (block, bin) of a batch.
// E = float selects the FP32 kernel, __bf16 / _Float16 the 16-bit-input kernel.
template <int MP, typename E, class Next>
__device__ __forceinline__ void corr_bin(const float2 *Xf, int T, int M, int64_t sT, float scale,
                                         int accumulate, float2 *Rf, float2 (&v)[kChunkRegs<MP>],
                                         Next &&next)
{
    if constexpr (sizeof(E) == 4)
        corr_f32_bin<MP>(Xf, T, M, sT, scale, accumulate, Rf, v, next);
    else
        corr_lp_bin<MP, E>(Xf, T, M, sT, scale, accumulate, Rf, v, next);
}

// A resident grid of workgroups strides over the bins (a bin is a few microseconds of work: one
// launch-time workgroup per bin spends as long being dispatched as computing), loading each
// bin's first chunk under the previous bin's products.
template <int MP, typename E>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void corr_single(const float2 *__restrict__ X, int F, int T,
                                                        int M, int64_t sF, int64_t sT, float scale,
                                                        int accumulate, float2 *__restrict__ R)
{
    const int tid = threadIdx.x;
    const int nf0 = min(kChunk, T);
    float2 v[kChunkRegs<MP>];
    if (blockIdx.x < F) load_chunk<MP>(X + (size_t)blockIdx.x * sF, 0, nf0, M, sT, tid, v);
    for (int f = blockIdx.x; f < F; f += gridDim.x) {
        const int fn = f + gridDim.x;
        corr_bin<MP, E>(X + (size_t)f * sF, T, M, sT, scale, accumulate, R + (size_t)f * M * M, v,
                        [&](float2 (&w)[kChunkRegs<MP>]) {
                            if (fn < F) load_chunk<MP>(X + (size_t)fn * sF, 0, nf0, M, sT, tid, w);
                        });
    }
}

template <int MP, typename E>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void corr_batch(const BlockDev *__restrict__ blk,
                                                       const int2 *__restrict__ items, int n_items)
{
    const int tid = threadIdx.x;
    auto first_chunk = [&](int i, float2 (&w)[kChunkRegs<MP>]) {
        const int2 it = items[i];
        const BlockDev &B = blk[it.x];
        load_chunk<MP>(B.X + (size_t)it.y * B.sF, 0, min(kChunk, B.T), B.M, B.sT, tid, w);
    };
    float2 v[kChunkRegs<MP>];
    if ((int)blockIdx.x < n_items) first_chunk(blockIdx.x, v);
    for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
        const int2 it = items[i];
        const BlockDev &B = blk[it.x];
        const int in = i + gridDim.x;
        corr_bin<MP, E>(B.X + (size_t)it.y * B.sF, B.T, B.M, B.sT, B.scale, 0,
                        B.R + (size_t)it.y * B.M * B.M, v, [&](float2 (&w)[kChunkRegs<MP>]) {
                            if (in < n_items) first_chunk(in, w);
                        });
    }
}

// Workgroups of `kernel` resident on the whole device at once, capped at n.
template <typename K>
int resident_grid(K kernel, int n)
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kThreads, 0) != hipSuccess)
        return n;
    const int g = (cus > 0 ? cus : 1) * (per > 0 ? per : 1);
    return n < g ? n : g;
}

// ---------------------------------------------------------------------------------------------
// FP64 accumulation (noise correlation K) on v_mfma_f64_16x16x4f64: the complex64 frames are
// widened exactly to FP64 operands and the products accumulate in FP64.  With x = a + i b,
//   Re K_ij += a_i a_j + b_i b_j,     Im K_ij += b_i a_j - a_i b_j
// over k-steps of 4 frames: A[i][k] = x_{t+k}[16I + i] from lane i + 16k, B[k][j] = x_{t+k}[16J + j]
// from lane j + 16k.  Each wave owns 16x16 tiles of the upper block triangle; the result goes
// through LDS (the lower triangle as the conjugate of the same registers: K is Hermitian to the
// bit, with a zero imaginary diagonal) and leaves in rows.  The FP64 result layout: element e of
// lane l is row l/16 + 4e, column l%16 of the tile.
typedef double doublex4 __attribute__((ext_vector_type(4)));

// mode 0: R = scale S;  1: R = R0 + scale S;  2: R = alpha R0 + (1 - alpha) (scale S),
// S = sum_t x x^H (the blend of the EMA noise update, in the same arithmetic as
// noise_blend_c128).  R0 is read from R0f: Rf itself, or another matrix of the same shape.
constexpr int kStore = 0, kAccumulate = 1, kBlend = 2;

template <int MP>
__device__ __forceinline__ void corr_f64_bin(const float2 *__restrict__ Xf, int T, int M,
                                             int64_t sT, double scale, int mode, double alpha,
                                             const double2 *R0f, double2 *Rf)
{
    constexpr int NT = MP / 16;
    constexpr int NTILE = NT * (NT + 1) / 2;
    constexpr int TPW = (NTILE + 3) / 4;
    constexpr int S = MP + 16;                 // frame row stride: the 4 rows of a step on other banks
    constexpr int RS = MP + 1;                 // result row stride (complex128)
    constexpr int ZB = kChunk * S * 8, RB = MP * RS * 16;
    __shared__ __attribute__((aligned(16))) char buf[ZB > RB ? ZB : RB];
    float2 *Z = reinterpret_cast<float2 *>(buf);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    doublex4 acc_re[TPW], acc_im[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        acc_re[q] = doublex4{0.0, 0.0, 0.0, 0.0};
        acc_im[q] = doublex4{0.0, 0.0, 0.0, 0.0};
    }
    for (int t0 = 0; t0 < T; t0 += kChunk) {
        const int nf = min(kChunk, T - t0);
        float2 v[kChunkRegs<MP>];
        load_chunk<MP>(Xf, t0, nf, M, sT, tid, v);               // every load in flight
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kChunkRegs<MP>; ++u) {               // frame e / MP, channel e % MP
            const int e = tid + u * kThreads;
            Z[(e / MP) * S + e % MP] = v[u];
        }
        __syncthreads();
        const int nsteps = (nf + 3) >> 2;
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            const int tile = wave + 4 * q;
            if (tile < NTILE) {
                int I, J;
                tile_coords(tile, NT, I, J);
                const int ca = 16 * I + (lane & 15), cb = 16 * J + (lane & 15);
                for (int s = 0; s < nsteps; ++s) {
                    const int row = (4 * s + (lane >> 4)) * S;
                    const float2 a = Z[row + ca], b = Z[row + cb];
                    const double ar = a.x, ai = a.y, br = b.x, bi = b.y;
                    acc_re[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, acc_re[q], 0, 0, 0);
                    acc_re[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bi, acc_re[q], 0, 0, 0);
                    acc_im[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, br, acc_im[q], 0, 0, 0);
                    acc_im[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ar, bi, acc_im[q], 0, 0, 0);
                }
            }
        }
    }
    __syncthreads();                           // frames no longer needed: buf holds the result
    double2 *Rs = reinterpret_cast<double2 *>(buf);
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        const int tile = wave + 4 * q;
        if (tile < NTILE) {
            int I, J;
            tile_coords(tile, NT, I, J);
            const int j = 16 * J + (lane & 15);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = 16 * I + (lane >> 4) + 4 * e;
                if (I == J && i > j) continue;           // mirrored from the (j, i) lane
                const double vr = acc_re[q][e] * scale;
                const double vi = (i == j) ? 0.0 : acc_im[q][e] * scale;
                Rs[i * RS + j] = make_double2(vr, vi);
                if (i != j) Rs[j * RS + i] = make_double2(vr, -vi);
            }
        }
    }
    __syncthreads();
    for (int i = wave; i < M; i += kThreads / 64) {              // row by wave, column by lane
        const int j = lane;
        if (j >= M) continue;
        double2 v = Rs[i * RS + j];
        if (mode == kAccumulate) {
            const double2 a = gload(R0f + (size_t)i * M + j);
            v.x += a.x;
            v.y += a.y;
        } else if (mode == kBlend) {
            const double2 a = gload(R0f + (size_t)i * M + j);
            v = make_double2(fma(alpha, a.x, (1.0 - alpha) * v.x),
                             fma(alpha, a.y, (1.0 - alpha) * v.y));
        }
        gstore(Rf + (size_t)i * M + j, v);
    }
}

template <int MP>
__global__ __launch_bounds__(kThreads) void corr_f64(const float2 *__restrict__ X, int T, int M,
                                                     int64_t sF, int64_t sT, double scale,
                                                     int accumulate, double2 *__restrict__ R)
{
    const int f = blockIdx.x;
    double2 *Rf = R + (size_t)f * M * M;
    corr_f64_bin<MP>(X + (size_t)f * sF, T, M, sT, scale, accumulate ? kAccumulate : kStore, 0.0,
                     Rf, Rf);
}

// Item (handle, bin): K[f] <- alpha Ks[f] + (1 - alpha) (1/T) sum_t x x^H of the handle's frames.
template <int MP>
__global__ __launch_bounds__(kThreads) void noise_corr_blend(const NoiseUpdDev *__restrict__ h,
                                                             const int2 *__restrict__ items,
                                                             double alpha)
{
    const int2 it = items[blockIdx.x];
    const NoiseUpdDev &H = h[it.x];
    const int M = H.M, T = H.T, f = it.y;
    corr_f64_bin<MP>(H.X + (size_t)f * T * M, T, M, M, 1.0 / T, kBlend, alpha,
                     H.Ks + (size_t)f * M * M, H.K + (size_t)f * M * M);
}

template <int MP, typename E>
hipError_t launch_mp_t(const float2 *Xp, int F, int T, int M, int64_t sF, int64_t sT, float scale,
                       int accumulate, float2 *Rp, hipStream_t st)
{
    const int g = resident_grid(corr_single<MP, E>, F);
    hipLaunchKernelGGL((corr_single<MP, E>), dim3(g), dim3(kThreads), 0, st, Xp, F, T, M, sF, sT,
                       scale, accumulate, Rp);
    return hipGetLastError();
}

template <int MP>
hipError_t launch_mp(const ssl_c64 *X, int F, int T, int M, int64_t sF, int64_t sT, double scale,
                     int accumulate, ssl_prec prec, void *R, hipStream_t st)
{
    const float2 *Xp = reinterpret_cast<const float2 *>(X);
    float2 *Rp = reinterpret_cast<float2 *>(R);
    if (prec == SSL_FP32)
        return launch_mp_t<MP, float>(Xp, F, T, M, sF, sT, (float)scale, accumulate, Rp, st);
    if (prec == SSL_BF16)
        return launch_mp_t<MP, __bf16>(Xp, F, T, M, sF, sT, (float)scale, accumulate, Rp, st);
    return launch_mp_t<MP, _Float16>(Xp, F, T, M, sF, sT, (float)scale, accumulate, Rp, st);
}

template <int MP, typename E>
hipError_t launch_mp_batch_t(const BlockDev *blk, const int2 *items, int n, hipStream_t st)
{
    const int g = resident_grid(corr_batch<MP, E>, n);
    hipLaunchKernelGGL((corr_batch<MP, E>), dim3(g), dim3(kThreads), 0, st, blk, items, n);
    return hipGetLastError();
}

template <int MP>
hipError_t launch_mp_batch(const BlockDev *blk, const int2 *items, int n, ssl_prec prec,
                           hipStream_t st)
{
    if (prec == SSL_FP32) return launch_mp_batch_t<MP, float>(blk, items, n, st);
    if (prec == SSL_BF16) return launch_mp_batch_t<MP, __bf16>(blk, items, n, st);
    return launch_mp_batch_t<MP, _Float16>(blk, items, n, st);
}

}  // namespace

hipError_t launch_corr(const ssl_c64 *X, int F, int T, int M, int64_t sF, int64_t sT, double scale,
                       int accumulate, ssl_prec prec, void *R, hipStream_t st)
{
    if (prec == SSL_FP64) {
        const float2 *Xp = reinterpret_cast<const float2 *>(X);
        double2 *Rp = reinterpret_cast<double2 *>(R);
        if (M <= 16)
            hipLaunchKernelGGL(corr_f64<16>, dim3(F), dim3(kThreads), 0, st, Xp, T, M, sF, sT,
                               scale, accumulate, Rp);
        else if (M <= 32)
            hipLaunchKernelGGL(corr_f64<32>, dim3(F), dim3(kThreads), 0, st, Xp, T, M, sF, sT,
                               scale, accumulate, Rp);
        else
            hipLaunchKernelGGL(corr_f64<64>, dim3(F), dim3(kThreads), 0, st, Xp, T, M, sF, sT,
                               scale, accumulate, Rp);
        return hipGetLastError();
    }
    switch (corr_class(M)) {
    case 16: return launch_mp<16>(X, F, T, M, sF, sT, scale, accumulate, prec, R, st);
    case 32: return launch_mp<32>(X, F, T, M, sF, sT, scale, accumulate, prec, R, st);
    case 48: return launch_mp<48>(X, F, T, M, sF, sT, scale, accumulate, prec, R, st);
    default: return launch_mp<64>(X, F, T, M, sF, sT, scale, accumulate, prec, R, st);
    }
}

hipError_t launch_noise_corr_blend(const NoiseUpdDev *h, const int2 *items, int n_items, int cls,
                                   double alpha, hipStream_t st)
{
    if (n_items <= 0) return hipSuccess;
    if (cls == 16)
        hipLaunchKernelGGL(noise_corr_blend<16>, dim3(n_items), dim3(kThreads), 0, st, h, items,
                           alpha);
    else if (cls == 32)
        hipLaunchKernelGGL(noise_corr_blend<32>, dim3(n_items), dim3(kThreads), 0, st, h, items,
                           alpha);
    else
        hipLaunchKernelGGL(noise_corr_blend<64>, dim3(n_items), dim3(kThreads), 0, st, h, items,
                           alpha);
    return hipGetLastError();
}

hipError_t launch_corr_batch(const BlockDev *blk, const int2 *items, int n_items, int cls,
                             ssl_prec prec, hipStream_t st)
{
    if (n_items <= 0) return hipSuccess;
    switch (cls) {
    case 16: return launch_mp_batch<16>(blk, items, n_items, prec, st);
    case 32: return launch_mp_batch<32>(blk, items, n_items, prec, st);
    case 48: return launch_mp_batch<48>(blk, items, n_items, prec, st);
    default: return launch_mp_batch<64>(blk, items, n_items, prec, st);
    }
}
