// MUSIC pseudo-spectrum, eq.5 of arXiv 2504.03373 (CalcAveragePower):
//   G[f] = H[f]^H E_n[f]      (D x M) . (M x Nn) complex product per bin, Nn = M - Ns
//   den  = sum_c |G_dc|^p     (p = 2: the projector form; p = 1: the literal form of eq.5)
//   P    = |H_d|^2 / max(den, FLT_MIN)
//
// Complex product as one real MFMA product.  Flatten H row d to 2M reals h = (Re H_d0, Im H_d0,
// Re H_d1, ...) -- exactly its complex64 storage -- and give each noise vector e_c two real
// columns, (Re e, Im e)-interleaved and (Im e, -Re e)-interleaved; then
//   h . col(2c) = Re(H_d^H e_c),   h . col(2c+1) = Im(H_d^H e_c),
// so G is a [D x 2M] . [2M x 2Nn] real product and |G_dc|^2 is the sum of squares of the two
// adjacent outputs.  The B operand (E_n, <= 64 KB) is staged once per workgroup in LDS as
// [column][k]; the A operand streams from HBM (the steering table is the dominant traffic).
// Workgroup = 8 waves x 16 directions; a wave owns 16 rows x all 2Nn columns in accumulators.
#include "ssl_internal.h"

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int kThreads = 512;            // 8 waves x 16 directions
constexpr int kRowsPerBlock = 128;
constexpr int kMaxColTiles = 8;          // 2 * Nn <= 126 -> 8 tiles of 16 columns

template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float sum16(float v)
{
    v += dpp<0xB1>(v);
    v += dpp<0x4E>(v);
    v += dpp<0x141>(v);
    v += dpp<0x140>(v);
    return v;
}

// Shared epilogue.  acc[ct][r] = G-column (16 ct + l%16) of row (4 (l/16) + r) of this wave's
// 16-row strip.  hn = partial |h|^2 of row l%16 over this lane's k-slice.
template <int NCT>
__device__ __forceinline__ void finish_rows(const floatx4 (&acc)[NCT], float hn, int p, int lane,
                                            int wave, int d0, int D, bool bin_ok,
                                            float *__restrict__ Pf, float *den_s, float *nrm_s)
{
    float part[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        float s = 0.f;
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
            const float v = acc[ct][r];
            if (p == 2) {
                s = fmaf(v, v, s);
            } else {
                const float w = dpp<0xB1>(v);                 // partner column (2c <-> 2c+1)
                const float mag = sqrtf(fmaf(v, v, w * w));
                s += (lane & 1) ? 0.f : mag;
            }
        }
        part[r] = sum16(s);
    }
    // |h|^2: combine the 4 k-slices (lanes l, l^16, l^32, l^48)
    hn += __shfl_xor(hn, 16);
    hn += __shfl_xor(hn, 32);
    if ((lane & 15) == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) den_s[wave * 16 + 4 * (lane >> 4) + r] = part[r];
    }
    if (lane < 16) nrm_s[wave * 16 + lane] = hn;
    __syncthreads();
    if (lane < 16) {
        const int d = d0 + wave * 16 + lane;
        if (d < D) {
            const float den = den_s[wave * 16 + lane];
            Pf[d] = bin_ok ? nrm_s[wave * 16 + lane] / fmaxf(den, 1.17549435e-38f) : 0.0f;
        }
    }
}

// Stage E_n[f] as the real B operand: Bs[col * KS + k], col < 16*NCT, k < KP (zero padded).
template <typename E>
__device__ __forceinline__ void stage_b(const float2 *__restrict__ Enf, int M, int Nn, E *Bs,
                                        int KS, int NCOL, int KP, int tid)
{
    for (int e = tid; e < (NCOL / 2) * (KP / 2); e += kThreads) {
        const int col2 = e / (KP / 2);           // pair of columns (2c, 2c+1)
        const int m = e - col2 * (KP / 2);       // k = 2m, 2m+1
        float er = 0.f, ei = 0.f;
        if (col2 < Nn && m < M) {
            const float2 v = Enf[(size_t)col2 * M + m];
            er = v.x;
            ei = v.y;
        }
        Bs[(2 * col2) * KS + 2 * m] = (E)er;
        Bs[(2 * col2) * KS + 2 * m + 1] = (E)ei;
        Bs[(2 * col2 + 1) * KS + 2 * m] = (E)ei;
        Bs[(2 * col2 + 1) * KS + 2 * m + 1] = (E)(-er);
    }
}

// ---------------------------------------------------------------------------------------------
// FP32: v_mfma_f32_16x16x4f32.  Lane l = (row i = l%16, slice s = l/16) reads the float4
// h[16 kq + 4 s .. +3] of its row; MFMA step e (0..3) contracts k = 16 kq + 4 s + e, and the B
// operand of the same k is the float4 Bs[col][16 kq + 4 s .. +3].
// One workgroup tile: directions d0 .. d0 + kRowsPerBlock - 1 of one bin.  Hf = the bin's [D][2M]
// table, Enf = its [Nn][M] noise subspace, Pf = its [D] output, ok = bin status is SSL_BIN_OK.
template <int NCT>
__device__ __forceinline__ void steer_f32_tile(const float *__restrict__ Hf,
                                               const float2 *__restrict__ Enf, bool ok, int D,
                                               int M, int Ns, int p, float *__restrict__ Pf,
                                               int d0)
{
    constexpr int KS_MAX = 128 + 4;
    __shared__ __attribute__((aligned(16))) float Bs[16 * NCT * KS_MAX];
    __shared__ float den_s[kRowsPerBlock];
    __shared__ float nrm_s[kRowsPerBlock];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int Nn = M - Ns;
    const int K2 = 2 * M;
    const int KQ = (K2 + 15) / 16;
    const int KP = 16 * KQ;
    const int KS = KP + 4;
    const int NCOL = 16 * NCT;
    stage_b<float>(Enf, M, Nn, Bs, KS, NCOL, KP, tid);
    __syncthreads();

    const int row = d0 + wave * 16 + (lane & 15);
    const int sl = lane >> 4;
    const float *hrow = Hf + (size_t)(row < D ? row : 0) * K2;
    // the wave's whole 16-row strip of H in registers first: every load in flight at once
    constexpr int KQ_MAX = 8;
    float4 a[KQ_MAX];
    float hn = 0.f;
#pragma unroll
    for (int kq = 0; kq < KQ_MAX; ++kq) {
        const int k0 = 16 * kq + 4 * sl;
        float2 lo = make_float2(0.f, 0.f), hi = make_float2(0.f, 0.f);
        if (kq < KQ && row < D) {
            if (k0 < K2) lo = *(const float2 *)(hrow + k0);          // complex element k0/2
            if (k0 + 2 < K2) hi = *(const float2 *)(hrow + k0 + 2);
        }
        a[kq] = make_float4(lo.x, lo.y, hi.x, hi.y);
    }
#pragma unroll
    for (int kq = 0; kq < KQ_MAX; ++kq)
        hn = fmaf(a[kq].x, a[kq].x, fmaf(a[kq].y, a[kq].y, fmaf(a[kq].z, a[kq].z, fmaf(a[kq].w, a[kq].w, hn))));
    floatx4 acc[NCT];
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) acc[ct] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kq = 0; kq < KQ_MAX; ++kq) {
        if (kq < KQ) {
            const int k0 = 16 * kq + 4 * sl;
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct) {
                const float4 b = *(const float4 *)&Bs[(16 * ct + (lane & 15)) * KS + k0];
                acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[kq].x, b.x, acc[ct], 0, 0, 0);
                acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[kq].y, b.y, acc[ct], 0, 0, 0);
                acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[kq].z, b.z, acc[ct], 0, 0, 0);
                acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[kq].w, b.w, acc[ct], 0, 0, 0);
            }
        }
    }
    finish_rows<NCT>(acc, hn, p, lane, wave, d0, D, ok, Pf, den_s, nrm_s);
}

// ---------------------------------------------------------------------------------------------
// bf16 / fp16: v_mfma_f32_16x16x32_{bf16,f16}.  H is stored as interleaved 16-bit pairs; lane
// (row i = l%16, slice s = l/16) reads 8 consecutive k = 32 ks + 8 s .. +7.
template <typename E> struct LpMfma;
template <> struct LpMfma<__bf16> {
    typedef bf16x8 vec;
    static __device__ __forceinline__ floatx4 run(vec a, vec b, floatx4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct LpMfma<_Float16> {
    typedef halfx8 vec;
    static __device__ __forceinline__ floatx4 run(vec a, vec b, floatx4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

template <int NCT, typename E>
__device__ __forceinline__ void steer_lp_tile(const E *__restrict__ Hf,
                                              const float2 *__restrict__ Enf, bool ok, int D,
                                              int M, int Ns, int p, float *__restrict__ Pf,
                                              int d0)
{
    typedef typename LpMfma<E>::vec vec;
    constexpr int KS_MAX = 128 + 8;
    __shared__ __attribute__((aligned(16))) E Bs[16 * NCT * KS_MAX];
    __shared__ float den_s[kRowsPerBlock];
    __shared__ float nrm_s[kRowsPerBlock];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int Nn = M - Ns;
    const int K2 = 2 * M;
    const int KQ = (K2 + 31) / 32;
    const int KP = 32 * KQ;
    const int KS = KP + 8;
    const int NCOL = 16 * NCT;
    stage_b<E>(Enf, M, Nn, Bs, KS, NCOL, KP, tid);
    __syncthreads();

    const int row = d0 + wave * 16 + (lane & 15);
    const int sl = lane >> 4;
    const E *hrow = Hf + (size_t)(row < D ? row : 0) * K2;
    // the strip in registers first; each complex element is one 32-bit (re, im) pair
    constexpr int KQ_MAX = 4;
    vec a[KQ_MAX];
    float hn = 0.f;
#pragma unroll
    for (int kq = 0; kq < KQ_MAX; ++kq) {
        const int m0 = 16 * kq + 4 * sl;                 // complex element of k0 = 32 kq + 8 s
        uint32_t w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            w[i] = (kq < KQ && row < D && m0 + i < M)
                       ? *(const uint32_t *)(hrow + 2 * (m0 + i)) : 0u;
        a[kq] = __builtin_bit_cast(vec, w);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float fv = (float)a[kq][e];
            hn = fmaf(fv, fv, hn);
        }
    }
    floatx4 acc[NCT];
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) acc[ct] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kq = 0; kq < KQ_MAX; ++kq) {
        if (kq < KQ) {
            const int k0 = 32 * kq + 8 * sl;
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct) {
                const vec b = *(const vec *)&Bs[(16 * ct + (lane & 15)) * KS + k0];
                acc[ct] = LpMfma<E>::run(a[kq], b, acc[ct]);
            }
        }
    }
    finish_rows<NCT>(acc, hn, p, lane, wave, d0, D, ok, Pf, den_s, nrm_s);
}

// E = float selects the FP32 tile, __bf16 / _Float16 the 16-bit tile.
template <int NCT, typename E>
__device__ __forceinline__ void steer_tile(const E *Hf, const float2 *Enf, bool ok, int D, int M,
                                           int Ns, int p, float *Pf, int d0)
{
    if constexpr (sizeof(E) == 4)
        steer_f32_tile<NCT>(Hf, Enf, ok, D, M, Ns, p, Pf, d0);
    else
        steer_lp_tile<NCT, E>(Hf, Enf, ok, D, M, Ns, p, Pf, d0);
}

template <int NCT, typename E>
__global__ __launch_bounds__(kThreads) void steer_single(const E *__restrict__ H,
                                                         const float2 *__restrict__ En,
                                                         const int32_t *__restrict__ bin_status,
                                                         int D, int M, int Ns, int p,
                                                         float *__restrict__ P)
{
    const int f = blockIdx.y;
    const bool ok = bin_status == nullptr || bin_status[f] == SSL_BIN_OK;
    steer_tile<NCT, E>(H + (size_t)f * D * 2 * M, En + (size_t)f * (M - Ns) * M, ok, D, M, Ns, p,
                       P + (size_t)f * D, blockIdx.x * kRowsPerBlock);
}

template <int NCT, typename E>
__global__ __launch_bounds__(kThreads) void steer_batch(const BlockDev *__restrict__ blk,
                                                        const int2 *__restrict__ items)
{
    const int2 it = items[blockIdx.x];            // items on x: a batch may exceed 65535 of them
    const BlockDev &B = blk[it.x];
    const int d0 = blockIdx.y * kRowsPerBlock;
    if (d0 >= B.D) return;
    const int f = it.y, M = B.M, Ns = B.Ns, D = B.D;
    const bool ok = B.status[f] == SSL_BIN_OK;
    steer_tile<NCT, E>(static_cast<const E *>(B.H) + (size_t)f * D * 2 * M,
                       B.En + (size_t)f * (M - Ns) * M, ok, D, M, Ns, B.p, B.P + (size_t)f * D,
                       d0);
}

template <int NCT>
hipError_t launch_nct(const void *H, ssl_prec hprec, const ssl_c64 *En, int F, int D, int M,
                      int Ns, int p, const int32_t *bin_status, float *P, hipStream_t st)
{
    const dim3 grid((D + kRowsPerBlock - 1) / kRowsPerBlock, F);
    const float2 *Ep = reinterpret_cast<const float2 *>(En);
    if (hprec == SSL_FP32)
        hipLaunchKernelGGL((steer_single<NCT, float>), grid, dim3(kThreads), 0, st,
                           static_cast<const float *>(H), Ep, bin_status, D, M, Ns, p, P);
    else if (hprec == SSL_BF16)
        hipLaunchKernelGGL((steer_single<NCT, __bf16>), grid, dim3(kThreads), 0, st,
                           static_cast<const __bf16 *>(H), Ep, bin_status, D, M, Ns, p, P);
    else
        hipLaunchKernelGGL((steer_single<NCT, _Float16>), grid, dim3(kThreads), 0, st,
                           static_cast<const _Float16 *>(H), Ep, bin_status, D, M, Ns, p, P);
    return hipGetLastError();
}

template <int NCT>
hipError_t launch_nct_batch(const BlockDev *blk, const int2 *items, int n_items, int max_dtiles,
                            ssl_prec hprec, hipStream_t st)
{
    const dim3 grid(n_items, max_dtiles);
    if (hprec == SSL_FP32)
        hipLaunchKernelGGL((steer_batch<NCT, float>), grid, dim3(kThreads), 0, st, blk, items);
    else if (hprec == SSL_BF16)
        hipLaunchKernelGGL((steer_batch<NCT, __bf16>), grid, dim3(kThreads), 0, st, blk, items);
    else
        hipLaunchKernelGGL((steer_batch<NCT, _Float16>), grid, dim3(kThreads), 0, st, blk, items);
    return hipGetLastError();
}

}  // namespace

int steer_rows_per_block() { return kRowsPerBlock; }

hipError_t launch_steer(const void *H, ssl_prec hprec, const ssl_c64 *En, int F, int D, int M,
                        int Ns, int p, const int32_t *bin_status, float *P, hipStream_t st)
{
    switch (steer_class(M, Ns)) {
    case 1: return launch_nct<1>(H, hprec, En, F, D, M, Ns, p, bin_status, P, st);
    case 2: return launch_nct<2>(H, hprec, En, F, D, M, Ns, p, bin_status, P, st);
    case 4: return launch_nct<4>(H, hprec, En, F, D, M, Ns, p, bin_status, P, st);
    default: return launch_nct<kMaxColTiles>(H, hprec, En, F, D, M, Ns, p, bin_status, P, st);
    }
}

hipError_t launch_steer_batch(const BlockDev *blk, const int2 *items, int n_items, int cls,
                              int max_dtiles, ssl_prec hprec, hipStream_t st)
{
    if (n_items <= 0) return hipSuccess;
    switch (cls) {
    case 1: return launch_nct_batch<1>(blk, items, n_items, max_dtiles, hprec, st);
    case 2: return launch_nct_batch<2>(blk, items, n_items, max_dtiles, hprec, st);
    case 4: return launch_nct_batch<4>(blk, items, n_items, max_dtiles, hprec, st);
    default: return launch_nct_batch<kMaxColTiles>(blk, items, n_items, max_dtiles, hprec, st);
    }
}
