// MUSIC pseudo-spectrum, eq.5 of arXiv 2504.03373 (CalcAveragePower):
//   G[f] = H[f]^H E_n[f]      (D x M) . (M x Nn) complex product per bin, Nn = M - Ns
//   den  = sum_c |G_dc|^p     (p = 2: the projector form; p = 1: the literal form of eq.5)
//   P    = |H_d|^2 / max(den, FLT_MIN)
//
// Complex product as real MFMA products.  Flatten steering row d to 2M reals
// h = (Re H_d0, Im H_d0, Re H_d1, ...) -- exactly its storage -- and let h' = (-Im H_d0, Re H_d0,
// -Im H_d1, ...).  With the noise vector e_c flattened the same way (its complex64 storage),
//   h . e_c = Re(H_d^H e_c),   h' . e_c = Im(H_d^H e_c),
// so one B operand (E_n in its natural layout, <= 64 columns) serves two A operands, and
// |G_dc|^2 = (h . e_c)^2 + (h' . e_c)^2 needs no cross-lane exchange.  h' is formed in registers
// from h (a swap and a sign flip), so the steering table is read once.
//
// Workgroup = WV waves x 16 directions of one bin (WV = 4, 8 or 16, chosen per size class and
// precision, 8 unless tuned); a wave keeps its 16-row strip of H (and h') in registers and owns
// all Nn columns in accumulators.  Workgroups are mapped XCD by XCD so that
// all direction tiles of a bin share one L2.  The batched kernel loops over every block
// that shares the steering table: H is read once per (bin, direction tile) for all of them and
// only E_n (staged in LDS) changes from block to block.
#include "ssl_internal.h"

#include <type_traits>

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

namespace {

template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

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

// Per-type layout constants.  FP32: v_mfma_f32_16x16x4f32, a k-chunk of 16 reals per kq, lane
// slice s = l/16 holding reals 16 kq + 4 s .. +3 (four MFMA steps).  16-bit: 16x16x32, a k-chunk of
// 32 reals, lane slice holding reals 32 kq + 8 s .. +7 (one MFMA step).
template <typename E> struct SteerCfg {
    static constexpr bool F32 = sizeof(E) == 4;
    static constexpr int KC = F32 ? 16 : 32;          // reals per k-chunk
    static constexpr int KQ_MAX = 128 / KC;           // 2M <= 128
    // B row stride KS_MAX (compile-time, so every LDS offset is an immediate): 128 reals plus 32
    // bytes, 8 banks mod 64, so the 16-byte B fragments of the 32 lanes of a half wave (16 rows x
    // 2 k-slices) fall on distinct banks (counted: no LDS bank conflicts)
    static constexpr int PAD = F32 ? 8 : 16;
    static constexpr int KS_MAX = 128 + PAD;
};

// A operands of one wave: rows d0 + 16 w .. +15 of the bin's table, h and h' per k-chunk.
template <typename E> struct AStrip;
template <> struct AStrip<float> {
    float4 a[8];                                       // h' is derived per k-chunk in mma()
};
template <typename E> struct AStrip {
    typename LpMfma<E>::vec a[4], b[4];                // h and h'
};

// (re, im) 16-bit pairs -> (-im, re): swap the halves, flip the sign bit of the new low half.
template <typename V>
__device__ __forceinline__ V twist(V a)
{
    uint32_t w[4];
    __builtin_memcpy(w, &a, 16);
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = __builtin_amdgcn_alignbit(w[i], w[i], 16) ^ 0x8000u;
    return __builtin_bit_cast(V, w);
}

// Loads the strip and returns the partial |h|^2 of this lane's row slice.
template <typename E>
__device__ __forceinline__ float load_strip(const E *__restrict__ Hf, int D, int M, int row,
                                            int sl, AStrip<E> &S)
{
    typedef SteerCfg<E> C;
    const int K2 = 2 * M;
    const int KQ = (K2 + C::KC - 1) / C::KC;
    const E *hrow = Hf + (size_t)(row < D ? row : 0) * K2;
    float hn = 0.f;
    if constexpr (C::F32) {
#pragma unroll
        for (int kq = 0; kq < C::KQ_MAX; ++kq) {
            const int k0 = 16 * kq + 4 * sl;
            float2 lo = make_float2(0.f, 0.f), hi = make_float2(0.f, 0.f);
            if (kq < KQ && row < D) {
                if (k0 < K2) lo = gload((const float2 *)(hrow + k0));    // complex element k0/2
                if (k0 + 2 < K2) hi = gload((const float2 *)(hrow + k0 + 2));
            }
            S.a[kq] = make_float4(lo.x, lo.y, hi.x, hi.y);
            hn = fmaf(lo.x, lo.x, fmaf(lo.y, lo.y, fmaf(hi.x, hi.x, fmaf(hi.y, hi.y, hn))));
        }
    } else {
        typedef typename LpMfma<E>::vec vec;
#pragma unroll
        for (int kq = 0; kq < C::KQ_MAX; ++kq) {
            const int m0 = 16 * kq + 4 * sl;            // complex element of real 32 kq + 8 s
            uint32_t w[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                w[i] = (kq < KQ && row < D && m0 + i < M)
                           ? gload((const uint32_t *)(hrow + 2 * (m0 + i))) : 0u;
            S.a[kq] = __builtin_bit_cast(vec, w);
            S.b[kq] = twist(S.a[kq]);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float fv = (float)S.a[kq][e];
                hn = fmaf(fv, fv, hn);
            }
        }
    }
    return hn;
}

// E_n[f] as the B operand: Bs[c * KS + k] = real k of noise vector c (k < 2M), zero for c >= Nn
// or k >= 2M up to the k-chunk padding KP (KS = KS_MAX).  Thread tid owns elements e = tid + 64 WV u of a
// 16 NCT x 64 complex grid (column c = e / 64 = tid / 64 + WV u, element m = e % 64 = tid % 64);
// load_b puts them in registers (all loads in flight at once), store_b writes those with
// m < KP / 2.
template <int NCT, int WV> struct BStage {
    static constexpr int NIT = 16 * NCT / WV;
    float2 v[NIT];
};

template <int NCT, int WV>
__device__ __forceinline__ void load_b(const float2 *__restrict__ Enf, int M, int Nn, int tid,
                                       BStage<NCT, WV> &st)
{
    // element u of this thread: column c0 + 8u, row m (fixed): one base address and a stride
    const int c0 = tid >> 6, m = tid & 63;
    const float2 *src = Enf + (size_t)c0 * M + m;
    const bool mok = m < M;
#pragma unroll
    for (int u = 0; u < BStage<NCT, WV>::NIT; ++u)
        st.v[u] = (mok && c0 + WV * u < Nn) ? gload(src + (size_t)u * WV * M) : make_float2(0.f, 0.f);
}

template <int NCT, int WV, typename E>
__device__ __forceinline__ void store_b(const BStage<NCT, WV> &st, E *Bs, int KS, int KP, int tid)
{
    const int c0 = tid >> 6, m = tid & 63;
    if (2 * m >= KP) return;
    E *dst = Bs + c0 * KS + 2 * m;
#pragma unroll
    for (int u = 0; u < BStage<NCT, WV>::NIT; ++u) {
        const float2 v = st.v[u];
        if constexpr (sizeof(E) == 4) {
            *(float2 *)(dst + u * WV * KS) = v;
        } else {
            E pr[2] = {(E)v.x, (E)v.y};
            *(uint32_t *)(dst + u * WV * KS) = __builtin_bit_cast(uint32_t, pr);
        }
    }
}

// acc1/acc2[ct] += A(h / h') . B over the k-chunks.
template <int NCT, typename E>
__device__ __forceinline__ void mma(const AStrip<E> &S, const E *Bs, int KS, int KQ, int lane,
                                    floatx4 (&acc1)[NCT], floatx4 (&acc2)[NCT])
{
    typedef SteerCfg<E> C;
    const int sl = lane >> 4;
    const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kq = 0; kq < C::KQ_MAX; ++kq) {
        if (kq >= KQ) break;
        if constexpr (C::F32) {
            const int k0 = 16 * kq + 4 * sl;
            const float4 a = S.a[kq];
            const float4 a2 = make_float4(-a.y, a.x, -a.w, a.z);      // h'
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct) {
                const float4 b = *(const float4 *)&Bs[(16 * ct + (lane & 15)) * KS + k0];
                acc1[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, kq ? acc1[ct] : zero, 0, 0, 0);
                acc2[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2.x, b.x, kq ? acc2[ct] : zero, 0, 0, 0);
                acc1[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc1[ct], 0, 0, 0);
                acc2[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2.y, b.y, acc2[ct], 0, 0, 0);
                acc1[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, acc1[ct], 0, 0, 0);
                acc2[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2.z, b.z, acc2[ct], 0, 0, 0);
                acc1[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, acc1[ct], 0, 0, 0);
                acc2[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2.w, b.w, acc2[ct], 0, 0, 0);
            }
        } else {
            typedef typename LpMfma<E>::vec vec;
            const int k0 = 32 * kq + 8 * sl;
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct) {
                const vec b = *(const vec *)&Bs[(16 * ct + (lane & 15)) * KS + k0];
                acc1[ct] = LpMfma<E>::run(S.a[kq], b, kq ? acc1[ct] : zero);
                acc2[ct] = LpMfma<E>::run(S.b[kq], b, kq ? acc2[ct] : zero);
            }
            // keep the next k-chunk's operand loads from all being hoisted here (register cap)
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// Epilogue.  acc[ct][r] = column 16 ct + l%16 of row 4 (l/16) + r of the wave's strip; den of a
// row is the sum over columns (the 16 lanes of a row group) of |G|^p.  The four row sums of a
// lane are reduced and scattered at once: a mirror exchange across the 16 lanes leaves rows
// {0, 1} on lanes c < 8 and {2, 3} on the others, a half mirror leaves one row per lane (row
// c / 4), and two quad exchanges complete the sums, so lane c of row group g ends with den of row
// 4 g + c / 4.  nrm_s holds |h|^2 of the workgroup's rows.
template <int NCT>
__device__ __forceinline__ void finish_rows(const floatx4 (&acc1)[NCT], const floatx4 (&acc2)[NCT],
                                            int p, int lane, int wave, int d0, int D, bool bin_ok,
                                            float *__restrict__ Pf,
                                            const float *nrm_s)
{
    float part[4];
    if (p == 2) {                          // uniform branch: no square roots on the p = 2 path
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float s = 0.f;
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct)
                s = fmaf(acc1[ct][r], acc1[ct][r], fmaf(acc2[ct][r], acc2[ct][r], s));
            part[r] = s;
        }
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float s = 0.f;
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct)
                s += sqrtf(fmaf(acc1[ct][r], acc1[ct][r], acc2[ct][r] * acc2[ct][r]));
            part[r] = s;
        }
    }
    const int c = lane & 15;
    const bool lo = c < 8, lo2 = (c & 7) < 4;
    const float a0 = (lo ? part[0] : part[2]) + dpp<0x140>(lo ? part[2] : part[0]);   // row_mirror
    const float a1 = (lo ? part[1] : part[3]) + dpp<0x140>(lo ? part[3] : part[1]);
    float den = (lo2 ? a0 : a1) + dpp<0x141>(lo2 ? a1 : a0);                        // row_half_mirror
    den += dpp<0xB1>(den);
    den += dpp<0x4E>(den);
    if ((c & 3) == 0) {
        const int row = wave * 16 + 4 * (lane >> 4) + (c >> 2);
        const int d = d0 + row;
        if (d < D) {
            // hardware reciprocal (1 ulp): P is compared at 1e-4, den >= FLT_MIN
            gstore(Pf + d, bin_ok ? nrm_s[row] * __builtin_amdgcn_rcpf(fmaxf(den, 1.17549435e-38f))
                                  : 0.0f);
        }
    }
}

// One workgroup: directions d0 .. d0 + 16 WV - 1 of bin f for nb blocks sharing the table Hf (the
// bin's [D][2M] rows).  blk(i) gives block i's (E_n of the bin, status ok, Ns, P row of the bin).
template <int NCT, int WV, typename E, class BlockAt>
__device__ __forceinline__ void steer_tile(const E *__restrict__ Hf, int D, int M, int p, int d0,
                                           int nb, BlockAt &&blk)
{
    typedef SteerCfg<E> C;
    constexpr int BSZ = 16 * NCT * C::KS_MAX;
    __shared__ __attribute__((aligned(16))) E Bbuf[2 * BSZ];   // two B stages, alternating by block
    __shared__ float nrm_s[16 * WV];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int K2 = 2 * M;
    const int KQ = (K2 + C::KC - 1) / C::KC;
    const int KP = C::KC * KQ;
    constexpr int KS = C::KS_MAX;

    AStrip<E> S;
    float hn = load_strip<E>(Hf, D, M, d0 + wave * 16 + (lane & 15), lane >> 4, S);
    // |h|^2: combine the 4 k-slices (lanes l, l^16, l^32, l^48)
    hn += __shfl_xor(hn, 16);
    hn += __shfl_xor(hn, 32);
    if (lane < 16) nrm_s[wave * 16 + lane] = hn;

    // software pipeline over the blocks: block i + 1's E_n loads are issued before block i's
    // MFMAs and written to the other LDS stage right after them, then block i's epilogue runs on
    // registers.  One barrier per block: the stage written for block i + 1 was last read by block
    // i - 1's MFMAs, which every wave finished before the previous barrier, so waves need not
    // wait for each other between their MFMAs and their stores, and one wave's stores and
    // epilogue overlap another's MFMAs.  The block descriptors (a chain of dependent reads) are
    // fetched one block further ahead still.
    struct Blk {
        const float2 *En;
        bool ok;
        int Ns;
        float *P;
    };
    Blk cur, nxt, nn;                  // blocks i, i + 1, i + 2 (unused entries stay unread)
    blk(0, cur.En, cur.ok, cur.Ns, cur.P);
    if (nb > 1) blk(1, nxt.En, nxt.ok, nxt.Ns, nxt.P);
    {
        BStage<NCT, WV> st;
        load_b<NCT, WV>(cur.En, M, M - cur.Ns, tid, st);
        store_b<NCT, WV, E>(st, Bbuf, KS, KP, tid);
    }
    __syncthreads();
    for (int i = 0; i < nb; ++i) {
        // opaque copies of the thread indices: the operand addresses derived from them are
        // recomputed per block instead of being hoisted out of the loop and held in registers
        int tid_i = tid, lane_i = lane;
        asm volatile("" : "+v"(tid_i), "+v"(lane_i));
        const bool more = i + 1 < nb;
        E *Bs = Bbuf + (i & 1) * BSZ;
        if (i + 2 < nb) blk(i + 2, nn.En, nn.ok, nn.Ns, nn.P);
        BStage<NCT, WV> st;
        if (more) load_b<NCT, WV>(nxt.En, M, M - nxt.Ns, tid_i, st);
        floatx4 acc1[NCT], acc2[NCT];
        mma<NCT, E>(S, Bs, KS, KQ, lane_i, acc1, acc2);
        if (more) store_b<NCT, WV, E>(st, Bbuf + ((i + 1) & 1) * BSZ, KS, KP, tid_i);
        finish_rows<NCT>(acc1, acc2, p, lane, wave, d0, D, cur.ok, cur.P, nrm_s);
        __syncthreads();                   // next B staged; this B free for block i + 2
        cur = nxt;
        nxt = nn;
    }
}

// Workgroup -> (item, direction tile).  Workgroups are dealt to the 8 XCDs round-robin by linear
// id, so workgroup w runs on XCD w % 8; giving XCD x the items x, x + 8, ... with all their tiles
// back to back keeps every tile of an item (which all stage the same E_n) on one L2.
constexpr int kXcds = 8;
__host__ __device__ inline int xcd_grid(int n_items, int n_tiles)
{
    return kXcds * ((n_items + kXcds - 1) / kXcds) * n_tiles;
}
__device__ __forceinline__ bool xcd_item(int n_items, int n_tiles, int &item, int &tile)
{
    const int w = blockIdx.x;
    const int slot = w / kXcds;
    item = (slot / n_tiles) * kXcds + w % kXcds;
    tile = slot % n_tiles;
    return item < n_items;
}

template <int NCT, typename E, int WV>
__global__ __launch_bounds__(64 * WV) __attribute__((amdgpu_waves_per_eu(4))) void steer_single(const E *__restrict__ H,
                                                         const float2 *__restrict__ En,
                                                         const int32_t *__restrict__ bin_status,
                                                         int F, int D, int M, int Ns, int p,
                                                         float *__restrict__ P, int n_tiles)
{
    int f, tile;
    if (!xcd_item(F, n_tiles, f, tile)) return;
    steer_tile<NCT, WV, E>(H + (size_t)f * D * 2 * M, D, M, p, tile * 16 * WV, 1,
                       [&](int, const float2 *&Enf, bool &ok, int &ns, float *&Pf) {
                           Enf = En + (size_t)f * (M - Ns) * M;
                           ok = bin_status == nullptr || bin_status[f] == SSL_BIN_OK;
                           ns = Ns;
                           Pf = P + (size_t)f * D;
                       });
}

// Batched: item = (group, bin), groups[g] = (first, count) into gblocks, the blocks of one
// steering table.
template <int NCT, typename E, int WV>
__global__ __launch_bounds__(64 * WV) __attribute__((amdgpu_waves_per_eu(4))) void steer_batch(const BlockDev *__restrict__ blk,
                                                        const int2 *__restrict__ items,
                                                        int n_items, int n_tiles,
                                                        const int2 *__restrict__ groups,
                                                        const int *__restrict__ gblocks)
{
    int ii, tile;
    if (!xcd_item(n_items, n_tiles, ii, tile)) return;
    const int2 it = items[ii];
    const int2 gr = groups[it.x];
    const BlockDev &B0 = blk[gblocks[gr.x]];
    const int d0 = tile * 16 * WV;
    if (d0 >= B0.D) return;
    const int f = it.y, M = B0.M, D = B0.D;
    steer_tile<NCT, WV, E>(static_cast<const E *>(B0.H) + (size_t)f * D * 2 * M, D, M, B0.p, d0, gr.y,
                       [&](int i, const float2 *&Enf, bool &ok, int &ns, float *&Pf) {
                           const BlockDev &B = blk[gblocks[gr.x + i]];
                           Enf = B.En + (size_t)f * (M - B.Ns) * M;
                           ok = gload(B.status + f) == SSL_BIN_OK;
                           ns = B.Ns;
                           Pf = B.P + (size_t)f * D;
                       });
}

// Calls fn(NCT, WV, (E *)nullptr) with the compile-time variant for (class, waves, precision).
template <class Fn>
hipError_t dispatch(int cls, int waves, ssl_prec prec, Fn &&fn)
{
    auto by_type = [&](auto nct, auto wv) -> hipError_t {
        if (prec == SSL_FP32) return fn(nct, wv, (float *)nullptr);
        if (prec == SSL_BF16) return fn(nct, wv, (__bf16 *)nullptr);
        return fn(nct, wv, (_Float16 *)nullptr);
    };
    auto by_waves = [&](auto nct) -> hipError_t {
        if (waves == 4) return by_type(nct, std::integral_constant<int, 4>{});
        if (waves == 16) return by_type(nct, std::integral_constant<int, 16>{});
        return by_type(nct, std::integral_constant<int, 8>{});
    };
    if (cls == 1) return by_waves(std::integral_constant<int, 1>{});
    if (cls == 2) return by_waves(std::integral_constant<int, 2>{});
    return by_waves(std::integral_constant<int, 4>{});
}

}  // namespace

bool steer_waves_ok(int waves) { return waves == 4 || waves == 8 || waves == 16; }
int steer_rows_per_block(int waves) { return 16 * waves; }

hipError_t launch_steer(const void *H, ssl_prec hprec, const ssl_c64 *En, int F, int D, int M,
                        int Ns, int p, const int32_t *bin_status, float *P, int waves,
                        hipStream_t st)
{
    const float2 *Ep = reinterpret_cast<const float2 *>(En);
    return dispatch(steer_class(M, Ns), waves, hprec, [&](auto nct, auto wv, auto *tag) {
        typedef std::remove_pointer_t<decltype(tag)> E;
        constexpr int NCT = decltype(nct)::value, WV = decltype(wv)::value;
        const int nt = (D + 16 * WV - 1) / (16 * WV);
        hipLaunchKernelGGL((steer_single<NCT, E, WV>), dim3(xcd_grid(F, nt)), dim3(64 * WV), 0,
                           st, static_cast<const E *>(H), Ep, bin_status, F, D, M, Ns, p, P, nt);
        return hipGetLastError();
    });
}

hipError_t launch_steer_batch(const BlockDev *blk, const int2 *items, int n_items,
                              const int2 *groups, const int *gblocks, int cls, int waves,
                              int max_dtiles, ssl_prec hprec, hipStream_t st)
{
    if (n_items <= 0) return hipSuccess;
    return dispatch(cls, waves, hprec, [&](auto nct, auto wv, auto *tag) {
        typedef std::remove_pointer_t<decltype(tag)> E;
        constexpr int NCT = decltype(nct)::value, WV = decltype(wv)::value;
        hipLaunchKernelGGL((steer_batch<NCT, E, WV>), dim3(xcd_grid(n_items, max_dtiles)),
                           dim3(64 * WV), 0, st, blk, items, n_items, max_dtiles, groups,
                           gblocks);
        return hipGetLastError();
    });
}
