// MUSIC pseudo-spectrum, eq.5 of arXiv 2504.03373 with p = 2, through the signal subspace.
//
// With U = [E_s E_n] unitary, sum over the noise vectors of |h^H e|^2 = |h|^2 - |E_s^H h|^2, so the
// denominator needs the Ns signal vectors instead of the M - Ns noise vectors (2 instead of 58 on
// the 60-channel workload).  The difference cancels where h lies close to the signal subspace --
// at the peaks -- so it is formed in FP64 from FP64 products of the stored complex64 inputs, and
// with the exact projector onto span E_s, E_s (E_s^H E_s)^{-1} E_s^H (the Jacobi solve supplies
// L^{-1}, L the Cholesky factor of the Gram matrix in FP64), so that the O(2^-24) departure of the
// stored vectors from orthonormality does not enter:
//   g = E_s^H h (FP64),   den = |h|^2 - |L^{-1} g|^2,   P = |h|^2 / max(den, FLT_MIN).
// What remains of the stored vectors' rounding is a rotation of their span, whose effect on den is
// first order in sqrt(den), as for the noise-vector form (the solver's own subspace error enters
// both forms the same way).
//
// Workgroup = 4 waves x 16 directions of one bin; a wave keeps its 16 rows of H in registers
// (complex64) and computes g for 16 columns at once on v_mfma_f64_16x16x4f64 -- the signal vectors
// of 16 / Ns_max blocks sharing the steering table, staged in LDS -- with
//   Re g = sum a c + b d,   Im g = sum b c - a d     (h = a + ib, e = c + id, FP64 operands:
// g_s = e_s^H h, the conjugate of h^H e_s, so that y = L^{-1} g with L from E_s^H E_s = L L^H),
// on three real products instead of four (Gauss's trick): P1 = sum a c, P2 = sum b (-d),
// P3 = sum (a + b)(c - d), Re g = P1 - P2, Im g = P3 - P1 - P2.  a + b and c - d are sums of two
// FP32-representable values, exact in FP64 unless their exponents differ by more than 29.
// The 16 x 16 result goes through LDS so that each lane finishes whole (direction, block) items.
#include "ssl_internal.h"

namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kRows = 16 * kWaves;          // directions per workgroup
constexpr int kCols = 16;                   // signal vectors per MFMA tile
constexpr int kKq = SSL_MAX_M / 4;          // k-steps of 4 complex elements at M = 64
constexpr int kEs = SSL_MAX_M + 2;          // complex64 stride of a staged signal vector
constexpr int kChunk = kThreads;            // blocks whose descriptors are held in LDS at once

// Steering-table readers: one complex element per word, complex64 (FP32 tables) or a pair of
// 16-bit values (re at the lower address) for bf16 / fp16 tables, widened exactly to FP32.
struct TabF32 {
    typedef float2 W;
    static __device__ __forceinline__ float2 get(const W *p) { return gload(p); }
};
struct TabBF16 {
    typedef unsigned int W;
    static __device__ __forceinline__ float2 get(const W *p)
    {
        const unsigned int w = gload(p);
        return make_float2(__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u));
    }
};
struct TabF16 {
    typedef unsigned int W;
    static __device__ __forceinline__ float2 get(const W *p)
    {
        const unsigned int w = gload(p);
        return make_float2((float)__builtin_bit_cast(_Float16, (unsigned short)(w & 0xffffu)),
                           (float)__builtin_bit_cast(_Float16, (unsigned short)(w >> 16)));
    }
};

// One workgroup: directions d0 .. d0 + 63 of bin f for nb blocks sharing the table Hf (the bin's
// [D][M] complex64 rows).  blk(i, Es, L, ns, ok, P) gives block i's signal vectors and L^{-1} of
// the bin, its Ns, whether the bin is valid, and its P row of the bin.
template <class Tab, class BlockAt>
__device__ __forceinline__ void sig_tile(const typename Tab::W *__restrict__ Hf, int D, int M,
                                         int d0, int nb, int nsmax, BlockAt &&blk)
{
    __shared__ float2 Es[2][kCols * kEs];                    // signal vectors, by tile parity
    __shared__ double2 Ls[2][kCols][6];
    __shared__ double2 Gs[kWaves][16 * kCols];
    __shared__ float *Pp[kChunk];                            // per block of the chunk
    __shared__ const float2 *Ep[kChunk];
    __shared__ const double2 *Lp[kChunk];
    __shared__ int Nsb[kChunk];
    __shared__ double nrm_s[kRows];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int KQ = (M + 3) >> 2;
    const int bpt = kCols / nsmax;                           // blocks per tile

    // this lane's A operands: row (lane & 15), complex elements 4 q + (lane >> 4)
    const int row = d0 + 16 * wave + (lane & 15);
    const typename Tab::W *hrow = Hf + (size_t)(row < D ? row : 0) * M;
    float2 ha[kKq];
    double hn = 0.0;
#pragma unroll
    for (int q = 0; q < kKq; ++q) {
        const int m = 4 * q + (lane >> 4);
        ha[q] = (q < KQ && m < M && row < D) ? Tab::get(hrow + m) : make_float2(0.f, 0.f);
        hn = fma((double)ha[q].x, (double)ha[q].x, fma((double)ha[q].y, (double)ha[q].y, hn));
    }
    hn += __shfl_xor(hn, 16);
    hn += __shfl_xor(hn, 32);
    if (lane < 16) nrm_s[16 * wave + lane] = hn;

    // One tile's operands into registers: thread x < kCols * SSL_MAX_M (kPer per thread) holds
    // element m of column j = block j / nsmax, vector j % nsmax (zero if absent); threads below
    // kCols * 6 hold one L^{-1} entry.  Loaded one tile ahead, so that the loads are in flight
    // under the current tile's products and epilogue; stored to the other parity's buffers.
    constexpr int kPer = kCols * SSL_MAX_M / kThreads;
    float2 ev[kPer];
    double2 lv;
    auto load_tile = [&](int c0, int nt) {                   // c0: first block, chunk-relative
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int x = tid + kThreads * i;
            const int j = x / SSL_MAX_M, m = x - j * SSL_MAX_M;
            const int bi = j / nsmax, s = j - bi * nsmax;
            ev[i] = (bi < nt && m < M && s < Nsb[c0 + bi]) ? gload(Ep[c0 + bi] + (size_t)s * M + m)
                                                           : make_float2(0.f, 0.f);
        }
        const int bi = tid / 6, k = tid - bi * 6;
        lv = (tid < kCols * 6 && bi < nt && Nsb[c0 + bi] > 0) ? gload(Lp[c0 + bi] + k)
                                                              : make_double2(0.0, 0.0);
    };
    auto store_tile = [&](int buf) {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int x = tid + kThreads * i;
            const int j = x / SSL_MAX_M, m = x - j * SSL_MAX_M;
            Es[buf][j * kEs + m] = ev[i];
        }
        if (tid < kCols * 6) Ls[buf][tid / 6][tid % 6] = lv;
    };

    for (int h0 = 0; h0 < nb; h0 += kChunk) {               // chunks of the blocks' descriptors
        const int nc = min(kChunk, nb - h0);
        __syncthreads();                                     // the previous chunk is finished
        if (tid < nc) {
            const float2 *e;
            const double2 *L;
            float *P;
            int ns = 0;
            bool ok = false;
            blk(h0 + tid, e, L, ns, ok, P);
            Nsb[tid] = ok ? ns : 0;
            Pp[tid] = P;
            Ep[tid] = e;
            Lp[tid] = L;
        }
        __syncthreads();
        const int ntiles = (nc + bpt - 1) / bpt;
        load_tile(0, min(bpt, nc));
        store_tile(0);
        __syncthreads();
        for (int t = 0; t < ntiles; ++t) {
            const int buf = t & 1, c0 = t * bpt, nt = min(bpt, nc - c0);
            if (t + 1 < ntiles) load_tile(c0 + bpt, min(bpt, nc - c0 - bpt));
            doublex4 p1 = {0.0, 0.0, 0.0, 0.0}, p2 = {0.0, 0.0, 0.0, 0.0}, p3 = {0.0, 0.0, 0.0, 0.0};
            const float2 *ecol = Es[buf] + (lane & 15) * kEs + (lane >> 4);
#pragma unroll
            for (int q = 0; q < kKq; ++q) {
                if (q < KQ) {                                // uniform
                    const float2 e = ecol[4 * q];
                    const double a = ha[q].x, b = ha[q].y, c = e.x, d = e.y;
                    p1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, c, p1, 0, 0, 0);
                    p2 = __builtin_amdgcn_mfma_f64_16x16x4f64(b, -d, p2, 0, 0, 0);
                    p3 = __builtin_amdgcn_mfma_f64_16x16x4f64(a + b, c - d, p3, 0, 0, 0);
                }
            }
            const doublex4 gre = p1 - p2, gim = p3 - p1 - p2;
            // FP64 result layout: element e of lane l is row l / 16 + 4 e, column l % 16
#pragma unroll
            for (int e = 0; e < 4; ++e)
                Gs[wave][((lane >> 4) + 4 * e) * kCols + (lane & 15)] =
                    make_double2(gre[e], gim[e]);
            __syncthreads();
            // items (direction row i of this wave, block bi): den = |h|^2 - |L^{-1} g|^2
            for (int it = lane; it < 16 * nt; it += 64) {
                const int i = it / nt, bi = it - i * nt;
                const int d = d0 + 16 * wave + i;
                float *P = Pp[c0 + bi];
                if (d >= D || P == nullptr) continue;
                const int ns = Nsb[c0 + bi];
                const double hh = nrm_s[16 * wave + i];
                float out = 0.0f;
                if (ns > 0) {
                    const double2 *g = &Gs[wave][i * kCols + bi * nsmax];
                    const double2 *L = Ls[buf][bi];
                    double2 y0 = make_double2(0.0, 0.0), y1 = y0, y2 = y0;
                    // y = L^{-1} g, L^{-1} lower triangular by rows (00, 10, 11, 20, 21, 22)
                    const double2 g0 = g[0];
                    y0 = make_double2(L[0].x * g0.x, L[0].x * g0.y);
                    double q2 = y0.x * y0.x + y0.y * y0.y;
                    if (ns >= 2) {
                        const double2 g1 = g[1];
                        y1 = make_double2(L[1].x * g0.x - L[1].y * g0.y + L[2].x * g1.x,
                                          L[1].x * g0.y + L[1].y * g0.x + L[2].x * g1.y);
                        q2 += y1.x * y1.x + y1.y * y1.y;
                    }
                    if (ns >= 3) {
                        const double2 g1 = g[1], g2 = g[2];
                        y2 = make_double2(L[3].x * g0.x - L[3].y * g0.y + L[4].x * g1.x -
                                              L[4].y * g1.y + L[5].x * g2.x,
                                          L[3].x * g0.y + L[3].y * g0.x + L[4].x * g1.y +
                                              L[4].y * g1.x + L[5].x * g2.y);
                        q2 += y2.x * y2.x + y2.y * y2.y;
                    }
                    const double den = fmax(hh - q2, 1.17549435e-38);
                    out = (float)(hh / den);
                }
                gstore(P + d, out);
            }
            // the other parity was last read in the previous tile, before this tile's barrier
            if (t + 1 < ntiles) store_tile(buf ^ 1);
            __syncthreads();
        }
    }
}

// Workgroup -> (item, direction tile), dealt XCD by XCD as in the noise-vector projection.
constexpr int kXcds = 8;
__host__ __device__ inline int sig_grid(int n_items, int n_tiles)
{
    return kXcds * ((n_items + kXcds - 1) / kXcds) * n_tiles;
}
__device__ __forceinline__ bool sig_item(int n_items, int n_tiles, int &item, int &tile)
{
    const int w = blockIdx.x;
    const int slot = w / kXcds;
    item = (slot / n_tiles) * kXcds + w % kXcds;
    tile = slot % n_tiles;
    return item < n_items;
}

template <class Tab>
__global__ __launch_bounds__(kThreads) void steer_sig_single(
    const typename Tab::W *__restrict__ H, const float2 *__restrict__ Es,
    const double2 *__restrict__ Esl,
    const int32_t *__restrict__ bin_status, int F, int D, int M, int Ns, float *__restrict__ P,
    int n_tiles)
{
    int f, tile;
    if (!sig_item(F, n_tiles, f, tile)) return;
    sig_tile<Tab>(H + (size_t)f * D * M, D, M, tile * kRows, 1, Ns,
             [&](int, const float2 *&e, const double2 *&L, int &ns, bool &ok, float *&Pf) {
                 e = Es + (size_t)f * Ns * M;
                 L = Esl + 6 * (size_t)f;
                 ns = Ns;
                 ok = bin_status == nullptr || bin_status[f] == SSL_BIN_OK;
                 Pf = P + (size_t)f * D;
             });
}

// Batched: item = (group, bin), groups[g] = (first, count) into gblocks, the blocks of one
// steering table; nsmax = the largest Ns of the batch.
// (3 waves per SIMD: the next tile's operands in registers would otherwise cost one)
template <class Tab>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(3))) void steer_sig_batch(
    const BlockDev *__restrict__ blk, const int2 *__restrict__ items, int n_items, int n_tiles,
    const int2 *__restrict__ groups, const int *__restrict__ gblocks, int nsmax)
{
    int ii, tile;
    if (!sig_item(n_items, n_tiles, ii, tile)) return;
    const int2 it = items[ii];
    const int2 gr = groups[it.x];
    const BlockDev &B0 = blk[gblocks[gr.x]];
    const int d0 = tile * kRows;
    if (d0 >= B0.D) return;
    const int f = it.y, M = B0.M, D = B0.D;
    sig_tile<Tab>(static_cast<const typename Tab::W *>(B0.H) + (size_t)f * D * M, D, M, d0, gr.y,
                  nsmax,
             [&](int i, const float2 *&e, const double2 *&L, int &ns, bool &ok, float *&Pf) {
                 const BlockDev &B = blk[gblocks[gr.x + i]];
                 e = B.Es + (size_t)f * B.Ns * M;
                 L = B.Esl + 6 * (size_t)f;
                 ns = B.Ns;
                 ok = gload(B.status + f) == SSL_BIN_OK;
                 Pf = B.P + (size_t)f * D;
             });
}

// Calls fn with the table reader of prec.
template <class Fn>
hipError_t with_table(ssl_prec prec, Fn &&fn)
{
    if (prec == SSL_BF16) return fn(TabBF16());
    if (prec == SSL_FP16) return fn(TabF16());
    return fn(TabF32());
}

}  // namespace

int steer_sig_tiles(int D) { return (D + kRows - 1) / kRows; }

hipError_t launch_steer_sig(const void *H, ssl_prec hprec, const ssl_c64 *Es,
                            const ssl_c128 *Esl, int F, int D, int M, int Ns,
                            const int32_t *bin_status, float *P, hipStream_t st)
{
    const int nt = steer_sig_tiles(D);
    return with_table(hprec, [&](auto tab) {
        typedef decltype(tab) Tab;
        hipLaunchKernelGGL(steer_sig_single<Tab>, dim3(sig_grid(F, nt)), dim3(kThreads), 0, st,
                           static_cast<const typename Tab::W *>(H),
                           reinterpret_cast<const float2 *>(Es),
                           reinterpret_cast<const double2 *>(Esl), bin_status, F, D, M, Ns, P, nt);
        return hipGetLastError();
    });
}

hipError_t launch_steer_sig_batch(const BlockDev *blk, const int2 *items, int n_items,
                                  const int2 *groups, const int *gblocks, int max_dtiles,
                                  int nsmax, ssl_prec hprec, hipStream_t st)
{
    if (n_items <= 0) return hipSuccess;
    return with_table(hprec, [&](auto tab) {
        typedef decltype(tab) Tab;
        hipLaunchKernelGGL(steer_sig_batch<Tab>, dim3(sig_grid(n_items, max_dtiles)),
                           dim3(kThreads), 0, st, blk, items, n_items, max_dtiles, groups,
                           gblocks, nsmax);
        return hipGetLastError();
    });
}
