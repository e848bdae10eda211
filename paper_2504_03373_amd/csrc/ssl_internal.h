// Internal declarations of the HIP library: context and noise-handle layouts, kernel launchers.
// Not part of the public ABI (include/ssl.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "ssl.h"

#define SSL_MAX_M 64
#define SSL_DEFAULT_SWEEPS 20

// Bin-sum chunking of the spectrum reduction: bins are summed in ascending order inside fixed
// chunks of SSL_BINSUM_CHUNK bins, then the chunk partials in ascending chunk order.
#define SSL_BINSUM_CHUNK 16

struct ssl_ctx_s {
    int device;
    size_t budget;          // 0 = unlimited
    size_t held;            // bytes currently allocated by this context
    // workspace for ssl_localize / ssl_music_spectrum (grown on demand, never shrunk)
    void *ws;
    size_t ws_bytes;
    // bin-sum scratch: partials [chunks][D]
    float *binsum_part;
    size_t binsum_floats;
    // per-kernel event timing (ssl_ctx_timing)
    struct Timed {
        int id;
        hipEvent_t start, stop;
    };
    bool timing = false;
    std::vector<Timed> pending;
    std::vector<Timed> event_pool;
    int64_t launches[SSL_K_COUNT] = {};
    double total_ms[SSL_K_COUNT] = {};
    // batched path (ssl_localize_batch)
    void *bdesc_dev = nullptr;           // device copy of descriptors + work-item lists
    void *bdesc_host = nullptr;          // pinned staging buffer of the same
    size_t bdesc_bytes = 0;
    hipEvent_t bdesc_ev = nullptr;       // completion of the last staging copy
    unsigned int *counters = nullptr;    // zero-initialised, every kernel leaves them at zero
    size_t n_counters = 0;
    hipStream_t cap_stream = nullptr;    // capture stream for graph construction
    bool use_graphs = true;
    struct GraphEntry {
        std::vector<int64_t> key;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;
    int cu_count = 0;
    // this device's address of the fixed scratch of ssl_localize_noalloc
    char *scratch = nullptr;
    // SVD backend of every entry point (ssl_ctx_set_svd)
    int svd = SSL_SVD_JACOBI;
    // subspace method for calls with a noise handle (ssl_ctx_set_subspace)
    int subspace = SSL_SUBSPACE_GSVD;
    int sub_stop = SSL_STOP_LOCALIZE;   // ssl_stop: where the Jacobi solve may stop at the subspace
    int proj = SSL_PROJ_SIGNAL;         // ssl_projection: form of eq.5 on the FP32 path
    // Jacobi variant (lanes per column pair) per size class 8/16/32/64 channels
    int jac_lanes[4] = {8, 8, 8, 8};     // lanes per Jacobi column pair, classes 8/16/32/64
    // waves per projection workgroup, [steer class 1/2/4][SSL_FP32, SSL_BF16, SSL_FP16]
    int steer_waves[3][3] = {{8, 8, 8}, {8, 8, 8}, {8, 8, 8}};
};

struct ssl_noise_s {
    ssl_ctx ctx;
    int F, M;
    bool is_set;
    ssl_c128 *K;       // [F][M][M] current noise correlation
    ssl_c128 *Kinv;    // [F][M][M] FP64 inverse by Gauss-Jordan elimination
    int32_t *status;   // [F] SSL_BIN_OK / SSL_BIN_NOT_PD
    // GEVD-MUSIC (ssl_noise_enable_gevd): K^{-1/2}, recomputed with every refactor once enabled
    ssl_c128 *Kisq = nullptr;
    bool gevd = false;
};

// Frame stream of eq.3 (ssl_sliding_*): the ring of the last T frames of every bin, the FP64 sum
// S of their outer products, and the sorted left singular vectors of the last solve (the start
// of a warm-started one).
struct ssl_sliding_s {
    ssl_ctx ctx;
    int F, M, T;
    int64_t pushed = 0;          // frames pushed so far
    int64_t since_refresh = 0;   // frames pushed since S was last recomputed from the ring
    ssl_c64 *ring = nullptr;     // [F][T][M]; frame k in slot k mod T
    ssl_c128 *S = nullptr;       // [F][M][M]
    ssl_c64 *U = nullptr;        // [F][M][M] column-major per bin
    bool have_U = false;
    int64_t cold_at = 0;         // frames pushed at the last cold solve
    size_t bytes = 0;
};

void ssl_set_error(const char *fmt, ...);

// Device view of one block of a batch: caller pointers, shapes and the block's slices of the
// batch workspace.  Filled on the host, copied to HBM once per batch call.
struct BlockDev {
    const float2 *X;
    int64_t sF, sT;
    int F, T, M, Ns, D, n_az, n_el, p;
    float scale;                    // (float)(1/T), the same value the single-block path uses
    int hprec;                      // ssl_prec of H
    const double2 *Kinv;            // noise handle: FP64 inverse, per-bin status
    const double2 *Kisq;            // K^{-1/2} when the block runs GEVD-MUSIC, else null
    const int32_t *kstatus;
    const void *H;
    float2 *R, *A, *En;             // workspace slices
    float2 *Es;                     // signal vectors [F][Ns][M] (workspace) or null
    double2 *Esl;                   // per bin: L^{-1} of their Gram matrix's Cholesky factor, [F][6]
    float *P, *part;
    int32_t *peaks, *status;        // caller outputs
    float *peak_val, *Pbar;
    int32_t *conv;                  // [F][3] Jacobi statistics or null
};

// Device view of one noise-handle update of ssl_noise_update_frames(_from): the noise-only
// frames [F][T][M] (contiguous), the source K read by the blend (Ks; the destination K itself for
// an update in place), and the destination's K, K^{-1} and per-bin status.
struct NoiseUpdDev {
    const float2 *X;
    int F, T, M;
    const double2 *Ks;
    double2 *K, *Kinv;
    int32_t *status;
};

// Device pointers read from descriptors are generic: loads through them compile to FLAT
// instructions, which count against the LDS counter as well, so a wait for an LDS read would also
// wait for every such load in flight.  gload / gstore access one element through a global-memory
// pointer (global_load / global_store, counted by the vector-memory counter only).
template <int N> struct GWord;
template <> struct GWord<4> { typedef unsigned int type; };
template <> struct GWord<8> { typedef unsigned long long type; };
template <> struct GWord<16> { typedef unsigned int type __attribute__((ext_vector_type(4))); };
template <typename T>
__device__ __forceinline__ T gload(const T *p)
{
    typedef typename GWord<sizeof(T)>::type W;
    return __builtin_bit_cast(T, *(const __attribute__((address_space(1))) W *)p);
}
template <typename T>
__device__ __forceinline__ void gstore(T *p, T v)
{
    typedef typename GWord<sizeof(T)>::type W;
    *(__attribute__((address_space(1))) W *)p = __builtin_bit_cast(W, v);
}

// Size classes shared by the single-block and batched launches, so that a bin is computed by the
// same kernel variant whichever entry point schedules it.
inline int corr_class(int M) { return M <= 16 ? 16 : M <= 32 ? 32 : M <= 48 ? 48 : 64; }
inline int whiten_class(int M) { return M <= 16 ? 16 : M <= 32 ? 32 : 64; }
inline int jacobi_class(int M) { return M <= 8 ? 8 : M <= 16 ? 16 : M <= 32 ? 32 : 64; }
inline int steer_class(int M, int Ns)
{
    const int nn = M - Ns;                 // noise vectors = B columns, 16 per column tile
    return nn <= 16 ? 1 : nn <= 32 ? 2 : 4;
}

// Batched launchers.  `items` lists (block, bin) pairs whose blocks share the kernel's size class.
hipError_t launch_corr_batch(const BlockDev *blk, const int2 *items, int n_items, int cls,
                             ssl_prec prec, hipStream_t st);
// Whitening items are (chunk, bin): chunks[c] = (first, count) into cblocks, a run of blocks that
// share one noise set, whose K^{-1} the workgroup loads once.
hipError_t launch_whiten_batch(const BlockDev *blk, const int2 *items, int n_items,
                               const int2 *chunks, const int *cblocks, int cls, hipStream_t st);
int whiten_wg_per_cu(int cls);
// Persistent: `grid` workgroups draw items from *queue (0 on entry, re-armed to 0 on exit).
// sub_full >= 0: blocks with p = 2 stop once their noise subspace has converged (launch_jacobi).
hipError_t launch_jacobi_batch(const BlockDev *blk, const int2 *items, int n_items, int cls,
                               int lanes, int max_sweeps, unsigned int *queue, int grid,
                               hipStream_t st, int sub_full = -1);
// eq.5 (p = 2) through the signal subspace, FP64 (steer_sig.hip): Es [F][Ns][M] and Esl [F][6]
// from the Jacobi solve, H [F][D][M] complex64 or [F][D][2M] bf16 / fp16 pairs (hprec),
// Ns <= 3; direction tiles of steer_sig_tiles(D).
int steer_sig_tiles(int D);
hipError_t launch_steer_sig(const void *H, ssl_prec hprec, const ssl_c64 *Es,
                            const ssl_c128 *Esl, int F, int D, int M, int Ns,
                            const int32_t *bin_status, float *P, hipStream_t st);
hipError_t launch_steer_sig_batch(const BlockDev *blk, const int2 *items, int n_items,
                                  const int2 *groups, const int *gblocks, int max_dtiles,
                                  int nsmax, ssl_prec hprec, hipStream_t st);
hipError_t launch_steer_batch(const BlockDev *blk, const int2 *items, int n_items,
                              const int2 *groups, const int *gblocks, int cls, int waves,
                              int max_dtiles, ssl_prec hprec, hipStream_t st);
hipError_t launch_binsum_batch(const BlockDev *blk, int nblocks, int max_dchunks,
                               int max_fchunks, hipStream_t st);
int jacobi_threads(int cls, int lanes);
inline int jacobi_class_index(int cls) { return cls == 8 ? 0 : cls == 16 ? 1 : cls == 32 ? 2 : 3; }
inline int steer_class_index(int cls) { return cls == 1 ? 0 : cls == 2 ? 1 : 2; }
bool steer_waves_ok(int waves);          // 4, 8 or 16 waves (16 directions each) per workgroup
int steer_rows_per_block(int waves);
int binsum_threads();

// --- launchers (each returns hipSuccess or the launch error) ---
// GEVD-MUSIC: W = K^{-1/2} per bin (FP64 Jacobi eigen-decomposition of K; wstatus may alias
// kstatus), C = W R W, and E_n <- W E_n; batched forms over (block, bin) items
hipError_t launch_noise_isqrt(const ssl_c128 *K, const int32_t *kstatus, int F, int M,
                              ssl_c128 *W, int32_t *wstatus, hipStream_t st);
hipError_t launch_gevd_whiten(const ssl_c128 *W, const ssl_c64 *R, ssl_c64 *C, int F, int M,
                              hipStream_t st);
hipError_t launch_gevd_back(const ssl_c128 *W, ssl_c64 *En, int F, int M, int Ns, hipStream_t st);
hipError_t launch_gevd_whiten_batch(const BlockDev *blk, const int2 *items, int n_items, int cls,
                                    hipStream_t st);
hipError_t launch_gevd_back_batch(const BlockDev *blk, const int2 *items, int n_items, int cls,
                                  hipStream_t st);
// eq.3 frame stream: S += sum over the n new frames of x x^H - o o^H (o: the frame each displaces
// from the ring, zero while fewer than T frames were pushed), ring updated; R = S * inv_t
hipError_t launch_sliding_push(const ssl_c64 *X, int n, int64_t sF, int64_t sT, int F, int M,
                               int T, int64_t pushed, ssl_c64 *ring, ssl_c128 *S, hipStream_t st);
hipError_t launch_sliding_scale(const ssl_c128 *S, int64_t n, double inv_t, void *R, bool fp64,
                                hipStream_t st);
// eq.1: pcm [n_samples][M] float -> X [nfft/2 + 1][T][M]; nfft a power of two in [16, 4096]
hipError_t launch_stft(const float *pcm, int M, int nfft, int hop, const float *win, int T,
                       ssl_c64 *X, hipStream_t st);
hipError_t launch_corr(const ssl_c64 *X, int F, int T, int M, int64_t sF, int64_t sT, double scale,
                       int accumulate, ssl_prec prec, void *R, hipStream_t st);
hipError_t launch_noise_factor(ssl_c128 *K, ssl_c128 *Kinv, int32_t *status, int F, int M,
                               hipStream_t st);
hipError_t launch_noise_load(ssl_c128 *K, const void *Kin, ssl_prec kprec, int F, int M,
                             hipStream_t st);
hipError_t launch_noise_blend(ssl_c128 *K, const void *Khat, ssl_prec kprec, double alpha,
                              int F, int M, hipStream_t st);
hipError_t launch_whiten(const ssl_c128 *Kinv, const ssl_c64 *R, ssl_c64 *A, int F, int M,
                         hipStream_t st);
// Batched EMA noise update, items (handle, bin) of one size class (16 / 32 / 64 channels):
// K <- alpha K + (1 - alpha) (1/T) sum_t x x^H (FP64 MFMA correlation, blend fused), then the
// Gauss-Jordan inverse of the updated K.  Both launches read the same items.
hipError_t launch_noise_corr_blend(const NoiseUpdDev *h, const int2 *items, int n_items, int cls,
                                   double alpha, hipStream_t st);
hipError_t launch_noise_factor_batch(const NoiseUpdDev *h, const int2 *items, int n_items,
                                     int cls, hipStream_t st);
inline int noise_class(int M) { return M <= 16 ? 16 : M <= 32 ? 32 : 64; }
// A is library workspace and is overwritten (it parks the QR reflectors between phases).
// lanes = lanes per column pair of the Jacobi variant (jacobi_variant_ok).
// U (optional): all M sorted left singular vectors, [F][M][M] column-major per bin (identity for
// a failed bin) -- the start of a warm-started solve (launch_jacobi_warm).
// sub_full >= 0 (with sigma and U null, 1 <= Ns <= 3): E_n is an orthonormal basis of the noise
// subspace, the solve stopping once that subspace has converged after sub_full full sweeps.
// Es ([F][Ns][M], optional): the signal vectors; Esl ([F][6], with Es, Ns <= 3): the inverse
// Cholesky factor of their FP64 Gram matrix (for the signal-subspace form of eq.5).
hipError_t launch_jacobi(ssl_c64 *A, const int32_t *kstatus, int F, int M, int Ns,
                         int max_sweeps, int lanes, ssl_c64 *En, float *sigma,
                         int32_t *bin_status, int32_t *conv, hipStream_t st,
                         ssl_c64 *U = nullptr, int sub_full = -1, ssl_c64 *Es = nullptr,
                         ssl_c128 *Esl = nullptr);
// Full sweeps before the subspace phase (p = 2): none.  The signal set is chosen on the column
// norms of X = R1^H, which the pivoted QR already grades, and only the pairs with a signal column
// are ever visited (about 2.4 subspace sweeps instead of one full sweep and 1.3 subspace sweeps on
// the 60-channel workload; a launch of many bins per CU, bound by VALU issue, runs about 6%
// faster, a one-block launch, bound by the latency of the serial subspace rounds, about 6% slower).
// The same value on every path keeps batched and one-block results bit-identical.
constexpr int kSubFullSweeps = 0;
// Warm-started solve: U [F][M][M] (column-major per bin) holds a unitary start on entry (the
// previous solve's sorted singular vectors) and this solve's on exit; A is read only.
hipError_t launch_jacobi_warm(const ssl_c64 *A, const int32_t *kstatus, int F, int M, int Ns,
                              int max_sweeps, ssl_c64 *U, ssl_c64 *En, int32_t *bin_status,
                              int32_t *conv, hipStream_t st);
bool jacobi_variant_ok(int cls, int lanes);
// The paper's SVD (Householder bidiagonalisation, phase transform, implicit-shift QR, sort,
// back-transformation): A is read only; conv = (QR steps, zero-diagonal chases, M) per bin.
hipError_t launch_gk_svd(const ssl_c64 *A, const int32_t *kstatus, int F, int M, int Ns,
                         int max_steps, ssl_c64 *En, float *sigma, int32_t *bin_status,
                         int32_t *conv, hipStream_t st);
hipError_t launch_gk_svd_batch(const BlockDev *blk, const int2 *items, int n_items, int cls,
                               int max_steps, hipStream_t st);
int jacobi_persistent_wg_per_cu(int cls, int lanes);
hipError_t launch_steer(const void *H, ssl_prec hprec, const ssl_c64 *En, int F, int D, int M,
                        int Ns, int p, const int32_t *bin_status, float *P, int waves,
                        hipStream_t st);
hipError_t launch_binsum_peaks(const float *P, int F, int D, float *Pbar, float *part,
                               int n_az, int n_el, int Ns, int32_t *peaks, float *peak_val,
                               hipStream_t st);
hipError_t launch_peaks(const float *Pbar, int n_az, int n_el, int Ns, int32_t *peaks,
                        float *peak_val, hipStream_t st);
