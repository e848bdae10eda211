// C ABI of the GSVD-MUSIC library (declared in include/ssl.h): argument validation, contexts,
// noise handles, workspace under an HBM budget, and the launch sequences of the entry points.
// Every arithmetic step runs in the HIP kernels of corr.hip, noise.hip, jacobi.hip, steer.hip and
// peaks.hip; this file only checks, allocates and enqueues.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <tuple>

#include "ssl_internal.h"

namespace {

thread_local char g_err[512] = "";

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

bool ok_prec(ssl_prec p) { return p == SSL_FP32 || p == SSL_BF16 || p == SSL_FP16 || p == SSL_FP64; }

ssl_status hip_fail(hipError_t e, const char *what)
{
    ssl_set_error("%s: %s", what, hipGetErrorString(e));
    return SSL_ERR_HIP;
}

// Makes ctx->device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

ssl_status dev_alloc(ssl_ctx ctx, void **p, size_t bytes, const char *what)
{
    if (ctx->budget && ctx->held + bytes > ctx->budget) {
        ssl_set_error("%s: %zu bytes would exceed the HBM budget (%zu held of %zu)", what, bytes,
                      ctx->held, ctx->budget);
        return SSL_ERR_BUDGET;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        ssl_set_error("%s: hipMalloc(%zu) failed: %s", what, bytes, hipGetErrorString(e));
        return SSL_ERR_NOMEM;
    }
    ctx->held += bytes;
    return SSL_OK;
}

void dev_free(ssl_ctx ctx, void *p, size_t bytes)
{
    if (p) {
        (void)hipFree(p);
        ctx->held -= bytes;
    }
}

// Captured graphs bake in workspace addresses: drop them whenever a buffer moves.
void clear_graphs(ssl_ctx ctx)
{
    for (auto &g : ctx->graphs) (void)hipGraphExecDestroy(g.exec);
    ctx->graphs.clear();
}

// Grows the context workspace to at least `bytes` (never shrinks).  hipFree of the old block
// synchronises the device, so in-flight work that used it has finished.
ssl_status ws_reserve(ssl_ctx ctx, size_t bytes)
{
    if (ctx->ws_bytes >= bytes) return SSL_OK;
    if (ctx->budget && ctx->held - ctx->ws_bytes + bytes > ctx->budget) {
        ssl_set_error("workspace of %zu bytes exceeds the HBM budget (%zu)", bytes, ctx->budget);
        return SSL_ERR_BUDGET;
    }
    clear_graphs(ctx);
    dev_free(ctx, ctx->ws, ctx->ws_bytes);
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
    ssl_status s = dev_alloc(ctx, &ctx->ws, bytes, "workspace");
    if (s == SSL_OK) ctx->ws_bytes = bytes;
    return s;
}

// Bin-sum scratch: [chunks][D] partials.
ssl_status binsum_reserve(ssl_ctx ctx, int F, int D)
{
    const size_t nch = (size_t)(F + SSL_BINSUM_CHUNK - 1) / SSL_BINSUM_CHUNK;
    const size_t need = nch * (size_t)D;
    if (ctx->binsum_floats >= need && ctx->binsum_part) return SSL_OK;
    if (ctx->binsum_part) {
        dev_free(ctx, ctx->binsum_part, ctx->binsum_floats * sizeof(float));
        ctx->binsum_part = nullptr;
        ctx->binsum_floats = 0;
    }
    void *p = nullptr;
    ssl_status s = dev_alloc(ctx, &p, need * sizeof(float), "bin-sum scratch");
    if (s != SSL_OK) return s;
    ctx->binsum_part = static_cast<float *>(p);
    ctx->binsum_floats = need;
    return SSL_OK;
}

// Runs one kernel launch, bracketed by timing events on its stream when the context times.
template <class Fn>
hipError_t timed(ssl_ctx ctx, int id, hipStream_t st, Fn &&launch)
{
    if (!ctx->timing) return launch();
    ssl_ctx_s::Timed t{id, nullptr, nullptr};
    if (!ctx->event_pool.empty()) {
        t = ctx->event_pool.back();
        ctx->event_pool.pop_back();
        t.id = id;
    } else {
        hipError_t e = hipEventCreate(&t.start);
        if (e == hipSuccess) e = hipEventCreate(&t.stop);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipEventRecord(t.start, st);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(t.stop, st);
    if (e == hipSuccess) ctx->pending.push_back(t);
    else ctx->event_pool.push_back(t);
    return e;
}

int jac_lanes(ssl_ctx ctx, int M) { return ctx->jac_lanes[jacobi_class_index(jacobi_class(M))]; }

// QR steps allowed to the bidiagonal solve: about 2 per singular value suffice in practice
int gk_max_steps(int M) { return 40 * M; }

// The SVD of the context's backend for F bins of A (the Jacobi kernel overwrites A, the
// bidiagonal one reads it only); U (Jacobi only) receives all sorted singular vectors.
hipError_t launch_svd(ssl_ctx ctx, ssl_c64 *A, const int32_t *kst, int F, int M, int Ns,
                      int max_sweeps, ssl_c64 *En, float *sigma, int32_t *stt, int32_t *conv,
                      hipStream_t st, ssl_c64 *U = nullptr, int sub_full = -1,
                      ssl_c64 *Es = nullptr, ssl_c128 *Esl = nullptr)
{
    if (ctx->svd == SSL_SVD_BIDIAG_QR)
        return launch_gk_svd(A, kst, F, M, Ns, gk_max_steps(M), En, sigma, stt, conv, st);
    return launch_jacobi(A, kst, F, M, Ns, max_sweeps, jac_lanes(ctx, M), En, sigma, stt, conv, st,
                         U, sub_full, Es, Esl);
}
// Whether eq.5 is evaluated through the signal subspace (FP64, steer_sig.hip): p = 2, the Jacobi
// backend, GSVD or SEVD (U unitary), Ns <= 3, any table precision, unless the context asks for
// the noise-vector projection.
bool use_sig(ssl_ctx ctx, ssl_prec prec, int p, int Ns, bool gevd)
{
    (void)prec;
    return ctx->proj == SSL_PROJ_SIGNAL && p == 2 && ctx->svd == SSL_SVD_JACOBI && !gevd &&
           Ns >= 1 && Ns <= 3;
}

// Whether a localization path stops the Jacobi solve at the noise subspace (p = 2: eq.5 reads only
// its projector): the batched path from SSL_STOP_BATCH on, the one-block paths from
// SSL_STOP_LOCALIZE on.
int sub_full_for(ssl_ctx ctx, int p, bool batched)
{
    const int need = batched ? SSL_STOP_BATCH : SSL_STOP_LOCALIZE;
    return p == 2 && ctx->sub_stop >= need ? kSubFullSweeps : -1;
}
int st_waves(ssl_ctx ctx, int M, int Ns, ssl_prec prec)
{
    return ctx->steer_waves[steer_class_index(steer_class(M, Ns))][prec];
}

ssl_status check_common(int F, int M, int Ns)
{
    if (F < 1 || F > 65535) {
        ssl_set_error("F = %d out of range [1, 65535]", F);
        return SSL_ERR_ARG;
    }
    if (M < 1 || M > SSL_MAX_M) {
        ssl_set_error("M = %d out of range [1, %d]", M, SSL_MAX_M);
        return SSL_ERR_ARG;
    }
    if (Ns != -1 && (Ns < 1 || Ns >= M)) {
        ssl_set_error("Ns = %d must satisfy 1 <= Ns < M = %d", Ns, M);
        return SSL_ERR_ARG;
    }
    return SSL_OK;
}

ssl_status check_grid(int n_az, int n_el, int Ns)
{
    if (n_az < 1 || n_el < 1 || (int64_t)n_az * n_el > (1 << 24)) {
        ssl_set_error("direction grid %d x %d invalid", n_el, n_az);
        return SSL_ERR_ARG;
    }
    if (Ns < 1 || Ns >= SSL_MAX_M) {
        ssl_set_error("Ns = %d out of range", Ns);
        return SSL_ERR_ARG;
    }
    return SSL_OK;
}

ssl_status check_x(const ssl_c64 *X, int T, int M, int64_t sF, int64_t sT)
{
    if (!X) {
        ssl_set_error("X is NULL");
        return SSL_ERR_ARG;
    }
    if (T < 1) {
        ssl_set_error("T = %d must be >= 1", T);
        return SSL_ERR_ARG;
    }
    if (sT < M || sF < 0) {
        ssl_set_error("strides (strideF %lld, strideT %lld) invalid for M = %d", (long long)sF,
                      (long long)sT, M);
        return SSL_ERR_ARG;
    }
    return SSL_OK;
}

// A noise handle for F bins of M channels that has been set, or NULL (SEVD-MUSIC: no whitening).
ssl_status check_noise(ssl_noise K, int F, int M)
{
    if (!K) return SSL_OK;
    if (K->F != F || K->M != M) {
        ssl_set_error("noise handle is %d x %d, call has F = %d, M = %d", K->F, K->M, F, M);
        return SSL_ERR_ARG;
    }
    if (!K->is_set) {
        ssl_set_error("noise handle was never set");
        return SSL_ERR_STATE;
    }
    return SSL_OK;
}

// GEVD-MUSIC needs the handle's K^{-1/2} (ssl_noise_enable_gevd)
bool use_gevd(ssl_ctx ctx, ssl_noise K) { return K && ctx->subspace == SSL_SUBSPACE_GEVD; }
ssl_status check_gevd(ssl_ctx ctx, ssl_noise K)
{
    if (use_gevd(ctx, K) && !K->gevd) {
        ssl_set_error("GEVD-MUSIC selected but ssl_noise_enable_gevd was not called on the handle");
        return SSL_ERR_STATE;
    }
    return SSL_OK;
}

ssl_status check_localize(ssl_ctx ctx, const ssl_c64 *X, int F, int T, int M, int64_t strideF,
                          int64_t strideT, ssl_noise K, const void *H, ssl_prec prec, int n_az,
                          int n_el, int Ns, int p, int32_t *peaks, float *peak_val)
{
    if (!ctx || !H || !peaks || !peak_val) {
        ssl_set_error("ctx, H, peaks or peak_val is NULL");
        return SSL_ERR_ARG;
    }
    ssl_status s = check_common(F, M, Ns);
    if (s != SSL_OK) return s;
    if ((s = check_x(X, T, M, strideF, strideT)) != SSL_OK) return s;
    if ((s = check_grid(n_az, n_el, Ns)) != SSL_OK) return s;
    if (p != 1 && p != 2) {
        ssl_set_error("p = %d must be 1 or 2", p);
        return SSL_ERR_ARG;
    }
    if (prec != SSL_FP32 && prec != SSL_BF16 && prec != SSL_FP16) {
        ssl_set_error("prec must be SSL_FP32, SSL_BF16 or SSL_FP16");
        return SSL_ERR_ARG;
    }
    ssl_status s2 = check_noise(K, F, M);
    return s2 != SSL_OK ? s2 : check_gevd(ctx, K);
}

// Workspace of one block's path: R | A | En | P | Pbar | status, then (scratch only) the bin-sum
// partials [chunks][D].
struct LocalizeWs {
    size_t bR, bE, bP, bB, bS, bEs, bEl, total, with_part;
    size_t off_es() const { return 2 * bR + bE + bP + bB + bS; }
};

LocalizeWs localize_ws(int F, int M, int Ns, int D)
{
    LocalizeWs L;
    L.bR = align256((size_t)F * M * M * sizeof(ssl_c64));
    L.bE = align256((size_t)F * (M - Ns) * M * sizeof(ssl_c64));
    L.bP = align256((size_t)F * D * sizeof(float));
    L.bB = align256((size_t)D * sizeof(float));
    L.bS = align256((size_t)F * sizeof(int32_t));
    L.bEs = align256((size_t)F * Ns * M * sizeof(ssl_c64));          // signal vectors
    L.bEl = align256((size_t)F * 6 * sizeof(ssl_c128));              // their L^{-1}
    L.total = 2 * L.bR + L.bE + L.bP + L.bB + L.bS + L.bEs + L.bEl;
    const size_t nch = (size_t)(F + SSL_BINSUM_CHUNK - 1) / SSL_BINSUM_CHUNK;
    L.with_part = L.total + align256(nch * (size_t)D * sizeof(float));
    return L;
}

// The five launches of one block (eq.2-6 and the peak search) on workspace w laid out as L and
// bin-sum partials `part`.  With `may_time` false no timing event is ever created or recorded.
ssl_status localize_enqueue(ssl_ctx ctx, bool may_time, char *w, const LocalizeWs &L, float *part,
                            const ssl_c64 *X, int F, int T, int M, int64_t strideF,
                            int64_t strideT, ssl_noise K, const void *H, ssl_prec prec, int n_az,
                            int n_el, int Ns, int p, int32_t *peaks, float *peak_val, float *Pbar,
                            int32_t *bin_status, hipStream_t st)
{
    const int D = n_az * n_el;
    ssl_c64 *R = reinterpret_cast<ssl_c64 *>(w);
    ssl_c64 *A = reinterpret_cast<ssl_c64 *>(w + L.bR);
    ssl_c64 *En = reinterpret_cast<ssl_c64 *>(w + 2 * L.bR);
    float *P = reinterpret_cast<float *>(w + 2 * L.bR + L.bE);
    float *Pb = Pbar ? Pbar : reinterpret_cast<float *>(w + 2 * L.bR + L.bE + L.bP);
    int32_t *stt = bin_status ? bin_status
                              : reinterpret_cast<int32_t *>(w + 2 * L.bR + L.bE + L.bP + L.bB);
    auto run = [&](int id, auto &&launch) {
        return may_time ? timed(ctx, id, st, launch) : launch();
    };
    hipError_t e = run(SSL_K_CORR, [&] {
        return launch_corr(X, F, T, M, strideF, strideT, 1.0 / T, 0, prec, R, st);
    });
    if (e != hipSuccess) return hip_fail(e, "corr launch");
    const bool gevd = use_gevd(ctx, K);
    if (gevd) {
        e = run(SSL_K_WHITEN, [&] { return launch_gevd_whiten(K->Kisq, R, A, F, M, st); });
        if (e != hipSuccess) return hip_fail(e, "GEVD whitening launch");
    } else if (K) {
        e = run(SSL_K_WHITEN, [&] { return launch_whiten(K->Kinv, R, A, F, M, st); });
        if (e != hipSuccess) return hip_fail(e, "whiten launch");
    } else {
        A = R;                                   // SEVD-MUSIC: the decomposition of R itself
    }
    const bool sig = use_sig(ctx, prec, p, Ns, gevd);
    ssl_c64 *Es = sig ? reinterpret_cast<ssl_c64 *>(w + L.off_es()) : nullptr;
    ssl_c128 *Esl = sig ? reinterpret_cast<ssl_c128 *>(w + L.off_es() + L.bEs) : nullptr;
    e = run(SSL_K_JACOBI, [&] {
        // through the signal subspace the noise vectors are neither formed nor stored
        return launch_svd(ctx, A, K ? K->status : nullptr, F, M, Ns, SSL_DEFAULT_SWEEPS,
                          sig ? nullptr : En, nullptr, stt, nullptr, st, nullptr,
                          sub_full_for(ctx, p, false), Es, Esl);
    });
    if (e != hipSuccess) return hip_fail(e, "jacobi launch");
    if (gevd) {
        e = run(SSL_K_WHITEN, [&] { return launch_gevd_back(K->Kisq, En, F, M, Ns, st); });
        if (e != hipSuccess) return hip_fail(e, "GEVD back-transformation launch");
    }
    e = run(SSL_K_STEER, [&] {
        if (sig)
            return launch_steer_sig(H, prec, Es, Esl, F, D, M, Ns, stt, P, st);
        return launch_steer(H, prec, En, F, D, M, Ns, p, stt, P, st_waves(ctx, M, Ns, prec), st);
    });
    if (e != hipSuccess) return hip_fail(e, "steer launch");
    e = run(SSL_K_BINSUM, [&] {
        return launch_binsum_peaks(P, F, D, Pb, part, n_az, n_el, Ns, peaks, peak_val, st);
    });
    return e == hipSuccess ? SSL_OK : hip_fail(e, "bin-sum launch");
}

// Fixed device scratch of ssl_localize_noalloc.  Every device the library runs on holds its own
// copy for the life of the process; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device (scratch_address), never through the name.
static __device__ __align__(256) unsigned char scratch[SSL_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_addr[kMaxDevices] = {};

// The device address of `scratch` on `device`, which must be the current device; looked up once
// per device.
ssl_status scratch_address(int device, char **out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) {
        ssl_set_error("device %d beyond the %d devices the scratch table covers", device,
                      kMaxDevices);
        return SSL_ERR_ARG;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                            "hipGetSymbolAddress(scratch)");
        }
        g_scratch_addr[device] = static_cast<char *>(ptr);
    }
    *out = g_scratch_addr[device];
    return SSL_OK;
}

}  // namespace

void ssl_set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

extern "C" {

const char *ssl_last_error(void) { return g_err; }

int ssl_version(void) { return 100; }

ssl_status ssl_ctx_create(ssl_ctx *out, int device, size_t hbm_budget_bytes)
{
    if (!out) {
        ssl_set_error("out is NULL");
        return SSL_ERR_ARG;
    }
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= n) {
        ssl_set_error("device %d not present (%d devices)", device, n);
        return SSL_ERR_ARG;
    }
    ssl_ctx c = new (std::nothrow) ssl_ctx_s();
    if (!c) {
        ssl_set_error("out of host memory");
        return SSL_ERR_NOMEM;
    }
    c->device = device;
    c->budget = hbm_budget_bytes;
    {
        DeviceGuard dg(device);
        ssl_status s = dg.ok ? scratch_address(device, &c->scratch)
                             : hip_fail(hipErrorInvalidDevice, "hipSetDevice");
        if (s != SSL_OK) {
            delete c;
            return s;
        }
    }
    if (hipDeviceGetAttribute(&c->cu_count, hipDeviceAttributeMultiprocessorCount, device) !=
            hipSuccess ||
        c->cu_count <= 0)
        c->cu_count = 256;
    *out = c;
    return SSL_OK;
}

void ssl_ctx_destroy(ssl_ctx ctx)
{
    if (!ctx) return;
    DeviceGuard dg(ctx->device);
    for (auto &t : ctx->pending) ctx->event_pool.push_back(t);
    for (auto &t : ctx->event_pool) {
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    clear_graphs(ctx);
    if (ctx->bdesc_ev) {
        (void)hipEventSynchronize(ctx->bdesc_ev);
        (void)hipEventDestroy(ctx->bdesc_ev);
    }
    if (ctx->bdesc_host) (void)hipHostFree(ctx->bdesc_host);
    dev_free(ctx, ctx->bdesc_dev, ctx->bdesc_bytes);
    dev_free(ctx, ctx->counters, ctx->n_counters * sizeof(unsigned int));
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    dev_free(ctx, ctx->ws, ctx->ws_bytes);
    if (ctx->binsum_part) dev_free(ctx, ctx->binsum_part, ctx->binsum_floats * sizeof(float));
    delete ctx;
}

size_t ssl_ctx_workspace_bytes(ssl_ctx ctx) { return ctx ? ctx->held : 0; }

ssl_status ssl_ctx_timing(ssl_ctx ctx, int enable)
{
    if (!ctx) {
        ssl_set_error("ctx is NULL");
        return SSL_ERR_ARG;
    }
    ctx->timing = enable != 0;
    return SSL_OK;
}

ssl_status ssl_ctx_timing_read(ssl_ctx ctx, int64_t *launches, double *total_ms, int reset)
{
    if (!ctx) {
        ssl_set_error("ctx is NULL");
        return SSL_ERR_ARG;
    }
    DeviceGuard dg(ctx->device);
    ssl_status s = SSL_OK;
    for (auto &t : ctx->pending) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(t.stop);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.start, t.stop);
        if (e != hipSuccess && s == SSL_OK) s = hip_fail(e, "timing event");
        ctx->launches[t.id] += 1;
        ctx->total_ms[t.id] += ms;
        ctx->event_pool.push_back(t);
    }
    ctx->pending.clear();
    for (int k = 0; k < SSL_K_COUNT; ++k) {
        if (launches) launches[k] = ctx->launches[k];
        if (total_ms) total_ms[k] = ctx->total_ms[k];
        if (reset) {
            ctx->launches[k] = 0;
            ctx->total_ms[k] = 0.0;
        }
    }
    return s;
}

ssl_status ssl_stft(ssl_ctx ctx, const float *pcm, int64_t n_samples, int M, int nfft, int hop,
                    int T, const float *window, ssl_c64 *X, void *stream)
{
    if (!ctx || !pcm || !X) {
        ssl_set_error("ctx, pcm or X is NULL");
        return SSL_ERR_ARG;
    }
    if (nfft < 16 || nfft > 4096 || (nfft & (nfft - 1)) != 0) {
        ssl_set_error("nfft = %d must be a power of two in [16, 4096]", nfft);
        return SSL_ERR_ARG;
    }
    if (M < 1 || M > 4096 || hop < 1 || T < 1 || T > 65535) {
        ssl_set_error("M = %d, hop = %d, T = %d out of range", M, hop, T);
        return SSL_ERR_ARG;
    }
    if ((int64_t)(T - 1) * hop + nfft > n_samples) {
        ssl_set_error("T = %d frames of %d samples at hop %d need %lld samples, pcm has %lld", T,
                      nfft, hop, (long long)((int64_t)(T - 1) * hop + nfft),
                      (long long)n_samples);
        return SSL_ERR_ARG;
    }
    DeviceGuard dg(ctx->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = timed(ctx, SSL_K_CORR, st,
                         [&] { return launch_stft(pcm, M, nfft, hop, window, T, X, st); });
    return e == hipSuccess ? SSL_OK : hip_fail(e, "stft launch");
}

ssl_status ssl_corr_accum(ssl_ctx ctx, const ssl_c64 *X, int F, int T, int M, int64_t strideF,
                          int64_t strideT, double scale, int accumulate, ssl_prec prec, void *R,
                          void *stream)
{
    if (!ctx || !R) {
        ssl_set_error("ctx or R is NULL");
        return SSL_ERR_ARG;
    }
    ssl_status s = check_common(F, M, -1);
    if (s != SSL_OK) return s;
    if ((s = check_x(X, T, M, strideF, strideT)) != SSL_OK) return s;
    if (!ok_prec(prec)) {
        ssl_set_error("bad precision %d", (int)prec);
        return SSL_ERR_ARG;
    }
    DeviceGuard dg(ctx->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = timed(ctx, SSL_K_CORR, st, [&] {
        return launch_corr(X, F, T, M, strideF, strideT, scale, accumulate, prec, R, st);
    });
    return e == hipSuccess ? SSL_OK : hip_fail(e, "corr launch");
}

ssl_status ssl_noise_create(ssl_ctx ctx, int F, int M, ssl_noise *out)
{
    if (!ctx || !out) {
        ssl_set_error("ctx or out is NULL");
        return SSL_ERR_ARG;
    }
    *out = nullptr;
    ssl_status s = check_common(F, M, -1);
    if (s != SSL_OK) return s;
    DeviceGuard dg(ctx->device);
    ssl_noise n = new (std::nothrow) ssl_noise_s();
    if (!n) {
        ssl_set_error("out of host memory");
        return SSL_ERR_NOMEM;
    }
    n->ctx = ctx;
    n->F = F;
    n->M = M;
    const size_t mat = (size_t)F * M * M * sizeof(ssl_c128);
    void *k = nullptr, *w = nullptr, *st = nullptr;
    if ((s = dev_alloc(ctx, &k, mat, "noise K")) != SSL_OK) goto fail;
    if ((s = dev_alloc(ctx, &w, mat, "noise K^-1")) != SSL_OK) goto fail;
    if ((s = dev_alloc(ctx, &st, align256((size_t)F * sizeof(int32_t)), "noise status")) != SSL_OK)
        goto fail;
    n->K = static_cast<ssl_c128 *>(k);
    n->Kinv = static_cast<ssl_c128 *>(w);
    n->status = static_cast<int32_t *>(st);
    *out = n;
    return SSL_OK;
fail:
    dev_free(ctx, k, k ? mat : 0);
    dev_free(ctx, w, w ? mat : 0);
    delete n;
    return s;
}

void ssl_noise_destroy(ssl_noise n)
{
    if (!n) return;
    DeviceGuard dg(n->ctx->device);
    const size_t mat = (size_t)n->F * n->M * n->M * sizeof(ssl_c128);
    dev_free(n->ctx, n->K, mat);
    dev_free(n->ctx, n->Kinv, mat);
    if (n->Kisq) dev_free(n->ctx, n->Kisq, mat);
    dev_free(n->ctx, n->status, align256((size_t)n->F * sizeof(int32_t)));
    delete n;
}

static ssl_status noise_refactor(ssl_noise n, int32_t *bin_status, hipStream_t st)
{
    hipError_t e = timed(n->ctx, SSL_K_NOISE, st, [&] {
        return launch_noise_factor(n->K, n->Kinv, n->status, n->F, n->M, st);
    });
    if (e != hipSuccess) return hip_fail(e, "noise factor launch");
    if (n->gevd) {
        e = timed(n->ctx, SSL_K_NOISE, st, [&] {
            return launch_noise_isqrt(n->K, n->status, n->F, n->M, n->Kisq, n->status, st);
        });
        if (e != hipSuccess) return hip_fail(e, "K^-1/2 launch");
    }
    if (bin_status) {
        e = hipMemcpyAsync(bin_status, n->status, (size_t)n->F * sizeof(int32_t),
                           hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "status copy");
    }
    n->is_set = true;
    return SSL_OK;
}

ssl_status ssl_noise_set(ssl_noise n, const void *Kin, ssl_prec kprec, int32_t *bin_status,
                         void *stream)
{
    if (!n || !Kin) {
        ssl_set_error("noise handle or K is NULL");
        return SSL_ERR_ARG;
    }
    if (kprec != SSL_FP64 && kprec != SSL_FP32) {
        ssl_set_error("K must be complex128 (SSL_FP64) or complex64 (SSL_FP32)");
        return SSL_ERR_ARG;
    }
    DeviceGuard dg(n->ctx->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = timed(n->ctx, SSL_K_NOISE, st,
                         [&] { return launch_noise_load(n->K, Kin, kprec, n->F, n->M, st); });
    if (e != hipSuccess) return hip_fail(e, "noise load");
    return noise_refactor(n, bin_status, st);
}

ssl_status ssl_noise_update(ssl_noise n, const void *Khat, ssl_prec kprec, double alpha,
                            int32_t *bin_status, void *stream)
{
    if (!n || !Khat) {
        ssl_set_error("noise handle or Khat is NULL");
        return SSL_ERR_ARG;
    }
    if (!n->is_set) {
        ssl_set_error("noise handle was never set");
        return SSL_ERR_STATE;
    }
    if (kprec != SSL_FP64 && kprec != SSL_FP32) {
        ssl_set_error("Khat must be complex128 (SSL_FP64) or complex64 (SSL_FP32)");
        return SSL_ERR_ARG;
    }
    if (!(alpha >= 0.0 && alpha <= 1.0)) {
        ssl_set_error("alpha = %g must lie in [0, 1]", alpha);
        return SSL_ERR_ARG;
    }
    DeviceGuard dg(n->ctx->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = timed(n->ctx, SSL_K_NOISE, st, [&] {
        return launch_noise_blend(n->K, Khat, kprec, alpha, n->F, n->M, st);
    });
    if (e != hipSuccess) return hip_fail(e, "noise blend launch");
    return noise_refactor(n, bin_status, st);
}

ssl_status ssl_noise_get(ssl_noise n, ssl_c128 *K_out, void *stream)
{
    if (!n || !K_out) {
        ssl_set_error("noise handle or K_out is NULL");
        return SSL_ERR_ARG;
    }
    if (!n->is_set) {
        ssl_set_error("noise handle was never set");
        return SSL_ERR_STATE;
    }
    DeviceGuard dg(n->ctx->device);
    hipError_t e = hipMemcpyAsync(K_out, n->K, (size_t)n->F * n->M * n->M * sizeof(ssl_c128),
                                  hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SSL_OK : hip_fail(e, "noise get");
}

ssl_status ssl_noise_enable_gevd(ssl_noise n, void *stream)
{
    if (!n) {
        ssl_set_error("noise handle is NULL");
        return SSL_ERR_ARG;
    }
    DeviceGuard dg(n->ctx->device);
    if (!n->Kisq) {
        void *w = nullptr;
        ssl_status s = dev_alloc(n->ctx, &w, (size_t)n->F * n->M * n->M * sizeof(ssl_c128),
                                 "noise K^-1/2");
        if (s != SSL_OK) return s;
        n->Kisq = static_cast<ssl_c128 *>(w);
    }
    n->gevd = true;
    if (!n->is_set) return SSL_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const hipError_t e = timed(n->ctx, SSL_K_NOISE, st, [&] {
        return launch_noise_isqrt(n->K, n->status, n->F, n->M, n->Kisq, n->status, st);
    });
    return e == hipSuccess ? SSL_OK : hip_fail(e, "K^-1/2 launch");
}

ssl_status ssl_ctx_set_subspace(ssl_ctx ctx, ssl_subspace method)
{
    if (!ctx) {
        ssl_set_error("ctx is NULL");
        return SSL_ERR_ARG;
    }
    if (method != SSL_SUBSPACE_GSVD && method != SSL_SUBSPACE_GEVD) {
        ssl_set_error("unknown subspace method %d", (int)method);
        return SSL_ERR_ARG;
    }
    ctx->subspace = method;
    return SSL_OK;
}

int ssl_ctx_get_subspace(ssl_ctx ctx) { return ctx ? ctx->subspace : -1; }

ssl_status ssl_gsvd(ssl_ctx ctx, const ssl_c64 *R, ssl_noise K, int F, int M, int Ns, ssl_c64 *En,
                    float *sigma, int32_t *bin_status, int32_t *conv, int max_sweeps,
                    void *stream)
{
    if (!ctx || !R || !En) {
        ssl_set_error("ctx, R or En is NULL");
        return SSL_ERR_ARG;
    }
    ssl_status s = check_common(F, M, Ns);
    if (s != SSL_OK) return s;
    if ((s = check_noise(K, F, M)) != SSL_OK) return s;
    if ((s = check_gevd(ctx, K)) != SSL_OK) return s;
    if (max_sweeps < 0 || max_sweeps > 1000) {
        ssl_set_error("max_sweeps = %d out of range [0, 1000]", max_sweeps);
        return SSL_ERR_ARG;
    }
    if (max_sweeps == 0) max_sweeps = SSL_DEFAULT_SWEEPS;
    DeviceGuard dg(ctx->device);
    if ((s = ws_reserve(ctx, align256((size_t)F * M * M * sizeof(ssl_c64)))) != SSL_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    ssl_c64 *A = static_cast<ssl_c64 *>(ctx->ws);
    hipError_t e;
    const bool gevd = use_gevd(ctx, K);
    if (gevd) {
        e = timed(ctx, SSL_K_WHITEN, st,
                  [&] { return launch_gevd_whiten(K->Kisq, R, A, F, M, st); });
        if (e != hipSuccess) return hip_fail(e, "GEVD whitening launch");
    } else if (K) {
        e = timed(ctx, SSL_K_WHITEN, st, [&] { return launch_whiten(K->Kinv, R, A, F, M, st); });
        if (e != hipSuccess) return hip_fail(e, "whiten launch");
    } else {                                     // SEVD-MUSIC: the kernel overwrites its input
        e = hipMemcpyAsync(A, R, (size_t)F * M * M * sizeof(ssl_c64), hipMemcpyDeviceToDevice,
                           st);
        if (e != hipSuccess) return hip_fail(e, "copy of R");
    }
    e = timed(ctx, SSL_K_JACOBI, st, [&] {
        return launch_svd(ctx, A, K ? K->status : nullptr, F, M, Ns, max_sweeps, En, sigma,
                          bin_status, conv, st, nullptr,
                          ctx->sub_stop == SSL_STOP_ALSO_GSVD && !sigma ? kSubFullSweeps : -1);
    });
    if (e != hipSuccess) return hip_fail(e, "jacobi launch");
    if (gevd) {
        e = timed(ctx, SSL_K_WHITEN, st, [&] { return launch_gevd_back(K->Kisq, En, F, M, Ns, st); });
        if (e != hipSuccess) return hip_fail(e, "GEVD back-transformation launch");
    }
    return SSL_OK;
}

ssl_status ssl_music_spectrum(ssl_ctx ctx, const void *H, ssl_prec hprec, const ssl_c64 *En, int F,
                              int D, int M, int Ns, int p, float *P, float *Pbar,
                              const int32_t *bin_status, void *stream)
{
    if (!ctx || !H || !En || !Pbar) {
        ssl_set_error("ctx, H, En or Pbar is NULL");
        return SSL_ERR_ARG;
    }
    ssl_status s = check_common(F, M, Ns);
    if (s != SSL_OK) return s;
    if (D < 1 || D > (1 << 24)) {
        ssl_set_error("D = %d out of range", D);
        return SSL_ERR_ARG;
    }
    if (p != 1 && p != 2) {
        ssl_set_error("p = %d must be 1 or 2", p);
        return SSL_ERR_ARG;
    }
    if (hprec != SSL_FP32 && hprec != SSL_BF16 && hprec != SSL_FP16) {
        ssl_set_error("H precision must be SSL_FP32, SSL_BF16 or SSL_FP16");
        return SSL_ERR_ARG;
    }
    DeviceGuard dg(ctx->device);
    float *Pw = P;
    if (!Pw) {
        if ((s = ws_reserve(ctx, align256((size_t)F * D * sizeof(float)))) != SSL_OK) return s;
        Pw = static_cast<float *>(ctx->ws);
    }
    if ((s = binsum_reserve(ctx, F, D)) != SSL_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = timed(ctx, SSL_K_STEER, st, [&] {
        return launch_steer(H, hprec, En, F, D, M, Ns, p, bin_status, Pw,
                            st_waves(ctx, M, Ns, hprec), st);
    });
    if (e != hipSuccess) return hip_fail(e, "steer launch");
    e = timed(ctx, SSL_K_BINSUM, st, [&] {
        return launch_binsum_peaks(Pw, F, D, Pbar, ctx->binsum_part, D, 1, 1, nullptr, nullptr,
                                   st);
    });
    return e == hipSuccess ? SSL_OK : hip_fail(e, "bin-sum launch");
}

ssl_status ssl_peaks(ssl_ctx ctx, const float *Pbar, int n_az, int n_el, int Ns, int32_t *peaks,
                     float *peak_val, void *stream)
{
    if (!ctx || !Pbar || !peaks || !peak_val) {
        ssl_set_error("ctx, Pbar, peaks or peak_val is NULL");
        return SSL_ERR_ARG;
    }
    ssl_status s = check_grid(n_az, n_el, Ns);
    if (s != SSL_OK) return s;
    DeviceGuard dg(ctx->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = timed(ctx, SSL_K_BINSUM, st, [&] {
        return launch_peaks(Pbar, n_az, n_el, Ns, peaks, peak_val, st);
    });
    return e == hipSuccess ? SSL_OK : hip_fail(e, "peaks launch");
}

ssl_status ssl_localize(ssl_ctx ctx, const ssl_c64 *X, int F, int T, int M, int64_t strideF,
                        int64_t strideT, ssl_noise K, const void *H, ssl_prec prec, int n_az,
                        int n_el, int Ns, int p, int32_t *peaks, float *peak_val, float *Pbar,
                        int32_t *bin_status, void *stream)
{
    ssl_status s = check_localize(ctx, X, F, T, M, strideF, strideT, K, H, prec, n_az, n_el, Ns,
                                  p, peaks, peak_val);
    if (s != SSL_OK) return s;
    const LocalizeWs L = localize_ws(F, M, Ns, n_az * n_el);
    DeviceGuard dg(ctx->device);
    if ((s = ws_reserve(ctx, L.total)) != SSL_OK) return s;
    if ((s = binsum_reserve(ctx, F, n_az * n_el)) != SSL_OK) return s;
    return localize_enqueue(ctx, true, static_cast<char *>(ctx->ws), L, ctx->binsum_part, X, F, T,
                            M, strideF, strideT, K, H, prec, n_az, n_el, Ns, p, peaks, peak_val,
                            Pbar, bin_status, static_cast<hipStream_t>(stream));
}

size_t ssl_localize_noalloc_bytes(int F, int M, int Ns, int D)
{
    if (F < 1 || M < 1 || M > SSL_MAX_M || Ns < 1 || Ns >= M || D < 1 || D > (1 << 24)) return 0;
    return localize_ws(F, M, Ns, D).with_part;
}

ssl_status ssl_localize_noalloc(ssl_ctx ctx, const ssl_c64 *X, int F, int T, int M,
                                int64_t strideF, int64_t strideT, ssl_noise K, const void *H,
                                ssl_prec prec, int n_az, int n_el, int Ns, int p, int32_t *peaks,
                                float *peak_val, float *Pbar, int32_t *bin_status, void *stream)
{
    ssl_status s = check_localize(ctx, X, F, T, M, strideF, strideT, K, H, prec, n_az, n_el, Ns,
                                  p, peaks, peak_val);
    if (s != SSL_OK) return s;
    const LocalizeWs L = localize_ws(F, M, Ns, n_az * n_el);
    if (L.with_part > SSL_NOALLOC_SCRATCH_BYTES) {
        ssl_set_error("ssl_localize_noalloc: F = %d, M = %d, Ns = %d, D = %d needs %zu bytes of "
                      "scratch, the fixed scratch holds %zu",
                      F, M, Ns, n_az * n_el, L.with_part, (size_t)SSL_NOALLOC_SCRATCH_BYTES);
        return SSL_ERR_ARG;
    }
    char *scr = ctx->scratch;
    if (!scr) {
        ssl_set_error("ssl_localize_noalloc: no scratch address for device %d", ctx->device);
        return SSL_ERR_STATE;
    }
    DeviceGuard dg(ctx->device);
    return localize_enqueue(ctx, false, scr, L, reinterpret_cast<float *>(scr + L.total), X, F, T,
                            M, strideF, strideT, K, H, prec, n_az, n_el, Ns, p, peaks, peak_val,
                            Pbar, bin_status, static_cast<hipStream_t>(stream));
}

ssl_status ssl_sliding_create(ssl_ctx ctx, int F, int M, int T, ssl_sliding *out)
{
    if (!ctx || !out) {
        ssl_set_error("ctx or out is NULL");
        return SSL_ERR_ARG;
    }
    *out = nullptr;
    if (F < 1 || F > 65535 || M < 1 || M > SSL_MAX_M || T < 1 || T > 65535) {
        ssl_set_error("F = %d, M = %d, T = %d out of range", F, M, T);
        return SSL_ERR_ARG;
    }
    ssl_sliding s = new (std::nothrow) ssl_sliding_s();
    if (!s) {
        ssl_set_error("out of host memory");
        return SSL_ERR_NOMEM;
    }
    s->ctx = ctx;
    s->F = F;
    s->M = M;
    s->T = T;
    DeviceGuard dg(ctx->device);
    const size_t bRing = (size_t)F * T * M * sizeof(ssl_c64),
                 bS = (size_t)F * M * M * sizeof(ssl_c128), bU = (size_t)F * M * M * sizeof(ssl_c64);
    ssl_status st = dev_alloc(ctx, (void **)&s->ring, bRing, "frame ring");
    if (st == SSL_OK) st = dev_alloc(ctx, (void **)&s->S, bS, "sliding correlation");
    if (st == SSL_OK) st = dev_alloc(ctx, (void **)&s->U, bU, "singular vectors");
    if (st == SSL_OK) {
        s->bytes = bRing + bS + bU;
        const hipError_t e = hipMemset(s->S, 0, bS);
        if (e != hipSuccess) st = hip_fail(e, "hipMemset");
    }
    if (st != SSL_OK) {
        dev_free(ctx, s->ring, s->ring ? bRing : 0);
        dev_free(ctx, s->S, s->S ? bS : 0);
        dev_free(ctx, s->U, s->U ? bU : 0);
        delete s;
        return st;
    }
    *out = s;
    return SSL_OK;
}

void ssl_sliding_destroy(ssl_sliding s)
{
    if (!s) return;
    DeviceGuard dg(s->ctx->device);
    (void)hipDeviceSynchronize();
    dev_free(s->ctx, s->ring, (size_t)s->F * s->T * s->M * sizeof(ssl_c64));
    dev_free(s->ctx, s->S, (size_t)s->F * s->M * s->M * sizeof(ssl_c128));
    dev_free(s->ctx, s->U, (size_t)s->F * s->M * s->M * sizeof(ssl_c64));
    delete s;
}

int64_t ssl_sliding_frames(ssl_sliding s) { return s ? s->pushed : -1; }

ssl_status ssl_sliding_push(ssl_sliding s, const ssl_c64 *X, int n, int64_t strideF,
                            int64_t strideT, void *stream)
{
    if (!s || !X) {
        ssl_set_error("stream state or X is NULL");
        return SSL_ERR_ARG;
    }
    if (n < 1 || n > 65535 || strideT < s->M || strideF < 0) {
        ssl_set_error("n = %d, strides (%lld, %lld) invalid for M = %d", n, (long long)strideF,
                      (long long)strideT, s->M);
        return SSL_ERR_ARG;
    }
    DeviceGuard dg(s->ctx->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = timed(s->ctx, SSL_K_CORR, st, [&] {
        return launch_sliding_push(X, n, strideF, strideT, s->F, s->M, s->T, s->pushed, s->ring,
                                   s->S, st);
    });
    if (e != hipSuccess) return hip_fail(e, "sliding push launch");
    s->pushed += n;
    s->since_refresh += n;
    if (s->pushed >= s->T && s->since_refresh >= s->T) {
        // exact recomputation of S from the ring (FP64), so that update rounding never builds up
        e = timed(s->ctx, SSL_K_CORR, st, [&] {
            return launch_corr(s->ring, s->F, s->T, s->M, (int64_t)s->T * s->M, s->M, 1.0, 0,
                               SSL_FP64, s->S, st);
        });
        if (e != hipSuccess) return hip_fail(e, "sliding refresh launch");
        s->since_refresh = 0;
    }
    return SSL_OK;
}

ssl_status ssl_sliding_corr(ssl_sliding s, ssl_c128 *R, void *stream)
{
    if (!s || !R) {
        ssl_set_error("stream state or R is NULL");
        return SSL_ERR_ARG;
    }
    DeviceGuard dg(s->ctx->device);
    const hipError_t e = launch_sliding_scale(s->S, (int64_t)s->F * s->M * s->M, 1.0 / s->T, R,
                                              true, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? SSL_OK : hip_fail(e, "sliding scale launch");
}

ssl_status ssl_sliding_localize(ssl_sliding s, ssl_noise K, const void *H, ssl_prec prec,
                                int n_az, int n_el, int Ns, int p, int warm, int32_t *peaks,
                                float *peak_val, float *Pbar, int32_t *bin_status, int32_t *conv,
                                void *stream)
{
    if (!s || !H || !peaks || !peak_val) {
        ssl_set_error("stream state, H, peaks or peak_val is NULL");
        return SSL_ERR_ARG;
    }
    const int F = s->F, M = s->M;
    ssl_status st_ = check_common(F, M, Ns);
    if (st_ != SSL_OK) return st_;
    if ((st_ = check_grid(n_az, n_el, Ns)) != SSL_OK) return st_;
    if ((st_ = check_noise(K, F, M)) != SSL_OK) return st_;
    if ((st_ = check_gevd(s->ctx, K)) != SSL_OK) return st_;
    if (p != 1 && p != 2) {
        ssl_set_error("p = %d must be 1 or 2", p);
        return SSL_ERR_ARG;
    }
    if (prec != SSL_FP32 && prec != SSL_BF16 && prec != SSL_FP16) {
        ssl_set_error("prec must be SSL_FP32, SSL_BF16 or SSL_FP16");
        return SSL_ERR_ARG;
    }
    if (s->pushed < s->T) {
        ssl_set_error("%lld frames pushed, the window needs T = %d", (long long)s->pushed, s->T);
        return SSL_ERR_STATE;
    }
    ssl_ctx ctx = s->ctx;
    const int D = n_az * n_el;
    const LocalizeWs L = localize_ws(F, M, Ns, D);
    DeviceGuard dg(ctx->device);
    if ((st_ = ws_reserve(ctx, L.total)) != SSL_OK) return st_;
    if ((st_ = binsum_reserve(ctx, F, D)) != SSL_OK) return st_;
    char *w = static_cast<char *>(ctx->ws);
    ssl_c64 *R = reinterpret_cast<ssl_c64 *>(w);
    ssl_c64 *A = reinterpret_cast<ssl_c64 *>(w + L.bR);
    ssl_c64 *En = reinterpret_cast<ssl_c64 *>(w + 2 * L.bR);
    float *P = reinterpret_cast<float *>(w + 2 * L.bR + L.bE);
    float *Pb = Pbar ? Pbar : reinterpret_cast<float *>(w + 2 * L.bR + L.bE + L.bP);
    int32_t *stt = bin_status ? bin_status
                              : reinterpret_cast<int32_t *>(w + 2 * L.bR + L.bE + L.bP + L.bB);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = timed(ctx, SSL_K_CORR, st, [&] {
        return launch_sliding_scale(s->S, (int64_t)F * M * M, 1.0 / s->T, R, false, st);
    });
    if (e != hipSuccess) return hip_fail(e, "sliding scale launch");
    const bool gevd = use_gevd(ctx, K);
    if (gevd) {
        e = timed(ctx, SSL_K_WHITEN, st,
                  [&] { return launch_gevd_whiten(K->Kisq, R, A, F, M, st); });
        if (e != hipSuccess) return hip_fail(e, "GEVD whitening launch");
    } else if (K) {
        e = timed(ctx, SSL_K_WHITEN, st, [&] { return launch_whiten(K->Kinv, R, A, F, M, st); });
        if (e != hipSuccess) return hip_fail(e, "whiten launch");
    } else {
        A = R;
    }
    const int32_t *kst = K ? K->status : nullptr;
    if (warm && s->have_U && s->pushed - s->cold_at < s->T) {
        e = timed(ctx, SSL_K_JACOBI, st, [&] {
            return launch_jacobi_warm(A, kst, F, M, Ns, SSL_DEFAULT_SWEEPS, s->U, En, stt, conv,
                                      st);
        });
    } else {
        e = timed(ctx, SSL_K_JACOBI, st, [&] {
            return launch_svd(ctx, A, kst, F, M, Ns, SSL_DEFAULT_SWEEPS, En, nullptr, stt, conv,
                              st, s->U);
        });
        if (e == hipSuccess && ctx->svd == SSL_SVD_JACOBI) {     // the Jacobi solve wrote U
            s->have_U = true;
            s->cold_at = s->pushed;
        }
    }
    if (e != hipSuccess) return hip_fail(e, "jacobi launch");
    if (gevd) {
        e = timed(ctx, SSL_K_WHITEN, st, [&] { return launch_gevd_back(K->Kisq, En, F, M, Ns, st); });
        if (e != hipSuccess) return hip_fail(e, "GEVD back-transformation launch");
    }
    e = timed(ctx, SSL_K_STEER, st, [&] {
        return launch_steer(H, prec, En, F, D, M, Ns, p, stt, P, st_waves(ctx, M, Ns, prec), st);
    });
    if (e != hipSuccess) return hip_fail(e, "steer launch");
    e = timed(ctx, SSL_K_BINSUM, st, [&] {
        return launch_binsum_peaks(P, F, D, Pb, ctx->binsum_part, n_az, n_el, Ns, peaks, peak_val,
                                   st);
    });
    return e == hipSuccess ? SSL_OK : hip_fail(e, "bin-sum launch");
}

}  // extern "C"

// ------------------------------------------------------------------------------------------------
// batched path
// ------------------------------------------------------------------------------------------------
namespace {

constexpr int kJacobiQueues = 4;     // counters[0..3]: work queues of Jacobi classes 8/16/32/64

int jacobi_queue(int cls) { return cls == 8 ? 0 : cls == 16 ? 1 : cls == 32 ? 2 : 3; }

struct Seg {
    int cls, start, count, extra;
    int waves = 0;                         // projection: waves per workgroup
    bool sig = false;                      // projection: through the signal subspace
};

// Launch plan of one batch shape: per kernel, contiguous runs of items sharing a size class.
struct Plan {
    std::vector<Seg> corr, whiten, jac, steer;
    int nblocks = 0, n_items = 0, max_dc = 0, max_fc = 0;
    std::vector<Seg> gevd;                 // (block, bin) items of GEVD-MUSIC blocks, by class
    int nsmax = 1;                         // largest Ns of the blocks projected by steer_sig
};

// Device tail of the descriptor buffer after the four item lists: steering groups (first, count)
// into a block-index list, a group = the blocks of one size class that share a steering table;
// whitening chunks (first, count) into a second block-index list, a chunk = a run of blocks that
// share a noise set.  Layout: groups int2[nblocks], chunks int2[nblocks], gblocks int[nblocks],
// cblocks int[nblocks].
struct GroupArrays {
    const int2 *groups;
    const int *gblocks;
    const int2 *chunks;
    const int *cblocks;
};

// Blocks per whitening workgroup for groups of sizes n[g] with F[g] bins on `slots` resident
// workgroups: K^{-1} of a bin is loaded once per run, which costs about 0.3 of one block's
// product, while longer runs mean fewer workgroups to fill the device.  Minimises
// (rounds of the launch) x (0.3 + run length).
int whiten_run_length(const std::vector<int> &n, const std::vector<int> &F, int slots)
{
    int maxn = 1;
    for (int v : n) maxn = std::max(maxn, v);
    int best_c = 1;
    double best = 0.0;
    for (int c = 1; c <= maxn; ++c) {
        int64_t wg = 0;
        for (size_t g = 0; g < n.size(); ++g) wg += (int64_t)((n[g] + c - 1) / c) * F[g];
        const double cost = (double)((wg + slots - 1) / slots) * (0.3 + c);
        if (c == 1 || cost < best) {
            best = cost;
            best_c = c;
        }
    }
    return best_c;
}

ssl_status counters_reserve(ssl_ctx ctx, size_t n)
{
    if (ctx->n_counters >= n) return SSL_OK;
    size_t want = n < 256 ? 256 : n;
    if (want < 2 * ctx->n_counters) want = 2 * ctx->n_counters;
    clear_graphs(ctx);
    dev_free(ctx, ctx->counters, ctx->n_counters * sizeof(unsigned int));
    ctx->counters = nullptr;
    ctx->n_counters = 0;
    void *p = nullptr;
    ssl_status s = dev_alloc(ctx, &p, want * sizeof(unsigned int), "batch counters");
    if (s != SSL_OK) return s;
    hipError_t e = hipMemset(p, 0, want * sizeof(unsigned int));
    if (e != hipSuccess) {
        dev_free(ctx, p, want * sizeof(unsigned int));
        return hip_fail(e, "hipMemset");
    }
    ctx->counters = static_cast<unsigned int *>(p);
    ctx->n_counters = want;
    return SSL_OK;
}

ssl_status bdesc_reserve(ssl_ctx ctx, size_t bytes)
{
    if (ctx->bdesc_bytes >= bytes) return SSL_OK;
    size_t want = bytes < (1u << 16) ? (1u << 16) : bytes;
    if (want < 2 * ctx->bdesc_bytes) want = 2 * ctx->bdesc_bytes;
    hipError_t e;
    if (!ctx->bdesc_ev) {
        e = hipEventCreateWithFlags(&ctx->bdesc_ev, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
    (void)hipEventSynchronize(ctx->bdesc_ev);     // the old staging buffer is no longer read
    clear_graphs(ctx);
    if (ctx->bdesc_host) (void)hipHostFree(ctx->bdesc_host);
    dev_free(ctx, ctx->bdesc_dev, ctx->bdesc_bytes);
    ctx->bdesc_host = nullptr;
    ctx->bdesc_dev = nullptr;
    ctx->bdesc_bytes = 0;
    ssl_status s = dev_alloc(ctx, &ctx->bdesc_dev, want, "batch descriptors");
    if (s != SSL_OK) return s;
    e = hipHostMalloc(&ctx->bdesc_host, want, hipHostMallocDefault);
    if (e != hipSuccess) {
        dev_free(ctx, ctx->bdesc_dev, want);
        ctx->bdesc_dev = nullptr;
        return hip_fail(e, "hipHostMalloc");
    }
    ctx->bdesc_bytes = want;
    return SSL_OK;
}

// Item lists of one kernel: blocks grouped by class (ascending), bins in order inside a block.
void build_list(const std::vector<int> &cls_of_block, const std::vector<int> &F_of_block,
                int2 *out, std::vector<Seg> &segs)
{
    std::vector<int> classes(cls_of_block);
    std::sort(classes.begin(), classes.end());
    classes.erase(std::unique(classes.begin(), classes.end()), classes.end());
    int pos = 0;
    for (int c : classes) {
        Seg s{c, pos, 0, 0};
        for (size_t b = 0; b < cls_of_block.size(); ++b) {
            if (cls_of_block[b] != c) continue;
            for (int f = 0; f < F_of_block[b]; ++f) out[pos++] = make_int2((int)b, f);
        }
        s.count = pos - s.start;
        segs.push_back(s);
    }
}

hipError_t enqueue_batch(ssl_ctx ctx, const Plan &P, const BlockDev *blk, const int2 *lists,
                         GroupArrays ga, const int2 *l_gevd, ssl_prec prec, hipStream_t st)
{
    const int2 *l_corr = lists, *l_wh = lists + P.n_items, *l_jac = lists + 2 * P.n_items,
               *l_st = lists + 3 * P.n_items;
    hipError_t e = hipSuccess;
    for (const Seg &s : P.corr) {
        e = timed(ctx, SSL_K_CORR, st, [&] {
            return launch_corr_batch(blk, l_corr + s.start, s.count, s.cls, prec, st);
        });
        if (e != hipSuccess) return e;
    }
    for (const Seg &s : P.whiten) {
        e = timed(ctx, SSL_K_WHITEN, st, [&] {
            return launch_whiten_batch(blk, l_wh + s.start, s.count, ga.chunks, ga.cblocks, s.cls,
                                       st);
        });
        if (e != hipSuccess) return e;
    }
    for (const Seg &s : P.gevd) {
        e = timed(ctx, SSL_K_WHITEN, st, [&] {
            return launch_gevd_whiten_batch(blk, l_gevd + s.start, s.count, s.cls, st);
        });
        if (e != hipSuccess) return e;
    }
    for (const Seg &s : P.jac) {
        e = timed(ctx, SSL_K_JACOBI, st, [&] {
            if (ctx->svd == SSL_SVD_BIDIAG_QR)
                return launch_gk_svd_batch(blk, l_jac + s.start, s.count, s.cls,
                                           gk_max_steps(s.cls), st);
            return launch_jacobi_batch(blk, l_jac + s.start, s.count, s.cls,
                                       ctx->jac_lanes[jacobi_class_index(s.cls)],
                                       SSL_DEFAULT_SWEEPS, ctx->counters + jacobi_queue(s.cls),
                                       s.extra, st, sub_full_for(ctx, 2, true));
        });
        if (e != hipSuccess) return e;
    }
    for (const Seg &s : P.gevd) {
        e = timed(ctx, SSL_K_WHITEN, st, [&] {
            return launch_gevd_back_batch(blk, l_gevd + s.start, s.count, s.cls, st);
        });
        if (e != hipSuccess) return e;
    }
    for (const Seg &s : P.steer) {
        e = timed(ctx, SSL_K_STEER, st, [&] {
            if (s.sig)
                return launch_steer_sig_batch(blk, l_st + s.start, s.count, ga.groups, ga.gblocks,
                                              s.extra, P.nsmax, prec, st);
            return launch_steer_batch(blk, l_st + s.start, s.count, ga.groups, ga.gblocks, s.cls,
                                      s.waves, s.extra, prec, st);
        });
        if (e != hipSuccess) return e;
    }
    return timed(ctx, SSL_K_BINSUM, st, [&] {
        return launch_binsum_batch(blk, P.nblocks, P.max_dc, P.max_fc, st);
    });
}

}  // namespace

extern "C" {

ssl_status ssl_ctx_set_jacobi_lanes(ssl_ctx ctx, int M, int lanes)
{
    if (!ctx || M < 1 || M > SSL_MAX_M || !jacobi_variant_ok(jacobi_class(M), lanes)) {
        ssl_set_error("no Jacobi variant with %d lanes for M = %d", lanes, M);
        return SSL_ERR_ARG;
    }
    ctx->jac_lanes[jacobi_class_index(jacobi_class(M))] = lanes;
    return SSL_OK;
}

int ssl_ctx_get_jacobi_lanes(ssl_ctx ctx, int M)
{
    if (!ctx || M < 1 || M > SSL_MAX_M) return -1;
    return jac_lanes(ctx, M);
}

ssl_status ssl_autotune_jacobi(ssl_ctx ctx, const ssl_c64 *R, ssl_noise K, int F, int M, int Ns,
                               int nblocks, int reps, int *best_lanes, double *ms_per_variant,
                               void *stream)
{
    if (!ctx || !R || !K || !best_lanes) {
        ssl_set_error("ctx, R, K or best_lanes is NULL");
        return SSL_ERR_ARG;
    }
    ssl_status s = check_common(F, M, Ns);
    if (s != SSL_OK) return s;
    if (K->F != F || K->M != M || !K->is_set) {
        ssl_set_error("noise handle does not match (or was never set)");
        return SSL_ERR_ARG;
    }
    if (reps < 1 || reps > 1000) {
        ssl_set_error("reps = %d out of range [1, 1000]", reps);
        return SSL_ERR_ARG;
    }
    if (nblocks < 1 || nblocks > 65535) {
        ssl_set_error("nblocks = %d out of range [1, 65535]", nblocks);
        return SSL_ERR_ARG;
    }
    DeviceGuard dg(ctx->device);
    // workspace: A and E_n per block, then (batched form) bin status, descriptors and items
    const size_t nb = (size_t)nblocks;
    const size_t perA = (size_t)F * M * M, perE = (size_t)F * (M - Ns) * M;
    const size_t bA = align256(nb * perA * sizeof(ssl_c64));
    const size_t bE = align256(nb * perE * sizeof(ssl_c64));
    const size_t bS = align256(nb * F * sizeof(int32_t));
    const size_t bB = align256(nb * sizeof(BlockDev));
    const size_t bI = align256(nb * F * sizeof(int2));
    if ((s = ws_reserve(ctx, bA + bE + bS + bB + bI)) != SSL_OK) return s;
    if (nblocks > 1 && (s = counters_reserve(ctx, kJacobiQueues)) != SSL_OK) return s;
    char *w = static_cast<char *>(ctx->ws);
    ssl_c64 *A = reinterpret_cast<ssl_c64 *>(w);
    ssl_c64 *En = reinterpret_cast<ssl_c64 *>(w + bA);
    int32_t *dstat = reinterpret_cast<int32_t *>(w + bA + bE);
    BlockDev *dblk = reinterpret_cast<BlockDev *>(w + bA + bE + bS);
    int2 *ditems = reinterpret_cast<int2 *>(w + bA + bE + bS + bB);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int cls = jacobi_class(M);
    hipError_t e = hipSuccess;
    if (nblocks > 1) {
        std::vector<BlockDev> hb(nb);
        std::vector<int2> hi(nb * F);
        for (size_t b = 0; b < nb; ++b) {
            BlockDev &B = hb[b];
            memset(&B, 0, sizeof(B));
            B.F = F;
            B.M = M;
            B.Ns = Ns;
            B.p = 2;                                   // timed as the p = 2 localization runs
            B.kstatus = K->status;
            B.A = reinterpret_cast<float2 *>(A + b * perA);
            B.En = reinterpret_cast<float2 *>(En + b * perE);
            B.status = dstat + b * F;
            for (int f = 0; f < F; ++f) hi[b * F + f] = make_int2((int)b, f);
        }
        e = hipMemcpyAsync(dblk, hb.data(), nb * sizeof(BlockDev), hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ditems, hi.data(), nb * F * sizeof(int2), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);    // host staging goes out of scope
        if (e != hipSuccess) return hip_fail(e, "autotune staging");
    }
    auto launch = [&](int lanes) {
        if (nblocks == 1)
            return launch_jacobi(A, K->status, F, M, Ns, SSL_DEFAULT_SWEEPS, lanes, En, nullptr,
                                 nullptr, nullptr, st, nullptr, sub_full_for(ctx, 2, false));
        const int n_items = nblocks * F;
        const int grid = std::min(n_items, ctx->cu_count * jacobi_persistent_wg_per_cu(cls, lanes));
        return launch_jacobi_batch(dblk, ditems, n_items, cls, lanes, SSL_DEFAULT_SWEEPS,
                                   ctx->counters + jacobi_queue(cls), grid, st,
                                   sub_full_for(ctx, 2, true));
    };
    const int cand[3] = {4, 8, 16};
    hipEvent_t a = nullptr, b = nullptr;
    e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    int best = -1;
    double best_ms = 0.0;
    for (int i = 0; i < 3 && e == hipSuccess; ++i) {
        if (ms_per_variant) ms_per_variant[i] = -1.0;
        if (!jacobi_variant_ok(cls, cand[i])) continue;
        double total = 0.0;
        for (int r = 0; r <= reps && e == hipSuccess; ++r) {
            // A is consumed by each launch: whiten it again, outside the timed window
            for (size_t bb = 0; bb < nb && e == hipSuccess; ++bb)
                e = launch_whiten(K->Kinv, R, A + bb * perA, F, M, st);
            if (e == hipSuccess) e = hipEventRecord(a, st);
            if (e == hipSuccess) e = launch(cand[i]);
            if (e == hipSuccess) e = hipEventRecord(b, st);
            if (e == hipSuccess) e = hipEventSynchronize(b);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
            if (r > 0) total += ms;                               // launch 0 is the warm-up
        }
        const double mean = total / reps;
        if (ms_per_variant) ms_per_variant[i] = mean;
        if (best < 0 || mean < best_ms) {
            best = cand[i];
            best_ms = mean;
        }
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (e != hipSuccess) return hip_fail(e, "autotune");
    ctx->jac_lanes[jacobi_class_index(cls)] = best;
    *best_lanes = best;
    return SSL_OK;
}

ssl_status ssl_ctx_set_steer_waves(ssl_ctx ctx, int M, int Ns, ssl_prec hprec, int waves)
{
    if (!ctx || M < 1 || M > SSL_MAX_M || Ns < 1 || Ns >= M ||
        (hprec != SSL_FP32 && hprec != SSL_BF16 && hprec != SSL_FP16) || !steer_waves_ok(waves)) {
        ssl_set_error("no projection variant with %d waves for M = %d, Ns = %d, prec = %d", waves,
                      M, Ns, (int)hprec);
        return SSL_ERR_ARG;
    }
    ctx->steer_waves[steer_class_index(steer_class(M, Ns))][hprec] = waves;
    return SSL_OK;
}

int ssl_ctx_get_steer_waves(ssl_ctx ctx, int M, int Ns, ssl_prec hprec)
{
    if (!ctx || M < 1 || M > SSL_MAX_M || Ns < 1 || Ns >= M ||
        (hprec != SSL_FP32 && hprec != SSL_BF16 && hprec != SSL_FP16))
        return -1;
    return st_waves(ctx, M, Ns, hprec);
}

ssl_status ssl_autotune_steer(ssl_ctx ctx, const void *H, ssl_prec hprec, const ssl_c64 *En,
                              int F, int D, int M, int Ns, int p, int nblocks, int reps,
                              int *best_waves, double *ms_per_variant, void *stream)
{
    if (!ctx || !H || !En || !best_waves) {
        ssl_set_error("ctx, H, En or best_waves is NULL");
        return SSL_ERR_ARG;
    }
    ssl_status s = check_common(F, M, Ns);
    if (s != SSL_OK) return s;
    if (D < 1 || D > (1 << 24)) {
        ssl_set_error("D = %d out of range", D);
        return SSL_ERR_ARG;
    }
    if (p != 1 && p != 2) {
        ssl_set_error("p = %d must be 1 or 2", p);
        return SSL_ERR_ARG;
    }
    if (hprec != SSL_FP32 && hprec != SSL_BF16 && hprec != SSL_FP16) {
        ssl_set_error("H precision must be SSL_FP32, SSL_BF16 or SSL_FP16");
        return SSL_ERR_ARG;
    }
    if (reps < 1 || reps > 1000) {
        ssl_set_error("reps = %d out of range [1, 1000]", reps);
        return SSL_ERR_ARG;
    }
    if (nblocks < 1 || nblocks > 65535) {
        ssl_set_error("nblocks = %d out of range [1, 65535]", nblocks);
        return SSL_ERR_ARG;
    }
    DeviceGuard dg(ctx->device);
    // workspace: P per block, then (batched form) the descriptors, the (group, bin) items, one
    // group, its block list and an all-OK bin status
    const size_t bP = align256((size_t)nblocks * F * D * sizeof(float));
    const size_t bB = align256((size_t)nblocks * sizeof(BlockDev));
    const size_t bI = align256((size_t)F * sizeof(int2));
    const size_t bG = align256(sizeof(int2));
    const size_t bL = align256((size_t)nblocks * sizeof(int));
    const size_t bS = align256((size_t)F * sizeof(int32_t));
    if ((s = ws_reserve(ctx, bP + bB + bI + bG + bL + bS)) != SSL_OK) return s;
    char *w = static_cast<char *>(ctx->ws);
    float *P = reinterpret_cast<float *>(w);
    BlockDev *dblk = reinterpret_cast<BlockDev *>(w + bP);
    int2 *ditems = reinterpret_cast<int2 *>(w + bP + bB);
    int2 *dgroup = reinterpret_cast<int2 *>(w + bP + bB + bI);
    int *dlist = reinterpret_cast<int *>(w + bP + bB + bI + bG);
    int32_t *dstat = reinterpret_cast<int32_t *>(w + bP + bB + bI + bG + bL);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = hipSuccess;
    const int cls = steer_class(M, Ns);
    if (nblocks > 1) {
        std::vector<BlockDev> hb(nblocks);
        std::vector<int2> hi(F);
        std::vector<int> hl(nblocks);
        for (int b = 0; b < nblocks; ++b) {
            BlockDev &B = hb[b];
            memset(&B, 0, sizeof(B));
            B.F = F;
            B.M = M;
            B.Ns = Ns;
            B.D = D;
            B.p = p;
            B.hprec = hprec;
            B.H = H;
            B.En = const_cast<float2 *>(reinterpret_cast<const float2 *>(En));
            B.P = P + (size_t)b * F * D;
            B.status = dstat;
            hl[b] = b;
        }
        for (int f = 0; f < F; ++f) hi[f] = make_int2(0, f);
        const int2 grp = make_int2(0, nblocks);
        e = hipMemcpyAsync(dblk, hb.data(), nblocks * sizeof(BlockDev), hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ditems, hi.data(), F * sizeof(int2), hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(dgroup, &grp, sizeof(int2), hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(dlist, hl.data(), nblocks * sizeof(int), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemsetAsync(dstat, 0, F * sizeof(int32_t), st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);    // host staging goes out of scope
        if (e != hipSuccess) return hip_fail(e, "autotune staging");
    }
    auto launch = [&](int waves) {
        if (nblocks == 1)
            return launch_steer(H, hprec, En, F, D, M, Ns, p, nullptr, P, waves, st);
        const int rows = steer_rows_per_block(waves);
        return launch_steer_batch(dblk, ditems, F, dgroup, dlist, cls, waves,
                                  (D + rows - 1) / rows, hprec, st);
    };
    const int cand[3] = {4, 8, 16};
    hipEvent_t a = nullptr, b = nullptr;
    e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    int best = -1;
    double best_ms = 0.0;
    for (int i = 0; i < 3 && e == hipSuccess; ++i) {
        double total = 0.0;
        for (int r = 0; r <= reps && e == hipSuccess; ++r) {
            e = hipEventRecord(a, st);
            if (e == hipSuccess) e = launch(cand[i]);
            if (e == hipSuccess) e = hipEventRecord(b, st);
            if (e == hipSuccess) e = hipEventSynchronize(b);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
            if (r > 0) total += ms;                               // launch 0 is the warm-up
        }
        const double mean = total / reps;
        if (ms_per_variant) ms_per_variant[i] = mean;
        if (best < 0 || mean < best_ms) {
            best = cand[i];
            best_ms = mean;
        }
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (e != hipSuccess) return hip_fail(e, "autotune");
    ctx->steer_waves[steer_class_index(cls)][hprec] = best;
    *best_waves = best;
    return SSL_OK;
}

ssl_status ssl_ctx_set_svd(ssl_ctx ctx, ssl_svd method)
{
    if (!ctx) {
        ssl_set_error("ctx is NULL");
        return SSL_ERR_ARG;
    }
    if (method != SSL_SVD_JACOBI && method != SSL_SVD_BIDIAG_QR) {
        ssl_set_error("unknown SVD method %d", (int)method);
        return SSL_ERR_ARG;
    }
    ctx->svd = method;
    return SSL_OK;
}

int ssl_ctx_get_svd(ssl_ctx ctx) { return ctx ? ctx->svd : -1; }

ssl_status ssl_ctx_set_stop(ssl_ctx ctx, ssl_stop mode)
{
    if (!ctx) {
        ssl_set_error("ctx is NULL");
        return SSL_ERR_ARG;
    }
    if (mode < SSL_STOP_NEVER || mode > SSL_STOP_ALSO_GSVD) {
        ssl_set_error("unknown stop mode %d", (int)mode);
        return SSL_ERR_ARG;
    }
    ctx->sub_stop = mode;
    return SSL_OK;
}

int ssl_ctx_get_stop(ssl_ctx ctx) { return ctx ? ctx->sub_stop : -1; }

ssl_status ssl_ctx_set_projection(ssl_ctx ctx, ssl_projection mode)
{
    if (!ctx) {
        ssl_set_error("ctx is NULL");
        return SSL_ERR_ARG;
    }
    if (mode != SSL_PROJ_NOISE && mode != SSL_PROJ_SIGNAL) {
        ssl_set_error("unknown projection %d", (int)mode);
        return SSL_ERR_ARG;
    }
    ctx->proj = mode;
    return SSL_OK;
}

int ssl_ctx_get_projection(ssl_ctx ctx) { return ctx ? ctx->proj : -1; }

ssl_status ssl_ctx_use_graphs(ssl_ctx ctx, int enable)
{
    if (!ctx) {
        ssl_set_error("ctx is NULL");
        return SSL_ERR_ARG;
    }
    ctx->use_graphs = enable != 0;
    return SSL_OK;
}

ssl_status ssl_localize_batch(ssl_ctx ctx, const ssl_block_desc *descs, int nblocks,
                              ssl_prec prec, int p, void *stream)
{
    if (!ctx || !descs) {
        ssl_set_error("ctx or descs is NULL");
        return SSL_ERR_ARG;
    }
    if (nblocks < 1 || nblocks > 65535) {
        ssl_set_error("nblocks = %d out of range [1, 65535]", nblocks);
        return SSL_ERR_ARG;
    }
    if (p != 1 && p != 2) {
        ssl_set_error("p = %d must be 1 or 2", p);
        return SSL_ERR_ARG;
    }
    if (prec != SSL_FP32 && prec != SSL_BF16 && prec != SSL_FP16) {
        ssl_set_error("prec must be SSL_FP32, SSL_BF16 or SSL_FP16");
        return SSL_ERR_ARG;
    }
    ssl_status s;
    size_t ws_total = 0;
    int64_t n_items = 0;
    std::vector<char> sigb(nblocks);        // block projected through the signal subspace
    int nsmax = 1;
    std::vector<int64_t> key;
    key.reserve(10 + 6 * (size_t)nblocks);
    key.push_back(nblocks);
    key.push_back(prec);
    key.push_back(p);
    for (int i = 0; i < 4; ++i) key.push_back(ctx->jac_lanes[i]);   // kernel variants captured
    key.push_back(ctx->svd);
    key.push_back(ctx->sub_stop);
    key.push_back(ctx->proj);
    for (int c = 0; c < 3; ++c) key.push_back(ctx->steer_waves[c][prec]);
    for (int b = 0; b < nblocks; ++b) {
        const ssl_block_desc &d = descs[b];
        if ((s = check_common(d.F, d.M, d.Ns)) != SSL_OK ||
            (s = check_x(d.X, d.T, d.M, d.strideF, d.strideT)) != SSL_OK ||
            (s = check_grid(d.n_az, d.n_el, d.Ns)) != SSL_OK) {
            char msg[512];
            snprintf(msg, sizeof(msg), "block %d: %s", b, ssl_last_error());
            ssl_set_error("%s", msg);
            return s;
        }
        if (!d.H || !d.peaks || !d.peak_val) {
            ssl_set_error("block %d: H, peaks or peak_val is NULL", b);
            return SSL_ERR_ARG;
        }
        if (d.K && (d.K->F != d.F || d.K->M != d.M || !d.K->is_set)) {
            ssl_set_error("block %d: noise handle does not match (or was never set)", b);
            return SSL_ERR_ARG;
        }
        if ((s = check_gevd(ctx, d.K)) != SSL_OK) {
            char msg[512];
            snprintf(msg, sizeof(msg), "block %d: %s", b, ssl_last_error());
            ssl_set_error("%s", msg);
            return s;
        }
        key.push_back(d.K ? (use_gevd(ctx, d.K) ? 2 : 1) : 0);
        sigb[b] = use_sig(ctx, prec, p, d.Ns, use_gevd(ctx, d.K)) ? 1 : 0;
        if (sigb[b]) nsmax = std::max(nsmax, d.Ns);
        key.push_back(sigb[b]);
        const size_t F = d.F, M = d.M, D = (size_t)d.n_az * d.n_el, Nn = d.M - d.Ns;
        const size_t nch = (F + SSL_BINSUM_CHUNK - 1) / SSL_BINSUM_CHUNK;
        ws_total += 2 * align256(F * M * M * sizeof(ssl_c64)) + align256(F * Nn * M * sizeof(ssl_c64)) +
                    align256(F * D * sizeof(float)) + align256(nch * D * sizeof(float)) +
                    align256(F * sizeof(int32_t)) + align256(D * sizeof(float)) +
                    align256(F * d.Ns * M * sizeof(ssl_c64)) + align256(F * 6 * sizeof(ssl_c128));
        n_items += d.F;
        key.push_back(d.F);
        key.push_back(d.T);
        key.push_back(d.M);
        key.push_back(d.Ns);
        key.push_back(d.n_az);
        key.push_back(d.n_el);
    }
    if (n_items > (int64_t)1 << 30) {
        ssl_set_error("batch too large");
        return SSL_ERR_ARG;
    }
    key.push_back(nsmax);
    DeviceGuard dg(ctx->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t desc_bytes = align256(sizeof(BlockDev) * nblocks);
    // four item lists, the group / chunk tail, then the GEVD items
    const size_t tail_bytes = 2 * (sizeof(int2) + sizeof(int)) * (size_t)nblocks;
    const size_t list_bytes = sizeof(int2) * 5 * (size_t)n_items + tail_bytes;
    if ((s = ws_reserve(ctx, ws_total)) != SSL_OK) return s;
    if ((s = counters_reserve(ctx, kJacobiQueues)) != SSL_OK) return s;
    if ((s = bdesc_reserve(ctx, desc_bytes + list_bytes)) != SSL_OK) return s;

    // the previous call's staging copy must have completed before the buffer is rewritten
    hipError_t e = hipEventSynchronize(ctx->bdesc_ev);
    if (e != hipSuccess) return hip_fail(e, "staging event");
    BlockDev *hb = static_cast<BlockDev *>(ctx->bdesc_host);
    int2 *hl = reinterpret_cast<int2 *>(static_cast<char *>(ctx->bdesc_host) + desc_bytes);
    const BlockDev *db = static_cast<const BlockDev *>(ctx->bdesc_dev);
    const int2 *dl =
        reinterpret_cast<const int2 *>(static_cast<char *>(ctx->bdesc_dev) + desc_bytes);
    const int2 *dtail = dl + 4 * n_items;
    const GroupArrays ga{dtail, reinterpret_cast<const int *>(dtail + 2 * nblocks), dtail + nblocks,
                         reinterpret_cast<const int *>(dtail + 2 * nblocks) + nblocks};
    const int2 *dgevd = reinterpret_cast<const int2 *>(reinterpret_cast<const char *>(dtail) +
                                                       tail_bytes);
    int2 *hgevd = reinterpret_cast<int2 *>(reinterpret_cast<char *>(hl + 4 * n_items) + tail_bytes);

    Plan plan;
    plan.nblocks = nblocks;
    plan.n_items = (int)n_items;
    plan.nsmax = nsmax;
    std::vector<int> c_corr(nblocks), c_wh(nblocks), c_jac(nblocks), c_st(nblocks), Fs(nblocks);
    char *w = static_cast<char *>(ctx->ws);
    for (int b = 0; b < nblocks; ++b) {
        const ssl_block_desc &d = descs[b];
        const size_t F = d.F, M = d.M, D = (size_t)d.n_az * d.n_el, Nn = d.M - d.Ns;
        const size_t nch = (F + SSL_BINSUM_CHUNK - 1) / SSL_BINSUM_CHUNK;
        BlockDev &B = hb[b];
        B.X = reinterpret_cast<const float2 *>(d.X);
        B.sF = d.strideF;
        B.sT = d.strideT;
        B.F = d.F;
        B.T = d.T;
        B.M = d.M;
        B.Ns = d.Ns;
        B.D = (int)D;
        B.n_az = d.n_az;
        B.n_el = d.n_el;
        B.p = p;
        B.scale = (float)(1.0 / d.T);
        B.hprec = prec;
        B.Kinv = d.K ? reinterpret_cast<const double2 *>(d.K->Kinv) : nullptr;
        B.Kisq = use_gevd(ctx, d.K) ? reinterpret_cast<const double2 *>(d.K->Kisq) : nullptr;
        B.kstatus = d.K ? d.K->status : nullptr;
        B.H = d.H;
        B.R = reinterpret_cast<float2 *>(w);
        w += align256(F * M * M * sizeof(ssl_c64));
        B.A = d.K ? reinterpret_cast<float2 *>(w) : B.R;   // SEVD-MUSIC: Jacobi on R
        w += align256(F * M * M * sizeof(ssl_c64));
        B.En = sigb[b] ? nullptr : reinterpret_cast<float2 *>(w);   // not formed for eq.5 via E_s
        w += align256(F * Nn * M * sizeof(ssl_c64));
        B.P = reinterpret_cast<float *>(w);
        w += align256(F * D * sizeof(float));
        B.part = reinterpret_cast<float *>(w);
        w += align256(nch * D * sizeof(float));
        B.status = d.bin_status ? d.bin_status : reinterpret_cast<int32_t *>(w);
        w += align256(F * sizeof(int32_t));
        B.Pbar = d.Pbar ? d.Pbar : reinterpret_cast<float *>(w);
        w += align256(D * sizeof(float));
        B.Es = sigb[b] ? reinterpret_cast<float2 *>(w) : nullptr;
        w += align256(F * d.Ns * M * sizeof(ssl_c64));
        B.Esl = sigb[b] ? reinterpret_cast<double2 *>(w) : nullptr;
        w += align256(F * 6 * sizeof(ssl_c128));
        B.peaks = d.peaks;
        B.peak_val = d.peak_val;
        B.conv = d.conv;
        c_corr[b] = corr_class(d.M);
        c_wh[b] = whiten_class(d.M);
        c_jac[b] = jacobi_class(d.M);
        c_st[b] = steer_class(d.M, d.Ns);
        Fs[b] = d.F;
        plan.max_dc = std::max(plan.max_dc, (int)((D + binsum_threads() - 1) / binsum_threads()));
        plan.max_fc = std::max(plan.max_fc, (int)nch);
    }
    build_list(c_corr, Fs, hl, plan.corr);
    for (int cls : {16, 32, 64}) {                    // GEVD products: (block, bin) by class
        Seg sg{cls, 0, 0, 0};
        sg.start = plan.gevd.empty() ? 0 : plan.gevd.back().start + plan.gevd.back().count;
        for (int b = 0; b < nblocks; ++b)
            if (hb[b].Kisq && c_wh[b] == cls)
                for (int f = 0; f < hb[b].F; ++f) hgevd[sg.start + sg.count++] = make_int2(b, f);
        if (sg.count) plan.gevd.push_back(sg);
    }
    {
        // whitening: blocks of one class sharing a noise set, cut into runs of near-equal length
        // (whiten_run_length); items (chunk, bin), bin-major inside a group so that the runs of
        // one bin (one K^{-1}) are dispatched together
        int2 *hc = hl + 4 * n_items + nblocks;
        int *hcb = reinterpret_cast<int *>(hl + 4 * n_items + 2 * nblocks) + nblocks;
        std::vector<int> first;
        std::vector<std::vector<int>> members;
        std::map<std::tuple<int, const void *>, int> group_of;
        for (int b = 0; b < nblocks; ++b) {
            if (!hb[b].Kinv || hb[b].Kisq) {          // SEVD / GEVD block: not whitened here
                key.push_back(-1);
                continue;
            }
            const auto ins = group_of.emplace(std::make_tuple(c_wh[b], (const void *)hb[b].Kinv),
                                              (int)first.size());
            const int g = ins.first->second;
            if (ins.second) {
                first.push_back(b);
                members.emplace_back();
            }
            members[g].push_back(b);
            key.push_back(g);                         // the sharing pattern shapes the launch
        }
        std::vector<int> classes;
        for (int b = 0; b < nblocks; ++b)
            if (hb[b].Kinv && !hb[b].Kisq) classes.push_back(c_wh[b]);
        std::sort(classes.begin(), classes.end());
        classes.erase(std::unique(classes.begin(), classes.end()), classes.end());
        int2 *out = hl + n_items;
        int pos = 0, nchunk = 0, at = 0;
        for (int c : classes) {
            Seg sg{c, pos, 0, 0};
            std::vector<int> gs, gn, gf;
            for (size_t g = 0; g < members.size(); ++g)
                if (c_wh[first[g]] == c) {
                    gs.push_back((int)g);
                    gn.push_back((int)members[g].size());
                    gf.push_back(hb[first[g]].F);
                }
            const int run = whiten_run_length(gn, gf, ctx->cu_count * whiten_wg_per_cu(c));
            for (int g : gs) {
                const std::vector<int> &mb = members[g];
                const int n = (int)mb.size(), k = (n + run - 1) / run;
                const int c0 = nchunk;
                for (int r = 0, b0 = 0; r < k; ++r) {
                    const int len = n / k + (r < n % k ? 1 : 0);
                    hc[nchunk++] = make_int2(at, len);
                    for (int i = 0; i < len; ++i) hcb[at++] = mb[b0 + i];
                    b0 += len;
                }
                for (int f = 0; f < hb[first[g]].F; ++f)
                    for (int r = 0; r < k; ++r) out[pos++] = make_int2(c0 + r, f);
            }
            sg.count = pos - sg.start;
            plan.whiten.push_back(sg);
        }
    }
    build_list(c_jac, Fs, hl + 2 * n_items, plan.jac);
    {
        // steering groups (first-appearance order), then (group, bin) items by ascending class
        int2 *hg = hl + 4 * n_items;
        int *hgb = reinterpret_cast<int *>(hg + 2 * nblocks);
        std::vector<int> first;                       // first block of each group
        std::vector<std::vector<int>> members;
        std::map<std::tuple<int, const void *, int, int, int, int>, int> group_of;
        for (int b = 0; b < nblocks; ++b) {
            const BlockDev &B = hb[b];
            const auto ins = group_of.emplace(
                std::make_tuple(c_st[b], B.H, B.F, B.D, B.M, (int)sigb[b]), (int)first.size());
            const int g = ins.first->second;
            if (ins.second) {
                first.push_back(b);
                members.emplace_back();
            }
            members[g].push_back(b);
            key.push_back(g);                         // the sharing pattern shapes the launch
        }
        int at = 0;
        for (size_t g = 0; g < members.size(); ++g) {
            hg[g] = make_int2(at, (int)members[g].size());
            for (int b : members[g]) hgb[at++] = b;
        }
        std::vector<int> classes(c_st);
        std::sort(classes.begin(), classes.end());
        classes.erase(std::unique(classes.begin(), classes.end()), classes.end());
        int2 *out = hl + 3 * n_items;
        int pos = 0;
        for (int c : classes)
            for (int kind = 0; kind < 2; ++kind) {         // noise-vector, then signal-subspace
                Seg sg{c, pos, 0, 0};
                sg.sig = kind == 1;
                for (size_t g = 0; g < members.size(); ++g) {
                    if (c_st[first[g]] != c || sigb[first[g]] != kind) continue;
                    for (int f = 0; f < hb[first[g]].F; ++f) out[pos++] = make_int2((int)g, f);
                }
                sg.count = pos - sg.start;
                if (sg.count) plan.steer.push_back(sg);
            }
    }
    for (Seg &sg : plan.jac)
        sg.extra = std::min(sg.count, ctx->cu_count * jacobi_persistent_wg_per_cu(
                                                         sg.cls, ctx->jac_lanes[jacobi_class_index(sg.cls)]));
    for (Seg &sg : plan.steer) {
        sg.waves = ctx->steer_waves[steer_class_index(sg.cls)][prec];
        const int rows = steer_rows_per_block(sg.waves);
        int dt = 0;
        for (int b = 0; b < nblocks; ++b)
            if (c_st[b] == sg.cls && sigb[b] == (sg.sig ? 1 : 0))
                dt = std::max(dt, sg.sig ? steer_sig_tiles(hb[b].D) : (hb[b].D + rows - 1) / rows);
        sg.extra = dt;
    }

    e = hipMemcpyAsync(ctx->bdesc_dev, ctx->bdesc_host, desc_bytes + list_bytes,
                       hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(ctx->bdesc_ev, st);
    if (e != hipSuccess) return hip_fail(e, "descriptor copy");

    if (!ctx->use_graphs || ctx->timing) {
        e = enqueue_batch(ctx, plan, db, dl, ga, dgevd, prec, st);
        return e == hipSuccess ? SSL_OK : hip_fail(e, "batch launch");
    }
    hipGraphExec_t exec = nullptr;
    for (auto &g : ctx->graphs)
        if (g.key == key) {
            exec = g.exec;
            break;
        }
    if (!exec) {
        if (!ctx->cap_stream) {
            e = hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking);
            if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
        }
        e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        hipError_t le = enqueue_batch(ctx, plan, db, dl, ga, dgevd, prec, ctx->cap_stream);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(ctx->cap_stream, &graph);
        if (le != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return hip_fail(le, "batch capture");
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        if (ctx->graphs.size() >= 32) clear_graphs(ctx);
        ctx->graphs.push_back({key, exec});
    }
    e = hipGraphLaunch(exec, st);
    return e == hipSuccess ? SSL_OK : hip_fail(e, "hipGraphLaunch");
}

ssl_status ssl_noise_update_frames_from(ssl_ctx ctx, int n, const ssl_noise *dst,
                                        const ssl_noise *src, const ssl_c64 *const *Xn,
                                        const int *T, double alpha, void *stream)
{
    if (!ctx || n < 0 || (n > 0 && (!dst || !src || !Xn || !T))) {
        ssl_set_error("ctx, dst, src, Xn or T is NULL (or n < 0)");
        return SSL_ERR_ARG;
    }
    if (!(alpha >= 0.0 && alpha <= 1.0)) {
        ssl_set_error("alpha = %g must lie in [0, 1]", alpha);
        return SSL_ERR_ARG;
    }
    // entries run in list order: entry i goes to the round after the last one that wrote its
    // source or its destination, or read its destination; the entries of one round touch
    // disjoint matrices (apart from an update in place), so each round is one batched launch pair
    // per size class
    std::vector<int> round(n);
    std::map<ssl_noise, int> last_w, last_r;
    auto last = [](const std::map<ssl_noise, int> &m, ssl_noise h) {
        auto it = m.find(h);
        return it == m.end() ? -1 : it->second;
    };
    int n_rounds = 0;
    int64_t n_items = 0;
    for (int i = 0; i < n; ++i) {
        const ssl_noise h = dst[i], hs = src[i];
        if (!h || !hs || !Xn[i]) {
            ssl_set_error("entry %d: noise handle or frames are NULL", i);
            return SSL_ERR_ARG;
        }
        if (!hs->is_set && !last_w.count(hs)) {          // nor written by an earlier entry
            ssl_set_error("entry %d: source noise handle was never set", i);
            return SSL_ERR_STATE;
        }
        if (h->ctx->device != ctx->device || hs->ctx->device != ctx->device) {
            ssl_set_error("entry %d: noise handles live on devices %d / %d, ctx on %d", i,
                          h->ctx->device, hs->ctx->device, ctx->device);
            return SSL_ERR_ARG;
        }
        if (hs->F != h->F || hs->M != h->M) {
            ssl_set_error("entry %d: source handle is %d x %d x %d, destination %d x %d x %d", i,
                          hs->F, hs->M, hs->M, h->F, h->M, h->M);
            return SSL_ERR_ARG;
        }
        if (T[i] < 1) {
            ssl_set_error("entry %d: T = %d must be >= 1", i, T[i]);
            return SSL_ERR_ARG;
        }
        const int r = 1 + std::max({last(last_w, hs), last(last_w, h), last(last_r, h)});
        round[i] = r;
        last_w[h] = r;
        last_r[hs] = std::max(last(last_r, hs), r);
        n_rounds = std::max(n_rounds, r + 1);
        n_items += h->F;
    }
    if (n == 0) return SSL_OK;
    if (n_items > (int64_t)1 << 30) {
        ssl_set_error("too many bins");
        return SSL_ERR_ARG;
    }
    DeviceGuard dg(ctx->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    // staging: descriptors [n], then the items of (round, class) segments
    const size_t desc_bytes = align256(sizeof(NoiseUpdDev) * n);
    const size_t item_bytes = sizeof(int2) * (size_t)n_items;
    ssl_status s = bdesc_reserve(ctx, desc_bytes + item_bytes);
    if (s != SSL_OK) return s;
    hipError_t e = hipEventSynchronize(ctx->bdesc_ev);   // the previous staging copy is done
    if (e != hipSuccess) return hip_fail(e, "staging event");
    NoiseUpdDev *hd = static_cast<NoiseUpdDev *>(ctx->bdesc_host);
    int2 *hi = reinterpret_cast<int2 *>(static_cast<char *>(ctx->bdesc_host) + desc_bytes);
    for (int i = 0; i < n; ++i) {
        const ssl_noise h = dst[i];
        hd[i] = NoiseUpdDev{reinterpret_cast<const float2 *>(Xn[i]), h->F, T[i], h->M,
                            reinterpret_cast<const double2 *>(src[i]->K),
                            reinterpret_cast<double2 *>(h->K), reinterpret_cast<double2 *>(h->Kinv),
                            h->status};
    }
    struct Seg {
        int cls, start, count;
    };
    std::vector<std::vector<Seg>> segs(n_rounds);
    int pos = 0;
    for (int r = 0; r < n_rounds; ++r)
        for (int c : {16, 32, 64}) {
            Seg sg{c, pos, 0};
            for (int i = 0; i < n; ++i)
                if (round[i] == r && noise_class(dst[i]->M) == c)
                    for (int f = 0; f < dst[i]->F; ++f) hi[pos++] = make_int2(i, f);
            sg.count = pos - sg.start;
            if (sg.count) segs[r].push_back(sg);
        }
    e = hipMemcpyAsync(ctx->bdesc_dev, ctx->bdesc_host, desc_bytes + item_bytes,
                       hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(ctx->bdesc_ev, st);
    if (e != hipSuccess) return hip_fail(e, "descriptor copy");
    const NoiseUpdDev *dd = static_cast<const NoiseUpdDev *>(ctx->bdesc_dev);
    const int2 *di = reinterpret_cast<const int2 *>(static_cast<char *>(ctx->bdesc_dev) + desc_bytes);
    for (int r = 0; r < n_rounds; ++r) {
        for (const Seg &sg : segs[r]) {
            e = timed(ctx, SSL_K_CORR, st, [&] {
                return launch_noise_corr_blend(dd, di + sg.start, sg.count, sg.cls, alpha, st);
            });
            if (e != hipSuccess) return hip_fail(e, "noise correlation launch");
        }
        for (const Seg &sg : segs[r]) {
            e = timed(ctx, SSL_K_NOISE, st, [&] {
                return launch_noise_factor_batch(dd, di + sg.start, sg.count, sg.cls, st);
            });
            if (e != hipSuccess) return hip_fail(e, "noise factor launch");
        }
    }
    for (int i = 0; i < n; ++i) {
        ssl_noise h = dst[i];
        h->is_set = true;
        bool first = true;                           // a handle listed twice: once suffices
        for (int j = i + 1; j < n; ++j) first = first && dst[j] != h;
        if (h->gevd && first) {
            e = timed(ctx, SSL_K_NOISE, st, [&] {
                return launch_noise_isqrt(h->K, h->status, h->F, h->M, h->Kisq, h->status, st);
            });
            if (e != hipSuccess) return hip_fail(e, "K^-1/2 launch");
        }
    }
    return SSL_OK;
}

ssl_status ssl_noise_update_frames(ssl_ctx ctx, int n, const ssl_noise *handles,
                                   const ssl_c64 *const *Xn, const int *T, double alpha,
                                   void *stream)
{
    return ssl_noise_update_frames_from(ctx, n, handles, handles, Xn, T, alpha, stream);
}

}  // extern "C"
