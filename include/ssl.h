/*
 * ssl.h -- C ABI of the MI355X (gfx950) GSVD-MUSIC sound-source-localization library.
 *
 * The method (arXiv 2504.03373, Sec. III-A and III-B):
 *   eq.2-3  R(w)  = (1/T) sum_t X(w,t) X(w,t)^H           correlation per frequency bin w
 *   eq.4    K(w)^{-1} R(w) = E Lambda E_r                 GSVD against the preset noise correlation K
 *           E_n(w) = [e_{Ns+1} .. e_M]                    noise subspace (left singular vectors)
 *   eq.5    P(theta,w) = |H^H H| / sum_i |H^H e_i|^p      MUSIC pseudo-spectrum (p = 2 default, 1 = literal)
 *   eq.6    Pbar(theta) = sum_w P(theta,w)                 sum over bins
 *   Sec. III-A, last paragraph: the preset number Ns of peaks of Pbar over the direction grid.
 *
 * Conventions for every entry point:
 *   - Array arguments are caller-owned DEVICE pointers (HBM of the context's device) unless the
 *     comment says "host".  The library never frees them and never keeps them past the completion
 *     of the work it enqueued on `stream`.
 *   - `stream` is a hipStream_t passed as void* (NULL = the legacy default stream).  Everything is
 *     enqueued asynchronously on it; the call returns before the GPU has finished.
 *   - Complex numbers are interleaved (re, im): ssl_c64 == torch.complex64, ssl_c128 == complex128.
 *   - Matrices are row-major per bin: element (i, j) of bin f of an [F][M][M] array is at
 *     f*M*M + i*M + j.  E_n is stored column-major per bin: column c of bin f at (f*(M-Ns)+c)*M.
 *   - Argument, shape and budget errors are reported synchronously by the return value; nothing is
 *     enqueued in that case and ssl_last_error() describes the problem.  Numerical failures are
 *     reported per bin, asynchronously, in `bin_status` (ssl_bin_status codes); a failed bin
 *     contributes 0 to Pbar and never poisons the other bins.
 *   - No C++ exception crosses this interface.  A context is not thread-safe: use one per host
 *     thread.  Calls that share a context must be ordered on one stream (its workspace is reused).
 *   - Limits: 1 <= M <= 64, 1 <= Ns < M, F, T, D >= 1, p in {1, 2}.
 */
#ifndef SSL_MI355X_H
#define SSL_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { float re, im; } ssl_c64;
typedef struct { double re, im; } ssl_c128;

typedef struct ssl_ctx_s *ssl_ctx;      /* library-owned: device, workspace (HBM budget) */
typedef struct ssl_noise_s *ssl_noise;  /* library-owned: one stream's K and its FP64 factor */
typedef struct ssl_sliding_s *ssl_sliding;  /* library-owned: a frame stream's eq.3 window */

typedef enum {
    SSL_OK = 0,
    SSL_ERR_ARG = -1,     /* bad argument or shape */
    SSL_ERR_NOMEM = -2,   /* device allocation failed */
    SSL_ERR_BUDGET = -3,  /* workspace would exceed the context's HBM budget */
    SSL_ERR_HIP = -4,     /* a HIP runtime call failed */
    SSL_ERR_STATE = -5    /* object used in the wrong state (e.g. noise handle never set) */
} ssl_status;

typedef enum {
    SSL_BIN_OK = 0,
    SSL_BIN_NOT_PD = 1,     /* K(w) is not numerically positive definite (FP64 Cholesky pivot
                               d_k <= 2^-40 * max_i K_ii, or not finite) */
    SSL_BIN_NO_CONV = 2,    /* the Jacobi SVD hit max_sweeps before converging */
    SSL_BIN_NONFINITE = 3   /* NaN or Inf in R(w) */
} ssl_bin_status;

typedef enum { SSL_FP32 = 0, SSL_BF16 = 1, SSL_FP16 = 2, SSL_FP64 = 3 } ssl_prec;

/* ---------------------------------------------------------------- context */

/* Creates a context on HIP device `device`.  hbm_budget_bytes bounds the workspace the context may
 * allocate (0 = unlimited).  Returns SSL_ERR_ARG for a bad device, SSL_ERR_HIP on runtime errors. */
ssl_status ssl_ctx_create(ssl_ctx *out, int device, size_t hbm_budget_bytes);
void ssl_ctx_destroy(ssl_ctx ctx);
/* Bytes of device workspace the context currently holds. */
size_t ssl_ctx_workspace_bytes(ssl_ctx ctx);
/* Per-kernel device timing.  While enabled, every kernel the context enqueues is bracketed by a
 * pair of HIP events recorded on the same stream.  ssl_ctx_timing_read() waits for the recorded
 * events and returns, per kernel class (ssl_kernel_id), the number of launches and the summed
 * device milliseconds since the last reset; reset != 0 clears the totals.  launches and total_ms
 * are host arrays of SSL_K_COUNT entries. */
typedef enum {
    SSL_K_CORR = 0,     /* correlation accumulation (eq.2-3) */
    SSL_K_NOISE = 1,    /* noise load / blend / FP64 inversion */
    SSL_K_WHITEN = 2,   /* A = K^{-1} R (FP64) */
    SSL_K_JACOBI = 3,   /* one-sided Jacobi SVD + sort + E_n */
    SSL_K_STEER = 4,    /* H^H E_n projection and P (eq.5) */
    SSL_K_BINSUM = 5,   /* bin sum (eq.6) + peak search */
    SSL_K_COUNT = 6
} ssl_kernel_id;
ssl_status ssl_ctx_timing(ssl_ctx ctx, int enable);
ssl_status ssl_ctx_timing_read(ssl_ctx ctx, int64_t *launches, double *total_ms, int reset);

/* Thread-local description of the last error of this thread (never NULL; "" if none). */
const char *ssl_last_error(void);
/* Library version as major*10000 + minor*100 + patch. */
int ssl_version(void);

/* ------------------------------------------------------------ STFT (eq.1) */

/* eq.1: the short-time Fourier transform of every channel of M-channel PCM,
 *   X_m(w, t) = sum_{n < nfft} win[n] x_m[t*hop + n] exp(-2 pi i w n / nfft),  w = 0 .. nfft/2,
 * for the complete frames t = 0 .. T-1 (frame t covers samples t*hop .. t*hop + nfft - 1; no
 * padding, no normalisation).  pcm: [n_samples][M] float32, channel-interleaved (device).
 * window: [nfft] float32 (device), or NULL for the periodic Hann window sin^2(pi n / nfft).
 * X: [nfft/2 + 1][T][M] complex64 (device), the layout ssl_corr_accum and ssl_localize read
 * (strideF = T*M, strideT = M).  nfft a power of two in [16, 4096]; 1 <= M <= 4096; hop >= 1;
 * 1 <= T <= 65535 with (T-1)*hop + nfft <= n_samples.  FP32 radix-2 FFT.  Timed (ssl_ctx_timing)
 * under SSL_K_CORR. */
ssl_status ssl_stft(ssl_ctx ctx, const float *pcm, int64_t n_samples, int M, int nfft, int hop,
                    int T, const float *window, ssl_c64 *X, void *stream);

/* ------------------------------------------------------- correlation (eq.2-3) */

/* AddCorrelation + NormalizeCorrelation (eq.2, eq.3):
 *   R[f] = scale * sum_{t<T} X[f,t,:] X[f,t,:]^H   (+ R[f] when accumulate != 0)
 * X: [F][T][M] complex64, M contiguous, element strides strideF, strideT (>= M).
 * prec: SSL_FP32 -> R is ssl_c64 [F][M][M], accumulated in FP32 on MFMA;
 *       SSL_BF16 / SSL_FP16 -> R is ssl_c64, X rounded to bf16/fp16 MFMA inputs, FP32 accumulation;
 *       SSL_FP64 -> R is ssl_c128 [F][M][M], FP64 accumulation (use it for the noise correlation K).
 * Both triangles are written from one computed value: R is Hermitian to the bit, diag imag = 0. */
ssl_status ssl_corr_accum(ssl_ctx ctx, const ssl_c64 *X, int F, int T, int M, int64_t strideF,
                          int64_t strideT, double scale, int accumulate, ssl_prec prec, void *R,
                          void *stream);

/* ------------------------------------------------- noise correlation handle */

/* A noise handle keeps one stream's preset noise correlation K(w) (the K of eq.4) resident on the
 * device in complex128 together with its FP64 factorisation, so each block only pays for the
 * whitening product.  Owned by the library; destroy with ssl_noise_destroy. */
ssl_status ssl_noise_create(ssl_ctx ctx, int F, int M, ssl_noise *out);
/* Copies K ([F][M][M]; ssl_c128 if kprec == SSL_FP64, ssl_c64 if SSL_FP32) into the handle and
 * inverts it per bin in FP64 by Gauss-Jordan elimination (the paper's method for K^{-1}); without
 * pivoting on a Hermitian positive definite K the elimination pivots are the Cholesky pivots
 * d_k = L_kk^2, which give the positive-definiteness test.  Per-bin result in bin_status ([F]
 * int32, may be NULL): SSL_BIN_OK or SSL_BIN_NOT_PD. */
ssl_status ssl_noise_set(ssl_noise K, const void *Kin, ssl_prec kprec, int32_t *bin_status,
                         void *stream);
/* Exponential averaging for streams whose noise field drifts:
 *   K <- alpha * K + (1 - alpha) * Khat, then refactor (same outputs as ssl_noise_set). */
ssl_status ssl_noise_update(ssl_noise K, const void *Khat, ssl_prec kprec, double alpha,
                            int32_t *bin_status, void *stream);
/* Serving form of ssl_noise_update, for many streams in one call: for each i < n, handle i's K is
 * blended with the FP64 correlation of its own noise-only frames Xn[i] ([F][T[i]][M] complex64,
 * device, contiguous, F and M those of the handle) and refactored:
 *   K <- alpha * K + (1 - alpha) * (1/T) sum_t x_t x_t^H.
 * Bit-identical, handle by handle, to ssl_corr_accum(ctx, Xn[i], F, T[i], M, T[i] M, M,
 * 1.0 / T[i], 0, SSL_FP64, Khat) followed by ssl_noise_update(handle, Khat, SSL_FP64, alpha,
 * NULL); a handle listed twice is updated twice, in list order.  All the bins of all the handles
 * run in one correlation-and-blend launch and one inverse launch per channel-count class (M <= 16,
 * <= 32, <= 64), on `stream`.  The descriptors go through ctx's batch staging buffers, so calls on
 * one ctx must be issued on one stream (or not overlap).  Handles must be on ctx's device.  Each
 * handle keeps its per-bin status (SSL_BIN_NOT_PD bins yield that status in ssl_gsvd). */
ssl_status ssl_noise_update_frames(ssl_ctx ctx, int n, const ssl_noise *handles,
                                   const ssl_c64 *const *Xn, const int *T, double alpha,
                                   void *stream);
/* ssl_noise_update_frames with a separate source per entry: for each i < n,
 *   dst[i].K <- alpha * src[i].K + (1 - alpha) * (1/T[i]) sum_t x_t x_t^H   (frames Xn[i]),
 * then dst[i]'s FP64 inverse and per-bin status are recomputed from the new K; src[i] is only
 * read (src[i] == dst[i] is the in-place update, bit-identical to ssl_noise_update_frames).  It
 * lets a stream keep two handles and blend into the one no batch is reading, so the update of
 * block n can run beside block n + 1 (which reads the other handle).  src[i] must be set (or be
 * the destination of an earlier entry) and have dst[i]'s F and M; dst[i] need not be set before.
 * Entries take effect in list order (an entry that reads or writes a matrix an earlier entry
 * writes, or writes one it reads, runs after it).
 * Errors (SSL_ERR_ARG / SSL_ERR_STATE, nothing launched): NULL arrays or entries, a source never
 * set, mismatched shapes or devices, T < 1, alpha outside [0, 1]. */
ssl_status ssl_noise_update_frames_from(ssl_ctx ctx, int n, const ssl_noise *dst,
                                        const ssl_noise *src, const ssl_c64 *const *Xn,
                                        const int *T, double alpha, void *stream);
/* Copies the current K (complex128 [F][M][M]) to K_out (device) for checkpointing. */
ssl_status ssl_noise_get(ssl_noise K, ssl_c128 *K_out, void *stream);
/* Prepares the handle for GEVD-MUSIC: allocates 16 F M^2 bytes (within the HBM budget) for
 * K^{-1/2}, computes it if K is set (FP64 one-sided Jacobi eigen-decomposition of K, rotate iff
 * |z_i^H z_j| > M 2^-53 |z_i||z_j|, at most 40 sweeps), and from then on recomputes it with every
 * ssl_noise_set / ssl_noise_update / ssl_noise_update_frames(_from) of the handle.  A bin whose K
 * is not positive definite, or whose decomposition does not converge, gets SSL_BIN_NOT_PD /
 * SSL_BIN_NO_CONV in the handle's status. */
ssl_status ssl_noise_enable_gevd(ssl_noise K, void *stream);
void ssl_noise_destroy(ssl_noise K);

/* --------------------------------------------------------------- GSVD (eq.4) */

/* For every bin f: A = K^{-1} R (FP64 product with the handle's inverse, rounded to complex64),
 * then the SVD A = U Sigma V^H by one-sided Jacobi in FP32 with the whole M x M problem resident in
 * LDS (a pair is rotated iff |b_i^H b_j| > 2 sqrt(M) 2^-24 |b_i||b_j|, the inner products
 * accumulated in FP32 and the comparison made in FP64; a sweep without a rotation ends the solve),
 * singular values sorted descending (ties: lower column first), and
 *   En[f] = U[:, Ns..M-1]   written column-major: [F][M-Ns][M] ssl_c64.
 * R: [F][M][M] ssl_c64 (e.g. from ssl_corr_accum).  K: a handle set for the same F and M, or
 * NULL for SEVD-MUSIC (the standard-eigenvalue baseline the paper compares against, Sec. II):
 * no whitening, the same SVD of R itself -- R is Hermitian positive semi-definite, so its left
 * singular vectors are its eigenvectors and its singular values its eigenvalues.
 * sigma: [F][M] float or NULL.  bin_status: [F] int32 or NULL.
 * conv: [F][3] int32 or NULL -> (sweeps run, rotations applied, numerical rank) per bin.
 * Numerical rank: the pivoted Householder QR that preconditions the Jacobi iteration stops at the
 * first pivot norm <= M 2^-24 times the first; the trailing rows are treated as zero (their
 * singular values are below the FP32 resolution of A), so only rank columns enter the sweeps.
 * max_sweeps: 0 selects the default (20).  Failed bins get En = 0 and sigma = 0. */
ssl_status ssl_gsvd(ssl_ctx ctx, const ssl_c64 *R, ssl_noise K, int F, int M, int Ns, ssl_c64 *En,
                    float *sigma, int32_t *bin_status, int32_t *conv, int max_sweeps, void *stream);

/* ------------------------------------------------- MUSIC spectrum (eq.5-6) */

/* den[f,d] = sum_{c<M-Ns} |H[f,d,:]^H En[f,:,c]|^p,   P[f,d] = |H[f,d,:]|^2 / max(den, FLT_MIN),
 * Pbar[d] = sum_f P[f,d] (bins in ascending order within fixed chunks; deterministic).
 * H: [F][D][M], ssl_c64 if hprec == SSL_FP32, or interleaved bf16/fp16 pairs (4 bytes per complex)
 * for SSL_BF16 / SSL_FP16 (the projection then runs on bf16/fp16 MFMA with FP32 accumulation; En
 * is rounded to the same type).  P: [F][D] float or NULL; Pbar: [D] float (required).
 * bin_status: [F] or NULL; bins whose status is not SSL_BIN_OK contribute P = 0. */
ssl_status ssl_music_spectrum(ssl_ctx ctx, const void *H, ssl_prec hprec, const ssl_c64 *En, int F,
                              int D, int M, int Ns, int p, float *P, float *Pbar,
                              const int32_t *bin_status, void *stream);

/* --------------------------------------------------------------- peak search */

/* The Ns largest local maxima of Pbar on the n_el x n_az grid (flat index d = el*n_az + az):
 * d is a local maximum when Pbar[d] >= each of its 8 neighbours (azimuth circular, elevation
 * clamped) and an equal neighbour has a higher index; maxima are ranked by value, then by lower
 * index.  peaks: [Ns] int32 (-1 where fewer maxima exist), peak_val: [Ns] float (0 there).
 * Non-finite Pbar entries are never peaks and never block one. */
ssl_status ssl_peaks(ssl_ctx ctx, const float *Pbar, int n_az, int n_el, int Ns, int32_t *peaks,
                     float *peak_val, void *stream);

/* ------------------------------------------- transfer-function tables (eq.5) */

/* Shape of a transfer-function table file: M channels, F bins of an nfft-point STFT at fs, a
 * regular n_el x n_az direction grid (azimuth az0 + k az_step, elevation el0 + l el_step degrees,
 * flat index d = l n_az + k) -- the layout of H in ssl_music_spectrum. */
typedef struct {
    int M, F, n_az, n_el, nfft;
    float fs, az0_deg, az_step_deg, el0_deg, el_step_deg;
} ssl_tf_info;

/* File layout (little-endian): 8-byte magic "SSLTF\0\0\1"; uint32 M, F, n_az, n_el, nfft; float32
 * fs, az0_deg, az_step_deg, el0_deg, el_step_deg; 16 zero bytes (64-byte header); float64
 * pos[M][3] (microphone positions, m); complex64 H[F][D][M].  Host only (no GPU work):
 * ssl_tf_write stores a table held in host memory; ssl_tf_info_read reads the header and, if pos
 * (host, [M][3]) is not NULL, the positions.  SSL_ERR_ARG for unreadable, malformed or truncated
 * files. */
ssl_status ssl_tf_write(const char *path, const ssl_tf_info *info, const double *pos,
                        const ssl_c64 *H);
ssl_status ssl_tf_info_read(const char *path, ssl_tf_info *info, double *pos);

/* Loads the table of a file into device memory H in the steering-table layout of `prec`:
 * SSL_FP32 -> [F][D][M] complex64; SSL_BF16 / SSL_FP16 -> [F][D][2M] interleaved (re, im) 16-bit
 * pairs, rounded to nearest even.  The file is streamed through pinned host memory in slabs of
 * whole bins (at most 16 MB each, allocated for the call) and converted on the device.  The call
 * synchronises `stream` and returns when H is complete. */
ssl_status ssl_tf_load(ssl_ctx ctx, const char *path, ssl_prec prec, void *H, void *stream);

/* Converts a complex64 steering table H [F][D][M] (device) into the 16-bit layout Hout
 * [F][D][2M] (device) of prec = SSL_BF16 or SSL_FP16, rounding to nearest even. */
ssl_status ssl_steering_convert(ssl_ctx ctx, const ssl_c64 *H, int F, int D, int M, ssl_prec prec,
                                void *Hout, void *stream);

/* ----------------------------------------------------------- whole path */

/* One block end to end: R = (1/T) sum X X^H (eq.2-3), A = K^{-1} R and E_n (eq.4), P (eq.5),
 * Pbar (eq.6), peaks.  X as in ssl_corr_accum; H as in ssl_music_spectrum with D = n_az*n_el;
 * prec selects the MFMA input type of the correlation and the storage type of H (SSL_FP32,
 * SSL_BF16 or SSL_FP16; H must be stored in that type); the projection is eq.5's signal-subspace
 * form in FP64 where it applies (see ssl_ctx_set_projection), else the noise-vector form on MFMA
 * at that type.  Pbar ([D]) and bin_status ([F]) may be NULL.
 * K NULL selects SEVD-MUSIC (E_n from R itself, as in ssl_gsvd).
 * Uses the context's workspace (allocated on first use within the HBM budget). */
ssl_status ssl_localize(ssl_ctx ctx, const ssl_c64 *X, int F, int T, int M, int64_t strideF,
                        int64_t strideT, ssl_noise K, const void *H, ssl_prec prec, int n_az,
                        int n_el, int Ns, int p, int32_t *peaks, float *peak_val, float *Pbar,
                        int32_t *bin_status, void *stream);

/* For callers that cannot allocate device memory -- code under HIP graph capture, allocation-free
 * serving loops, harnesses that forbid hipMalloc: ssl_localize with the same arguments, results
 * and errors, that allocates nothing.  Its workspace is a fixed scratch array of
 * SSL_NOALLOC_SCRATCH_BYTES in device memory, one per device, held until the process ends (its
 * address on a device is looked up once, by ssl_ctx_create on that device).  Needs
 * ssl_localize_noalloc_bytes(F, M, Ns, n_az * n_el) <= SSL_NOALLOC_SCRATCH_BYTES, otherwise
 * returns SSL_ERR_ARG and enqueues nothing (the 60-channel, 257-bin, 1368-direction block needs
 * about 24 MB).  Never times its launches (ssl_ctx_timing does not apply), never creates events.
 * Every call on one device shares that device's scratch, and nothing it reads starts from a
 * previous call's contents: calls on one device must be ordered (one stream, or events between
 * them); calls that overlap in time on one device race and give wrong results. */
#define SSL_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
ssl_status ssl_localize_noalloc(ssl_ctx ctx, const ssl_c64 *X, int F, int T, int M,
                                int64_t strideF, int64_t strideT, ssl_noise K, const void *H,
                                ssl_prec prec, int n_az, int n_el, int Ns, int p, int32_t *peaks,
                                float *peak_val, float *Pbar, int32_t *bin_status, void *stream);
/* Scratch bytes ssl_localize_noalloc needs for one block of this shape (0 for invalid shapes). */
size_t ssl_localize_noalloc_bytes(int F, int M, int Ns, int D);

/* ------------------------------------------------- frame stream (eq.3 window) */

/* Localization at frame rate, eq.3 as printed: R(w, f) = (1/T) sum_{i=-T+1}^{0} x(w, f+i)
 * x(w, f+i)^H over the T frames ending at the latest frame f, maintained as frames arrive (the
 * stream processing the paper leaves to future work, Sec. VI).  The state keeps the last T frames
 * of every bin, their outer-product sum S in FP64 (each pushed frame x adds x x^H and removes the
 * o o^H of the frame o it displaces, a rank-2 update; S is recomputed exactly from the stored
 * frames each time T more frames have passed) and the singular vectors of the last solve.
 * create: F <= 65535 bins, 1 <= M <= 64 channels, 1 <= T <= 65535; allocates 8FTM + 24FM^2 bytes
 * from ctx (within its HBM budget).  destroy synchronises the device. */
ssl_status ssl_sliding_create(ssl_ctx ctx, int F, int M, int T, ssl_sliding *out);
void ssl_sliding_destroy(ssl_sliding s);
/* Appends n frames X [F][n][M] (complex64, device; element strides strideF, strideT, M
 * contiguous), oldest first. */
ssl_status ssl_sliding_push(ssl_sliding s, const ssl_c64 *X, int n, int64_t strideF,
                            int64_t strideT, void *stream);
/* Frames pushed so far (-1 for NULL). */
int64_t ssl_sliding_frames(ssl_sliding s);
/* The current window's R = S / T, [F][M][M] complex128 (device). */
ssl_status ssl_sliding_corr(ssl_sliding s, ssl_c128 *R, void *stream);
/* The whole method on the current window (as ssl_localize from R on; R rounded to complex64 from
 * the FP64 window sum; prec selects the projection's input type; K NULL: SEVD-MUSIC).
 * warm = 0: the cold solve of ssl_gsvd.  warm != 0 and a previous solve on this state: a
 * warm-started Jacobi -- Y = A^H U0 with U0 the previous window's sorted left singular vectors,
 * one-sided Jacobi on Y accumulating its rotations into U0 -- which needs a few sweeps when the
 * window moved by a few frames and the spectrum is well separated (same rotation rule and
 * tolerance as the cold solve; the result matches the cold solve's to within the parity bounds,
 * not bit for bit).  A warm solve is used only within T frames of the last cold solve, which
 * re-anchors the singular vectors (rounding in U = U0 V accumulates over warm solves).  Either
 * way the sorted singular vectors are kept for the next call.  Needs at least T pushed frames
 * (SSL_ERR_STATE).
 * conv: [F][3] int32 or NULL (sweeps, rotations, rank as in ssl_gsvd; M for a warm solve).
 * Uses the context's workspace; calls on one ctx must be ordered on one stream. */
ssl_status ssl_sliding_localize(ssl_sliding s, ssl_noise K, const void *H, ssl_prec prec,
                                int n_az, int n_el, int Ns, int p, int warm, int32_t *peaks,
                                float *peak_val, float *Pbar, int32_t *bin_status, int32_t *conv,
                                void *stream);

/* ------------------------------------------------------------ batched path */

/* One block of a batch.  Fields as in ssl_localize; blocks may differ in F, T, M, Ns and grid. */
typedef struct {
    const ssl_c64 *X;          /* [F][T][M], M contiguous, strides in elements */
    int64_t strideF, strideT;
    int F, T, M, Ns;
    ssl_noise K;               /* noise handle set for this F and M, or NULL: SEVD-MUSIC */
    const void *H;             /* [F][D][M] steering table in the batch's prec, D = n_az*n_el */
    int n_az, n_el;
    int32_t *peaks;            /* [Ns] out */
    float *peak_val;           /* [Ns] out */
    float *Pbar;               /* [D] out or NULL */
    int32_t *bin_status;       /* [F] out or NULL */
    int32_t *conv;             /* [F][3] out or NULL: per bin the Jacobi solve's sweeps,
                                  rotations and numerical rank (as ssl_gsvd's conv) */
} ssl_block_desc;

/* Whole path (as ssl_localize) for nblocks blocks of possibly different shapes, in one set of
 * launches: every kernel runs once per size class over all (block, bin) items of the batch, the
 * Jacobi SVD as a persistent work-queue kernel (bins that converge early free their CU).  descs is
 * a HOST array, read during the call only.  The launch sequence of a batch shape is captured once
 * into a HIP graph and replayed for later batches of the same shape (descriptors are copied to the
 * device each call, so pointers may change freely).  Results are bit-identical to ssl_localize
 * on each block alone.  All blocks share prec and p.  Limits: 1 <= nblocks <= 65535. */
ssl_status ssl_localize_batch(ssl_ctx ctx, const ssl_block_desc *descs, int nblocks,
                              ssl_prec prec, int p, void *stream);

/* SVD backend of every entry point of the context (ssl_gsvd, ssl_localize, ssl_localize_noalloc,
 * ssl_localize_batch, cold solves of ssl_sliding_localize):
 *   SSL_SVD_JACOBI (default)  one-sided Jacobi preconditioned by two Householder QRs (the paper's
 *                             Sec. III-B category 1), FP32;
 *   SSL_SVD_BIDIAG_QR         the paper's own method (Sec. III-B category 2, its steps SVD1..SVD6):
 *                             Householder bidiagonalisation, phase transform to a real
 *                             non-negative bidiagonal, tolerance M 2^-24 max_k (|d_k| + |e_k|),
 *                             implicit-shift QR iterations (Golub-Kahan steps, Wilkinson shift) on
 *                             it with the left rotations accumulated, sort, back-transformation;
 *                             FP32, at most 40 M QR steps (SSL_BIN_NO_CONV beyond), ssl_gsvd's
 *                             max_sweeps is not used and conv reports (QR steps, zero-diagonal
 *                             chases, M).  No warm start in ssl_sliding_localize.
 * The two agree to within the parity bounds (rounding differs), so results are bit-identical
 * between entry points for one backend only.  Changing it drops captured batch graphs' reuse. */
typedef enum { SSL_SVD_JACOBI = 0, SSL_SVD_BIDIAG_QR = 1 } ssl_svd;

/* Subspace method of every entry point of the context for calls that pass a noise handle (a NULL
 * handle is SEVD-MUSIC whatever this setting):
 *   SSL_SUBSPACE_GSVD (default)  eq.4: left singular vectors of K^{-1} R;
 *   SSL_SUBSPACE_GEVD            GEVD-MUSIC, the generalized-eigenvalue alternative the paper
 *                                names (Sec. II): the noise vectors are the generalized
 *                                eigenvectors R e = lambda K e of the M - Ns smallest lambda,
 *                                computed as e = K^{-1/2} y from the eigenvectors y of
 *                                C = K^{-1/2} R K^{-1/2} (FP64 products, C rounded to complex64
 *                                for the context's SVD backend, e mapped back in FP64); they are
 *                                K-orthonormal.  Every noise handle used must have had
 *                                ssl_noise_enable_gevd called (SSL_ERR_STATE otherwise). */
typedef enum { SSL_SUBSPACE_GSVD = 0, SSL_SUBSPACE_GEVD = 1 } ssl_subspace;
ssl_status ssl_ctx_set_subspace(ssl_ctx ctx, ssl_subspace method);
int ssl_ctx_get_subspace(ssl_ctx ctx);
ssl_status ssl_ctx_set_svd(ssl_ctx ctx, ssl_svd method);
int ssl_ctx_get_svd(ssl_ctx ctx);

/* Where the Jacobi solve may stop once the noise subspace has converged, rather than the full
 * SVD.  eq.5 with p = 2 reads only the projector E_n E_n^H, which the subspace determines, not
 * the noise singular vectors themselves.  From the start of the sweeps (the pivoted QR already
 * grades the column norms) the solve keeps the Ns columns of largest norm as the signal set S
 * and rotates only the pairs with a member in S, keeping the larger result in S, until such a
 * sweep changes nothing (X_S orthogonal to the rest to the rotation tolerance).  It then stops
 * if min over S of |x|^2 exceeds the sum of |x|^2 over the other columns, a bound on the rest's
 * largest squared singular value, so that X_S spans the Ns dominant singular vectors.  E_n is
 * then an orthonormal basis of the complement of X_S (Householder vectors), not the singular
 * vectors.  A failed check, 6 such sweeps without convergence, or a weakest signal column holding
 * less than the other columns' energy at the switch keep the full solve.  Only for the Jacobi
 * backend, 1 <= Ns <= 3 and a numerical rank of at least 3 Ns.  On the 60-channel workload the
 * stopped solve takes 2.4 sweeps over the signal pairs per bin on average, against 6.1 full
 * sweeps (3.2 for the signal-subspace form of eq.5, whose sweeps run without the second QR).
 *   SSL_STOP_NEVER       always the full SVD;
 *   SSL_STOP_BATCH       ssl_localize_batch with p = 2;
 *   SSL_STOP_LOCALIZE    (default) also ssl_localize and ssl_localize_noalloc with p = 2;
 *   SSL_STOP_ALSO_GSVD   also ssl_gsvd calls that pass sigma = NULL (their E_n is then a basis of
 *                        the noise subspace).
 * ssl_sliding_localize keeps the full solve (its singular vectors seed warm starts).  Results
 * agree with the full solve's within the parity bounds (rounding differs); batched and one-block
 * results are bit-identical when both run the same solve (every mode but SSL_STOP_BATCH).
 * Changing the mode drops captured batch graphs' reuse. */
typedef enum {
    SSL_STOP_NEVER = 0,
    SSL_STOP_BATCH = 1,
    SSL_STOP_LOCALIZE = 2,
    SSL_STOP_ALSO_GSVD = 3
} ssl_stop;
ssl_status ssl_ctx_set_stop(ssl_ctx ctx, ssl_stop mode);
int ssl_ctx_get_stop(ssl_ctx ctx);

/* Form of eq.5 (p = 2).  With U = [E_s E_n] unitary, the sum over the noise vectors of |h^H e|^2
 * equals |h|^2 - |E_s^H h|^2, which needs the Ns signal vectors instead of the M - Ns noise
 * vectors.  That difference cancels near the peaks, so it is evaluated in FP64 from FP64
 * products of the stored vectors and of the table's values (complex64, or bf16 / fp16 pairs
 * widened exactly; FP64 matrix cores), with the exact projector E_s (E_s^H E_s)^{-1} E_s^H onto
 * their span (the Jacobi solve returns the inverse Cholesky factor of their FP64 Gram matrix):
 * den = |h|^2 - |L^{-1} E_s^H h|^2, P = |h|^2 / max(den, FLT_MIN).  The Jacobi solve then forms
 * only the signal vectors.
 *   SSL_PROJ_SIGNAL   (default) this form wherever it applies: p = 2, the Jacobi backend, GSVD or
 *                     SEVD (not GEVD, whose noise vectors are not orthonormal), 1 <= Ns <= 3, any
 *                     table precision, in ssl_localize, ssl_localize_noalloc and
 *                     ssl_localize_batch (per block: a batch may mix blocks of both forms);
 *   SSL_PROJ_NOISE    always the noise-vector projection H^H E_n (MFMA at the table's
 *                     precision), as ssl_music_spectrum computes it.
 * p = 1, ssl_sliding_localize and ssl_music_spectrum always use the noise-vector projection.  The
 * two forms agree within the parity bounds (rounding differs). */
typedef enum { SSL_PROJ_NOISE = 0, SSL_PROJ_SIGNAL = 1 } ssl_projection;
ssl_status ssl_ctx_set_projection(ssl_ctx ctx, ssl_projection mode);
int ssl_ctx_get_projection(ssl_ctx ctx);

/* Graph replay for ssl_localize_batch (default on).  With timing enabled (ssl_ctx_timing) batches
 * always run as individually timed launches. */
ssl_status ssl_ctx_use_graphs(ssl_ctx ctx, int enable);

/* ------------------------------------------------------------------ tuning */

/* Jacobi SVD kernel variant per channel-count class (M <= 8, <= 16, <= 32, <= 64): the number of
 * lanes that cooperate on one column pair.  Available: 4 or 8 (M <= 8); 4, 8 or 16 (M <= 16);
 * 8 or 16 (M <= 32); 4, 8 or 16 (M <= 64).  Default 8 in every class.  A context applies its
 * current choice to every entry point, so batched and single-block results remain
 * bit-identical; variants differ from each other only by rounding.  Returns SSL_ERR_ARG for an
 * unavailable variant. */
ssl_status ssl_ctx_set_jacobi_lanes(ssl_ctx ctx, int M, int lanes);
int ssl_ctx_get_jacobi_lanes(ssl_ctx ctx, int M);

/* Autotuner: times every available Jacobi variant of M's class on the caller's problems -- the
 * whitened products K^{-1} R[f] of F bins -- `reps` launches each (after one untimed launch),
 * with HIP events on `stream`, keeps the fastest in the context and returns it in *best_lanes.
 * nblocks = 1 times the one-launch-per-block kernel of ssl_gsvd / ssl_localize; nblocks > 1 (up
 * to 65535) times the persistent kernel of ssl_localize_batch over nblocks copies of the F
 * bins, whose best variant can differ (occupancy against load balance).  ms_per_variant ([3],
 * host, or NULL) receives the mean milliseconds per launch for lanes = 4, 8, 16 (-1 where
 * unavailable).  R: [F][M][M] device, K set for F and M.  Uses context workspace (nblocks * F
 * bins of A and E_n).  The solve is timed as the p = 2 localization runs it (stopped at the noise
 * subspace unless the context's ssl_stop is SSL_STOP_NEVER).  Synchronous. */
ssl_status ssl_autotune_jacobi(ssl_ctx ctx, const ssl_c64 *R, ssl_noise K, int F, int M, int Ns,
                               int nblocks, int reps, int *best_lanes, double *ms_per_variant,
                               void *stream);

/* Steering-projection (eq.5) tile shape per noise-subspace class (M - Ns <= 16, <= 32, <= 64) and
 * steering-table precision (SSL_FP32, SSL_BF16, SSL_FP16): the number of 64-lane waves per
 * workgroup, each wave owning 16 directions of one bin.  Available: 4, 8 or 16.  Default 8.  Every
 * direction's value is computed by one wave in the same order whatever the tile, so the choice
 * changes speed only: P and Pbar are bit-identical across variants.  Applied by every entry
 * point of the context.  Returns SSL_ERR_ARG for an unavailable variant (get returns -1). */
ssl_status ssl_ctx_set_steer_waves(ssl_ctx ctx, int M, int Ns, ssl_prec hprec, int waves);
int ssl_ctx_get_steer_waves(ssl_ctx ctx, int M, int Ns, ssl_prec hprec);

/* Autotuner for the projection tile: times the projection kernel for every available tile shape
 * on the caller's problem -- H [F][D][M] in hprec and En [F][M][M - Ns] (both device) -- `reps`
 * launches each (after one untimed launch) with HIP events on `stream`, keeps the fastest in the
 * context and returns it in *best_waves.  nblocks = 1 times the single-block kernel of
 * ssl_music_spectrum / ssl_localize; nblocks > 1 (up to 65535) times the batched kernel of
 * ssl_localize_batch as it runs when nblocks blocks share the steering table (En repeated), the
 * case whose best tile differs because H is read once for all of them.  ms_per_variant ([3],
 * host, or NULL) receives the mean milliseconds per launch for 4, 8, 16 waves.  Uses context
 * workspace (nblocks * F * D floats for P, plus descriptors).  Synchronous. */
ssl_status ssl_autotune_steer(ssl_ctx ctx, const void *H, ssl_prec hprec, const ssl_c64 *En,
                              int F, int D, int M, int Ns, int p, int nblocks, int reps,
                              int *best_waves, double *ms_per_variant, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SSL_MI355X_H */
