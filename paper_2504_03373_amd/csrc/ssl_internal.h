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
    // bin-sum scratch: partials [chunks][D] + one completion counter, zeroed at allocation
    float *binsum_part;
    unsigned int *binsum_counter;
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
};

struct ssl_noise_s {
    ssl_ctx ctx;
    int F, M;
    bool is_set;
    ssl_c128 *K;       // [F][M][M] current noise correlation
    ssl_c128 *Kinv;    // [F][M][M] FP64 inverse from the Cholesky factor
    int32_t *status;   // [F] SSL_BIN_OK / SSL_BIN_NOT_PD
};

void ssl_set_error(const char *fmt, ...);

// --- launchers (each returns hipSuccess or the launch error) ---
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
// A is library workspace and is overwritten (it parks the QR reflectors between phases).
hipError_t launch_jacobi(ssl_c64 *A, const int32_t *kstatus, int F, int M, int Ns,
                         int max_sweeps, ssl_c64 *En, float *sigma, int32_t *bin_status,
                         int32_t *conv, hipStream_t st);
hipError_t launch_steer(const void *H, ssl_prec hprec, const ssl_c64 *En, int F, int D, int M,
                        int Ns, int p, const int32_t *bin_status, float *P, hipStream_t st);
hipError_t launch_binsum_peaks(const float *P, int F, int D, float *Pbar, float *part,
                               unsigned int *counter, int n_az, int n_el, int Ns, int32_t *peaks,
                               float *peak_val, hipStream_t st);
hipError_t launch_peaks(const float *Pbar, int n_az, int n_el, int Ns, int32_t *peaks,
                        float *peak_val, hipStream_t st);
