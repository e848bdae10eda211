// Transfer-function tables H(theta, w) of eq.5 -- in the paper measured for its 60-channel array
// (Sec. V-C) -- from files, and the conversion of a complex64 table to the interleaved 16-bit
// layout of the mixed-precision projection.
//
// File layout (little-endian), written by ssl_tf_write and read by ssl_tf_info_read / ssl_tf_load:
//   bytes  0..7    magic "SSLTF\0\0\1"
//   bytes  8..47   uint32 M, F, n_az, n_el, nfft; float32 fs, az0_deg, az_step_deg, el0_deg,
//                  el_step_deg
//   bytes 48..63   zero
//   then           float64 pos[M][3] (microphone positions, metres)
//   then           complex64 H[F][D][M], D = n_az n_el, direction d = el * n_az + az
// The table is streamed through a pinned staging buffer in slabs of whole bins and converted on
// the device slab by slab, so a load needs no host copy of the whole table.
#include <stdio.h>
#include <string.h>

#include <algorithm>

#include "ssl_internal.h"

namespace {

const char kMagic[8] = {'S', 'S', 'L', 'T', 'F', 0, 0, 1};

// c64 [n][M] -> interleaved (re, im) 16-bit pairs [n][2M], rounding to nearest even
template <typename E>
__global__ __launch_bounds__(256) void convert_pairs(const float2 *__restrict__ H, int64_t n,
                                                     E *__restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const float2 h = H[i];
        out[2 * i] = (E)h.x;
        out[2 * i + 1] = (E)h.y;
    }
}

hipError_t launch_convert(const ssl_c64 *H, int64_t n, ssl_prec prec, void *out, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks64 = (n + 255) / 256;
    const unsigned grid = (unsigned)(blocks64 < 65536 ? blocks64 : 65536);
    const float2 *h = reinterpret_cast<const float2 *>(H);
    if (prec == SSL_BF16)
        hipLaunchKernelGGL((convert_pairs<__bf16>), dim3(grid), dim3(256), 0, st, h, n,
                           static_cast<__bf16 *>(out));
    else
        hipLaunchKernelGGL((convert_pairs<_Float16>), dim3(grid), dim3(256), 0, st, h, n,
                           static_cast<_Float16 *>(out));
    return hipGetLastError();
}

struct FileCloser {
    FILE *f;
    ~FileCloser()
    {
        if (f) fclose(f);
    }
};

ssl_status read_header(FILE *f, const char *path, ssl_tf_info *info)
{
    unsigned char hdr[64];
    if (fread(hdr, 1, sizeof(hdr), f) != sizeof(hdr)) {
        ssl_set_error("%s: shorter than a table header", path);
        return SSL_ERR_ARG;
    }
    if (memcmp(hdr, kMagic, sizeof(kMagic)) != 0) {
        ssl_set_error("%s: not a transfer-function table (bad magic)", path);
        return SSL_ERR_ARG;
    }
    uint32_t u[5];
    float v[5];
    memcpy(u, hdr + 8, sizeof(u));
    memcpy(v, hdr + 28, sizeof(v));
    info->M = (int)u[0];
    info->F = (int)u[1];
    info->n_az = (int)u[2];
    info->n_el = (int)u[3];
    info->nfft = (int)u[4];
    info->fs = v[0];
    info->az0_deg = v[1];
    info->az_step_deg = v[2];
    info->el0_deg = v[3];
    info->el_step_deg = v[4];
    if (u[0] < 1 || u[0] > SSL_MAX_M || u[1] < 1 || u[1] > 65535 || u[2] < 1 || u[3] < 1 ||
        (uint64_t)u[2] * u[3] > (1u << 24)) {
        ssl_set_error("%s: table shape M = %u, F = %u, n_az = %u, n_el = %u out of range", path,
                      u[0], u[1], u[2], u[3]);
        return SSL_ERR_ARG;
    }
    return SSL_OK;
}

}  // namespace

extern "C" {

ssl_status ssl_tf_info_read(const char *path, ssl_tf_info *info, double *pos)
{
    if (!path || !info) {
        ssl_set_error("path or info is NULL");
        return SSL_ERR_ARG;
    }
    FileCloser fc{fopen(path, "rb")};
    if (!fc.f) {
        ssl_set_error("%s: cannot open", path);
        return SSL_ERR_ARG;
    }
    ssl_status s = read_header(fc.f, path, info);
    if (s != SSL_OK) return s;
    if (pos && fread(pos, sizeof(double), 3 * (size_t)info->M, fc.f) != 3 * (size_t)info->M) {
        ssl_set_error("%s: truncated microphone positions", path);
        return SSL_ERR_ARG;
    }
    return SSL_OK;
}

ssl_status ssl_tf_write(const char *path, const ssl_tf_info *info, const double *pos,
                        const ssl_c64 *H)
{
    if (!path || !info || !pos || !H) {
        ssl_set_error("path, info, pos or H is NULL");
        return SSL_ERR_ARG;
    }
    if (info->M < 1 || info->M > SSL_MAX_M || info->F < 1 || info->F > 65535 || info->n_az < 1 ||
        info->n_el < 1 || (int64_t)info->n_az * info->n_el > (1 << 24)) {
        ssl_set_error("table shape out of range");
        return SSL_ERR_ARG;
    }
    unsigned char hdr[64] = {};
    memcpy(hdr, kMagic, sizeof(kMagic));
    const uint32_t u[5] = {(uint32_t)info->M, (uint32_t)info->F, (uint32_t)info->n_az,
                           (uint32_t)info->n_el, (uint32_t)info->nfft};
    const float v[5] = {info->fs, info->az0_deg, info->az_step_deg, info->el0_deg,
                        info->el_step_deg};
    memcpy(hdr + 8, u, sizeof(u));
    memcpy(hdr + 28, v, sizeof(v));
    FileCloser fc{fopen(path, "wb")};
    if (!fc.f) {
        ssl_set_error("%s: cannot create", path);
        return SSL_ERR_ARG;
    }
    const size_t nH = (size_t)info->F * info->n_az * info->n_el * info->M;
    if (fwrite(hdr, 1, sizeof(hdr), fc.f) != sizeof(hdr) ||
        fwrite(pos, sizeof(double), 3 * (size_t)info->M, fc.f) != 3 * (size_t)info->M ||
        fwrite(H, sizeof(ssl_c64), nH, fc.f) != nH) {
        ssl_set_error("%s: write failed", path);
        return SSL_ERR_ARG;
    }
    if (fclose(fc.f) != 0) {
        fc.f = nullptr;
        ssl_set_error("%s: write failed", path);
        return SSL_ERR_ARG;
    }
    fc.f = nullptr;
    return SSL_OK;
}

ssl_status ssl_steering_convert(ssl_ctx ctx, const ssl_c64 *H, int F, int D, int M, ssl_prec prec,
                                void *Hout, void *stream)
{
    if (!ctx || !H || !Hout) {
        ssl_set_error("ctx, H or Hout is NULL");
        return SSL_ERR_ARG;
    }
    if (prec != SSL_BF16 && prec != SSL_FP16) {
        ssl_set_error("prec must be SSL_BF16 or SSL_FP16");
        return SSL_ERR_ARG;
    }
    if (F < 1 || D < 1 || M < 1 || M > SSL_MAX_M || D > (1 << 24) || F > 65535) {
        ssl_set_error("F = %d, D = %d, M = %d out of range", F, D, M);
        return SSL_ERR_ARG;
    }
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != ctx->device) (void)hipSetDevice(ctx->device);
    const hipError_t e = launch_convert(H, (int64_t)F * D * M, prec, Hout,
                                        static_cast<hipStream_t>(stream));
    if (prev >= 0 && prev != ctx->device) (void)hipSetDevice(prev);
    if (e != hipSuccess) {
        ssl_set_error("conversion launch: %s", hipGetErrorString(e));
        return SSL_ERR_HIP;
    }
    return SSL_OK;
}

ssl_status ssl_tf_load(ssl_ctx ctx, const char *path, ssl_prec prec, void *H, void *stream)
{
    if (!ctx || !path || !H) {
        ssl_set_error("ctx, path or H is NULL");
        return SSL_ERR_ARG;
    }
    if (prec != SSL_FP32 && prec != SSL_BF16 && prec != SSL_FP16) {
        ssl_set_error("prec must be SSL_FP32, SSL_BF16 or SSL_FP16");
        return SSL_ERR_ARG;
    }
    FileCloser fc{fopen(path, "rb")};
    if (!fc.f) {
        ssl_set_error("%s: cannot open", path);
        return SSL_ERR_ARG;
    }
    ssl_tf_info info;
    ssl_status s = read_header(fc.f, path, &info);
    if (s != SSL_OK) return s;
    if (fseek(fc.f, (long)(64 + 24 * (size_t)info.M), SEEK_SET) != 0) {
        ssl_set_error("%s: truncated", path);
        return SSL_ERR_ARG;
    }
    const size_t per_bin = (size_t)info.n_az * info.n_el * info.M;    // complex64 per bin
    const size_t slab_bins = std::max<size_t>(1, ((size_t)16 << 20) / (per_bin * sizeof(ssl_c64)));
    const size_t slab = slab_bins * per_bin;
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != ctx->device) (void)hipSetDevice(ctx->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    ssl_c64 *host = nullptr, *dev = nullptr;
    hipError_t e = hipHostMalloc((void **)&host, slab * sizeof(ssl_c64), hipHostMallocDefault);
    if (e == hipSuccess && prec != SSL_FP32) e = hipMalloc((void **)&dev, slab * sizeof(ssl_c64));
    for (size_t f0 = 0; e == hipSuccess && s == SSL_OK && f0 < (size_t)info.F; f0 += slab_bins) {
        const size_t nb = std::min(slab_bins, (size_t)info.F - f0), n = nb * per_bin;
        e = hipStreamSynchronize(st);                   // the previous slab has left the buffer
        if (e != hipSuccess) break;
        if (fread(host, sizeof(ssl_c64), n, fc.f) != n) {
            ssl_set_error("%s: truncated table (bin %zu)", path, f0);
            s = SSL_ERR_ARG;
            break;
        }
        if (prec == SSL_FP32) {
            e = hipMemcpyAsync(static_cast<ssl_c64 *>(H) + f0 * per_bin, host,
                               n * sizeof(ssl_c64), hipMemcpyHostToDevice, st);
        } else {
            e = hipMemcpyAsync(dev, host, n * sizeof(ssl_c64), hipMemcpyHostToDevice, st);
            if (e == hipSuccess)
                e = launch_convert(dev, (int64_t)n, prec,
                                   static_cast<char *>(H) + f0 * per_bin * 2 * sizeof(uint16_t), st);
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (dev) (void)hipFree(dev);
    if (host) (void)hipHostFree(host);
    if (prev >= 0 && prev != ctx->device) (void)hipSetDevice(prev);
    if (s != SSL_OK) return s;
    if (e != hipSuccess) {
        ssl_set_error("%s: upload failed: %s", path, hipGetErrorString(e));
        return SSL_ERR_HIP;
    }
    return SSL_OK;
}

}  // extern "C"
