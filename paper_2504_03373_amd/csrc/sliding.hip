// Frame-by-frame correlation of eq.3 as printed: R(w, f) = (1/T) sum_{i = -T+1}^{0} x(w, f + i)
// x(w, f + i)^H, the window of the T frames ending at frame f, kept up to date as frames arrive:
// each new frame x enters and the frame o it displaces from the window leaves,
//   S <- S + x x^H - o o^H,          R(w, f) = S / T,
// a rank-2 update per frame instead of the T outer products of a fresh sum.  S is FP64 (the
// running sum is exact to FP64 rounding; the host schedules an exact recomputation from the ring
// of the last T frames each time T more frames have passed, so rounding does not accumulate).
//
// GPU mapping: one workgroup per bin; each thread owns up to kMaxOwn entries (i, j) of S in FP64
// registers for the whole call; frame by frame, the new and the displaced frame of the bin are
// staged in LDS (one barrier), every thread updates its entries, then the new frame replaces the
// displaced one in the ring.
#include "ssl_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kMaxOwn = (SSL_MAX_M * SSL_MAX_M + kThreads - 1) / kThreads;   // 16

__global__ __launch_bounds__(kThreads) void sliding_push(const float2 *__restrict__ X, int n,
                                                         int64_t sF, int64_t sT, int M, int T,
                                                         int64_t pushed, float2 *__restrict__ ring,
                                                         double2 *__restrict__ S)
{
    __shared__ float2 xn[SSL_MAX_M], xo[SSL_MAX_M];
    const int f = blockIdx.x, tid = threadIdx.x;
    const int MM = M * M;
    double2 *Sf = S + (size_t)f * MM;
    float2 *ring_f = ring + (size_t)f * T * M;
    double2 acc[kMaxOwn];
#pragma unroll
    for (int k = 0; k < kMaxOwn; ++k) {
        const int e = tid + k * kThreads;
        acc[k] = e < MM ? Sf[e] : make_double2(0.0, 0.0);
    }
    for (int j = 0; j < n; ++j) {
        const int64_t frame = pushed + j;
        const int slot = (int)(frame % T);
        if (tid < M) {
            xn[tid] = X[(size_t)f * sF + (size_t)j * sT + tid];
            xo[tid] = frame >= T ? ring_f[(size_t)slot * M + tid] : make_float2(0.f, 0.f);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kMaxOwn; ++k) {
            const int e = tid + k * kThreads;
            if (e < MM) {
                const int a = e / M, b = e - a * M;
                // x_a conj(x_b) - o_a conj(o_b)
                const double xar = xn[a].x, xai = xn[a].y, xbr = xn[b].x, xbi = xn[b].y;
                const double oar = xo[a].x, oai = xo[a].y, obr = xo[b].x, obi = xo[b].y;
                acc[k].x += fma(xar, xbr, xai * xbi) - fma(oar, obr, oai * obi);
                acc[k].y += fma(xai, xbr, -xar * xbi) - fma(oai, obr, -oar * obi);
            }
        }
        __syncthreads();
        if (tid < M) ring_f[(size_t)slot * M + tid] = xn[tid];
    }
#pragma unroll
    for (int k = 0; k < kMaxOwn; ++k) {
        const int e = tid + k * kThreads;
        if (e < MM) Sf[e] = acc[k];
    }
}

// R = S / T, rounded to complex64 (the input of the whitening and of the SEVD path) or kept in
// FP64
template <typename Out>
__global__ __launch_bounds__(kThreads) void sliding_scale(const double2 *__restrict__ S,
                                                          int64_t n, double inv_t,
                                                          Out *__restrict__ R)
{
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
        const double2 v = S[i];
        R[i].x = v.x * inv_t;
        R[i].y = v.y * inv_t;
    }
}

}  // namespace

hipError_t launch_sliding_push(const ssl_c64 *X, int n, int64_t sF, int64_t sT, int F, int M,
                               int T, int64_t pushed, ssl_c64 *ring, ssl_c128 *S, hipStream_t st)
{
    hipLaunchKernelGGL(sliding_push, dim3(F), dim3(kThreads), 0, st,
                       reinterpret_cast<const float2 *>(X), n, sF, sT, M, T, pushed,
                       reinterpret_cast<float2 *>(ring), reinterpret_cast<double2 *>(S));
    return hipGetLastError();
}

hipError_t launch_sliding_scale(const ssl_c128 *S, int64_t n, double inv_t, void *R, bool fp64,
                                hipStream_t st)
{
    const int64_t blocks = (n + kThreads - 1) / kThreads;
    const dim3 grid((unsigned)(blocks < 65536 ? blocks : 65536));
    const double2 *s = reinterpret_cast<const double2 *>(S);
    if (fp64)
        hipLaunchKernelGGL((sliding_scale<double2>), grid, dim3(kThreads), 0, st, s, n, inv_t,
                           static_cast<double2 *>(R));
    else
        hipLaunchKernelGGL((sliding_scale<float2>), grid, dim3(kThreads), 0, st, s, n, inv_t,
                           static_cast<float2 *>(R));
    return hipGetLastError();
}
