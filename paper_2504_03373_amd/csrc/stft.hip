// Front end of the method (eq.1): the short-time Fourier transform of every channel,
//   X_m(w, t) = sum_{n < N} win[n] x_m[t hop + n] e^{-2 pi i w n / N},   w = 0 .. N/2,
// written as X [N/2 + 1][T][M] complex64, the layout the correlation reads (channels contiguous).
//
// GPU mapping (gfx950): the transform is HBM-bound (about 10 flops per input byte at N = 512), so
// it is a radix-2 FFT in LDS, not a DFT-as-GEMM.  One workgroup per (frame, group of CH channels):
// the windowed frame is loaded channel-interleaved -- for each sample, CH consecutive channels are
// one contiguous read of the [n_samples][M] PCM -- into bit-reversed positions of an [N][CH]
// complex LDS array; log2 N butterfly stages follow, each thread taking butterflies of all CH
// channels in turn (consecutive threads: consecutive channels of one butterfly, so one twiddle
// sin/cos per CH lanes and conflict-free LDS rows); the N/2 + 1 bins leave as rows of CH
// consecutive channels.  Twiddles come from sincospif of an exact dyadic fraction.
#include "ssl_internal.h"

namespace {

constexpr int kThreads = 256;

// channels per workgroup: the [N][CH] complex frame fills at most 64 KB of LDS
constexpr int stft_ch(int logn) { return (1 << logn) >= 8192 ? 1 : (8192 >> logn) < 16 ? (8192 >> logn) : 16; }

template <int LOGN>
__global__ __launch_bounds__(kThreads) void stft_frames(const float *__restrict__ pcm, int M,
                                                        int hop, const float *__restrict__ win,
                                                        int T, float2 *__restrict__ X)
{
    constexpr int N = 1 << LOGN;
    constexpr int CH = stft_ch(LOGN);
    constexpr int F = N / 2 + 1;
    __shared__ float2 buf[N * CH];
    const int t = blockIdx.x;
    const int c0 = blockIdx.y * CH;
    const int nc = min(CH, M - c0);
    const float *frame = pcm + (int64_t)t * hop * M + c0;
    for (int e = threadIdx.x; e < N * CH; e += kThreads) {
        const int n = e / CH, ch = e - n * CH;
        float v = 0.0f;
        if (ch < nc) {
            float w;
            if (win) {
                w = win[n];
            } else {                                // periodic Hann: sin^2(pi n / N)
                const float s = sinpif((float)n / (float)N);
                w = s * s;
            }
            v = w * frame[(int64_t)n * M + ch];
        }
        const int rn = (int)(__brev((unsigned int)n) >> (32 - LOGN));
        buf[rn * CH + ch] = make_float2(v, 0.0f);
    }
    __syncthreads();
#pragma unroll 1
    for (int s = 0; s < LOGN; ++s) {
        const int half = 1 << s;                    // butterflies span 2 half points
        for (int e = threadIdx.x; e < (N / 2) * CH; e += kThreads) {
            const int b = e / CH, ch = e - b * CH;
            const int j = b & (half - 1);
            const int i0 = ((b >> s) << (s + 1)) + j, i1 = i0 + half;
            float sn, cs;                           // e^{-i pi j / half}
            sincospif(-(float)j / (float)half, &sn, &cs);
            const float2 u = buf[i0 * CH + ch], v = buf[i1 * CH + ch];
            const float2 tv = make_float2(fmaf(v.x, cs, -v.y * sn), fmaf(v.x, sn, v.y * cs));
            buf[i0 * CH + ch] = make_float2(u.x + tv.x, u.y + tv.y);
            buf[i1 * CH + ch] = make_float2(u.x - tv.x, u.y - tv.y);
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < F * CH; e += kThreads) {
        const int w = e / CH, ch = e - w * CH;
        if (ch < nc) X[((int64_t)w * T + t) * M + c0 + ch] = buf[w * CH + ch];
    }
}

template <int LOGN>
hipError_t launch(const float *pcm, int M, int hop, const float *win, int T, ssl_c64 *X,
                  hipStream_t st)
{
    constexpr int CH = stft_ch(LOGN);
    hipLaunchKernelGGL((stft_frames<LOGN>), dim3(T, (M + CH - 1) / CH), dim3(kThreads), 0, st, pcm,
                       M, hop, win, T, reinterpret_cast<float2 *>(X));
    return hipGetLastError();
}

}  // namespace

hipError_t launch_stft(const float *pcm, int M, int nfft, int hop, const float *win, int T,
                       ssl_c64 *X, hipStream_t st)
{
    switch (nfft) {
    case 16: return launch<4>(pcm, M, hop, win, T, X, st);
    case 32: return launch<5>(pcm, M, hop, win, T, X, st);
    case 64: return launch<6>(pcm, M, hop, win, T, X, st);
    case 128: return launch<7>(pcm, M, hop, win, T, X, st);
    case 256: return launch<8>(pcm, M, hop, win, T, X, st);
    case 512: return launch<9>(pcm, M, hop, win, T, X, st);
    case 1024: return launch<10>(pcm, M, hop, win, T, X, st);
    case 2048: return launch<11>(pcm, M, hop, win, T, X, st);
    case 4096: return launch<12>(pcm, M, hop, win, T, X, st);
    default: return hipErrorInvalidValue;
    }
}
