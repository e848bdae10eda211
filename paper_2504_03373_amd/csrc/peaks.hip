// Bin integration (eq.6 of arXiv 2504.03373) and peak search (Sec. III-A, last paragraph).
//
// Pbar[d] = sum_f P[f, d].  Deterministic, atomics-free order: bins are summed in ascending order
// inside fixed chunks of SSL_BINSUM_CHUNK bins (one thread per (direction, chunk), the whole chip
// busy), then a second launch (one workgroup per block) sums the chunk partials in ascending chunk
// order and searches the peaks.  The launch boundary makes the partials visible: no device-scope
// fence per workgroup (each is an L2 write-back on this multi-XCD part) and no completion counter.
//
// Peak rule on the n_el x n_az grid (d = el * n_az + az): d is a local maximum when it beats each
// of its 8 neighbours -- azimuth circular, elevation clamped -- where "beats" means a larger value,
// or an equal value and a lower flat index.  Maxima are ranked by the same relation; the first
// Ns are returned, -1 / 0 beyond the number found.  Non-finite values never take part.
#include "ssl_internal.h"

namespace {

constexpr int kThreads = 256;         // partial sums
constexpr int kFinal = 1024;          // final sum + peak search, one workgroup per block
constexpr int kLdsPbar = 8192;        // Pbar staged in LDS when D <= this

__device__ __forceinline__ bool beats(float va, int a, float vb, int b)
{
    return va > vb || (va == vb && a < b);
}

__device__ bool is_local_max(const float *pb, int n_el, int n_az, int d)
{
    const float v = pb[d];
    if (!isfinite(v)) return false;
    const int el = d / n_az, az = d - el * n_az;
    for (int de = -1; de <= 1; ++de) {
        const int e = el + de;
        if (e < 0 || e >= n_el) continue;
        for (int da = -1; da <= 1; ++da) {
            if (de == 0 && da == 0) continue;
            int a = az + da;
            a = (a < 0) ? a + n_az : (a >= n_az ? a - n_az : a);
            const int nb = e * n_az + a;
            if (nb == d) continue;
            const float w = pb[nb];
            if (!isfinite(w)) continue;
            if (!beats(v, d, w, nb)) return false;
        }
    }
    return true;
}

// Whole-workgroup peak search over pb[0..D) (LDS or global).  cand is an LDS flag array of
// size >= D when D <= kLdsPbar, otherwise candidates are re-tested on the fly.
__device__ void search_peaks(const float *pb, int D, int n_az, int n_el, int Ns,
                             int32_t *__restrict__ peaks, float *__restrict__ peak_val,
                             unsigned char *cand, float *red_v, int *red_i, int *chosen)
{
    const int tid = threadIdx.x;
    const bool use_cand = D <= kLdsPbar;
    if (use_cand) {
        for (int d = tid; d < D; d += kFinal) cand[d] = is_local_max(pb, n_el, n_az, d) ? 1 : 0;
    }
    __syncthreads();
    for (int k = 0; k < Ns; ++k) {
        // each thread: best remaining candidate among its directions
        float bv = 0.f;
        int bi = -1;
        for (int d = tid; d < D; d += kFinal) {
            bool c = use_cand ? (cand[d] != 0) : is_local_max(pb, n_el, n_az, d);
            if (!c) continue;
            bool taken = false;
            for (int j = 0; j < k; ++j) taken |= (chosen[j] == d);
            if (taken) continue;
            const float v = pb[d];
            if (bi < 0 || beats(v, d, bv, bi)) {
                bv = v;
                bi = d;
            }
        }
        red_v[tid] = bv;
        red_i[tid] = bi;
        __syncthreads();
        for (int s = kFinal / 2; s > 0; s >>= 1) {
            if (tid < s) {
                const int oi = red_i[tid + s];
                const float ov = red_v[tid + s];
                if (oi >= 0 && (red_i[tid] < 0 || beats(ov, oi, red_v[tid], red_i[tid]))) {
                    red_v[tid] = ov;
                    red_i[tid] = oi;
                }
            }
            __syncthreads();
        }
        if (tid == 0) {
            chosen[k] = red_i[0];
            peaks[k] = red_i[0];
            peak_val[k] = red_i[0] >= 0 ? red_v[0] : 0.0f;
        }
        __syncthreads();
    }
}

// Partial sums: thread (dc, ch, tid) sums bins ch*CHUNK .. +CHUNK-1 of direction dc*kThreads+tid.
__device__ __forceinline__ void binsum_part_body(const float *__restrict__ P, int F, int D,
                                                 float *__restrict__ part, int dc, int ch)
{
    const int d = dc * kThreads + (int)threadIdx.x;
    if (d >= D) return;
    // all loads of the chunk in flight at once, then the sum in ascending bin order
    // (absent bins of a short last chunk add an exact 0)
    const int f0 = ch * SSL_BINSUM_CHUNK;
    const int nf = min(F - f0, SSL_BINSUM_CHUNK);
    float v[SSL_BINSUM_CHUNK];
#pragma unroll
    for (int i = 0; i < SSL_BINSUM_CHUNK; ++i)
        v[i] = (i < nf) ? P[(size_t)(f0 + i) * D + d] : 0.0f;
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < SSL_BINSUM_CHUNK; ++i) s += v[i];
    part[(size_t)ch * D + d] = s;
}

// Final sum over the nch chunk partials (ascending) and the peak search (peaks may be null).
__device__ __forceinline__ void binsum_final_body(const float *__restrict__ part, int nch, int D,
                                                  float *__restrict__ Pbar, int n_az, int n_el,
                                                  int Ns, int32_t *__restrict__ peaks,
                                                  float *__restrict__ peak_val)
{
    __shared__ float pb_s[kLdsPbar];
    __shared__ unsigned char cand[kLdsPbar];
    __shared__ float red_v[kFinal];
    __shared__ int red_i[kFinal];
    __shared__ int chosen[SSL_MAX_M];
    const int tid = threadIdx.x;
    const bool lds = D <= kLdsPbar;
    for (int e = tid; e < D; e += kFinal) {
        float s = 0.f;
        int c = 0;
        for (; c + 8 <= nch; c += 8) {
            float v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = part[(size_t)(c + i) * D + e];
#pragma unroll
            for (int i = 0; i < 8; ++i) s += v[i];
        }
        for (; c < nch; ++c) s += part[(size_t)c * D + e];
        Pbar[e] = s;
        if (lds) pb_s[e] = s;
    }
    __syncthreads();
    if (peaks != nullptr)
        search_peaks(lds ? pb_s : Pbar, D, n_az, n_el, Ns, peaks, peak_val, cand, red_v, red_i,
                     chosen);
}

__global__ __launch_bounds__(kThreads) void binsum_part(const float *__restrict__ P, int F, int D,
                                                        float *__restrict__ part)
{
    binsum_part_body(P, F, D, part, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(kFinal) void binsum_final(const float *__restrict__ part, int nch,
                                                       int D, float *__restrict__ Pbar, int n_az,
                                                       int n_el, int Ns,
                                                       int32_t *__restrict__ peaks,
                                                       float *__restrict__ peak_val)
{
    binsum_final_body(part, nch, D, Pbar, n_az, n_el, Ns, peaks, peak_val);
}

// Batch: grid z (partials) or x (final) = block; workgroups outside a block's own (direction,
// bin) chunk grid leave at once.
__global__ __launch_bounds__(kThreads) void binsum_part_batch(const BlockDev *__restrict__ blk)
{
    const BlockDev &B = blk[blockIdx.z];
    const int ndc = (B.D + kThreads - 1) / kThreads;
    const int nch = (B.F + SSL_BINSUM_CHUNK - 1) / SSL_BINSUM_CHUNK;
    if ((int)blockIdx.x >= ndc || (int)blockIdx.y >= nch) return;
    binsum_part_body(B.P, B.F, B.D, B.part, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(kFinal) void binsum_final_batch(const BlockDev *__restrict__ blk)
{
    const BlockDev &B = blk[blockIdx.x];
    const int nch = (B.F + SSL_BINSUM_CHUNK - 1) / SSL_BINSUM_CHUNK;
    binsum_final_body(B.part, nch, B.D, B.Pbar, B.n_az, B.n_el, B.Ns, B.peaks, B.peak_val);
}

__global__ __launch_bounds__(kFinal) void peaks_only(const float *__restrict__ Pbar, int D,
                                                     int n_az, int n_el, int Ns,
                                                     int32_t *__restrict__ peaks,
                                                     float *__restrict__ peak_val)
{
    __shared__ float pb_s[kLdsPbar];
    __shared__ unsigned char cand[kLdsPbar];
    __shared__ float red_v[kFinal];
    __shared__ int red_i[kFinal];
    __shared__ int chosen[SSL_MAX_M];
    const bool lds = D <= kLdsPbar;
    if (lds)
        for (int e = threadIdx.x; e < D; e += kFinal) pb_s[e] = Pbar[e];
    __syncthreads();
    search_peaks(lds ? pb_s : Pbar, D, n_az, n_el, Ns, peaks, peak_val, cand, red_v, red_i,
                 chosen);
}

}  // namespace

hipError_t launch_binsum_peaks(const float *P, int F, int D, float *Pbar, float *part,
                               int n_az, int n_el, int Ns, int32_t *peaks, float *peak_val,
                               hipStream_t st)
{
    const int nch = (F + SSL_BINSUM_CHUNK - 1) / SSL_BINSUM_CHUNK;
    hipLaunchKernelGGL(binsum_part, dim3((D + kThreads - 1) / kThreads, nch), dim3(kThreads), 0,
                       st, P, F, D, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(binsum_final, dim3(1), dim3(kFinal), 0, st, part, nch, D, Pbar, n_az, n_el,
                       Ns, peaks, peak_val);
    return hipGetLastError();
}

int binsum_threads() { return kThreads; }

hipError_t launch_binsum_batch(const BlockDev *blk, int nblocks, int max_dchunks, int max_fchunks,
                               hipStream_t st)
{
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(binsum_part_batch, dim3(max_dchunks, max_fchunks, nblocks),
                       dim3(kThreads), 0, st, blk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(binsum_final_batch, dim3(nblocks), dim3(kFinal), 0, st, blk);
    return hipGetLastError();
}

hipError_t launch_peaks(const float *Pbar, int n_az, int n_el, int Ns, int32_t *peaks,
                        float *peak_val, hipStream_t st)
{
    hipLaunchKernelGGL(peaks_only, dim3(1), dim3(kFinal), 0, st, Pbar, n_az * n_el, n_az, n_el,
                       Ns, peaks, peak_val);
    return hipGetLastError();
}
