// Bin integration (eq.6 of arXiv 2504.03373) and peak search (Sec. III-A, last paragraph).
//
// Pbar[d] = sum_f P[f, d].  Deterministic, atomics-free order: bins are summed in ascending order
// inside fixed chunks of SSL_BINSUM_CHUNK bins (one thread per (direction, chunk)), then the chunk
// partials in ascending chunk order.  The same launch finishes with the peak search: the last
// workgroup to complete (a ticket on a device counter, released with a device-scope fence) sums
// the partials and searches the peaks, then re-arms the counter for the next launch.  Nothing
// ever waits on another workgroup.
//
// Peak rule on the n_el x n_az grid (d = el * n_az + az): d is a local maximum when it beats each
// of its 8 neighbours -- azimuth circular, elevation clamped -- where "beats" means a larger value,
// or an equal value and a lower flat index.  Maxima are ranked by the same relation; the first
// Ns are returned, -1 / 0 beyond the number found.  Non-finite values never take part.
#include "ssl_internal.h"

namespace {

constexpr int kThreads = 256;
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
        for (int d = tid; d < D; d += kThreads) cand[d] = is_local_max(pb, n_el, n_az, d) ? 1 : 0;
    }
    __syncthreads();
    for (int k = 0; k < Ns; ++k) {
        // each thread: best remaining candidate among its directions
        float bv = 0.f;
        int bi = -1;
        for (int d = tid; d < D; d += kThreads) {
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
        for (int s = kThreads / 2; s > 0; s >>= 1) {
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

// Workgroup (dc, ch) of an ndc x nch grid over one block's [F][D] spectrum.
__device__ __forceinline__ void binsum_peaks_body(
    const float *__restrict__ P, int F, int D, float *__restrict__ Pbar, float *__restrict__ part,
    unsigned int *__restrict__ counter, int n_az, int n_el, int Ns, int32_t *__restrict__ peaks,
    float *__restrict__ peak_val, int dc, int ch, int ndc, int nch)
{
    __shared__ float pb_s[kLdsPbar];
    __shared__ unsigned char cand[kLdsPbar];
    __shared__ float red_v[kThreads];
    __shared__ int red_i[kThreads];
    __shared__ int chosen[SSL_MAX_M];
    __shared__ int is_last;
    const int tid = threadIdx.x;
    const int d = dc * kThreads + tid;
    if (d < D) {
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
    __threadfence();
    __syncthreads();
    if (tid == 0) {
        const unsigned int ticket = atomicAdd(counter, 1u);
        is_last = (ticket == (unsigned int)(ndc * nch) - 1u) ? 1 : 0;
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    const bool lds = D <= kLdsPbar;
    for (int e = tid; e < D; e += kThreads) {
        float s = 0.f;
        int c = 0;
        for (; c + 8 <= nch; c += 8) {
            float v[8];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                v[i] = __hip_atomic_load(&part[(size_t)(c + i) * D + e], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
            for (int i = 0; i < 8; ++i) s += v[i];
        }
        for (; c < nch; ++c)
            s += __hip_atomic_load(&part[(size_t)c * D + e], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        Pbar[e] = s;
        if (lds) pb_s[e] = s;
    }
    __syncthreads();
    if (tid == 0) *counter = 0u;     // re-arm for the next launch on this stream
    if (peaks != nullptr)
        search_peaks(lds ? pb_s : Pbar, D, n_az, n_el, Ns, peaks, peak_val, cand, red_v, red_i,
                     chosen);
}

__global__ __launch_bounds__(kThreads) void binsum_peaks(
    const float *__restrict__ P, int F, int D, float *__restrict__ Pbar, float *__restrict__ part,
    unsigned int *__restrict__ counter, int n_az, int n_el, int Ns, int32_t *__restrict__ peaks,
    float *__restrict__ peak_val)
{
    binsum_peaks_body(P, F, D, Pbar, part, counter, n_az, n_el, Ns, peaks, peak_val, blockIdx.x,
                      blockIdx.y, gridDim.x, gridDim.y);
}

// Batch: grid z = block; workgroups outside a block's own (direction, bin) chunk grid leave at once
// and never touch its counter.
__global__ __launch_bounds__(kThreads) void binsum_peaks_batch(const BlockDev *__restrict__ blk)
{
    const BlockDev &B = blk[blockIdx.z];
    const int ndc = (B.D + kThreads - 1) / kThreads;
    const int nch = (B.F + SSL_BINSUM_CHUNK - 1) / SSL_BINSUM_CHUNK;
    if ((int)blockIdx.x >= ndc || (int)blockIdx.y >= nch) return;
    binsum_peaks_body(B.P, B.F, B.D, B.Pbar, B.part, B.counter, B.n_az, B.n_el, B.Ns, B.peaks,
                      B.peak_val, blockIdx.x, blockIdx.y, ndc, nch);
}

__global__ __launch_bounds__(kThreads) void peaks_only(const float *__restrict__ Pbar, int D,
                                                       int n_az, int n_el, int Ns,
                                                       int32_t *__restrict__ peaks,
                                                       float *__restrict__ peak_val)
{
    __shared__ float pb_s[kLdsPbar];
    __shared__ unsigned char cand[kLdsPbar];
    __shared__ float red_v[kThreads];
    __shared__ int red_i[kThreads];
    __shared__ int chosen[SSL_MAX_M];
    const bool lds = D <= kLdsPbar;
    if (lds)
        for (int e = threadIdx.x; e < D; e += kThreads) pb_s[e] = Pbar[e];
    __syncthreads();
    search_peaks(lds ? pb_s : Pbar, D, n_az, n_el, Ns, peaks, peak_val, cand, red_v, red_i,
                 chosen);
}

}  // namespace

hipError_t launch_binsum_peaks(const float *P, int F, int D, float *Pbar, float *part,
                               unsigned int *counter, int n_az, int n_el, int Ns, int32_t *peaks,
                               float *peak_val, hipStream_t st)
{
    const int nch = (F + SSL_BINSUM_CHUNK - 1) / SSL_BINSUM_CHUNK;
    const dim3 grid((D + kThreads - 1) / kThreads, nch);
    hipLaunchKernelGGL(binsum_peaks, grid, dim3(kThreads), 0, st, P, F, D, Pbar, part, counter,
                       n_az, n_el, Ns, peaks, peak_val);
    return hipGetLastError();
}

int binsum_threads() { return kThreads; }

hipError_t launch_binsum_batch(const BlockDev *blk, int nblocks, int max_dchunks, int max_fchunks,
                               hipStream_t st)
{
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(binsum_peaks_batch, dim3(max_dchunks, max_fchunks, nblocks),
                       dim3(kThreads), 0, st, blk);
    return hipGetLastError();
}

hipError_t launch_peaks(const float *Pbar, int n_az, int n_el, int Ns, int32_t *peaks,
                        float *peak_val, hipStream_t st)
{
    hipLaunchKernelGGL(peaks_only, dim3(1), dim3(kThreads), 0, st, Pbar, n_az * n_el, n_az, n_el,
                       Ns, peaks, peak_val);
    return hipGetLastError();
}
