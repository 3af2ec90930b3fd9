// Event preprocessing of the divergence estimator (gfx950): the steps the
// paper applies before estimation (Sec. 6, "Preprocessing"): hot-pixel
// removal, and the "resized and resampled" variant that scales the image
// coordinates to a smaller sensor and keeps a random fraction of the events.
//
// Both produce compacted copies of the windows (order kept) with new CSR
// offsets.  The random keep decision is a counter-based draw: event k of
// window w (k counted from the window start) is kept iff the top 24 bits of
// SplitMix64 at counter seed + (w * 2^32 + k + 1) * 0x9E3779B97F4A7C15 fall
// below keep_frac * 2^24.
#include "ecmd_internal.hpp"

namespace ecmd {

constexpr int kPreThreads = 1024;

__device__ __forceinline__ unsigned long long splitmix64(unsigned long long s) {
    unsigned long long z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// keep flags for the resample: counter-based draw per event
__global__ __launch_bounds__(kPreThreads) void k_resample_keep(const long long* __restrict__ offsets, int B,
                                                              long long n, unsigned long long seed,
                                                              unsigned thresh24, unsigned char* __restrict__ keep) {
    const long long i = (long long)blockIdx.x * kPreThreads + threadIdx.x;
    if (i >= n) return;
    int lo = 0, hi = B;  // window of event i: largest w with offsets[w] <= i
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (offsets[mid] <= i + offsets[0]) lo = mid; else hi = mid;
    }
    const unsigned long long k = (unsigned long long)(i + offsets[0] - offsets[lo]);
    const unsigned long long ctr = ((unsigned long long)lo << 32) + k + 1ull;
    const unsigned long long z = splitmix64(seed + ctr * 0x9E3779B97F4A7C15ull);
    keep[i] = (unsigned)(z >> 40) < thresh24 ? 1 : 0;
}

// per-window pixel counts of the unwarped events
__global__ __launch_bounds__(kPreThreads) void k_pixel_counts(const float* __restrict__ x, const float* __restrict__ y,
                                                             const long long* __restrict__ offsets, int B, long long n,
                                                             int W, int H, unsigned* __restrict__ counts) {
    const long long i = (long long)blockIdx.x * kPreThreads + threadIdx.x;
    if (i >= n) return;
    int lo = 0, hi = B;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (offsets[mid] <= i + offsets[0]) lo = mid; else hi = mid;
    }
    const long long j = i + offsets[0];
    const float xv = x[j], yv = y[j];
    if (!(xv >= 0.0f && xv < (float)W && yv >= 0.0f && yv < (float)H)) return;
    const long long pix = (long long)lo * W * H + (long long)(int)floorf(yv) * W + (int)floorf(xv);
    atomicAdd(&counts[pix], 1u);
}

__global__ __launch_bounds__(kPreThreads) void k_hot_keep(const float* __restrict__ x, const float* __restrict__ y,
                                                         const long long* __restrict__ offsets, int B, long long n,
                                                         int W, int H, const unsigned* __restrict__ counts,
                                                         unsigned max_count, unsigned char* __restrict__ keep) {
    const long long i = (long long)blockIdx.x * kPreThreads + threadIdx.x;
    if (i >= n) return;
    int lo = 0, hi = B;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (offsets[mid] <= i + offsets[0]) lo = mid; else hi = mid;
    }
    const long long j = i + offsets[0];
    const float xv = x[j], yv = y[j];
    unsigned char k = 1;
    if (xv >= 0.0f && xv < (float)W && yv >= 0.0f && yv < (float)H) {
        const long long pix = (long long)lo * W * H + (long long)(int)floorf(yv) * W + (int)floorf(xv);
        k = counts[pix] > max_count ? 0 : 1;
    }
    keep[i] = k;
}

// stream compaction of the kept events: per-block counts, one scan, scatter
__global__ __launch_bounds__(kPreThreads) void k_keep_count(const unsigned char* __restrict__ keep, long long n,
                                                           long long* __restrict__ blk) {
    __shared__ int s;
    if (threadIdx.x == 0) s = 0;
    __syncthreads();
    const long long i = (long long)blockIdx.x * kPreThreads + threadIdx.x;
    if (i < n && keep[i]) atomicAdd(&s, 1);
    __syncthreads();
    if (threadIdx.x == 0) blk[blockIdx.x] = s;
}

__global__ __launch_bounds__(1024) void k_keep_scan(long long nb, long long* __restrict__ blk) {
    __shared__ long long s[1024];
    __shared__ long long carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (long long base = 0; base < nb; base += 1024) {
        const long long k = base + threadIdx.x;
        const long long v = k < nb ? blk[k] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const long long a = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0;
            __syncthreads();
            s[threadIdx.x] += a;
            __syncthreads();
        }
        const long long incl = s[threadIdx.x] + carry;
        if (k < nb) blk[k] = incl - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry = incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) blk[nb] = carry;
}

__global__ __launch_bounds__(kPreThreads) void k_keep_scatter(
    const float* __restrict__ x, const float* __restrict__ y, const float* __restrict__ t, long long off0, long long n,
    const unsigned char* __restrict__ keep, const long long* __restrict__ blk, float sx, float sy,
    float* __restrict__ xo, float* __restrict__ yo, float* __restrict__ to) {
    __shared__ int s[kPreThreads];
    const long long i = (long long)blockIdx.x * kPreThreads + threadIdx.x;
    const int k = (i < n && keep[i]) ? 1 : 0;
    s[threadIdx.x] = k;
    __syncthreads();
    for (int o = 1; o < kPreThreads; o <<= 1) {
        const int a = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0;
        __syncthreads();
        s[threadIdx.x] += a;
        __syncthreads();
    }
    if (k) {
        const long long d = blk[blockIdx.x] + s[threadIdx.x] - 1;
        const long long j = i + off0;
        xo[d] = x[j] * sx;
        yo[d] = y[j] * sy;
        to[d] = t[j];
    }
}

// new offsets: number of kept events before each window start
__global__ void k_keep_offsets(const long long* __restrict__ offsets, int B, const unsigned char* __restrict__ keep,
                               const long long* __restrict__ blk, long long* __restrict__ off_out) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w > B) return;
    const long long i = offsets[w] - offsets[0];  // first event of window w (local index)
    const long long b = i / kPreThreads;
    long long c = blk[b];
    for (long long k = b * kPreThreads; k < i; ++k) c += keep[k];
    off_out[w] = c;
}

hipError_t launch_compact(hipStream_t s, const float* x, const float* y, const float* t, const long long* offsets,
                          int B, long long off0, long long n, const unsigned char* keep, long long* blk, float sx,
                          float sy, float* xo, float* yo, float* to, long long* off_out) {
    const long long nb = (n + kPreThreads - 1) / kPreThreads;
    if (nb > 0) {
        k_keep_count<<<(unsigned)nb, kPreThreads, 0, s>>>(keep, n, blk);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    k_keep_scan<<<1, 1024, 0, s>>>(nb, blk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (nb > 0) {
        k_keep_scatter<<<(unsigned)nb, kPreThreads, 0, s>>>(x, y, t, off0, n, keep, blk, sx, sy, xo, yo, to);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    k_keep_offsets<<<(B + 1 + 255) / 256, 256, 0, s>>>(offsets, B, keep, blk, off_out);
    return hipGetLastError();
}

hipError_t launch_resample_keep(hipStream_t s, const long long* offsets, int B, long long n, unsigned long long seed,
                                unsigned thresh24, unsigned char* keep) {
    if (n <= 0) return hipSuccess;
    k_resample_keep<<<(unsigned)((n + kPreThreads - 1) / kPreThreads), kPreThreads, 0, s>>>(offsets, B, n, seed,
                                                                                           thresh24, keep);
    return hipGetLastError();
}

hipError_t launch_hot_keep(hipStream_t s, const float* x, const float* y, const long long* offsets, int B, long long n,
                           int W, int H, unsigned* counts, unsigned max_count, unsigned char* keep) {
    if (n <= 0) return hipSuccess;
    const unsigned nb = (unsigned)((n + kPreThreads - 1) / kPreThreads);
    k_pixel_counts<<<nb, kPreThreads, 0, s>>>(x, y, offsets, B, n, W, H, counts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_hot_keep<<<nb, kPreThreads, 0, s>>>(x, y, offsets, B, n, W, H, counts, max_count, keep);
    return hipGetLastError();
}

// ------------------------------------------------------------ stream windows

// offsets[k] = first event with t >= t_start + k * tau (t non-decreasing)
__global__ void k_stream_bounds(const double* __restrict__ t, long long n, double t_start, double tau, int K,
                                long long* __restrict__ offsets) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > K) return;
    const double b = t_start + (double)k * tau;
    long long lo = 0, hi = n;
    while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if (t[mid] < b) lo = mid + 1; else hi = mid;
    }
    offsets[k] = lo;
}

// t_rel of every event of the K windows, relative to its window start
__global__ __launch_bounds__(kPreThreads) void k_stream_trel(const double* __restrict__ t,
                                                            const long long* __restrict__ offsets, int K,
                                                            double t_start, double tau, float* __restrict__ t_rel) {
    const long long i = offsets[0] + (long long)blockIdx.x * kPreThreads + threadIdx.x;
    if (i >= offsets[K]) return;
    int lo = 0, hi = K;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (offsets[mid] <= i) lo = mid; else hi = mid;
    }
    t_rel[i - offsets[0]] = (float)(t[i] - (t_start + (double)lo * tau));
}

hipError_t launch_stream_bounds(hipStream_t s, const double* t, long long n, double t_start, double tau, int K,
                                long long* offsets) {
    k_stream_bounds<<<(K + 1 + 255) / 256, 256, 0, s>>>(t, n, t_start, tau, K, offsets);
    return hipGetLastError();
}

hipError_t launch_stream_trel(hipStream_t s, const double* t, const long long* offsets, long long n_sel, int K,
                              double t_start, double tau, float* t_rel) {
    if (n_sel <= 0) return hipSuccess;
    k_stream_trel<<<(unsigned)((n_sel + kPreThreads - 1) / kPreThreads), kPreThreads, 0, s>>>(t, offsets, K, t_start,
                                                                                             tau, t_rel);
    return hipGetLastError();
}

}  // namespace ecmd
