// Calibration kernels for the roofline of the evaluation kernel: the rate of
// conflict-free LDS atomic adds without return (the operation the
// event-image histograms use, counted per lane) and the HBM stream-read
// bandwidth, both measured on the device the context runs on.
#include "ecmd_internal.hpp"

namespace ecmd {

constexpr int kCalThreads = 1024;
constexpr int kCalWords = 8192;  // 32 KiB of counters per workgroup

// Every lane adds 1 to its own counter word, `iters` times, without using
// the old value (the form the histograms use); lanes of a wave hit 64
// consecutive words, i.e. no two lanes of an access share a bank.
__global__ __launch_bounds__(kCalThreads) void k_lds_atomics(int iters, unsigned* __restrict__ sink) {
    __shared__ unsigned cnt[kCalWords];
    for (int i = threadIdx.x; i < kCalWords; i += kCalThreads) cnt[i] = 0u;
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int k = 0; k < iters; ++k) {
        const int w = ((wave * 8 + (k & 7)) * 64 + lane) & (kCalWords - 1);
        atomicAdd(&cnt[w], 1u);
    }
    __syncthreads();
    const unsigned v = cnt[threadIdx.x & (kCalWords - 1)];
    if (v == 0xFFFFFFFFu) sink[blockIdx.x] = v;  // keeps the counters observable
}

// Sum of a buffer of float4, grid-stride, one partial per workgroup.
__global__ __launch_bounds__(256) void k_stream_read(const float4* __restrict__ a, long long n4,
                                                      float* __restrict__ partial) {
    float s = 0.0f;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n4; i += (long long)gridDim.x * 256) {
        const float4 v = a[i];
        s += (v.x + v.y) + (v.z + v.w);
    }
    __shared__ float red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

hipError_t launch_lds_atomics(hipStream_t s, int blocks, int iters, unsigned* sink) {
    k_lds_atomics<<<blocks, kCalThreads, 0, s>>>(iters, sink);
    return hipGetLastError();
}

hipError_t launch_stream_read(hipStream_t s, const void* a, long long bytes, int blocks, float* partial) {
    k_stream_read<<<blocks, 256, 0, s>>>(static_cast<const float4*>(a), bytes / 16, partial);
    return hipGetLastError();
}

}  // namespace ecmd
