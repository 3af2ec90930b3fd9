// Learned-incumbent network of the divergence estimator (gfx950).
//
// A small convolutional regressor proposes a divergence for each window from
// its unwarped 64x64 event-count image; the proposal seeds the incumbent of
// the branch and bound, which still certifies the optimum.  Layers:
//   conv3x3/s2/p1 1->16, ReLU (32x32), conv3x3/s2/p1 16->32, ReLU (16x16),
//   conv3x3/s2/p1 32->64, ReLU (8x8), mean over positions, linear 64->1.
// Weights and layer inputs are rounded to bfloat16 (nearest even) where they
// enter a product; products and sums are fp32.  The backward pass treats the
// rounding as the identity.  One workgroup per image keeps every activation
// of that image in LDS (128 KB); parameters are read from HBM/L2.
#include "ecmd_internal.hpp"

namespace ecmd {

namespace cnn {
constexpr int kThreads = 256;
constexpr int oW1 = 0, oB1 = oW1 + 16 * 1 * 9, oW2 = oB1 + 16, oB2 = oW2 + 32 * 16 * 9, oW3 = oB2 + 32,
              oB3 = oW3 + 64 * 32 * 9, oWfc = oB3 + 64, oBfc = oWfc + 64, kNParam = oBfc + 1;
static_assert(kNParam == 23361, "parameter count");
// LDS (floats): image, a1, a2, a3, pooled, scratch
constexpr int sImg = 0, sA1 = sImg + 64 * 64, sA2 = sA1 + 16 * 32 * 32, sA3 = sA2 + 32 * 16 * 16,
              sG = sA3 + 64 * 8 * 8, sRed = sG + 64, kLdsFloats = sRed + kThreads;
}  // namespace cnn

using namespace cnn;

__device__ __forceinline__ float bf(float v) {
    unsigned u = __float_as_uint(v);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xFFFF0000u);
}

__device__ __forceinline__ float bits_to_f(uint16_t b) { return __uint_as_float((unsigned)b << 16); }

// z[o][y][x] = b[o] + sum_{i,ky,kx} bf(W[o][i][ky][kx]) * bf(in[i][2y+ky-1][2x+kx-1]); out = relu(z)
template <int CI, int CO, int HI>
__device__ void conv_fwd(const float* __restrict__ in, float* __restrict__ out, const float* __restrict__ W,
                         const float* __restrict__ b, bool round_in) {
    constexpr int HO = HI / 2;
    for (int idx = threadIdx.x; idx < CO * HO * HO; idx += kThreads) {
        const int o = idx / (HO * HO), rem = idx % (HO * HO), y = rem / HO, x = rem % HO;
        float acc = 0.0f;
        for (int i = 0; i < CI; ++i) {
            const float* Wi = W + (o * CI + i) * 9;
            const float* ini = in + i * HI * HI;
            for (int ky = 0; ky < 3; ++ky) {
                const int iy = 2 * y + ky - 1;
                if (iy < 0 || iy >= HI) continue;
                for (int kx = 0; kx < 3; ++kx) {
                    const int ix = 2 * x + kx - 1;
                    if (ix < 0 || ix >= HI) continue;
                    const float v = round_in ? bf(ini[iy * HI + ix]) : ini[iy * HI + ix];
                    acc = fmaf(bf(Wi[ky * 3 + kx]), v, acc);
                }
            }
        }
        out[idx] = fmaxf(acc + b[o], 0.0f);
    }
}

// dW[o][i][ky][kx] = sum_{y,x} dz[o][y][x] * bf(in[i][2y+ky-1][2x+kx-1]); db[o] = sum dz[o]
template <int CI, int CO, int HI>
__device__ void conv_wgrad(const float* __restrict__ in, const float* __restrict__ dz, float* __restrict__ gW,
                           float* __restrict__ gb, bool round_in) {
    constexpr int HO = HI / 2;
    for (int idx = threadIdx.x; idx < CO * CI * 9; idx += kThreads) {
        const int o = idx / (CI * 9), rem = idx % (CI * 9), i = rem / 9, ky = (rem % 9) / 3, kx = rem % 3;
        const float* dzo = dz + o * HO * HO;
        const float* ini = in + i * HI * HI;
        float acc = 0.0f;
        for (int y = 0; y < HO; ++y) {
            const int iy = 2 * y + ky - 1;
            if (iy < 0 || iy >= HI) continue;
            for (int x = 0; x < HO; ++x) {
                const int ix = 2 * x + kx - 1;
                if (ix < 0 || ix >= HI) continue;
                const float v = round_in ? bf(ini[iy * HI + ix]) : ini[iy * HI + ix];
                acc = fmaf(dzo[y * HO + x], v, acc);
            }
        }
        gW[idx] = acc;
    }
    for (int o = threadIdx.x; o < CO; o += kThreads) {
        float acc = 0.0f;
        for (int p = 0; p < HO * HO; ++p) acc += dz[o * HO * HO + p];
        gb[o] = acc;
    }
}

// In place: act[i][iy][ix] <- (act > 0) * sum_{o,ky,kx} dz[o][y][x] * bf(W[o][i][ky][kx])
// over the output positions (y, x) whose window covers (iy, ix).
template <int CI, int CO, int HI>
__device__ void conv_dgrad_relu(float* __restrict__ act, const float* __restrict__ dz, const float* __restrict__ W) {
    constexpr int HO = HI / 2;
    for (int idx = threadIdx.x; idx < CI * HI * HI; idx += kThreads) {
        const int i = idx / (HI * HI), rem = idx % (HI * HI), iy = rem / HI, ix = rem % HI;
        float acc = 0.0f;
        if (act[idx] > 0.0f) {
            for (int ky = 0; ky < 3; ++ky) {
                const int ty = iy + 1 - ky;
                if (ty < 0 || (ty & 1) || (ty >> 1) >= HO) continue;
                const int y = ty >> 1;
                for (int kx = 0; kx < 3; ++kx) {
                    const int tx = ix + 1 - kx;
                    if (tx < 0 || (tx & 1) || (tx >> 1) >= HO) continue;
                    const int x = tx >> 1;
                    for (int o = 0; o < CO; ++o)
                        acc = fmaf(dz[(o * HO + y) * HO + x], bf(W[(o * CI + i) * 9 + ky * 3 + kx]), acc);
                }
            }
        }
        act[idx] = acc;
    }
}

// mode 0: forward only (out[b]); mode 1: forward + backward of the MSE
// loss with `inv_n` = 1 / batch, per-image gradients to pg[b][kNParam] and
// per-image loss to lossb[b].
__global__ __launch_bounds__(kThreads) void k_cnn(const float* __restrict__ P, const uint16_t* __restrict__ imgs,
                                                  int B, float* __restrict__ out, int mode,
                                                  const float* __restrict__ labels, float inv_n,
                                                  float* __restrict__ pg, float* __restrict__ lossb) {
    extern __shared__ float s[];
    const int b = blockIdx.x;
    if (b >= B) return;
    const int tid = threadIdx.x;
    float* img = s + sImg;
    float* a1 = s + sA1;
    float* a2 = s + sA2;
    float* a3 = s + sA3;
    float* g = s + sG;
    float* red = s + sRed;
    for (int k = tid; k < 64 * 64; k += kThreads) img[k] = bits_to_f(imgs[(long long)b * 4096 + k]);
    __syncthreads();
    conv_fwd<1, 16, 64>(img, a1, P + oW1, P + oB1, false);
    __syncthreads();
    conv_fwd<16, 32, 32>(a1, a2, P + oW2, P + oB2, true);
    __syncthreads();
    conv_fwd<32, 64, 16>(a2, a3, P + oW3, P + oB3, true);
    __syncthreads();
    if (tid < 64) {
        float acc = 0.0f;
        for (int p = 0; p < 64; ++p) acc += a3[tid * 64 + p];
        g[tid] = acc * (1.0f / 64.0f);
    }
    __syncthreads();
    if (tid < 64) red[tid] = bf(g[tid]) * bf(P[oWfc + tid]);
    __syncthreads();
    float d = 0.0f;
    if (tid == 0) {
        for (int c = 0; c < 64; ++c) d += red[c];
        d += P[oBfc];
        out[b] = d;
        red[64] = d;
    }
    if (mode == 0) return;
    __syncthreads();
    d = red[64];
    const float dd = 2.0f * (d - labels[b]) * inv_n;
    float* gp = pg + (long long)b * kNParam;
    if (tid == 0) {
        gp[oBfc] = dd;
        lossb[b] = (d - labels[b]) * (d - labels[b]) * inv_n;
    }
    if (tid < 64) gp[oWfc + tid] = dd * bf(g[tid]);
    // dz3 = (dd * bf(Wfc[c]) / 64) * (a3 > 0), in place
    for (int k = tid; k < 64 * 64; k += kThreads) {
        const int c = k >> 6;
        a3[k] = a3[k] > 0.0f ? dd * bf(P[oWfc + c]) * (1.0f / 64.0f) : 0.0f;
    }
    __syncthreads();
    conv_wgrad<32, 64, 16>(a2, a3, gp + oW3, gp + oB3, true);
    __syncthreads();
    conv_dgrad_relu<32, 64, 16>(a2, a3, P + oW3);
    __syncthreads();
    conv_wgrad<16, 32, 32>(a1, a2, gp + oW2, gp + oB2, true);
    __syncthreads();
    conv_dgrad_relu<16, 32, 32>(a1, a2, P + oW2);
    __syncthreads();
    conv_wgrad<1, 16, 64>(img, a1, gp + oW1, gp + oB1, false);
}

// Forward pass alone (the proposal of the learned incumbent), for a few
// images at a time: 1024 threads per image so that a batch of a few dozen
// windows is not bound by one wave per SIMD.  Each wave computes CB output
// channels (wave-uniform, so their weights are scalar loads) at every
// position it owns, reusing each input read for the CB channels; a layer
// whose output feeds a rounded input stores it rounded (bf(bf(v)) = bf(v)).
// Every output sums its products in the order of conv_fwd, so the results
// are conv_fwd's.
constexpr int kFwdThreads = 1024;
constexpr int kFwdWaves = kFwdThreads / 64;

template <int CI, int CO, int HI, int CB>
__device__ void conv_fwd_waves(const float* __restrict__ in, float* __restrict__ out, const float* __restrict__ W,
                               const float* __restrict__ b, bool round_out) {
    constexpr int HO = HI / 2, NP = HO * HO;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    for (int o0 = wave * CB; o0 < CO; o0 += kFwdWaves * CB) {
        for (int p = lane; p < NP; p += 64) {
            const int y = p / HO, x = p % HO;
            float acc[CB];
#pragma unroll
            for (int c = 0; c < CB; ++c) acc[c] = 0.0f;
            for (int i = 0; i < CI; ++i) {
                const float* ini = in + i * HI * HI;
                for (int ky = 0; ky < 3; ++ky) {
                    const int iy = 2 * y + ky - 1;
                    if (iy < 0 || iy >= HI) continue;
                    for (int kx = 0; kx < 3; ++kx) {
                        const int ix = 2 * x + kx - 1;
                        if (ix < 0 || ix >= HI) continue;
                        const float v = ini[iy * HI + ix];
#pragma unroll
                        for (int c = 0; c < CB; ++c) acc[c] = fmaf(bf(W[((o0 + c) * CI + i) * 9 + ky * 3 + kx]), v, acc[c]);
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < CB; ++c) {
                const float r = fmaxf(acc[c] + b[o0 + c], 0.0f);
                out[(o0 + c) * NP + p] = round_out ? bf(r) : r;
            }
        }
    }
}

__global__ __launch_bounds__(kFwdThreads) void k_cnn_fwd(const float* __restrict__ P,
                                                         const uint16_t* __restrict__ imgs, int B,
                                                         float* __restrict__ out) {
    extern __shared__ float s[];
    const int b = blockIdx.x;
    if (b >= B) return;
    const int tid = threadIdx.x;
    float* img = s + sImg;
    float* a1 = s + sA1;
    float* a2 = s + sA2;
    float* a3 = s + sA3;
    float* g = s + sG;
    for (int k = tid; k < 64 * 64; k += kFwdThreads) img[k] = bits_to_f(imgs[(long long)b * 4096 + k]);
    __syncthreads();
    conv_fwd_waves<1, 16, 64, 1>(img, a1, P + oW1, P + oB1, true);
    __syncthreads();
    conv_fwd_waves<16, 32, 32, 2>(a1, a2, P + oW2, P + oB2, true);
    __syncthreads();
    conv_fwd_waves<32, 64, 16, 4>(a2, a3, P + oW3, P + oB3, false);
    __syncthreads();
    if (tid < 64) {
        float acc = 0.0f;
        for (int p = 0; p < 64; ++p) acc += a3[tid * 64 + p];
        g[tid] = bf(acc * (1.0f / 64.0f)) * bf(P[oWfc + tid]);
    }
    __syncthreads();
    if (tid == 0) {
        float d = 0.0f;
        for (int c = 0; c < 64; ++c) d += g[c];
        out[b] = d + P[oBfc];
    }
}

// grad[p] = sum_b pg[b][p] (fixed order); loss = sum_b lossb[b]
__global__ void k_cnn_reduce(const float* __restrict__ pg, const float* __restrict__ lossb, int B,
                             float* __restrict__ grad, float* __restrict__ loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kNParam) {
        float acc = 0.0f;
        for (int b = 0; b < B; ++b) acc += pg[(long long)b * kNParam + p];
        grad[p] = acc;
    }
    if (p == 0) {
        float acc = 0.0f;
        for (int b = 0; b < B; ++b) acc += lossb[b];
        *loss = acc;
    }
}

__global__ void k_adam(float* __restrict__ P, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ grad, float lr, float c1, float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNParam) return;
    const float g = grad[p];
    const float mi = 0.9f * m[p] + 0.1f * g;
    const float vi = 0.999f * v[p] + 0.001f * g * g;
    m[p] = mi;
    v[p] = vi;
    P[p] -= lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
}

// Nearest grid index of each prediction as the seed divergence (NaN if not finite).
__global__ void k_seed_from_pred(const float* __restrict__ pred, int B, float d_lo, float d_hi,
                                 float* __restrict__ seeds) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const float d = pred[b];
    seeds[b] = isfinite(d) ? fminf(fmaxf(d, d_lo), d_hi) : __builtin_nanf("");
}

size_t cnn_lds_bytes() { return (size_t)kLdsFloats * sizeof(float); }
int cnn_nparam() { return kNParam; }

hipError_t cnn_set_lds() {
    hipError_t e =
        hipFuncSetAttribute((const void*)k_cnn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cnn_lds_bytes());
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_cnn_fwd, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)cnn_lds_bytes());
}

hipError_t launch_cnn(hipStream_t s, const float* P, const uint16_t* imgs, int B, float* out, int mode,
                      const float* labels, float* pg, float* lossb) {
    if (B <= 0) return hipSuccess;
    if (mode == 0)
        k_cnn_fwd<<<B, kFwdThreads, cnn_lds_bytes(), s>>>(P, imgs, B, out);
    else
        k_cnn<<<B, kThreads, cnn_lds_bytes(), s>>>(P, imgs, B, out, mode, labels, 1.0f / (float)B, pg, lossb);
    return hipGetLastError();
}

hipError_t launch_cnn_reduce(hipStream_t s, const float* pg, const float* lossb, int B, float* grad, float* loss) {
    k_cnn_reduce<<<(kNParam + 255) / 256, 256, 0, s>>>(pg, lossb, B, grad, loss);
    return hipGetLastError();
}

hipError_t launch_adam(hipStream_t s, float* P, float* m, float* v, const float* grad, float lr, int step) {
    const float c1 = 1.0f / (1.0f - powf(0.9f, (float)step));
    const float c2 = 1.0f / (1.0f - powf(0.999f, (float)step));
    k_adam<<<(kNParam + 255) / 256, 256, 0, s>>>(P, m, v, grad, lr, c1, c2);
    return hipGetLastError();
}

hipError_t launch_seed_from_pred(hipStream_t s, const float* pred, int B, float d_lo, float d_hi, float* seeds) {
    if (B <= 0) return hipSuccess;
    k_seed_from_pred<<<(B + 255) / 256, 256, 0, s>>>(pred, B, d_lo, d_hi, seeds);
    return hipGetLastError();
}

}  // namespace ecmd
