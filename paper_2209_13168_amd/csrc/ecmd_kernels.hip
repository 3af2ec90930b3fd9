// HIP kernels of the MI355X divergence estimator (gfx950).
//
// Method: arXiv 2209.13168 -- radial warp eq. (12), event image eq. (13),
// contrast eq. (14), upper bound eqs. (15)-(20), branch and bound Alg. 1.
// Built with -ffp-contract=off: every fp32/fp64 operation below rounds
// exactly as written (the readings are listed in include/ecmd.h).
#include "ecmd_internal.hpp"

namespace ecmd {

// ------------------------------------------------------------ arithmetic

__device__ __forceinline__ float rate_of(float d, float tau) {
    float a = d * tau;
    float den = 1.0f - a;
    return d / den;  // correctly rounded fp32 division
}

__device__ __forceinline__ float grid_d(float d_lo, float d_hi, int L, unsigned j) {
    double span = (double)d_hi - (double)d_lo;
    double v = (double)d_lo + span * ldexp((double)j, -L);
    return (float)v;
}

__device__ __forceinline__ bool inside(float xw, float yw, float Wf, float Hf) {
    return xw >= 0.0f && xw < Wf && yw >= 0.0f && yw < Hf;
}

// floor(v) as an integer in one instruction (saturating for huge |v|,
// which only ever means "outside the image").
__device__ __forceinline__ int cvt_flr(float v) {
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(v));
    return r;
}

// floor of v clamped to [-1, hi]: -1 and hi both mean "outside the image"
// (floor commutes with clamping to integer limits).
__device__ __forceinline__ int flr_clamp(float v, int hi) {
    return min(max(cvt_flr(v), -1), hi);
}

__device__ __forceinline__ i128 mk128(long long hi, unsigned long long lo) {
    unsigned __int128 u = ((unsigned __int128)(unsigned long long)hi << 64) | (unsigned __int128)lo;
    return (i128)u;
}

__device__ __forceinline__ void sp128(i128 v, long long& hi, unsigned long long& lo) {
    unsigned __int128 u = (unsigned __int128)v;
    lo = (unsigned long long)u;
    hi = (long long)(unsigned long long)(u >> 64);
}

__device__ __forceinline__ bool improvable(i128 key, unsigned ja, i128 Kinc, unsigned jinc) {
    return key > Kinc || (key == Kinc && (unsigned long long)ja + 1ull < (unsigned long long)jinc);
}

__device__ __forceinline__ int bitlen128(i128 v) {
    unsigned __int128 u = (unsigned __int128)v;
    unsigned long long hi = (unsigned long long)(u >> 64), lo = (unsigned long long)u;
    if (hi) return 128 - __clzll(hi);
    if (lo) return 64 - __clzll(lo);
    return 0;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ------------------------------------------------------------ window params

__global__ void k_winparam(const float* __restrict__ tau, const long long* __restrict__ offsets, int B,
                           float d_lo, float d_hi, WinParam* __restrict__ wp) {
    int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= B) return;
    WinParam p;
    p.tau = tau[w];
    p.r_lo = rate_of(d_lo, p.tau);
    p.r_hi = rate_of(d_hi, p.tau);
    p.pad = 0;
    p.n_events = offsets[w + 1] - offsets[w];
    wp[w] = p;
}

hipError_t launch_winparam(hipStream_t s, const float* tau, const long long* offsets, int B,
                           float d_lo, float d_hi, WinParam* wp) {
    if (B <= 0) return hipSuccess;
    k_winparam<<<(B + 255) / 256, 256, 0, s>>>(tau, offsets, B, d_lo, d_hi, wp);
    return hipGetLastError();
}

// ------------------------------------------------------------ prep (a1)

// Window of block b: the largest w with blk_start[w] <= b.
__device__ __forceinline__ int window_of_block(const int* blk_start, int B, int b) {
    int lo = 0, hi = B;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (blk_start[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int band_of(const int* cut, int n, int k) {
    int b = 0;
    while (b + 1 < n && cut[b + 1] <= k) ++b;
    return b;
}

// Tile rectangle [tx0, tx1] x [ty0, ty1] reachable by an event over the
// whole search range (the pixel box spanned by its root segment), or
// false when that box misses the image.
__device__ __forceinline__ bool event_tiles(const Geometry& g, float x, float y, float ax, float ay,
                                            float r_lo, float r_hi, int& tx0, int& tx1, int& ty0,
                                            int& ty1) {
    float xa = fmaf(ax, r_lo, x), xb = fmaf(ax, r_hi, x);
    float ya = fmaf(ay, r_lo, y), yb = fmaf(ay, r_hi, y);
    int kx0 = flr_clamp(fminf(xa, xb), g.W), kx1 = flr_clamp(fmaxf(xa, xb), g.W);
    int ky0 = flr_clamp(fminf(ya, yb), g.H), ky1 = flr_clamp(fmaxf(ya, yb), g.H);
    if (kx1 < 0 || kx0 > g.W - 1 || ky1 < 0 || ky0 > g.H - 1) return false;
    kx0 = max(kx0, 0); ky0 = max(ky0, 0);
    kx1 = min(kx1, g.W - 1); ky1 = min(ky1, g.H - 1);
    tx0 = band_of(g.colcut, g.ntx, kx0); tx1 = band_of(g.colcut, g.ntx, kx1);
    ty0 = band_of(g.rowcut, g.nty, ky0); ty1 = band_of(g.rowcut, g.nty, ky1);
    return true;
}

constexpr int kPrepThreads = 256;

__global__ __launch_bounds__(kPrepThreads) void k_prep_count(
    Geometry g, const float* __restrict__ x, const float* __restrict__ y, const float* __restrict__ t_rel,
    const long long* __restrict__ offsets, const WinParam* __restrict__ wp, int B,
    const int* __restrict__ blk_start, int chunk, int* __restrict__ cnt_own, int* __restrict__ cnt_guest,
    int* __restrict__ err_flag) {
    __shared__ int s_own[kMaxTiles], s_guest[kMaxTiles];
    const int T = g.T;
    for (int t = threadIdx.x; t < T; t += blockDim.x) { s_own[t] = 0; s_guest[t] = 0; }
    __syncthreads();
    const int w = window_of_block(blk_start, B, blockIdx.x);
    const int c = blockIdx.x - blk_start[w];
    const long long beg = offsets[w] + (long long)c * chunk;
    const long long end = min(beg + chunk, offsets[w + 1]);
    const WinParam p = wp[w];
    for (long long i = beg + threadIdx.x; i < end; i += blockDim.x) {
        float xv = x[i], yv = y[i], tv = t_rel[i];
        if (!(isfinite(xv) && isfinite(yv) && tv >= 0.0f && tv <= p.tau)) {
            atomicOr(err_flag, 1);
            continue;
        }
        float ux = xv - g.cx, uy = yv - g.cy, delta = p.tau - tv;
        float ax = ux * delta, ay = uy * delta;
        int tx0, tx1, ty0, ty1;
        if (!event_tiles(g, xv, yv, ax, ay, p.r_lo, p.r_hi, tx0, tx1, ty0, ty1)) continue;
        atomicAdd(&s_own[ty0 * g.ntx + tx0], 1);
        for (int ty = ty0; ty <= ty1; ++ty)
            for (int tx = tx0; tx <= tx1; ++tx)
                if (ty != ty0 || tx != tx0) atomicAdd(&s_guest[ty * g.ntx + tx], 1);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < T; t += blockDim.x) {
        if (s_own[t]) atomicAdd(&cnt_own[w * T + t], s_own[t]);
        if (s_guest[t]) atomicAdd(&cnt_guest[w * T + t], s_guest[t]);
    }
}

// Exclusive scan of segment sizes (one workgroup).
__global__ __launch_bounds__(1024) void k_prep_scan(int nseg, const int* __restrict__ cnt_own,
                                                    const int* __restrict__ cnt_guest,
                                                    long long* __restrict__ seg_off,
                                                    int* __restrict__ seg_own,
                                                    unsigned long long* __restrict__ cursor) {
    __shared__ long long s[1024];
    __shared__ long long carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nseg; base += 1024) {
        int k = base + threadIdx.x;
        long long v = k < nseg ? (long long)cnt_own[k] + cnt_guest[k] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            long long a = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
            __syncthreads();
            s[threadIdx.x] += a;
            __syncthreads();
        }
        long long incl = s[threadIdx.x] + carry;
        if (k < nseg) {
            long long off = incl - v;
            seg_off[k] = off;
            seg_own[k] = cnt_own[k];
            cursor[2 * k] = (unsigned long long)off;
            cursor[2 * k + 1] = (unsigned long long)(off + cnt_own[k]);
        }
        __syncthreads();
        if (threadIdx.x == 1023) carry = incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) seg_off[nseg] = carry;
}

__global__ __launch_bounds__(kPrepThreads) void k_prep_scatter(
    Geometry g, const float* __restrict__ x, const float* __restrict__ y, const float* __restrict__ t_rel,
    const long long* __restrict__ offsets, const WinParam* __restrict__ wp, int B,
    const int* __restrict__ blk_start, int chunk, unsigned long long* __restrict__ cursor,
    float4* __restrict__ ev) {
    __shared__ int s_cnt[2 * kMaxTiles];
    __shared__ unsigned long long s_base[2 * kMaxTiles];
    const int T = g.T;
    for (int t = threadIdx.x; t < 2 * T; t += blockDim.x) s_cnt[t] = 0;
    __syncthreads();
    const int w = window_of_block(blk_start, B, blockIdx.x);
    const int c = blockIdx.x - blk_start[w];
    const long long beg = offsets[w] + (long long)c * chunk;
    const long long end = min(beg + chunk, offsets[w + 1]);
    const WinParam p = wp[w];
    // pass 1: count per (tile, owned/guest) within the block
    for (long long i = beg + threadIdx.x; i < end; i += blockDim.x) {
        float xv = x[i], yv = y[i], tv = t_rel[i];
        if (!(isfinite(xv) && isfinite(yv) && tv >= 0.0f && tv <= p.tau)) continue;
        float ax = (xv - g.cx) * (p.tau - tv), ay = (yv - g.cy) * (p.tau - tv);
        int tx0, tx1, ty0, ty1;
        if (!event_tiles(g, xv, yv, ax, ay, p.r_lo, p.r_hi, tx0, tx1, ty0, ty1)) continue;
        for (int ty = ty0; ty <= ty1; ++ty)
            for (int tx = tx0; tx <= tx1; ++tx) {
                int own = (ty == ty0 && tx == tx0) ? 0 : 1;
                atomicAdd(&s_cnt[2 * (ty * g.ntx + tx) + own], 1);
            }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < 2 * T; k += blockDim.x) {
        int n = s_cnt[k];
        s_base[k] = n ? atomicAdd(&cursor[2 * (w * T) + k], (unsigned long long)n) : 0ull;
        s_cnt[k] = 0;
    }
    __syncthreads();
    // pass 2: write
    for (long long i = beg + threadIdx.x; i < end; i += blockDim.x) {
        float xv = x[i], yv = y[i], tv = t_rel[i];
        if (!(isfinite(xv) && isfinite(yv) && tv >= 0.0f && tv <= p.tau)) continue;
        float ax = (xv - g.cx) * (p.tau - tv), ay = (yv - g.cy) * (p.tau - tv);
        int tx0, tx1, ty0, ty1;
        if (!event_tiles(g, xv, yv, ax, ay, p.r_lo, p.r_hi, tx0, tx1, ty0, ty1)) continue;
        float4 e = make_float4(xv, yv, ax, ay);
        for (int ty = ty0; ty <= ty1; ++ty)
            for (int tx = tx0; tx <= tx1; ++tx) {
                int k = 2 * (ty * g.ntx + tx) + ((ty == ty0 && tx == tx0) ? 0 : 1);
                int r = atomicAdd(&s_cnt[k], 1);
                ev[s_base[k] + (unsigned long long)r] = e;
            }
    }
}

hipError_t launch_prep(hipStream_t s, int phase, const Geometry& g, const float* x, const float* y,
                       const float* t_rel, const long long* offsets, const WinParam* wp, int B,
                       const int* blk_start, int nblk, int chunk, int* cnt_own, int* cnt_guest,
                       long long* seg_off, int* seg_own, unsigned long long* cursor, float4* ev,
                       int* err_flag) {
    if (phase == 0) {
        if (nblk > 0) {
            k_prep_count<<<nblk, kPrepThreads, 0, s>>>(g, x, y, t_rel, offsets, wp, B, blk_start, chunk,
                                                       cnt_own, cnt_guest, err_flag);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        k_prep_scan<<<1, 1024, 0, s>>>(B * g.T, cnt_own, cnt_guest, seg_off, seg_own, cursor);
        return hipGetLastError();
    }
    if (nblk > 0) {
        k_prep_scatter<<<nblk, kPrepThreads, 0, s>>>(g, x, y, t_rel, offsets, wp, B, blk_start, chunk,
                                                     cursor, ev);
        return hipGetLastError();
    }
    return hipSuccess;
}

// ------------------------------------------------------------ evaluation (a2, a3)

// Add one to every pixel of this tile that the staircase walk from pixel
// (kxa, kya) to pixel (kxb, kyb) visits (eq. (17)).  Corner decisions follow
// the event's ray through (x, y) with direction (ax, ay), in fp64; within
// 2^-8 px of a corner both side pixels are counted.  Pixels outside the
// tile increment the thread's private spill word `spill` instead, whose
// returned counts are removed at the end (see k_eval).
__device__ __forceinline__ void walk_tile(unsigned* __restrict__ tile, unsigned spill, int x0, int y0,
                                          unsigned tw, unsigned th, int kxa, int kya, int kxb, int kyb,
                                          double x, double y, double ax, double ay,
                                          unsigned long long& sumold, unsigned& visits) {
    const int sx = (kxb > kxa) - (kxb < kxa);
    const int sy = (kyb > kya) - (kyb < kya);
    const double thr = (fabs(ax) + fabs(ay)) * 0.00390625;
    const double aax = fabs(ax), aay = fabs(ay);
    int kx = kxa, ky = kya;
    auto visit = [&](int px, int py) {
        const unsigned lx = (unsigned)(px - x0), ly = (unsigned)(py - y0);
        const unsigned a = (lx < tw && ly < th) ? __umul24(ly, tw) + lx : spill;
        sumold += atomicAdd(&tile[a], 1u);
        visits += 1;
    };
    visit(kx, ky);
    while (kx != kxb || ky != kyb) {
        if (kx == kxb) {
            ky += sy;
        } else if (ky == kyb) {
            kx += sx;
        } else {
            double X = (double)(kx + (sx > 0));
            double Y = (double)(ky + (sy > 0));
            double ex = fabs(X - x) * aay;
            double ey = fabs(Y - y) * aax;
            double e = ex - ey;
            if (e < -thr) {
                kx += sx;
            } else if (e > thr) {
                ky += sy;
            } else {
                visit(kx + sx, ky);
                visit(kx, ky + sy);
                kx += sx;
                ky += sy;
            }
        }
        visit(kx, ky);
    }
}

// LDS layout of k_eval: [tile: tw*th counters][spill: one word per thread]
// [reduction scratch][work item].
constexpr int kEvalWaves = kEvalThreads / 64;

size_t eval_lds_bytes(int max_tile_px) {
    return (size_t)(max_tile_px + kEvalThreads) * 4 + 3 * kEvalWaves * 8 + 16;
}

// Persistent evaluation kernel: each workgroup takes (hypothesis, tile)
// items from the queue until it is empty.  For each item it clears its LDS
// tile, bins the tile's events (point: one increment per event, interval:
// one per pixel of the walk) with atomics that return the previous count,
// so the sum of squares is sum(2*old + 1) with no pass over the tile.
__global__ __launch_bounds__(kEvalThreads) void k_eval(
    Geometry g, const float4* __restrict__ ev, const long long* __restrict__ seg_off,
    const int* __restrict__ seg_own, const Hyp* __restrict__ hyps, const Item* __restrict__ items,
    Queue* __restrict__ q, Queue* __restrict__ q_reset, Part* __restrict__ part, int HS,
    unsigned* __restrict__ img_out) {
    extern __shared__ unsigned smem[];
    const int tid = threadIdx.x;
    unsigned* const tile = smem;
    unsigned long long* const s_red =
        reinterpret_cast<unsigned long long*>(smem + g.max_tile_px + kEvalThreads);
    int* const s_item = reinterpret_cast<int*>(s_red + 3 * kEvalWaves);
    if (blockIdx.x == 0 && tid == 0 && q_reset) {
        q_reset->n_items = 0;
        q_reset->next = 0;
    }
    const int n_items = q->n_items;
    const float Wf = (float)g.W, Hf = (float)g.H;
    for (;;) {
        if (tid == 0) *s_item = atomicAdd(&q->next, 1);
        __syncthreads();
        const int it = *s_item;
        __syncthreads();
        if (it >= n_items) break;
        const Item item = items[it];
        const int w = item.wh / HS, t = item.t;
        const Hyp hp = hyps[item.wh];
        const int tx = t % g.ntx, ty = t / g.ntx;
        const int x0 = g.colcut[tx], y0 = g.rowcut[ty];
        const unsigned tw = (unsigned)(g.colcut[tx + 1] - x0), th = (unsigned)(g.rowcut[ty + 1] - y0);
        const int npx = (int)(tw * th);
        const unsigned spill = (unsigned)npx + (unsigned)tid;  // this thread's private word
        const long long seg = (long long)w * g.T + t;
        const long long beg = seg_off[seg], end = seg_off[seg + 1];
        const long long own_end = beg + seg_own[seg];

        for (int i = tid; i < npx + kEvalThreads; i += kEvalThreads) tile[i] = 0u;
        __syncthreads();

        unsigned long long sumold = 0, nlow = 0;
        unsigned visits = 0;
        if (hp.kind == HYP_POINT) {
            // Point hypothesis (eqs. (12)-(13)): U events per thread in
            // flight, loads first, then U increments without branches.
            const float r = hp.ra;
            constexpr int U = 4;
            constexpr long long S = kEvalThreads;
            long long i = beg + tid;
            for (; i + (U - 1) * S < end; i += U * S) {
                float4 e[U];
#pragma unroll
                for (int k = 0; k < U; ++k) e[k] = ev[i + k * S];
                unsigned a[U];
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    const unsigned lx = (unsigned)(cvt_flr(fmaf(e[k].z, r, e[k].x)) - x0);
                    const unsigned ly = (unsigned)(cvt_flr(fmaf(e[k].w, r, e[k].y)) - y0);
                    a[k] = (lx < tw && ly < th) ? __umul24(ly, tw) + lx : spill;
                }
                unsigned old[U];
#pragma unroll
                for (int k = 0; k < U; ++k) old[k] = atomicAdd(&tile[a[k]], 1u);
#pragma unroll
                for (int k = 0; k < U; ++k) sumold += old[k];
                visits += U;
            }
            for (; i < end; i += S) {
                const float4 e = ev[i];
                const unsigned lx = (unsigned)(cvt_flr(fmaf(e.z, r, e.x)) - x0);
                const unsigned ly = (unsigned)(cvt_flr(fmaf(e.w, r, e.y)) - y0);
                const unsigned a = (lx < tw && ly < th) ? __umul24(ly, tw) + lx : spill;
                sumold += atomicAdd(&tile[a], 1u);
                visits += 1;
            }
        } else {
            // Interval hypothesis (eqs. (17)-(20)): endpoints, N_low, walk.
            const float ra = hp.ra, rb = hp.rb;
            long long i = beg + tid;
            float4 e = i < end ? ev[i] : make_float4(0.f, 0.f, 0.f, 0.f);
            for (; i < end; i += kEvalThreads) {
                const long long inext = i + kEvalThreads;
                const float4 en = inext < end ? ev[inext] : e;  // prefetch while walking
                const float xa = fmaf(e.z, ra, e.x), ya = fmaf(e.w, ra, e.y);
                const float xb = fmaf(e.z, rb, e.x), yb = fmaf(e.w, rb, e.y);
                if (i < own_end && inside(xa, ya, Wf, Hf) && inside(xb, yb, Wf, Hf)) nlow += 1;
                walk_tile(tile, spill, x0, y0, tw, th, flr_clamp(xa, g.W), flr_clamp(ya, g.H),
                          flr_clamp(xb, g.W), flr_clamp(yb, g.H), (double)e.x, (double)e.y, (double)e.z,
                          (double)e.w, sumold, visits);
                e = en;
            }
        }
        // Remove the spill word: its m increments returned 0, 1, .., m-1.
        const unsigned m = tile[spill];
        sumold -= (unsigned long long)m * (m - 1ull) / 2ull;
        unsigned long long hits = (unsigned long long)(visits - m);
        // block reduction of (sumold, hits, nlow)
        sumold = wave_sum(sumold);
        hits = wave_sum(hits);
        nlow = wave_sum(nlow);
        const int wave = tid >> 6, lane = tid & 63;
        if (lane == 0) {
            s_red[wave] = sumold;
            s_red[kEvalWaves + wave] = hits;
            s_red[2 * kEvalWaves + wave] = nlow;
        }
        __syncthreads();
        if (tid == 0) {
            unsigned long long a = 0, b = 0, c = 0;
            for (int k = 0; k < kEvalWaves; ++k) {
                a += s_red[k];
                b += s_red[kEvalWaves + k];
                c += s_red[2 * kEvalWaves + k];
            }
            Part pt;
            pt.S = 2ull * a + b;
            pt.N = (long long)(hp.kind == HYP_POINT ? b : c);
            pt.U = b;
            pt.pad = 0;
            part[(long long)item.wh * g.T + t] = pt;
        }
        if (img_out) {
            const long long M = (long long)g.W * g.H;
            for (int k = tid; k < npx; k += kEvalThreads) {
                int lx = k % (int)tw, ly = k / (int)tw;
                img_out[(long long)item.wh * M + (long long)(y0 + ly) * g.W + (x0 + lx)] = tile[k];
            }
        }
    }
}

hipError_t eval_occupancy(int* blocks_per_cu, size_t lds_bytes) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_eval, kEvalThreads, lds_bytes);
}

hipError_t eval_set_lds(size_t bytes) {
    return hipFuncSetAttribute((const void*)k_eval, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_eval(hipStream_t s, const Geometry& g, int nblocks, size_t lds_bytes, const float4* ev,
                       const long long* seg_off, const int* seg_own, const Hyp* hyps, const Item* items,
                       Queue* q, Queue* q_reset, Part* part, int HS, unsigned* img_out) {
    k_eval<<<nblocks, kEvalThreads, lds_bytes, s>>>(g, ev, seg_off, seg_own, hyps, items, q, q_reset, part,
                                                   HS, img_out);
    return hipGetLastError();
}

// ------------------------------------------------------------ frontier (a4)

// Hypothesis slots of the selected nodes and the work items for them.
__device__ void emit_hyps(const Search& sp, const WinParam& p, int w, int T, const long long* seg_off,
                          const Sel* sl, int n_sel, Hyp* hy, Item* items, Queue* qf) {
    const int F = sp.F, HS = sp.HS;
    __shared__ int s_n_nonempty, s_base;
    __shared__ int s_tiles[kMaxTiles];
    __shared__ int s_active[3 * 1024];  // slots with work (HS <= 3 * 1024)
    __shared__ int s_nact;
    if (threadIdx.x == 0) { s_n_nonempty = 0; s_nact = 0; }
    __syncthreads();
    for (int t = threadIdx.x; t < T; t += blockDim.x) {
        long long seg = (long long)w * T + t;
        if (seg_off[seg + 1] > seg_off[seg]) s_tiles[atomicAdd(&s_n_nonempty, 1)] = t;
    }
    for (int h = threadIdx.x; h < HS; h += blockDim.x) {
        Hyp hp;
        hp.kind = HYP_NONE;
        hp.pad = 0;
        hp.ra = hp.rb = 0.0f;
        if (h < F) {
            if (h < n_sel) {
                hp.kind = HYP_POINT;
                hp.ra = hp.rb = rate_of(grid_d(sp.d_lo, sp.d_hi, sp.L, sl[h].jc), p.tau);
            }
        } else {
            int c = h - F, i = c >> 1;
            if (i < n_sel && sl[i].kids) {
                unsigned a = (c & 1) ? sl[i].jc : sl[i].ja;
                unsigned b = (c & 1) ? sl[i].jb : sl[i].jc;
                hp.kind = HYP_INTERVAL;
                hp.ra = rate_of(grid_d(sp.d_lo, sp.d_hi, sp.L, a), p.tau);
                hp.rb = rate_of(grid_d(sp.d_lo, sp.d_hi, sp.L, b), p.tau);
            }
        }
        hy[h] = hp;
        if (hp.kind != HYP_NONE) s_active[atomicAdd(&s_nact, 1)] = h;
    }
    __syncthreads();
    const int nt = s_n_nonempty, na = s_nact;
    if (threadIdx.x == 0) s_base = (na * nt) ? atomicAdd(&qf->n_items, na * nt) : 0;
    __syncthreads();
    for (int k = threadIdx.x; k < na * nt; k += blockDim.x) {
        Item it;
        it.wh = w * HS + s_active[k / nt];
        it.t = s_tiles[k % nt];
        items[s_base + k] = it;
    }
    __syncthreads();
}

__global__ __launch_bounds__(kFrontThreads) void k_init(Search sp, const WinParam* __restrict__ wp,
                                                        const float* __restrict__ seeds, int B,
                                                        WinState* __restrict__ st, Sel* __restrict__ sel,
                                                        Hyp* __restrict__ hyps, Item* __restrict__ items,
                                                        Queue* __restrict__ q, int T,
                                                        const long long* __restrict__ seg_off) {
    const int w = blockIdx.x;
    const unsigned top = 1u << sp.L;
    Sel* sl = sel + (long long)w * sp.F;
    __shared__ int s_nsel;
    if (threadIdx.x == 0) {
        WinState s = WinState{};
        s.Kinc_hi = -1;
        s.Kinc_lo = ~0ull;  // K_inc = -1: the first evaluated point replaces it
        s.j_inc = 0;
        s.active = 1;
        Sel root;
        root.ja = 0;
        root.jb = top;
        root.jc = top >> 1;
        root.kids = (top >= 4) ? 1u : 0u;
        sl[0] = root;
        int n_sel = 1;
        if (seeds) {
            float d = seeds[w];
            if (isfinite(d)) {
                double span = (double)sp.d_hi - (double)sp.d_lo;
                double v = ((double)d - (double)sp.d_lo) / span * (double)top;
                long long j = llround(v);
                j = j < 1 ? 1 : (j > (long long)top - 1 ? (long long)top - 1 : j);
                if ((unsigned)j != root.jc && sp.F > 1) {
                    Sel sd;
                    sd.ja = sd.jb = sd.jc = (unsigned)j;
                    sd.kids = 0;
                    sl[1] = sd;
                    n_sel = 2;
                }
                s.seeded = 1;
            }
        }
        s.n_sel = n_sel;
        s.nodes_expanded = 1;
        st[w] = s;
        s_nsel = n_sel;
    }
    __syncthreads();
    emit_hyps(sp, wp[w], w, T, seg_off, sl, s_nsel, hyps + (long long)w * sp.HS, items, q);
}

hipError_t launch_init(hipStream_t s, const Search& sp, const WinParam* wp, const float* seeds, int B,
                       WinState* st, Sel* sel, Hyp* hyps, Item* items, Queue* q, int T,
                       const long long* seg_off) {
    if (B <= 0) return hipSuccess;
    k_init<<<B, kFrontThreads, 0, s>>>(sp, wp, seeds, B, st, sel, hyps, items, q, T, seg_off);
    return hipGetLastError();
}

__global__ __launch_bounds__(kFrontThreads) void k_frontier(
    Search sp, const WinParam* __restrict__ wp, int B, int T, const long long* __restrict__ seg_off,
    WinState* __restrict__ st, Node* __restrict__ front, Sel* __restrict__ sel, Hyp* __restrict__ hyps,
    const Part* __restrict__ part, Item* __restrict__ items, Queue* __restrict__ qf,
    int* __restrict__ n_active) {
    const int w = blockIdx.x, tid = threadIdx.x;
    constexpr int NT = kFrontThreads;
    __shared__ WinState s;
    __shared__ long long s_khi[NT];
    __shared__ unsigned long long s_klo[NT];
    __shared__ unsigned s_j[NT];
    __shared__ int s_cnt, s_overflow, s_hist[130], s_quota_ctr, s_nsel_new, s_kids_new, s_out;
    __shared__ unsigned long long s_pix;
    __shared__ long long s_pruned, s_nbound;
    __shared__ int s_scan[NT];
    __shared__ int s_bstar, s_quota, s_stop;
    if (tid == 0) s = st[w];
    __syncthreads();
    if (!s.active) return;
    const int F = sp.F, HS = sp.HS, CAP = sp.CAP;
    const long long M = sp.M;
    const WinParam p = wp[w];
    Node* fr = front + (long long)w * CAP;
    Sel* sl = sel + (long long)w * F;
    const Part* pw = part + (long long)w * HS * T;
    const long long* so = seg_off + (long long)w * T;

    // (1) centre points: lexicographic max of (K, -j) with the incumbent
    i128 bK = mk128(s.Kinc_hi, s.Kinc_lo);
    unsigned bJ = s.j_inc;
    for (int i = tid; i < s.n_sel; i += NT) {
        unsigned long long S = 0;
        long long N = 0;
        for (int t = 0; t < T; ++t) {
            if (so[t + 1] > so[t]) {
                S += pw[(long long)i * T + t].S;
                N += pw[(long long)i * T + t].N;
            }
        }
        i128 K = (i128)M * (i128)S - (i128)N * (i128)N;
        unsigned jc = sl[i].jc;
        if (K > bK || (K == bK && jc < bJ)) { bK = K; bJ = jc; }
    }
    sp128(bK, s_khi[tid], s_klo[tid]);
    s_j[tid] = bJ;
    if (tid == 0) {
        s_cnt = s.n_front;
        s_overflow = 0;
        s_pix = 0;
        s_pruned = 0;
        s_nbound = 0;
        s_quota_ctr = 0;
        s_nsel_new = 0;
        s_kids_new = 0;
        s_stop = 0;
    }
    for (int b = tid; b < 130; b += NT) s_hist[b] = 0;
    __syncthreads();
    if (tid == 0) {
        i128 K0 = mk128(s_khi[0], s_klo[0]);
        unsigned j0 = s_j[0];
        for (int k = 1; k < NT; ++k) {
            i128 K = mk128(s_khi[k], s_klo[k]);
            if (K > K0 || (K == K0 && s_j[k] < j0)) { K0 = K; j0 = s_j[k]; }
        }
        sp128(K0, s.Kinc_hi, s.Kinc_lo);
        s.j_inc = j0;
        s.point_evals += s.n_sel;
        s.event_hyp += (long long)s.n_sel * p.n_events;
    }
    __syncthreads();
    const i128 Kinc = mk128(s.Kinc_hi, s.Kinc_lo);
    const unsigned jinc = s.j_inc;

    // (2) children of the expanded nodes: bound key, insert if improvable
    for (int c = tid; c < 2 * s.n_sel; c += NT) {
        const int i = c >> 1;
        if (!sl[i].kids) continue;
        unsigned long long S = 0, U = 0;
        long long N = 0;
        for (int t = 0; t < T; ++t) {
            if (so[t + 1] > so[t]) {
                const Part& q = pw[(long long)(F + c) * T + t];
                S += q.S;
                N += q.N;
                U += q.U;
            }
        }
        atomicAdd(&s_pix, U);
        atomicAdd((unsigned long long*)&s_nbound, 1ull);
        i128 Kb = (i128)M * (i128)S - (i128)N * (i128)N;
        unsigned ja = (c & 1) ? sl[i].jc : sl[i].ja;
        unsigned jb = (c & 1) ? sl[i].jb : sl[i].jc;
        if (improvable(Kb, ja, Kinc, jinc)) {
            int pos = atomicAdd(&s_cnt, 1);
            if (pos < CAP) {
                Node nd;
                sp128(Kb, nd.khi, nd.klo);
                nd.ja = ja;
                nd.jb = jb;
                fr[pos] = nd;
            } else {
                s_overflow = 1;
            }
        } else {
            atomicAdd((unsigned long long*)&s_pruned, 1ull);
        }
    }
    __syncthreads();
    if (tid == 0) {
        s.bound_evals += s_nbound;
        s.event_hyp += s_nbound * p.n_events;
        s.pixel_updates += (long long)s_pix;
        s.nodes_pruned += s_pruned;
    }
    const int n = min(s_cnt, CAP);

    // (3) which queued nodes can still improve; histogram of their gap sizes
    long long my_gap_hi = -1;
    unsigned long long my_gap_lo = 0;
    i128 best_gap = -1;
    for (int i = tid; i < n; i += NT) {
        Node nd = fr[i];
        i128 k = mk128(nd.khi, nd.klo);
        if (improvable(k, nd.ja, Kinc, jinc)) {
            i128 gap = k - Kinc;
            atomicAdd(&s_hist[bitlen128(gap)], 1);
            if (gap > best_gap) best_gap = gap;
        }
    }
    sp128(best_gap, my_gap_hi, my_gap_lo);
    s_khi[tid] = my_gap_hi;
    s_klo[tid] = my_gap_lo;
    __syncthreads();
    if (tid == 0) {
        i128 g = -1;
        for (int k = 0; k < NT; ++k) {
            i128 v = mk128(s_khi[k], s_klo[k]);
            if (v > g) g = v;
        }
        int n_keep = 0;
        for (int b = 0; b < 130; ++b) n_keep += s_hist[b];
        int stop = 0;
        if (s_overflow) {
            s.status = -5;  // ECMD_EFRONTIER
            sp128((i128)-1, s.gap_hi, s.gap_lo);
            stop = 1;
        } else if (n_keep == 0) {
            s.status = 0;
            s.gap_hi = 0;
            s.gap_lo = 0;
            stop = 1;
        } else if (sp.gamma_key >= 0 && g <= (i128)sp.gamma_key) {
            s.status = 0;
            sp128(g, s.gap_hi, s.gap_lo);
            s.nodes_pruned += n_keep;
            stop = 1;
        }
        int take = min(F, n_keep);
        if (!stop && sp.max_nodes > 0) {
            long long left = sp.max_nodes - s.nodes_expanded;
            if (left <= 0) {
                s.status = -4;  // ECMD_EBUDGET
                sp128(g, s.gap_hi, s.gap_lo);
                stop = 1;
            } else if (left < take) {
                take = (int)left;
            }
        }
        // threshold bucket: take every node of a larger gap class, and
        // `quota` of the class b*
        int cum = 0, bstar = 0, quota = 0;
        if (!stop) {
            for (int b = 129; b >= 0; --b) {
                if (cum + s_hist[b] >= take) { bstar = b; quota = take - cum; break; }
                cum += s_hist[b];
            }
        }
        s_bstar = bstar;
        s_quota = quota;
        s_stop = stop;
        s_out = 0;
    }
    __syncthreads();
    if (s_stop) {
        if (tid == 0) {
            s.active = 0;
            s.n_sel = 0;
            s.n_front = 0;
            st[w] = s;
            atomicSub(n_active, 1);
        }
        return;
    }

    // (4) split the queue into the nodes expanded now and the rest (in place)
    for (int base = 0; base < n; base += NT) {
        const int i = base + tid;
        Node nd;
        int keep = 0, take = 0;
        if (i < n) {
            nd = fr[i];
            i128 k = mk128(nd.khi, nd.klo);
            if (improvable(k, nd.ja, Kinc, jinc)) {
                int b = bitlen128(k - Kinc);
                if (b > s_bstar) take = 1;
                else if (b == s_bstar && atomicAdd(&s_quota_ctr, 1) < s_quota) take = 1;
                else keep = 1;
            }
        }
        s_scan[tid] = keep;
        __syncthreads();
        for (int o = 1; o < NT; o <<= 1) {
            int a = tid >= o ? s_scan[tid - o] : 0;
            __syncthreads();
            s_scan[tid] += a;
            __syncthreads();
        }
        const int out0 = s_out;
        if (keep) fr[out0 + s_scan[tid] - 1] = nd;
        if (take) {
            int k = atomicAdd(&s_nsel_new, 1);
            Sel x;
            x.ja = nd.ja;
            x.jb = nd.jb;
            x.jc = (nd.ja + nd.jb) >> 1;
            x.kids = (nd.jb - nd.ja >= 4) ? 1u : 0u;
            sl[k] = x;
        }
        __syncthreads();
        if (tid == NT - 1) s_out = out0 + s_scan[NT - 1];
        __syncthreads();
    }
    if (tid == 0) {
        s.n_front = s_out;
        s.n_sel = s_nsel_new;
        s.nodes_expanded += s_nsel_new;
        s.steps += 1;
        st[w] = s;
    }
    __syncthreads();
    emit_hyps(sp, p, w, T, seg_off, sl, s_nsel_new, hyps + (long long)w * HS, items, qf);
}

hipError_t launch_frontier(hipStream_t s, const Search& sp, const WinParam* wp, int B, int T,
                           const long long* seg_off, WinState* st, Node* front, Sel* sel, Hyp* hyps,
                           const Part* part, Item* items, Queue* q_fill, int* n_active) {
    if (B <= 0) return hipSuccess;
    k_frontier<<<B, kFrontThreads, 0, s>>>(sp, wp, B, T, seg_off, st, front, sel, hyps, part, items, q_fill,
                                          n_active);
    return hipGetLastError();
}

// ------------------------------------------------------------ probes

__global__ void k_rates(const float* __restrict__ d_a, const float* __restrict__ d_b, int m, float tau,
                        Hyp* __restrict__ hyps) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    Hyp h;
    h.ra = rate_of(d_a[k], tau);
    h.rb = d_b ? rate_of(d_b[k], tau) : h.ra;
    h.kind = d_b ? HYP_INTERVAL : HYP_POINT;
    h.pad = 0;
    hyps[k] = h;
}

hipError_t launch_rates(hipStream_t s, const float* d_a, const float* d_b, int m, float tau, Hyp* hyps) {
    if (m <= 0) return hipSuccess;
    k_rates<<<(m + 255) / 256, 256, 0, s>>>(d_a, d_b, m, tau, hyps);
    return hipGetLastError();
}

__global__ void k_probe_pixels(const float* __restrict__ x, const float* __restrict__ y,
                               const float* __restrict__ t_rel, long long n, float tau, float d, int W,
                               int H, float cx, float cy, int* __restrict__ pix) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float r = rate_of(d, tau);
    float ax = (x[i] - cx) * (tau - t_rel[i]);
    float ay = (y[i] - cy) * (tau - t_rel[i]);
    float xw = fmaf(ax, r, x[i]), yw = fmaf(ay, r, y[i]);
    pix[i] = inside(xw, yw, (float)W, (float)H) ? (int)floorf(yw) * W + (int)floorf(xw) : -1;
}

hipError_t launch_probe_pixels(hipStream_t s, const float* x, const float* y, const float* t_rel, long long n,
                               float tau, float d, int W, int H, float cx, float cy, int* pix) {
    if (n <= 0) return hipSuccess;
    k_probe_pixels<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, y, t_rel, n, tau, d, W, H, cx, cy, pix);
    return hipGetLastError();
}

// ------------------------------------------------------------ window selection

constexpr int kSelThreads = 1024;

__global__ __launch_bounds__(kSelThreads) void k_select_count(const double* __restrict__ t, long long n, double t0,
                                                              double t1, int* __restrict__ blk_cnt) {
    __shared__ int s_n;
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    long long i = (long long)blockIdx.x * kSelThreads + threadIdx.x;
    if (i < n && t[i] >= t0 && t[i] <= t1) atomicAdd(&s_n, 1);
    __syncthreads();
    if (threadIdx.x == 0) blk_cnt[blockIdx.x] = s_n;
}

__global__ __launch_bounds__(1024) void k_select_scan(int nb, int* __restrict__ blk_cnt, long long* __restrict__ total) {
    __shared__ long long s[1024];
    __shared__ long long carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nb; base += 1024) {
        int k = base + threadIdx.x;
        long long v = k < nb ? blk_cnt[k] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            long long a = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
            __syncthreads();
            s[threadIdx.x] += a;
            __syncthreads();
        }
        long long incl = s[threadIdx.x] + carry;
        if (k < nb) blk_cnt[k] = (int)(incl - v);
        __syncthreads();
        if (threadIdx.x == 1023) carry = incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kSelThreads) void k_select_write(const float* __restrict__ x, const float* __restrict__ y,
                                                              const double* __restrict__ t, long long n, double t0,
                                                              double t1, const int* __restrict__ blk_off,
                                                              float* __restrict__ xo, float* __restrict__ yo,
                                                              float* __restrict__ to) {
    __shared__ int s[kSelThreads];
    long long i = (long long)blockIdx.x * kSelThreads + threadIdx.x;
    int keep = (i < n && t[i] >= t0 && t[i] <= t1) ? 1 : 0;
    s[threadIdx.x] = keep;
    __syncthreads();
    for (int o = 1; o < kSelThreads; o <<= 1) {
        int a = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
        __syncthreads();
        s[threadIdx.x] += a;
        __syncthreads();
    }
    if (keep) {
        long long k = (long long)blk_off[blockIdx.x] + s[threadIdx.x] - 1;
        xo[k] = x[i];
        yo[k] = y[i];
        to[k] = (float)(t[i] - t0);
    }
}

hipError_t launch_select(hipStream_t s, const float* x, const float* y, const double* t, long long n, double t0,
                         double t1, float* xo, float* yo, float* to, int* blk_cnt, long long* total) {
    const int nb = (int)((n + kSelThreads - 1) / kSelThreads);
    if (nb > 0) {
        k_select_count<<<nb, kSelThreads, 0, s>>>(t, n, t0, t1, blk_cnt);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    k_select_scan<<<1, 1024, 0, s>>>(nb, blk_cnt, total);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nb == 0) return e;
    k_select_write<<<nb, kSelThreads, 0, s>>>(x, y, t, n, t0, t1, blk_cnt, xo, yo, to);
    return hipGetLastError();
}

// ------------------------------------------------------------ learned-incumbent input

__device__ __forceinline__ uint16_t bf16_rne(float v) {
    unsigned u = __float_as_uint(v);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

constexpr int kGrid = 64;

__global__ __launch_bounds__(256) void k_downsample_count(const float* __restrict__ x,
                                                          const float* __restrict__ y,
                                                          const long long* __restrict__ offsets, int B,
                                                          int W, int H, const int* __restrict__ blk_start,
                                                          int chunk, unsigned* __restrict__ counts) {
    __shared__ unsigned s_cnt[kGrid * kGrid];
    for (int k = threadIdx.x; k < kGrid * kGrid; k += blockDim.x) s_cnt[k] = 0;
    __syncthreads();
    const int w = window_of_block(blk_start, B, blockIdx.x);
    const int c = blockIdx.x - blk_start[w];
    const long long beg = offsets[w] + (long long)c * chunk;
    const long long end = min(beg + chunk, offsets[w + 1]);
    const float Wf = (float)W, Hf = (float)H, G = (float)kGrid;
    for (long long i = beg + threadIdx.x; i < end; i += blockDim.x) {
        int bx = (int)floorf((x[i] * G) / Wf);
        int by = (int)floorf((y[i] * G) / Hf);
        bx = min(max(bx, 0), kGrid - 1);
        by = min(max(by, 0), kGrid - 1);
        atomicAdd(&s_cnt[by * kGrid + bx], 1u);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kGrid * kGrid; k += blockDim.x)
        if (s_cnt[k]) atomicAdd(&counts[(long long)w * kGrid * kGrid + k], s_cnt[k]);
}

__global__ void k_downsample_finish(const unsigned* __restrict__ counts, const long long* __restrict__ offsets,
                                    int B, uint16_t* __restrict__ out) {
    const int w = blockIdx.x;
    const long long n = offsets[w + 1] - offsets[w];
    const float scale = n > 0 ? (float)(kGrid * kGrid) / (float)n : 0.0f;
    for (int k = threadIdx.x; k < kGrid * kGrid; k += blockDim.x)
        out[(long long)w * kGrid * kGrid + k] = bf16_rne((float)counts[(long long)w * kGrid * kGrid + k] * scale);
}

hipError_t launch_downsample(hipStream_t s, const float* x, const float* y, const long long* offsets, int B,
                             int W, int H, const int* blk_start, int nblk, int chunk, unsigned* counts,
                             uint16_t* out) {
    if (B <= 0) return hipSuccess;
    if (nblk > 0) {
        k_downsample_count<<<nblk, 256, 0, s>>>(x, y, offsets, B, W, H, blk_start, chunk, counts);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    k_downsample_finish<<<B, 256, 0, s>>>(counts, offsets, B, out);
    return hipGetLastError();
}

}  // namespace ecmd
