// HIP kernels of the MI355X divergence estimator (gfx950).
//
// Method: arXiv 2209.13168 -- radial warp eq. (12), event image eq. (13),
// contrast eq. (14), upper bound eqs. (15)-(20), branch and bound Alg. 1.
// Built with -ffp-contract=off: every fp32/fp64 operation below rounds
// exactly as written (the readings are listed in include/ecmd.h).
#include <hip/hip_ext.h>

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
    return cvt_flr(__builtin_amdgcn_fmed3f(v, -1.0f, (float)hi));
}

__device__ __forceinline__ unsigned umax(unsigned a, unsigned b) { return a > b ? a : b; }

__device__ __forceinline__ i128 mk128(long long hi, unsigned long long lo) {
    unsigned __int128 u = ((unsigned __int128)(unsigned long long)hi << 64) | (unsigned __int128)lo;
    return (i128)u;
}

__device__ __forceinline__ void sp128(i128 v, long long& hi, unsigned long long& lo) {
    unsigned __int128 u = (unsigned __int128)v;
    lo = (unsigned long long)u;
    hi = (long long)(unsigned long long)(u >> 64);
}

// Correctly rounded conversion of a 128-bit integer to double: the top 64
// significant bits, with a sticky bit for any below them, are converted
// (one rounding) and scaled by a power of two (exact).
__device__ __forceinline__ double i128_to_double(i128 v) {
    const bool neg = v < 0;
    const unsigned __int128 u = neg ? (unsigned __int128)0 - (unsigned __int128)v : (unsigned __int128)v;
    const unsigned long long hi = (unsigned long long)(u >> 64);
    double r;
    if (hi == 0) {
        r = (double)(unsigned long long)u;
    } else {
        const int sh = 64 - __clzll(hi);
        unsigned long long top = (unsigned long long)(u >> sh);
        top |= (u & ((((unsigned __int128)1) << sh) - 1)) != 0 ? 1ull : 0ull;
        r = ldexp((double)top, sh);
    }
    return neg ? -r : r;
}

// A float no smaller than v >= 0 (the double is within 2^-53 of v, the
// float within 2^-24 of the double, the factor covers both).
__device__ __forceinline__ float ub_float(i128 v) { return (float)(i128_to_double(v) * (1.0 + 0x1p-20)); }

// The smallest integer no smaller than the finite f >= 0.
__device__ __forceinline__ i128 ceil_i128(float f) {
    int e;
    const float m = frexpf(f, &e);  // f = m 2^e, m in [0.5, 1)
    const long long mi = (long long)ldexpf(m, 24);  // f = mi 2^(e - 24) exactly
    const int sh = e - 24;
    if (sh >= 0) return (i128)mi << sh;
    if (sh < -24) return mi > 0 ? (i128)1 : (i128)0;
    return ((i128)mi + (((i128)1 << -sh) - 1)) >> -sh;
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

// One step of a DPP wave reduction of a 64-bit value: add the value that
// DPP control CTRL routes to this lane (rows outside ROWMASK add zero).
template <int CTRL, int ROWMASK>
__device__ __forceinline__ unsigned long long dpp_add(unsigned long long v) {
    const unsigned lo = __builtin_amdgcn_update_dpp(0u, (unsigned)v, CTRL, ROWMASK, 0xf, false);
    const unsigned hi = __builtin_amdgcn_update_dpp(0u, (unsigned)(v >> 32), CTRL, ROWMASK, 0xf, false);
    return v + (((unsigned long long)hi << 32) | lo);
}

// The same for a 32-bit value whose wave total fits 32 bits.
__device__ __forceinline__ unsigned wave_total32(unsigned v) {
    v += __builtin_amdgcn_update_dpp(0u, v, 0xB1, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0u, v, 0x4E, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0u, v, 0x141, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0u, v, 0x140, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0u, v, 0x142, 0xa, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0u, v, 0x143, 0xc, 0xf, false);
    return v;
}

// Sum over the 64 lanes of a wave in registers (no LDS): quad swaps, half-row
// and row mirrors give every lane its row's sum; the two row broadcasts then
// carry rows 0-2 into row 3.  The total is valid in lane 63 (all lanes active).
__device__ __forceinline__ unsigned long long wave_total(unsigned long long v) {
    v = dpp_add<0xB1, 0xf>(v);   // quad_perm [1,0,3,2]
    v = dpp_add<0x4E, 0xf>(v);   // quad_perm [2,3,0,1]
    v = dpp_add<0x141, 0xf>(v);  // row_half_mirror
    v = dpp_add<0x140, 0xf>(v);  // row_mirror
    v = dpp_add<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_add<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// ------------------------------------------------------------ window params

// Walk-length classes: inside a tile segment, events are ordered by
// |ax| + |ay| (longest first).  For any interval an event's staircase walk
// is about (|ax| + |ay|)(r_b - r_a) pixels long, so neighbouring lanes of a
// wave then walk similar distances.
constexpr int kNB = 16;
// Guests keep half as many walk classes (kNB / 2 per guest bin).
constexpr int kNG = kNB / 2;
// Prep counters of one tile segment: owned by walk class, then guests by
// bin and walk class, so a segment holds its owned events first and its
// guest bins in increasing order.
constexpr int kTC = kNB + kGuestBins * kNG;

// Guest bin cuts of a window, uniform over its binning range [r_lo, r_hi]
// and non-decreasing whatever the rounding.
__device__ __forceinline__ void set_guest_cuts(WinParam& p) {
    const float span = p.r_hi - p.r_lo;
    float prev = p.r_lo;
    for (int m = 1; m < kGuestBins; ++m) {
        prev = fmaxf(prev, fmaf((float)m * (1.0f / kGuestBins), span, p.r_lo));
        p.gcut[m - 1] = prev;
    }
}

__global__ void k_winparam(const float* __restrict__ tau, const long long* __restrict__ offsets, int B,
                           float d_lo, float d_hi, int W, int H, float cx, float cy, WinParam* __restrict__ wp) {
    int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= B) return;
    WinParam p;
    p.tau = tau[w];
    p.r_lo = rate_of(d_lo, p.tau);
    p.r_hi = rate_of(d_hi, p.tau);
    const float key_max = (fmaxf(fabsf(cx), fabsf((float)W - cx)) + fmaxf(fabsf(cy), fabsf((float)H - cy))) * p.tau;
    p.kscale = key_max > 0.0f ? (float)kNB / key_max : 0.0f;
    p.n_events = offsets[w + 1] - offsets[w];
    set_guest_cuts(p);
    wp[w] = p;
}

hipError_t launch_winparam(hipStream_t s, const Geometry& g, const float* tau, const long long* offsets, int B,
                           float d_lo, float d_hi, WinParam* wp) {
    if (B <= 0) return hipSuccess;
    k_winparam<<<(B + 255) / 256, 256, 0, s>>>(tau, offsets, B, d_lo, d_hi, g.W, g.H, g.cx, g.cy, wp);
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
    // the cuts increase: the band is the count of inner cuts at or below k
    // (every lane runs the same loop, so the cuts are read as scalars)
    int b = 0;
    for (int j = 1; j < n; ++j) b += cut[j] <= k ? 1 : 0;
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

__device__ __forceinline__ int walk_class(float ax, float ay, float kscale) {
    int b = (int)((fabsf(ax) + fabsf(ay)) * kscale);
    return kNB - 1 - min(max(b, 0), kNB - 1);
}

// counters of an owned event and of a guest copy in bin m, inside a window
__device__ __forceinline__ int ctr_own(int t, int b) { return t * kTC + b; }
__device__ __forceinline__ int ctr_guest(int t, int m, int b) { return t * kTC + kNB + m * kNG + (b >> 1); }

// Cuts at which one coordinate of an event, warped by the evaluation's own
// fmaf (v + a r), is still short of the edge e of a band, e being the edge
// the coordinate moves towards as the rate grows (the lower one for a >= 0).
// The test is monotone in the rate, so the cuts at which it holds come
// first.  A guest copy's bin is the larger of its two coordinates' counts:
// the event has not reached the tile while either coordinate is short, and
// the union of two leading runs of cuts is the longer one.  A bin-m copy
// evaluated at rates that are all at most gcut[m - 1] lies outside the tile
// at both ends, on the same side, and adds only to the tile's border.
__device__ __forceinline__ int cuts_short(const WinParam& p, float v, float a, float e) {
    const bool neg = a < 0.0f;
    int m = 0;
#pragma unroll
    for (int k = 0; k < kGuestBins - 1; ++k) m += ((fmaf(a, p.gcut[k], v) < e) != neg) ? 1 : 0;
    return m;
}

// Band edges of the tile grid as floats, in LDS for the prep blocks.
struct PrepCuts {
    float col[kMaxTiles + 1], row[kMaxTiles + 1];
};

__device__ __forceinline__ void load_cuts(const Geometry& g, PrepCuts& c) {
    for (int k = threadIdx.x; k <= g.ntx; k += blockDim.x) c.col[k] = (float)g.colcut[k];
    for (int k = threadIdx.x; k <= g.nty; k += blockDim.x) c.row[k] = (float)g.rowcut[k];
}

// First segment of event i's image: the polarity-aware contrast keeps one
// event image per polarity (p > 0: the second), each tiled alike.
__device__ __forceinline__ int seg_base(const Geometry& g, const signed char* pol, long long i) {
    return (pol && pol[i] > 0) ? g.nsp : 0;
}

constexpr int kPrepThreads = 256;

// Counter of every copy of a prepared event (segment base sb), in the
// same order for the counting and the scattering passes.  The event's own
// copy (the one N_low and the certificates read) goes to the tile it
// starts in, at the low end of the binning range: the corner of its tile
// rectangle it moves away from.  Every other tile is a guest, reached at
// higher rates only.
template <class F>
__device__ __forceinline__ void for_each_copy(const Geometry& g, const WinParam& p, const PrepCuts& c, int sb,
                                              float x, float y, float ax, float ay, int tx0, int tx1, int ty0,
                                              int ty1, int cls, F&& f) {
    const int ox = ax < 0.0f ? tx1 : tx0, oy = ay < 0.0f ? ty1 : ty0;
    for (int ty = ty0; ty <= ty1; ++ty) {
        const int by = cuts_short(p, y, ay, c.row[ay < 0.0f ? ty + 1 : ty]);
        for (int tx = tx0; tx <= tx1; ++tx) {
            const int t = sb + ty * g.ntx + tx;
            if (ty == oy && tx == ox) {
                f(ctr_own(t, cls));
            } else {
                const int bx = cuts_short(p, x, ax, c.col[ax < 0.0f ? tx + 1 : tx]);
                f(ctr_guest(t, max(bx, by), cls));
            }
        }
    }
}

// Per-event prep: validity, (ax, ay), reachable tiles and walk class.
struct PrepEv {
    bool ok, valid;
    float x, y, ax, ay;
    int tx0, tx1, ty0, ty1, cls;
};

__device__ __forceinline__ PrepEv prep_event(const Geometry& g, const WinParam& p, float xv, float yv, float tv) {
    PrepEv e;
    e.valid = isfinite(xv) && isfinite(yv) && tv >= 0.0f && tv <= p.tau;
    e.ok = false;
    if (!e.valid) return e;
    const float ux = xv - g.cx, uy = yv - g.cy, delta = p.tau - tv;
    e.x = xv;
    e.y = yv;
    e.ax = ux * delta;
    e.ay = uy * delta;
    e.ok = event_tiles(g, xv, yv, e.ax, e.ay, p.r_lo, p.r_hi, e.tx0, e.tx1, e.ty0, e.ty1);
    e.cls = walk_class(e.ax, e.ay, p.kscale);
    return e;
}

__global__ __launch_bounds__(kPrepThreads) void k_prep_count(
    Geometry g, const float* __restrict__ x, const float* __restrict__ y, const float* __restrict__ t_rel,
    const signed char* __restrict__ pol, const long long* __restrict__ offsets, const WinParam* __restrict__ wp, int B,
    const int* __restrict__ blk_start, int chunk, int* __restrict__ cnt, int* __restrict__ err_flag) {
    extern __shared__ int s_cnt[];  // g.T * kTC counters
    __shared__ PrepCuts s_cuts;
    if ((int)blockIdx.x >= blk_start[B]) return;  // a grid sized for the largest batch
    const int nc = g.T * kTC;
    for (int k = threadIdx.x; k < nc; k += blockDim.x) s_cnt[k] = 0;
    load_cuts(g, s_cuts);
    __syncthreads();
    const int w = window_of_block(blk_start, B, blockIdx.x);
    const int c = blockIdx.x - blk_start[w];
    const long long beg = offsets[w] + (long long)c * chunk;
    const long long end = min(beg + chunk, offsets[w + 1]);
    const WinParam p = wp[w];
    for (long long i = beg + threadIdx.x; i < end; i += blockDim.x) {
        const PrepEv e = prep_event(g, p, x[i], y[i], t_rel[i]);
        if (!e.valid) atomicOr(&err_flag[w], 1);
        if (!e.ok) continue;
        for_each_copy(g, p, s_cuts, seg_base(g, pol, i), e.x, e.y, e.ax, e.ay, e.tx0, e.tx1, e.ty0, e.ty1, e.cls,
                      [&](int k) { atomicAdd(&s_cnt[k], 1); });
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nc; k += blockDim.x)
        if (s_cnt[k]) atomicAdd(&cnt[(long long)w * nc + k], s_cnt[k]);
}

// Exclusive scan of the counters of every (window, tile, owned/guest bin,
// class) in that order (one workgroup: a prefix sum inside each wave, the
// wave totals through LDS, 1024 counters per round); then the segment of
// (w, t) starts at its first counter, its owned events end where its first
// guest bin begins, and guest bin m ends where bin m + 1 (or the next
// segment) begins.
__global__ __launch_bounds__(1024) void k_prep_scan(int B, int T, const int* __restrict__ cnt,
                                                    long long* __restrict__ seg_off, int* __restrict__ seg_own,
                                                    unsigned long long* __restrict__ cursor) {
    __shared__ long long s_wave[16];
    __shared__ long long s_carry;
    const long long n = (long long)B * T * kTC;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (threadIdx.x == 0) s_carry = 0;
    for (long long base = 0; base < n; base += 1024) {
        const long long k = base + threadIdx.x;
        const long long v = k < n ? cnt[k] : 0;
        long long incl = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const long long a = __shfl_up(incl, o, 64);
            if (lane >= o) incl += a;
        }
        if (lane == 63) s_wave[wv] = incl;
        __syncthreads();  // the wave totals and the last round's carry are visible
        long long pre = s_carry;
        for (int j = 0; j < wv; ++j) pre += s_wave[j];
        if (k < n) cursor[k] = (unsigned long long)(pre + incl - v);
        __syncthreads();  // every read of s_wave and s_carry is done
        if (threadIdx.x == 1023) s_carry = pre + incl;
    }
    __syncthreads();  // the total and every cursor are visible
    const long long total = s_carry;
    const auto start = [&](long long k) { return k < n ? (long long)cursor[k] : total; };
    for (int st = threadIdx.x; st < B * T; st += 1024) {
        const long long c0 = (long long)st * kTC;
        const long long o0 = start(c0);
        seg_off[st] = o0;
        int* const so = seg_own + (long long)st * (kGuestBins + 1);
        so[0] = (int)(start(c0 + kNB) - o0);
        for (int m = 0; m < kGuestBins; ++m) so[1 + m] = (int)(start(c0 + kNB + (m + 1) * kNG) - o0);
    }
    if (threadIdx.x == 0) seg_off[(long long)B * T] = total;
}

__global__ __launch_bounds__(kPrepThreads) void k_prep_scatter(
    Geometry g, const float* __restrict__ x, const float* __restrict__ y, const float* __restrict__ t_rel,
    const signed char* __restrict__ pol, const long long* __restrict__ offsets, const WinParam* __restrict__ wp, int B,
    const int* __restrict__ blk_start, int chunk, unsigned long long* __restrict__ cursor,
    const long long* __restrict__ total, long long cap, float4* __restrict__ ev) {
    extern __shared__ unsigned long long s_prep[];  // g.T * kTC bases, then as many counts
    const int nc = g.T * kTC;
    unsigned long long* const s_base = s_prep;
    int* const s_cnt = reinterpret_cast<int*>(s_prep + nc);
    __shared__ PrepCuts s_cuts;
    if ((int)blockIdx.x >= blk_start[B]) return;
    if (total && *total > cap) return;  // the records would not fit the store: nothing is written
    load_cuts(g, s_cuts);
    for (int k = threadIdx.x; k < nc; k += blockDim.x) s_cnt[k] = 0;
    __syncthreads();
    const int w = window_of_block(blk_start, B, blockIdx.x);
    const int c = blockIdx.x - blk_start[w];
    const long long beg = offsets[w] + (long long)c * chunk;
    const long long end = min(beg + chunk, offsets[w + 1]);
    const WinParam p = wp[w];
    for (long long i = beg + threadIdx.x; i < end; i += blockDim.x) {
        const PrepEv e = prep_event(g, p, x[i], y[i], t_rel[i]);
        if (!e.ok) continue;
        for_each_copy(g, p, s_cuts, seg_base(g, pol, i), e.x, e.y, e.ax, e.ay, e.tx0, e.tx1, e.ty0, e.ty1, e.cls,
                      [&](int k) { atomicAdd(&s_cnt[k], 1); });
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nc; k += blockDim.x) {
        const int n = s_cnt[k];
        s_base[k] = n ? atomicAdd(&cursor[(long long)w * nc + k], (unsigned long long)n) : 0ull;
        s_cnt[k] = 0;
    }
    __syncthreads();
    for (long long i = beg + threadIdx.x; i < end; i += blockDim.x) {
        const PrepEv e = prep_event(g, p, x[i], y[i], t_rel[i]);
        if (!e.ok) continue;
        const float4 v = make_float4(e.x, e.y, e.ax, e.ay);
        for_each_copy(g, p, s_cuts, seg_base(g, pol, i), e.x, e.y, e.ax, e.ay, e.tx0, e.tx1, e.ty0, e.ty1, e.cls,
                      [&](int k) {
                          const int r = atomicAdd(&s_cnt[k], 1);
                          ev[s_base[k] + (unsigned long long)r] = v;
                      });
    }
}

size_t prep_counters(int B, int T) { return (size_t)B * T * kTC; }
size_t seg_own_words(int B, int T) { return (size_t)B * T * (kGuestBins + 1); }

hipError_t launch_prep(hipStream_t s, int phase, const Geometry& g, const float* x, const float* y,
                       const float* t_rel, const signed char* pol, const long long* offsets, const WinParam* wp, int B,
                       const int* blk_start, int nblk, int chunk, int* cnt, long long* seg_off, int* seg_own,
                       unsigned long long* cursor, float4* ev, int* err_flag, long long cap) {
    if (phase == 0) {
        if (nblk > 0) {
            k_prep_count<<<nblk, kPrepThreads, sizeof(int) * g.T * kTC, s>>>(g, x, y, t_rel, pol, offsets, wp, B,
                                                                             blk_start, chunk, cnt, err_flag);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        k_prep_scan<<<1, 1024, 0, s>>>(B, g.T, cnt, seg_off, seg_own, cursor);
        return hipGetLastError();
    }
    if (nblk > 0) {
        k_prep_scatter<<<nblk, kPrepThreads, (sizeof(unsigned long long) + sizeof(int)) * g.T * kTC, s>>>(
            g, x, y, t_rel, pol, offsets, wp, B, blk_start, chunk, cursor,
            cap >= 0 ? seg_off + (long long)B * g.T : nullptr, cap, ev);
        return hipGetLastError();
    }
    return hipSuccess;
}

// ------------------------------------------------------------ evaluation (a2, a3)

// Add one to every pixel of this tile that the staircase walk from pixel
// (kx, ky) to pixel (kxb, kyb) visits (eq. (17)); the start pixel is
// counted by the caller.  While both coordinates still move each step takes
// the corner test below; once one has reached its end the rest is a straight
// run with no test (the two loops visit exactly the pixels of one loop that
// tests every step, and skip its fp64 work on the run).  Corner decisions follow the event's ray through
// (x, y) with direction (ax, ay), in fp64: e = |X - x||ay| - |Y - y||ax|
// compares where the ray meets the next vertical and horizontal pixel
// edges; within 2^-8 px of the corner both side pixels are counted.
// Increments do not return the old count, so no step waits on the LDS;
// the item's sum of squares and its count of increments come from one pass
// over the tile afterwards (no walk counts its own steps).
// The corner test computes X - x as kx - (x - 1) or kx - x (the edge ahead
// is kx + 1 or kx), the same fp64 value as X - x, so decisions do not change.
// Pixels outside the tile are clamped onto its one-cell border (`Ring`),
// whose counts are removed at the end.

// The tile's counters in LDS with a one-cell border: pixel (kx, ky), clamped
// to [xlo, xhi] x [ylo, yhi] = [x0 - 1, x0 + tw] x [y0 - 1, y0 + th], is
// counter ky * rw + kx + base, rw = tw + 2.  Border counters collect every
// increment outside the tile (other tiles, outside the image).  `org` is
// the counter array shifted by base (org[ky * rw + kx] is pixel (kx, ky)),
// so an address is one 24-bit mad and one shift-add.
struct Ring {
    int xlo, xhi, ylo, yhi;
    int rw, base;
    int vxhi, vyhi;  // xhi, yhi held in vector registers (the clamp takes one scalar operand)
};

// v copied into a vector register that the compiler keeps (rather than
// copying it again before every use)
__device__ __forceinline__ int to_vgpr(int v) {
    int r;
    asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "s"(v));
    return r;
}

// a * b + c for 24-bit signed a, b in one instruction, b uniform (left to
// itself the compiler scales both terms of the index separately)
__device__ __forceinline__ int mad24(int a, int b, int c) {
    int r;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
    return r;
}

// v clamped to [lo, hi] (lo <= hi, lo uniform) in one instruction
__device__ __forceinline__ int clampi(int v, int lo, int hi) {
    int r;
    asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(v), "s"(lo), "v"(hi));
    return r;
}

__device__ __forceinline__ unsigned* ring_at(unsigned* org, const Ring& R, int kx, int ky) {
    return org + mad24(ky, R.rw, kx);
}

__device__ __forceinline__ void lds_inc(unsigned* p) {
    atomicAdd(p, 1u);  // the old count is not used: no wait for it
}

__device__ __forceinline__ void tile_add(unsigned* org, const Ring& R, int px, int py) {
    const int cx = clampi(px, R.xlo, R.vxhi), cy = clampi(py, R.ylo, R.vyhi);
    lds_inc(ring_at(org, R, cx, cy));
}

__device__ __forceinline__ void walk_tile(unsigned* org, const Ring& R, int kx, int ky, int kxb,
                                          int kyb, float xf, float yf, float axf, float ayf) {
    // a single step along a row or a column (|dx| + |dy| = 1, i.e.
    // dx^2 + dy^2 = 1) has no corner to test: it visits the end pixel only
    // (the coordinates are clamped to [-1, W] x [-1, H], so the squares are
    // 24-bit products)
    {
        const int dx = kxb - kx, dy = kyb - ky;
        if (__mul24(dx, dx) + __mul24(dy, dy) == 1) {
            tile_add(org, R, kxb, kyb);
            return;
        }
    }
    // step direction of each coordinate (not used once it is at its end)
    const bool px = kxb > kx, py = kyb > ky;
    const int sx = px ? 1 : -1, sy = py ? 1 : -1;
    if (kx != kxb && ky != kyb) {
        // the edges ahead are X = kx + px and Y = ky + py; with the origin
        // moved to (x - px, y - py) (exact in fp64), X - x = kx - xo exactly
        const double xo = (double)xf - (double)px, yo = (double)yf - (double)py;
        const double aax = fabs((double)axf), aay = fabs((double)ayf);
        const double thr = (aax + aay) * 0.00390625;
        // both coordinates still move: which edge does the ray meet first
        do {
            const double ex = fabs((double)kx - xo) * aay;
            const double ey = fabs((double)ky - yo) * aax;
            const double e = ex - ey;
            const bool lo = e < -thr, hi = e > thr;
            if (!lo && !hi) {  // the ray passes near the corner: both side pixels
                tile_add(org, R, kx + sx, ky);
                tile_add(org, R, kx, ky + sy);
            }
            kx += !hi ? sx : 0;
            ky += !lo ? sy : 0;
            tile_add(org, R, kx, ky);
        } while (kx != kxb && ky != kyb);
    }
    // one coordinate left: a straight run along a row or a column
    if (kx != kxb) {
        const int cy = clampi(ky, R.ylo, R.vyhi);
        do {
            kx += sx;
            lds_inc(org + mad24(cy, R.rw, clampi(kx, R.xlo, R.vxhi)));
        } while (kx != kxb);
    } else {
        const int cx = clampi(kx, R.xlo, R.vxhi);
        while (ky != kyb) {
            ky += sy;
            lds_inc(org + mad24(clampi(ky, R.ylo, R.vyhi), R.rw, cx));
        }
    }
}

// LDS layout of k_eval: [tile with its border: (tw + 2)(th + 2) counters]
// (region rounded up to 16 bytes)[reduction scratch][work item, queue sizes].  The
// reduction scratch is sized for the largest workgroup (1024 threads).
constexpr int kEvalWaves = kEvalThreads / 64;

// Counter words of the LDS tile region for tiles of up to ring_px counters
// (border included), rounded up to whole 16-byte units so the clear can use
// 16-byte stores.
__host__ __device__ __forceinline__ int eval_counter_words(int ring_px) { return (ring_px + 3) & ~3; }

size_t eval_lds_bytes(int ring_px) {
    return (size_t)eval_counter_words(ring_px) * 4 + 3 * kEvalWaves * 8 + 4 * (1 + kXcd);
}

// Persistent evaluation kernel: each workgroup takes work items (a window's
// tile segment and one or more hypotheses) from the queue until it is
// empty.  For each hypothesis it bins the tile's events in LDS (point: one
// increment per event, interval: one per pixel of the walk) with atomic adds
// that return nothing, then removes the border counters' share and sums the
// squares of the tile's counters in one 16-byte-wide pass that also zeroes
// them for the next hypothesis (the tile region is cleared once, at start).
// An interval takes the segment's owned events, then its guest copies,
// skipping a guest whose walk box misses the tile (all its increments would
// land on the border).  Points and intervals read the guest bins whose lower
// cut lies below the hypothesis's larger rate only (the others are short of
// the tile at every rate it takes).  An endpoint certificate reads the owned
// events only and touches no counter.
template <int NT>
__global__ __launch_bounds__(NT) void k_eval(
    Geometry g, const float4* __restrict__ ev, const long long* __restrict__ seg_off,
    const int* __restrict__ seg_own, const WinParam* __restrict__ wp, const Hyp* __restrict__ hyps,
    const int* __restrict__ act, const Item* __restrict__ items, int qcap, Queue* __restrict__ q, Queue* __restrict__ q_reset,
    Part* __restrict__ part, int HS, unsigned* __restrict__ img_out) {
    constexpr int NW = NT / 64;
    extern __shared__ __align__(16) unsigned smem[];
    const int tid = threadIdx.x;
    unsigned* const tile = smem;
    unsigned long long* const s_red =
        reinterpret_cast<unsigned long long*>(smem + eval_counter_words(g.ring_px));
    int* const s_item = reinterpret_cast<int*>(s_red + 3 * NW);
    if (blockIdx.x == 0 && tid < kXcd && q_reset) {
        q_reset[tid].n_items = 0;
        q_reset[tid].next = 0;
    }
    {  // every counter of the tile region starts at zero and is zeroed again
       // by the pass that sums each hypothesis's squares
        uint4* const t4 = reinterpret_cast<uint4*>(tile);
        const int n4 = eval_counter_words(g.ring_px) >> 2;
        for (int i = tid; i < n4; i += NT) t4[i] = make_uint4(0u, 0u, 0u, 0u);
    }
    const int home = blockIdx.x % kXcd;
    int qi = 0;  // queues tried so far, starting at this XCD's own (thread 0 only)
    int* const qn = s_item + 1;  // queue sizes, read once (thread 0 only; in LDS, not registers)
    if (tid == 0)
        for (int r = 0; r < kXcd; ++r) qn[r] = q[(home + r) % kXcd].n_items;
    for (;;) {
        if (tid == 0) {
            int got = -1;
            while (qi < kXcd) {
                const int r = (home + qi) % kXcd;
                if (qn[qi] > 0) {
                    const int k = atomicAdd(&q[r].next, 1);
                    if (k < qn[qi]) {
                        got = r * qcap + k;
                        break;
                    }
                }
                ++qi;
            }
            *s_item = got;
        }
        __syncthreads();
        const int it = *s_item;
        __syncthreads();
        if (it < 0) break;
        const Item item = items[it];
        const int w = item.w, t = item.t;
        const int ts = t % g.nsp;  // spatial tile of the segment
        const int tx = ts % g.ntx, ty = ts / g.ntx;
        const int x0 = g.colcut[tx], y0 = g.rowcut[ty];
        const int tw = g.colcut[tx + 1] - x0, th = g.rowcut[ty + 1] - y0;
        Ring R;
        R.xlo = x0 - 1;
        R.xhi = x0 + tw;
        R.ylo = y0 - 1;
        R.yhi = y0 + th;
        R.rw = tw + 2;
        R.base = -(R.ylo * R.rw + R.xlo);
        R.vxhi = to_vgpr(R.xhi);
        R.vyhi = to_vgpr(R.yhi);
        unsigned* const org = tile + R.base;   // org[ky * rw + kx]: pixel (kx, ky)
        const int ncnt = R.rw * (th + 2);       // counters, border included
        const int nring = 2 * R.rw + 2 * th;    // border counters
        const float fxlo = (float)R.xlo, fxhi = (float)R.xhi, fylo = (float)R.ylo, fyhi = (float)R.yhi;
        const long long seg = (long long)w * g.T + t;
        const long long beg = seg_off[seg];
        const int* const sown = seg_own + seg * (kGuestBins + 1);
        const float* const gcut = wp[w].gcut;
      for (int gk = 0; gk < item.cnt; ++gk) {
        const int wh = w * HS + act[w * HS + item.r0 + gk];
        const Hyp hp = hyps[wh];
        // guest bins read: those whose lower cut lies below the larger rate
        int nbin = 0;
        {
            const float rmax = fmaxf(hp.ra, hp.rb);
#pragma unroll
            for (int k = 0; k < kGuestBins - 1; ++k) nbin += gcut[k] < rmax ? 1 : 0;
        }

        unsigned long long nlow = 0;
        // the segment's events, indexed from its start with 32-bit offsets
        // (byte offsets fit 32 bits: a segment holds fewer than 2^28 events)
        const char* __restrict__ sev = reinterpret_cast<const char*>(ev + beg);
        const auto at = [sev](unsigned k) { return *reinterpret_cast<const float4*>(sev + (k << 4)); };
        const unsigned nown = (unsigned)sown[0], nseg = (unsigned)sown[1 + nbin];
        unsigned long long ucert = 0;  // certificate: walk pixels of the events inside at both ends
        if (hp.kind == HYP_CERT) {
            // Endpoint certificate of an interval (eqs. (17)-(20) without
            // the walk): the owned events only, no counter is touched.  An
            // event with both endpoint pixels in the image walks through
            // |dkx| + |dky| + 1 distinct image pixels at least.
            const float ra = hp.ra, rb = hp.rb;
            unsigned nl = 0;
            const auto one = [&](const float4& e) {
                const int kxa = flr_clamp(fmaf(e.z, ra, e.x), g.W), kya = flr_clamp(fmaf(e.w, ra, e.y), g.H);
                const int kxb = flr_clamp(fmaf(e.z, rb, e.x), g.W), kyb = flr_clamp(fmaf(e.w, rb, e.y), g.H);
                // both endpoints in the image, i.e. the far one (see the interval path)
                const bool full = ((unsigned)kxb < (unsigned)g.W) & ((unsigned)kyb < (unsigned)g.H);
                nl += full ? 1u : 0u;
                ucert += full ? (unsigned)(abs(kxb - kxa) + abs(kyb - kya) + 1) : 0u;
            };
            constexpr int U = 4;
            constexpr unsigned S = NT;
            unsigned i = tid;
            for (; i + (U - 1) * S < nown; i += U * S) {
                float4 e[U];
#pragma unroll
                for (int k = 0; k < U; ++k) e[k] = at(i + k * S);
#pragma unroll
                for (int k = 0; k < U; ++k) one(e[k]);
            }
            for (; i < nown; i += S) one(at(i));
            nlow = nl;
        } else if (hp.kind == HYP_POINT) {
            // Point hypothesis (eqs. (12)-(13)): U events per thread in
            // flight, loads first, then U increments without branches.
            const float r = hp.ra;
            constexpr int U = 4;
            constexpr unsigned S = NT;
            unsigned i = tid;
            for (; i + (U - 1) * S < nseg; i += U * S) {
                float4 e[U];
#pragma unroll
                for (int k = 0; k < U; ++k) e[k] = at(i + k * S);
                int a[U];
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    const int kx = cvt_flr(__builtin_amdgcn_fmed3f(fmaf(e[k].z, r, e[k].x), fxlo, fxhi));
                    const int ky = cvt_flr(__builtin_amdgcn_fmed3f(fmaf(e[k].w, r, e[k].y), fylo, fyhi));
                    a[k] = mad24(ky, R.rw, kx);
                }
#pragma unroll
                for (int k = 0; k < U; ++k) atomicAdd(org + a[k], 1u);
            }
            for (; i < nseg; i += S) {
                const float4 e = at(i);
                const int kx = cvt_flr(__builtin_amdgcn_fmed3f(fmaf(e.z, r, e.x), fxlo, fxhi));
                const int ky = cvt_flr(__builtin_amdgcn_fmed3f(fmaf(e.w, r, e.y), fylo, fyhi));
                atomicAdd(ring_at(org, R, kx, ky), 1u);
            }
        } else {
            // Interval hypothesis (eqs. (17)-(20)): endpoints, N_low, walk.
            const float ra = hp.ra, rb = hp.rb;
            unsigned nlow32 = 0;
            const auto one = [&](const float4& e, unsigned i) {
                const float xa = fmaf(e.z, ra, e.x), ya = fmaf(e.w, ra, e.y);
                const float xb = fmaf(e.z, rb, e.x), yb = fmaf(e.w, rb, e.y);
                const int kxa = flr_clamp(xa, g.W), kya = flr_clamp(ya, g.H);
                const int kxb = flr_clamp(xb, g.W), kyb = flr_clamp(yb, g.H);
                // both endpoints in the image, i.e. the far one (not clamped to
                // -1, huge as unsigned, nor to W, H): the warp only moves an
                // event away from the FOE as the rate grows, so an event inside
                // at rb is inside at ra <= rb
                nlow32 += (unsigned)(i < nown) & (unsigned)((unsigned)kxb < (unsigned)g.W) &
                          (unsigned)((unsigned)kyb < (unsigned)g.H);
                tile_add(org, R, kxa, kya);
                if (kxa != kxb || kya != kyb) walk_tile(org, R, kxa, kya, kxb, kyb, e.x, e.y, e.z, e.w);
            };
            // Owned events first (N_low counts them), then the guest copies:
            // a guest whose walk box for this interval misses the tile would
            // only increment the discarded border, so it is skipped, tested
            // on the warped coordinates before their floor (for an integer
            // edge e, floor(v) < e exactly when v < e, and the clamp to the
            // image cannot move a coordinate across an edge of the tile).
            // Two events in flight ahead of the one being binned (the loads
            // may read up to two strides past a range: the store is padded by
            // kEvalPad records).
            const float fx0 = (float)x0, fx1 = (float)(x0 + tw), fy0 = (float)y0, fy1 = (float)(y0 + th);
            const auto guest = [&](const float4& e, unsigned i) {
                const float xa = fmaf(e.z, ra, e.x), ya = fmaf(e.w, ra, e.y);
                const float xb = fmaf(e.z, rb, e.x), yb = fmaf(e.w, rb, e.y);
                const bool miss = fmaxf(xa, xb) < fx0 || fminf(xa, xb) >= fx1 || fmaxf(ya, yb) < fy0 || fminf(ya, yb) >= fy1;
                if (!miss) {
                    const int kxa = flr_clamp(xa, g.W), kya = flr_clamp(ya, g.H);
                    const int kxb = flr_clamp(xb, g.W), kyb = flr_clamp(yb, g.H);
                    tile_add(org, R, kxa, kya);
                    if (kxa != kxb || kya != kyb) walk_tile(org, R, kxa, kya, kxb, kyb, e.x, e.y, e.z, e.w);
                }
            };
            const auto run = [&](unsigned i, unsigned lim, auto&& f) {
                if (i < lim) {
                    float4 e0 = at(i), e1 = at(i + NT), e2;
                    for (;;) {
                        e2 = at(i + 2 * NT);
                        f(e0, i);
                        i += NT;
                        if (i >= lim) break;
                        e0 = at(i + 2 * NT);
                        f(e1, i);
                        i += NT;
                        if (i >= lim) break;
                        e1 = at(i + 2 * NT);
                        f(e2, i);
                        i += NT;
                        if (i >= lim) break;
                    }
                }
            };
            run((unsigned)tid, nown, one);
            run(nown + (unsigned)tid, nseg, guest);
            nlow = nlow32;
        }
        // The border counters' squares and counts are removed, then the sums
        // of the counters and of their squares are taken over the whole
        // counter region, 16 bytes per read, and the region is zeroed for the
        // next hypothesis (every counter is zero between hypotheses).  The
        // sum of the counters less the border's is the hypothesis's count of
        // in-tile increments (every increment lands in one counter).  Each
        // thread takes some counters (its own sums may wrap; the workgroup's
        // totals are exact).
        // (A certificate touched no counter: it skips both passes, not the
        // barrier, which also orders thread 0's reads of the reduction
        // scratch before the next writes.)
        __syncthreads();
        unsigned long long sq = ucert, hits = 0;
        if (hp.kind != HYP_CERT) {
            for (int k = tid; k < nring; k += NT) {
                int idx;
                if (k < R.rw) idx = k;                                      // top row
                else if (k < 2 * R.rw) idx = (th + 1) * R.rw + (k - R.rw);  // bottom row
                else idx = (1 + ((k - 2 * R.rw) >> 1)) * R.rw + (((k - 2 * R.rw) & 1) ? R.rw - 1 : 0);
                const unsigned m = tile[idx];
                sq -= (unsigned long long)m * m;
                hits -= m;
            }
            if (img_out) {  // hypothesis wh's image(s): W*H cells per polarity image
                const long long M = (long long)g.W * g.H;
                unsigned* const im = img_out + (long long)wh * M * (g.T / g.nsp) + (long long)(t / g.nsp) * M;
                for (int k = tid; k < tw * th; k += NT) {
                    const int lx = k % tw, ly = k / tw;
                    im[(long long)(y0 + ly) * g.W + (x0 + lx)] = tile[(ly + 1) * R.rw + lx + 1];
                }
            }
            __syncthreads();  // every read of single counters is done before the region is zeroed
            uint4* const t4 = reinterpret_cast<uint4*>(tile);
            const int n4 = (ncnt + 3) >> 2;  // the counters lie in the rounded-up region
            for (int i = tid; i < n4; i += NT) {
                const uint4 v = t4[i];
                t4[i] = make_uint4(0u, 0u, 0u, 0u);
                sq += (unsigned long long)v.x * v.x + (unsigned long long)v.y * v.y +
                      (unsigned long long)v.z * v.z + (unsigned long long)v.w * v.w;
                hits += (unsigned long long)v.x + v.y + v.z + v.w;
            }
        }
        // block reduction of (S, hits, nlow)
        sq = wave_total(sq);
        hits = wave_total(hits);
        // N_low counts owned events (fewer than 2^28 per segment); points have none
        if (hp.kind != HYP_POINT) nlow = wave_total32((unsigned)nlow);
        const int wave = tid >> 6, lane = tid & 63;
        if (lane == 63) {
            s_red[wave] = sq;
            s_red[NW + wave] = hits;
            s_red[2 * NW + wave] = nlow;
        }
        __syncthreads();
        if (tid == 0) {
            unsigned long long a = 0, b = 0, c = 0;
            for (int k = 0; k < NW; ++k) {
                a += s_red[k];
                b += s_red[NW + k];
                c += s_red[2 * NW + k];
            }
            Part pt;
            pt.S = a;
            pt.N = (long long)(hp.kind == HYP_POINT ? b : c);
            pt.U = b;
            pt.pad = 0;
            part[(long long)wh * g.T + t] = pt;
        }
        // no barrier here: every thread zeroed its counters before the one
        // above, and thread 0 reads s_red before the next hypothesis's first
        // barrier, after which s_red is written again
      }
    }
}

// The evaluation kernel for nt threads per workgroup (256, 512 or 1024).
static const void* eval_kernel(int nt) {
    switch (nt) {
        case 256: return (const void*)k_eval<256>;
        case 512: return (const void*)k_eval<512>;
        default: return (const void*)k_eval<1024>;
    }
}

hipError_t eval_occupancy(int* blocks_per_cu, size_t lds_bytes, int nt) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, eval_kernel(nt), nt, lds_bytes);
}

hipError_t eval_set_lds(size_t bytes) {
    for (int nt : {256, 512, 1024}) {
        hipError_t e = hipFuncSetAttribute(eval_kernel(nt), hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_eval(hipStream_t s, const Geometry& g, int nblocks, int nt, size_t lds_bytes, const float4* ev,
                       const long long* seg_off, const int* seg_own, const WinParam* wp, const Hyp* hyps,
                       const int* act,
                       const Item* items, int qcap, Queue* q, Queue* q_reset, Part* part, int HS,
                       unsigned* img_out, hipEvent_t t0, hipEvent_t t1) {
    // the events (nullable) take the kernel's start and end times from its dispatch
    switch (nt) {
        case 256:
            hipExtLaunchKernelGGL(k_eval<256>, dim3(nblocks), dim3(256), (uint32_t)lds_bytes, s, t0, t1, 0u, g, ev,
                                  seg_off, seg_own, wp, hyps, act, items, qcap, q, q_reset, part, HS, img_out);
            break;
        case 512:
            hipExtLaunchKernelGGL(k_eval<512>, dim3(nblocks), dim3(512), (uint32_t)lds_bytes, s, t0, t1, 0u, g, ev,
                                  seg_off, seg_own, wp, hyps, act, items, qcap, q, q_reset, part, HS, img_out);
            break;
        default:
            hipExtLaunchKernelGGL(k_eval<1024>, dim3(nblocks), dim3(1024), (uint32_t)lds_bytes, s, t0, t1, 0u, g,
                                  ev, seg_off, seg_own, wp, hyps, act, items, qcap, q, q_reset, part, HS, img_out);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ frontier (a4)

constexpr int NTF = kFrontThreads;
constexpr int NWF = NTF / 64;

// Exclusive prefix sum of v over the workgroup (in thread order); `total`
// receives the sum.  All threads must call it.
__device__ __forceinline__ int block_scan(int v, int* s_wave, int& total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_wave[wave] = x;
    __syncthreads();
    int base = 0, tot = 0;
    for (int k = 0; k < NWF; ++k) {
        const int t = s_wave[k];
        if (k < wave) base += t;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return base + x - v;
}

// Lexicographic maximum of (K, -j) over the workgroup: within each wave by
// lane exchanges, then across the NWF wave winners through LDS.
__device__ __forceinline__ bool lex_better(long long bh, unsigned long long bl, unsigned bj, long long ah,
                                           unsigned long long al, unsigned aj) {
    return bh > ah || (bh == ah && (bl > al || (bl == al && bj < aj)));
}

__device__ __forceinline__ void block_argmax(i128& K, unsigned& j, long long* s_hi, unsigned long long* s_lo,
                                             unsigned* s_j) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    long long h;
    unsigned long long l;
    sp128(K, h, l);
    unsigned jj = j;
    for (int o = 32; o > 0; o >>= 1) {
        const long long oh = __shfl_xor(h, o, 64);
        const unsigned long long ol = __shfl_xor(l, o, 64);
        const unsigned oj = __shfl_xor(jj, o, 64);
        if (lex_better(oh, ol, oj, h, l, jj)) {
            h = oh;
            l = ol;
            jj = oj;
        }
    }
    if (lane == 0) {
        s_hi[wave] = h;
        s_lo[wave] = l;
        s_j[wave] = jj;
    }
    __syncthreads();
    h = s_hi[0];
    l = s_lo[0];
    jj = s_j[0];
    for (int k = 1; k < NWF; ++k)
        if (lex_better(s_hi[k], s_lo[k], s_j[k], h, l, jj)) {
            h = s_hi[k];
            l = s_lo[k];
            jj = s_j[k];
        }
    K = mk128(h, l);
    j = jj;
    __syncthreads();
}

// Sum of the tiles' partial sums of one hypothesis slot.
__device__ __forceinline__ void slot_sums(const Part* pw, int slot, int T, const int* tiles, int nt,
                                          unsigned long long& S, long long& N, unsigned long long& U) {
    S = 0;
    N = 0;
    U = 0;
    for (int k = 0; k < nt; ++k) {
        const Part q = pw[(long long)slot * T + tiles[k]];
        S += q.S;
        N += q.N;
        U += q.U;
    }
}

// Work items of the na active slots act[0..na) of window w: groups of up
// to G slots on each non-empty tile, tile-major, appended to the window's
// queue in qf.
__device__ void emit_items(const Search& sp, int w, const int* tiles, int nt, int na, Item* items, int qcap,
                           Queue* qf) {
    int G = sp.G;
    const int qr = w % kXcd;  // this window's queue
    Item* qitems = items + (long long)qr * qcap;
    __shared__ int s_base;
    if (sp.gslots > 0) {  // this step's items with one hypothesis each, all windows alike
        const long long work = (long long)sp.B * na * nt;
        G = (int)max(1ll, min((long long)G, work / sp.gslots));
    }
    const int ng = (na + G - 1) / G;
    if (threadIdx.x == 0) s_base = (ng * nt) ? atomicAdd(&qf[qr].n_items, ng * nt) : 0;
    __syncthreads();
    for (int k = threadIdx.x; k < ng * nt; k += NTF) {
        const int ti = k / ng, gi = k % ng;  // tile-major: items sharing events are adjacent
        Item it;
        it.w = w;
        it.t = tiles[ti];
        it.r0 = gi * G;
        it.cnt = min(G, na - gi * G);
        // within a tile the groups with intervals (the longer items) first
        qitems[s_base + ti * ng + (ng - 1 - gi)] = it;
    }
    __syncthreads();
}

// Hypotheses of the selected nodes, the list of active slots, and the work
// items.  q_rem: nodes left in the queue; n_kids: selected nodes with
// children.  When every node the queue can hold after the next step is
// expanded at that step (q_rem + 2 n_kids <= F) and there is no node
// budget, a child's bound value decides nothing but whether it is kept, so
// the children get the endpoint certificate (exact bounds when it fails, in
// the same step).  For the gamma stop a certified child's points are
// bounded by its nearest exactly bounded ancestor's bound instead.
__device__ void emit_hyps(const Search& sp, const WinParam& p, int w, int T, const int* tiles, int nt,
                          const Sel* sl, int n_sel, int q_rem, int n_kids, float kinc, Hyp* hy, int* act,
                          Item* items, int qcap, Queue* qf, int* s_wave) {
    const int F = sp.F, HS = sp.HS;
    const bool cert = sp.cert && sp.max_nodes == 0 && q_rem + 2 * n_kids <= F && q_rem + 2 * n_kids <= sp.CAP;
    // a node's children take the certificate when it is expected to clear
    // the incumbent K_inc (kinc): a failed certificate costs its pass and the
    // exact bound (measured on the three batches: margins of 0.5 to 1.5 x
    // K_inc within 3%, 1.0 best; no prediction: +10% on 1280x720, +25% on
    // 346x260)
    int na = 0;  // active slots so far
    for (int h0 = 0; h0 < HS; h0 += NTF) {
        const int h = h0 + threadIdx.x;
        Hyp hp;
        hp.kind = HYP_NONE;
        hp.pad = 0;
        hp.ra = hp.rb = 0.0f;
        if (h < F) {
            if (h < n_sel) {
                hp.kind = HYP_POINT;
                hp.ra = hp.rb = rate_of(grid_d(sp.d_lo, sp.d_hi, sp.L, sl[h].jc), p.tau);
            }
        } else if (h < HS) {
            const int c = h - F, i = c >> 1;
            if (i < n_sel && sl[i].kids) {
                const unsigned a = (c & 1) ? sl[i].jc : sl[i].ja;
                const unsigned b = (c & 1) ? sl[i].jb : sl[i].jc;
                hp.kind = (cert && sl[i].lc > kinc) ? HYP_CERT : HYP_INTERVAL;
                hp.ra = rate_of(grid_d(sp.d_lo, sp.d_hi, sp.L, a), p.tau);
                hp.rb = rate_of(grid_d(sp.d_lo, sp.d_hi, sp.L, b), p.tau);
            }
        }
        if (h < HS) hy[h] = hp;
        int tot;
        const int r = block_scan(hp.kind != HYP_NONE ? 1 : 0, s_wave, tot);
        if (hp.kind != HYP_NONE) act[na + r] = h;
        na += tot;
    }
    emit_items(sp, w, tiles, nt, na, items, qcap, qf);
}

__device__ __forceinline__ void nonempty_tiles(int w, int T, const long long* seg_off, int* tiles, int* s_nt,
                                               int* s_wave) {
    const int t = threadIdx.x;
    int ne = 0;
    if (t < T) {
        const long long seg = (long long)w * T + t;
        ne = seg_off[seg + 1] > seg_off[seg] ? 1 : 0;
    }
    int tot;
    const int r = block_scan(ne, s_wave, tot);
    if (ne) tiles[r] = t;
    if (threadIdx.x == 0) *s_nt = tot;
    __syncthreads();
}

__global__ __launch_bounds__(NTF) void k_init(Search sp, const WinParam* __restrict__ wp,
                                              const float* __restrict__ seeds, int B, WinState* __restrict__ st,
                                              Sel* __restrict__ sel, Hyp* __restrict__ hyps, int* __restrict__ act,
                                              Item* __restrict__ items, int qcap, Queue* __restrict__ q, int T,
                                              const long long* __restrict__ seg_off, InitCheck chk) {
    const int w = blockIdx.x;
    const unsigned top = 1u << sp.L;
    Sel* sl = sel + (long long)w * sp.F;
    __shared__ int s_nsel, s_nt, s_wave[NWF];
    __shared__ int s_tiles[kMaxTiles];
    if (chk.wstat) {
        const int bad = chk.wstat[w] ? chk.wstat[w]
                        : chk.werr[w] ? -1                                  // ECMD_EINVAL
                        : seg_off[(long long)B * T] > chk.cap ? -2 : 0;     // ECMD_ENOMEM
        if (bad) {
            if (threadIdx.x == 0) {
                WinState s = WinState{};
                s.status = bad;
                st[w] = s;
            }
            return;
        }
    }
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
        root.lc = INFINITY;  // no evaluation yet: the root's children try the certificate
        root.ub = INFINITY;  // and no bound above them
        sl[0] = root;
        int n_sel = 1;
        if (seeds) {
            const float d = seeds[w];
            if (isfinite(d)) {
                const double span = (double)sp.d_hi - (double)sp.d_lo;
                const double v = ((double)d - (double)sp.d_lo) / span * (double)top;
                long long j = llround(v);
                j = j < 1 ? 1 : (j > (long long)top - 1 ? (long long)top - 1 : j);
                if ((unsigned)j != root.jc && sp.F > 1) {
                    Sel sd;
                    sd.ja = sd.jb = sd.jc = (unsigned)j;
                    sd.kids = 0;
                    sd.lc = 0.0f;
                    sd.ub = INFINITY;
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
    nonempty_tiles(w, T, seg_off, s_tiles, &s_nt, s_wave);
    emit_hyps(sp, wp[w], w, T, s_tiles, s_nt, sl, s_nsel, 0, 1, -1.0f, hyps + (long long)w * sp.HS,
              act + (long long)w * sp.HS, items, qcap, q, s_wave);
}

hipError_t launch_init(hipStream_t s, const Search& sp, const WinParam* wp, const float* seeds, int B,
                       WinState* st, Sel* sel, Hyp* hyps, int* act, Item* items, int qcap, Queue* q, int T,
                       const long long* seg_off, InitCheck chk) {
    if (B <= 0) return hipSuccess;
    k_init<<<B, NTF, 0, s>>>(sp, wp, seeds, B, st, sel, hyps, act, items, qcap, q, T, seg_off, chk);
    return hipGetLastError();
}

// The certificate a node's children can expect, from the node's own sums:
// U walk pixels over N_low events inside at both ends, i.e. mean walk
// length l = U / N_low - 1; a child's walks are about half as long, so its
// certificate is about N_low^2 (l/2)(l/2 + 2).  Only the choice between the
// certificate and the exact bound depends on it, never a result.
__device__ __forceinline__ float child_cert(unsigned long long U, long long N) {
    if (N <= 0) return 0.0f;
    const float l = fmaxf((float)U / (float)N - 1.0f, 0.0f) * 0.5f;
    return (float)N * (float)N * l * (l + 2.0f);
}

// Append the children whose keep flag is set to the queue (array order),
// noting an overflow of the capacity.
__device__ __forceinline__ void queue_append(Node* fr, int& n, int CAP, bool keep, const Node& nd, int* s_wave,
                                             int& overflow) {
    int tot;
    const int r = block_scan(keep ? 1 : 0, s_wave, tot);
    if (keep && n + r < CAP) fr[n + r] = nd;
    if (n + tot > CAP) overflow = 1;
    n = min(n + tot, CAP);
}

// Phase 0 of one step of Algorithm 1 for window blockIdx.x: absorb the
// evaluated hypotheses, update the incumbent and queue the improvable
// children.  A child evaluated by its endpoint certificate L <= K_bar is
// queued with key L (marked kNodeCert) when L already shows it improvable;
// otherwise it is queued in its place as a placeholder (kNodeRepair) and its
// exact bound goes to the evaluation launch between the phases, so the
// queue keeps the exact search's order.  Every order below is the array
// order (scans, no atomic slot races), so the search is reproducible.
__global__ __launch_bounds__(NTF) void k_frontier_a(
    Search sp, const WinParam* __restrict__ wp, int B, int T, const long long* __restrict__ seg_off,
    WinState* __restrict__ st, Node* __restrict__ front, Sel* __restrict__ sel, Hyp* __restrict__ hyps,
    int* __restrict__ act, const Part* __restrict__ part, Item* __restrict__ items, int qcap,
    Queue* __restrict__ qf, int* __restrict__ n_active) {
    const int w = blockIdx.x, tid = threadIdx.x;
    __shared__ WinState s;
    __shared__ long long s_hi[NTF];
    __shared__ unsigned long long s_lo[NTF];
    __shared__ unsigned s_j[NTF];
    __shared__ int s_wave[NWF], s_tiles[kMaxTiles], s_nt;
    __shared__ unsigned long long s_pix;
    __shared__ long long s_nbound, s_pruned, s_ncert;
    if (tid == 0) s = st[w];
    __syncthreads();
    if (!s.active) return;
    const int F = sp.F, HS = sp.HS, CAP = sp.CAP;
    const long long M = sp.M;
    const WinParam p = wp[w];
    Node* fr = front + (long long)w * CAP;
    Sel* sl = sel + (long long)w * F;
    Hyp* hy = hyps + (long long)w * HS;
    int* ac = act + (long long)w * HS;
    const Part* pw = part + (long long)w * HS * T;
    nonempty_tiles(w, T, seg_off, s_tiles, &s_nt, s_wave);
    const int nt = s_nt;
    const int n_sel = s.n_sel;

    // (1) centre points: lexicographic max of (K, -j) with the incumbent
    i128 bK = mk128(s.Kinc_hi, s.Kinc_lo);
    unsigned bJ = s.j_inc;
    for (int i = tid; i < n_sel; i += NTF) {
        unsigned long long S, U;
        long long N;
        slot_sums(pw, i, T, s_tiles, nt, S, N, U);
        const i128 K = (i128)M * (i128)S - (i128)N * (i128)N;
        const unsigned jc = sl[i].jc;
        if (K > bK || (K == bK && jc < bJ)) { bK = K; bJ = jc; }
    }
    block_argmax(bK, bJ, s_hi, s_lo, s_j);
    const i128 Kinc = bK;
    const unsigned jinc = bJ;
    if (tid == 0) {
        sp128(Kinc, s.Kinc_hi, s.Kinc_lo);
        s.j_inc = jinc;
        s.point_evals += n_sel;
        s.event_hyp += (long long)n_sel * p.n_events;
        s_pix = 0;
        s_nbound = 0;
        s_pruned = 0;
        s_ncert = 0;
    }
    __syncthreads();

    // (2) children of the expanded nodes, appended in slot order
    int n = s.n_front;
    const int n0 = n;
    int overflow = 0, nrep = 0;
    for (int c0 = 0; c0 < 2 * n_sel; c0 += NTF) {
        const int c = c0 + tid;
        bool keep = false, rep = false;
        Node nd;
        if (c < 2 * n_sel && sl[c >> 1].kids) {
            unsigned long long S, U;
            long long N;
            slot_sums(pw, F + c, T, s_tiles, nt, S, N, U);
            const Sel x = sl[c >> 1];
            nd.ja = (c & 1) ? x.jc : x.ja;
            nd.jb = (c & 1) ? x.jb : x.jc;
            nd.ub = x.ub;  // every grid point of the child is one of the parent's
            if (hy[F + c].kind == HYP_CERT) {
                // S holds U (walk pixels of the events inside at both ends),
                // a lower bound of sum H_bar.  Two lower bounds of K_bar:
                // M S_bar >= U^2 (Cauchy-Schwarz over the M cells), and, as
                // the centre d_c of the expanded node (evaluated this step:
                // S_c, N_c) is an end of the child, H_bar >= H(d_c) pixel by
                // pixel, so with X = H_bar - H(d_c) >= 0,
                // S_bar >= S_c + (sum X)^2 / M and sum X >= U - N_c.
                unsigned long long Sc, Uc;
                long long Nc;
                slot_sums(pw, c >> 1, T, s_tiles, nt, Sc, Nc, Uc);
                const i128 N2 = (i128)N * (i128)N;
                const i128 L1 = (i128)S * (i128)S - N2;
                const i128 X = (long long)S > Nc ? (i128)((long long)S - Nc) : (i128)0;
                const i128 L2 = (i128)M * (i128)Sc + X * X - N2;
                const i128 Lb = L1 > L2 ? L1 : L2;
                nd.lc = child_cert(S, N);
                keep = true;
                if (improvable(Lb, nd.ja, Kinc, jinc)) {
                    sp128(Lb, nd.khi, nd.klo);
                    nd.jb |= kNodeCert;
                    atomicAdd((unsigned long long*)&s_ncert, 1ull);
                } else {
                    rep = true;
                    nd.khi = kNodeRepair;
                    nd.klo = (unsigned long long)(F + c);
                }
            } else {
                atomicAdd(&s_pix, U);
                atomicAdd((unsigned long long*)&s_nbound, 1ull);
                const i128 Kb = (i128)M * (i128)S - (i128)N * (i128)N;
                sp128(Kb, nd.khi, nd.klo);
                nd.lc = child_cert(U, N);
                keep = improvable(Kb, nd.ja, Kinc, jinc);
                if (!keep) atomicAdd((unsigned long long*)&s_pruned, 1ull);
            }
        }
        queue_append(fr, n, CAP, keep, nd, s_wave, overflow);
        // the children to bound exactly between the phases
        int tot;
        const int r = block_scan(rep ? 1 : 0, s_wave, tot);
        if (rep) {
            hy[F + c].kind = HYP_INTERVAL;  // same end rates
            ac[nrep + r] = F + c;
        }
        nrep += tot;
    }
    __syncthreads();
    if (tid == 0) {
        s.bound_evals += s_nbound;
        s.event_hyp += s_nbound * p.n_events;
        s.pixel_updates += (long long)s_pix;
        s.nodes_pruned += s_pruned;
        s.cert_evals += s_ncert;
        s.n_front = n;
        s.n_front0 = n0;
        s.overflow = overflow;
        s.n_repair = nrep;
        st[w] = s;
    }
    if (nrep) emit_items(sp, w, s_tiles, nt, nrep, items, qcap, qf);
}

// Phase 1 of the step: put the exact bounds of the children whose
// certificate failed into their placeholders, drop queued nodes that can no
// longer improve, decide whether to stop, select the next nodes, emit their
// hypotheses.
__global__ __launch_bounds__(NTF) void k_frontier_b(
    Search sp, const WinParam* __restrict__ wp, int B, int T, const long long* __restrict__ seg_off,
    WinState* __restrict__ st, Node* __restrict__ front, Sel* __restrict__ sel, Hyp* __restrict__ hyps,
    int* __restrict__ act, const Part* __restrict__ part, Item* __restrict__ items, int qcap,
    Queue* __restrict__ qf, int* __restrict__ n_active) {
    const int w = blockIdx.x, tid = threadIdx.x;
    __shared__ WinState s;
    __shared__ long long s_hi[NTF];
    __shared__ unsigned long long s_lo[NTF];
    __shared__ unsigned s_j[NTF];
    __shared__ int s_wave[NWF], s_tiles[kMaxTiles], s_nt;
    __shared__ int s_hist[130];
    __shared__ int s_bstar, s_quota, s_stop, s_take, s_anycert, s_ubmax;
    __shared__ unsigned long long s_pix;
    __shared__ long long s_nbound, s_pruned;
    if (tid == 0) s = st[w];
    __syncthreads();
    if (!s.active) return;
    const int F = sp.F, HS = sp.HS, CAP = sp.CAP;
    const long long M = sp.M;
    const WinParam p = wp[w];
    Node* fr = front + (long long)w * CAP;
    Sel* sl = sel + (long long)w * F;
    const Part* pw = part + (long long)w * HS * T;
    nonempty_tiles(w, T, seg_off, s_tiles, &s_nt, s_wave);
    const int nt = s_nt;
    const i128 Kinc = mk128(s.Kinc_hi, s.Kinc_lo);
    const unsigned jinc = s.j_inc;
    if (tid == 0) {
        s_pix = 0;
        s_nbound = 0;
        s_pruned = 0;
        s_anycert = 0;
        s_ubmax = 0;  // 0.0f
    }
    for (int b = tid; b < 130; b += NTF) s_hist[b] = 0;
    __syncthreads();

    // (2') the exact bounds of the children whose certificate failed, into
    // their placeholders (this step's children sit at [n_front0, n_front));
    // one that cannot improve is dropped below with the other such nodes
    const int n = s.n_front;
    const int overflow = s.overflow;
    if (s.n_repair) {
        for (int i = s.n_front0 + tid; i < n; i += NTF) {
            Node nd = fr[i];
            if (nd.khi != kNodeRepair) continue;
            unsigned long long S, U;
            long long N;
            slot_sums(pw, (int)nd.klo, T, s_tiles, nt, S, N, U);
            atomicAdd(&s_pix, U);
            atomicAdd((unsigned long long*)&s_nbound, 1ull);
            const i128 Kb = (i128)M * (i128)S - (i128)N * (i128)N;
            sp128(Kb, nd.khi, nd.klo);
            if (!improvable(Kb, nd.ja, Kinc, jinc)) atomicAdd((unsigned long long*)&s_pruned, 1ull);
            fr[i] = nd;
        }
    }
    __syncthreads();

    // (3) which queued nodes can still improve; histogram of their gap
    // sizes; the node Algorithm 1 would pop next (largest bound, ties to the
    // smaller grid index; queued intervals are disjoint, so ja names it).
    // A certificate key is only a lower bound of K_bar: such a node's points
    // are bounded above by its ub (an ancestor's exact bound), and the gap
    // certified while it is queued is taken from that (infinite when some
    // such node has no exactly bounded ancestor).
    i128 best_gap = -1;
    unsigned best_ja = 0xFFFFFFFFu;
    for (int i = tid; i < n; i += NTF) {
        const Node nd = fr[i];
        const i128 k = mk128(nd.khi, nd.klo);
        if (improvable(k, nd.ja, Kinc, jinc)) {
            const i128 gap = k - Kinc;
            atomicAdd(&s_hist[bitlen128(gap)], 1);
            if (nd.jb & kNodeCert) {
                s_anycert = 1;
                atomicMax(&s_ubmax, __float_as_int(nd.ub));  // ub >= 0: int order is float order
            }
            if (gap > best_gap || (gap == best_gap && nd.ja < best_ja)) {
                best_gap = gap;
                best_ja = nd.ja;
            }
        }
    }
    block_argmax(best_gap, best_ja, s_hi, s_lo, s_j);
    // the gap classes from the largest down, one thread each: `before` =
    // improvable nodes in larger classes, n_keep = all of them
    const int hb = tid < 130 ? s_hist[129 - tid] : 0;
    int n_keep = 0;
    const int before = block_scan(hb, s_wave, n_keep);
    if (tid == 0) {
        s.bound_evals += s_nbound;
        s.event_hyp += s_nbound * p.n_events;
        s.pixel_updates += (long long)s_pix;
        s.nodes_pruned += s_pruned;
        // the gap certified so far (queued and selected nodes), kept for a
        // search that is cut short after this step (-1: none certified)
        i128 gap = best_gap < 0 ? (i128)0 : best_gap;
        bool gap_inf = false;
        if (s_anycert) {
            const float u = __int_as_float(s_ubmax);
            if (!(u < INFINITY)) {
                gap_inf = true;
            } else {
                const i128 g = ceil_i128(u) - Kinc;
                if (g > gap) gap = g;
            }
        }
        sp128(gap_inf ? (i128)-1 : gap, s.gap_hi, s.gap_lo);
        int stop = 0;
        if (overflow) {
            s.status = -5;  // ECMD_EFRONTIER
            sp128((i128)-1, s.gap_hi, s.gap_lo);
            stop = 1;
        } else if (n_keep == 0) {
            s.status = 0;
            s.gap_hi = 0;
            s.gap_lo = 0;
            stop = 1;
        } else if (sp.gamma_key >= 0 && !gap_inf && gap <= (i128)sp.gamma_key) {
            s.status = 0;
            sp128(gap, s.gap_hi, s.gap_lo);
            s.nodes_pruned += n_keep;
            stop = 1;
        }
        int take = min(F, n_keep);
        if (!stop && sp.max_nodes > 0) {
            const long long left = sp.max_nodes - s.nodes_expanded;
            if (left <= 0) {
                s.status = -4;  // ECMD_EBUDGET
                sp128(best_gap, s.gap_hi, s.gap_lo);
                stop = 1;
            } else if (left < take) {
                take = (int)left;
            }
        }
        s_stop = stop;
        s_take = take;
    }
    __syncthreads();
    // take every node of a larger gap class and the first `quota` of class
    // b*, the class where the running count reaches `take`
    if (!s_stop && tid < 130 && before < s_take && s_take <= before + hb) {
        s_bstar = 129 - tid;
        s_quota = s_take - before;
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

    // (4) split the queue into the nodes expanded now and the rest (in
    // place).  One node: Algorithm 1's pop, the best node found above.
    // More: every node of the larger gap classes and the first `quota`
    // of class b* in queue order.
    const bool pop_one = s_take == 1;
    int out = 0, nsel = 0, inb = 0, nkids = 0;
    for (int base = 0; base < n; base += NTF) {
        const int i = base + tid;
        Node nd = Node{};
        int keep = 0, cand = 0, big = 0;
        if (i < n) {
            nd = fr[i];
            const i128 k = mk128(nd.khi, nd.klo);
            if (improvable(k, nd.ja, Kinc, jinc)) {
                if (pop_one) {
                    big = nd.ja == best_ja;
                    keep = !big;
                } else {
                    const int b = bitlen128(k - Kinc);
                    big = b > s_bstar;
                    cand = b == s_bstar;
                    keep = !big && !cand;
                }
            }
        }
        int tot_c;
        const int rc = block_scan(cand, s_wave, tot_c);
        const int take = big || (cand && inb + rc < s_quota);
        if (cand && !take) keep = 1;
        inb += tot_c;
        const unsigned jb = nd.jb & ~kNodeCert;
        const int kids = take && jb - nd.ja >= 4;
        int tot_k, tot_t, tot_d;
        const int rk = block_scan(keep, s_wave, tot_k);
        const int rt = block_scan(take, s_wave, tot_t);
        block_scan(kids, s_wave, tot_d);
        if (keep) fr[out + rk] = nd;
        if (take) {
            Sel x;
            x.ja = nd.ja;
            x.jb = jb;
            x.jc = (nd.ja + jb) >> 1;
            x.kids = kids ? 1u : 0u;
            x.lc = nd.lc;
            x.ub = (nd.jb & kNodeCert) ? nd.ub : ub_float(mk128(nd.khi, nd.klo));
            sl[nsel + rt] = x;
        }
        out += tot_k;
        nsel += tot_t;
        nkids += tot_d;
    }
    __syncthreads();
    if (tid == 0) {
        s.n_front = out;
        s.n_sel = nsel;
        s.nodes_expanded += nsel;
        s.steps += 1;
        st[w] = s;
    }
    emit_hyps(sp, p, w, T, s_tiles, nt, sl, nsel, out, nkids, (float)i128_to_double(Kinc), hyps + (long long)w * HS,
              act + (long long)w * HS, items, qcap, qf, s_wave);
}

// Grid range still alive in each active window: the queued nodes and those
// selected for the next step.  Every later hypothesis is a grid interval or
// point inside it and the warp is monotone in d, so events binned with this
// range still reach every tile they can reach for the rest of the search;
// binning again with it drops the guest copies that only the early, wide
// intervals needed.
__global__ __launch_bounds__(NTF) void k_live_range(Search sp, const WinState* __restrict__ st,
                                                    const Node* __restrict__ front, const Sel* __restrict__ sel,
                                                    WinParam* __restrict__ wp) {
    const int w = blockIdx.x, tid = threadIdx.x;
    __shared__ unsigned s_lo, s_hi;
    const WinState s = st[w];
    if (!s.active) return;
    if (tid == 0) {
        s_lo = 0xFFFFFFFFu;
        s_hi = 0u;
    }
    __syncthreads();
    const Node* fr = front + (long long)w * sp.CAP;
    const Sel* sl = sel + (long long)w * sp.F;
    unsigned lo = 0xFFFFFFFFu, hi = 0u;
    for (int i = tid; i < s.n_front; i += NTF) {
        lo = min(lo, fr[i].ja);
        hi = max(hi, fr[i].jb & ~kNodeCert);
    }
    for (int i = tid; i < s.n_sel; i += NTF) {
        lo = min(lo, sl[i].ja);
        hi = max(hi, sl[i].jb);
    }
    atomicMin(&s_lo, lo);
    atomicMax(&s_hi, hi);
    __syncthreads();
    if (tid == 0 && s_lo <= s_hi) {
        WinParam p = wp[w];
        p.r_lo = rate_of(grid_d(sp.d_lo, sp.d_hi, sp.L, s_lo), p.tau);
        p.r_hi = rate_of(grid_d(sp.d_lo, sp.d_hi, sp.L, s_hi), p.tau);
        set_guest_cuts(p);
        wp[w] = p;
    }
}

hipError_t launch_live_range(hipStream_t s, const Search& sp, const WinState* st, const Node* front, const Sel* sel,
                             WinParam* wp, int B) {
    if (B <= 0) return hipSuccess;
    k_live_range<<<B, NTF, 0, s>>>(sp, st, front, sel, wp);
    return hipGetLastError();
}

hipError_t launch_frontier(hipStream_t s, int phase, const Search& sp, const WinParam* wp, int B, int T,
                           const long long* seg_off, WinState* st, Node* front, Sel* sel, Hyp* hyps, int* act,
                           const Part* part, Item* items, int qcap, Queue* q_fill, int* n_active, hipEvent_t t0,
                           hipEvent_t t1) {
    if (B <= 0) return hipSuccess;
    if (phase == 0)
        hipExtLaunchKernelGGL(k_frontier_a, dim3(B), dim3(NTF), 0u, s, t0, t1, 0u, sp, wp, B, T, seg_off, st, front,
                              sel, hyps, act, part, items, qcap, q_fill, n_active);
    else
        hipExtLaunchKernelGGL(k_frontier_b, dim3(B), dim3(NTF), 0u, s, t0, t1, 0u, sp, wp, B, T, seg_off, st, front,
                              sel, hyps, act, part, items, qcap, q_fill, n_active);
    return hipGetLastError();
}

// ------------------------------------------------------------ asynchronous plan

// The host-side checks of a synchronous call, made on the device for the
// launches of a plan: window w is valid when its offsets are non-negative and
// non-decreasing, it holds fewer than 2^28 events, its exact sums fit 64
// bits, tau > 0 is finite and d_hi * tau < 1 (eq. (11)).  n: its events.
__device__ __forceinline__ bool window_ok(const long long* off, const float* tau, int w, float d_hi, int W, int H,
                                          long long& n) {
    const long long a = off[w], b = off[w + 1];
    n = b - a;
    if (a < 0 || n < 0 || n >= kMaxWindowEvents) return false;
    const double bound = (double)n * (double)n * 2.0 * ((double)W + H + 3.0);
    if (bound >= 9.0e18) return false;
    const float t = tau[w];
    if (!(t > 0.0f) || !isfinite(t)) return false;
    return d_hi * t < 1.0f;
}

constexpr int kCheckThreads = 1024;

// One workgroup: wstat[w] = 0 for a valid window, else ECMD_EINVAL (every
// window when the valid ones hold more than max_events events); blk = the
// exclusive prefix of the prep blocks (`chunk` events each) of the valid
// windows, B + 1 entries; werr, both queue sets and n_active cleared.
// Thread k checks the windows [k * per, (k + 1) * per).
__global__ __launch_bounds__(kCheckThreads) void k_plan_check(
    const long long* __restrict__ off, const float* __restrict__ tau, int B, float d_hi, int W, int H,
    long long max_events, int chunk, int* __restrict__ wstat, int* __restrict__ werr, int* __restrict__ blk,
    Queue* __restrict__ q, int* __restrict__ n_active) {
    __shared__ long long s_ev[kCheckThreads / 64];
    __shared__ int s_scan[kCheckThreads];
    const int tid = threadIdx.x;
    if (tid < 2 * kXcd) {
        q[tid].n_items = 0;
        q[tid].next = 0;
    }
    if (tid == 0) *n_active = 0;
    const int per = (B + kCheckThreads - 1) / kCheckThreads;
    const int w0 = min(B, tid * per), w1 = min(B, w0 + per);
    long long ev = 0;
    int nb = 0;
    for (int w = w0; w < w1; ++w) {
        long long n;
        if (window_ok(off, tau, w, d_hi, W, H, n)) {
            ev += n;
            nb += (int)((n + chunk - 1) / chunk);
        }
    }
    // events of the valid windows: wave sums, then the workgroup's
    for (int o = 32; o > 0; o >>= 1) ev += __shfl_xor(ev, o);
    if ((tid & 63) == 0) s_ev[tid >> 6] = ev;
    // inclusive scan of the block counts (Hillis-Steele)
    s_scan[tid] = nb;
    __syncthreads();
    for (int o = 1; o < kCheckThreads; o <<= 1) {
        const int a = tid >= o ? s_scan[tid - o] : 0;
        __syncthreads();
        s_scan[tid] += a;
        __syncthreads();
    }
    long long total = 0;
    for (int k = 0; k < kCheckThreads / 64; ++k) total += s_ev[k];
    const bool over = total > max_events;
    int run = over ? 0 : s_scan[tid] - nb;
    for (int w = w0; w < w1; ++w) {
        long long n;
        const bool ok = window_ok(off, tau, w, d_hi, W, H, n) && !over;
        wstat[w] = ok ? 0 : -1;  // ECMD_EINVAL
        werr[w] = 0;
        blk[w] = run;
        if (ok) run += (int)((n + chunk - 1) / chunk);
    }
    if (tid == kCheckThreads - 1) blk[B] = over ? 0 : s_scan[tid];
}

__global__ void k_fill_u32(unsigned* __restrict__ p, long long n, unsigned v) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

// Per-window results of a plan launch, written to `out` (device memory or
// pinned host memory), with the same arithmetic as a synchronous call.
__global__ void k_plan_results(Search sp, int B, const WinState* __restrict__ st, const long long* __restrict__ off,
                               const float* __restrict__ tau, ecmd_result* __restrict__ out) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= B) return;
    const WinState s = st[w];
    ecmd_result r = {};
    r.L = (uint32_t)sp.L;
    if (s.status == -1 || s.status == -2) {  // rejected before the search: only the status
        r.status = s.status;
        out[w] = r;
        return;
    }
    r.status = s.active ? -4 : s.status;  // still running when the steps ran out: ECMD_EBUDGET
    r.j_star = s.j_inc;
    r.d_hat = grid_d(sp.d_lo, sp.d_hi, sp.L, s.j_inc);
    r.K_lo = s.Kinc_lo;
    r.K_hi = s.Kinc_hi;
    const double M2 = (double)sp.M * (double)sp.M;
    r.contrast = i128_to_double(mk128(s.Kinc_hi, s.Kinc_lo)) / M2;
    const double t = (double)tau[w];
    r.d_end = (double)r.d_hat / (1.0 - (double)r.d_hat * t);
    // no finite gap certified: a frontier overflow, or a search cut short
    // while a node kept on its endpoint certificate, with no exactly bounded
    // ancestor, was queued
    r.gap = (s.status == -5 || s.gap_hi < 0) ? (double)INFINITY : i128_to_double(mk128(s.gap_hi, s.gap_lo)) / M2;
    r.n_events = off[w + 1] - off[w];
    r.nodes_expanded = s.nodes_expanded;
    r.nodes_pruned = s.nodes_pruned;
    r.point_evals = s.point_evals;
    r.bound_evals = s.bound_evals;
    r.event_hyp_evals = s.event_hyp;
    r.pixel_updates = s.pixel_updates;
    r.steps = s.steps;
    r.seeded = s.seeded;
    r.bound_certs = s.cert_evals;
    out[w] = r;
}

hipError_t launch_plan_check(hipStream_t s, const long long* off, const float* tau, int B, float d_hi, int W, int H,
                             long long max_events, int chunk, int* wstat, int* werr, int* blk, Queue* q,
                             int* n_active) {
    k_plan_check<<<1, kCheckThreads, 0, s>>>(off, tau, B, d_hi, W, H, max_events, chunk, wstat, werr, blk, q,
                                             n_active);
    return hipGetLastError();
}

hipError_t launch_fill_u32(hipStream_t s, unsigned* p, long long n, unsigned v) {
    if (n <= 0) return hipSuccess;
    const long long nb = (n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192;
    k_fill_u32<<<(int)nb, 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_plan_results(hipStream_t s, const Search& sp, int B, const WinState* st, const long long* off,
                               const float* tau, ecmd_result* out) {
    if (B <= 0) return hipSuccess;
    k_plan_results<<<(B + 255) / 256, 256, 0, s>>>(sp, B, st, off, tau, out);
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
            long long a = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0;
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
                                                              const double* __restrict__ t,
                                                              const signed char* __restrict__ p, long long n,
                                                              double t0, double t1, const int* __restrict__ blk_off,
                                                              float* __restrict__ xo, float* __restrict__ yo,
                                                              float* __restrict__ to, signed char* __restrict__ po) {
    __shared__ int s[kSelThreads];
    long long i = (long long)blockIdx.x * kSelThreads + threadIdx.x;
    int keep = (i < n && t[i] >= t0 && t[i] <= t1) ? 1 : 0;
    s[threadIdx.x] = keep;
    __syncthreads();
    for (int o = 1; o < kSelThreads; o <<= 1) {
        int a = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0;
        __syncthreads();
        s[threadIdx.x] += a;
        __syncthreads();
    }
    if (keep) {
        long long k = (long long)blk_off[blockIdx.x] + s[threadIdx.x] - 1;
        xo[k] = x[i];
        yo[k] = y[i];
        to[k] = (float)(t[i] - t0);
        if (p) po[k] = p[i];
    }
}

hipError_t launch_select(hipStream_t s, const float* x, const float* y, const double* t, const signed char* p,
                         long long n, double t0, double t1, float* xo, float* yo, float* to, signed char* po,
                         int* blk_cnt, long long* total) {
    const int nb = (int)((n + kSelThreads - 1) / kSelThreads);
    if (nb > 0) {
        k_select_count<<<nb, kSelThreads, 0, s>>>(t, n, t0, t1, blk_cnt);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    k_select_scan<<<1, 1024, 0, s>>>(nb, blk_cnt, total);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nb == 0) return e;
    k_select_write<<<nb, kSelThreads, 0, s>>>(x, y, t, p, n, t0, t1, blk_cnt, xo, yo, to, po);
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
