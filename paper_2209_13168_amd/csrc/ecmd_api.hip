// Host runtime and C ABI of the MI355X divergence estimator.
//
// One call = prep (tile binning of every window's events, a1) -> init of the
// per-window branch and bound (Alg. 1) -> repeated [evaluate hypotheses
// (a2, a3), frontier step (a4)] until every window is certified.  All
// search state stays in device memory; the host only launches and polls a
// single counter of windows still running.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <string>
#include <vector>

#include "ecmd.h"
#include "ecmd_internal.hpp"

using namespace ecmd;

namespace {

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t bytes) {
        if (bytes <= cap) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
        size_t want = std::max(bytes, (size_t)256);
        hipError_t e = hipMalloc(&p, want);
        if (e == hipSuccess) cap = want;
        return e;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

struct HostBuf {
    void* p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t bytes) {
        if (bytes <= cap) return hipSuccess;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
        size_t want = std::max(bytes, (size_t)256);
        hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
        if (e == hipSuccess) cap = want;
        return e;
    }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
    }
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

constexpr int kChunk = 4096;          // events per prep workgroup
constexpr int kDefaultF = 96;         // nodes expanded together (measured: 64 to 192 within 3%; 96 best)
constexpr int kDefaultCap = 16384;    // queued nodes per window
constexpr int kMaxSteps = 1 << 20;    // hard stop of the step loop
constexpr int kMaxRebins = 2;         // re-binnings of the events per search

}  // namespace

struct ecmd_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    std::vector<ecmd_cnn*> nets;  // live networks created on this context
    std::vector<ecmd_batch_plan*> plans;  // live plans created on this context
    int num_cu = 0;
    size_t max_lds = 0;
    size_t eval_lds = 0;   // LDS bytes of the last evaluation set-up (0 = none yet)
    int eval_nt = 0;       // threads per evaluation workgroup of that set-up
    int eval_nb = 0;       // evaluation workgroups for that size
    // staging of host inputs
    DevBuf sx, sy, st, soff, stau, sseed, spol;
    // prep
    DevBuf wp, blk, cnt_own, cnt_guest, seg_off, seg_own, cursor, ev, err_flag;
    // search
    DevBuf state, front, sel, hyps, act, items, queues, part, n_active;
    // probes / window selection / downsample
    DevBuf pix, img, keep, counts, misc;
    HostBuf pinned;
    std::vector<long long> h_off;
    std::vector<float> h_tau;
    // launch tuning and the captured step graph
    ecmd_tuning tune{};
    hipStream_t own_stream = nullptr;  // work stream when the caller gives the null stream
    hipGraphExec_t gexec = nullptr;
    std::vector<unsigned char> gkey;
    // phase timers
    bool profiling = false;
    ecmd_profile prof{};
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
};

// Event pair around a launch when profiling (kind: 0 eval, 1 frontier, 2 prep).
struct Mark {
    hipEvent_t a, b;
    int kind;
};

static hipEvent_t pool_event(ecmd_ctx* c) {
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->ev_pool.push_back(e);
    }
    return c->ev_pool[c->ev_used++];
}

struct Timers {
    ecmd_ctx* c;
    std::vector<Mark> marks;
    hipEvent_t pending = nullptr;
    hipEvent_t last = nullptr;  // end event of the previous launch, if nothing was enqueued since
    explicit Timers(ecmd_ctx* ctx) : c(ctx) { c->ev_used = 0; }
    void begin() {
        if (!c->profiling) return;
        if (last) {  // back-to-back launches share the boundary event
            pending = last;
            last = nullptr;
            return;
        }
        pending = pool_event(c);
        if (pending) (void)hipEventRecord(pending, c->stream);
    }
    void end(int kind) {
        if (!c->profiling || !pending) return;
        hipEvent_t b = pool_event(c);
        if (!b) return;
        (void)hipEventRecord(b, c->stream);
        marks.push_back(Mark{pending, b, kind});
        pending = nullptr;
        last = b;
    }
    // other work is enqueued next: the following launch records its own start
    void cut() { last = nullptr; }
    // A pair of events for one kernel launched with them (the dispatch takes
    // the kernel's own start and end times; no event is recorded on the
    // stream), or two nulls when not profiling.
    void pair(int kind, hipEvent_t& a, hipEvent_t& b) {
        a = b = nullptr;
        if (!c->profiling) return;
        a = pool_event(c);
        b = pool_event(c);
        if (!a || !b) {
            a = b = nullptr;
            return;
        }
        marks.push_back(Mark{a, b, kind});
        last = nullptr;
    }
    // after the stream has been synchronised
    void collect() {
        if (!c->profiling) return;
        for (const Mark& m : marks) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, m.a, m.b) != hipSuccess) continue;
            if (m.kind == 0) { c->prof.eval_ms += ms; c->prof.eval_launches += 1; }
            else if (m.kind == 1) { c->prof.frontier_ms += ms; c->prof.frontier_launches += 1; }
            else c->prof.prep_ms += ms;
        }
        c->prof.calls += 1;
        marks.clear();
    }
};

struct ecmd_cnn {
    ecmd_ctx* ctx = nullptr;  // NULL once the context is destroyed
    DevBuf P, m, v, grad, pg, lossb, loss, out, imgs, labels, seeds;
    int step = 0;
};

static void cnn_release(ecmd_cnn* n) {
    DevBuf* bufs[] = {&n->P, &n->m, &n->v, &n->grad, &n->pg, &n->lossb, &n->loss, &n->out, &n->imgs, &n->labels,
                      &n->seeds};
    for (DevBuf* b : bufs) b->release();
}

static int fail(ecmd_ctx* c, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

#define HIPCHK(ctx, expr)                                                                    \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail((ctx), e_ == hipErrorOutOfMemory ? ECMD_ENOMEM : ECMD_EDEVICE,       \
                        "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
    } while (0)

// ---------------------------------------------------------------- helpers

// Grid point j of depth L (fp64 then fp32; identical to the device's).
static float host_grid_d(float d_lo, float d_hi, int L, unsigned j) {
    double span = (double)d_hi - (double)d_lo;
    double v = (double)d_lo + span * ldexp((double)j, -L);
    return (float)v;
}

static int grid_depth(float d_lo, float d_hi, float eps) {
    double span = (double)d_hi - (double)d_lo;
    for (int L = 1; L <= 30; ++L)
        if (ldexp(span, -L) <= (double)eps) return L;
    return -1;
}

// Tile plan: column and row cuts at the FOE lines when the FOE is an
// integer point strictly inside the sensor (no event crosses them), then
// each band split evenly until every tile's counters, (w + 2)(h + 2) with
// the one-cell border, fit the budget max_px.
// npol = 1, or 2 for the polarity-aware contrast (one tiled image per
// polarity); segments = tiles x npol stay within kMaxTiles.
static bool plan_geometry(int W, int H, float cx, float cy, int max_px, int npol, Geometry& g) {
    memset(&g, 0, sizeof g);
    g.W = W;
    g.H = H;
    g.cx = cx;
    g.cy = cy;
    std::vector<int> bx = {0}, by = {0};
    if (cx == floorf(cx) && cx > 0.0f && cx < (float)W) bx.push_back((int)cx);
    if (cy == floorf(cy) && cy > 0.0f && cy < (float)H) by.push_back((int)cy);
    bx.push_back(W);
    by.push_back(H);
    auto split = [](const std::vector<int>& base, int k) {
        std::vector<int> cut;
        for (size_t b = 0; b + 1 < base.size(); ++b) {
            int a = base[b], e = base[b + 1];
            for (int i = 0; i < k; ++i) cut.push_back(a + (int)((long long)(e - a) * i / k));
        }
        cut.push_back(base.back());
        return cut;
    };
    auto max_band = [](const std::vector<int>& cut) {
        int m = 0;
        for (size_t i = 0; i + 1 < cut.size(); ++i) m = std::max(m, cut[i + 1] - cut[i]);
        return m;
    };
    int best = -1;
    std::vector<int> bc, br;
    for (int kx = 1; kx <= 32; ++kx) {
        for (int ky = 1; ky <= 32; ++ky) {
            std::vector<int> c = split(bx, kx), r = split(by, ky);
            int ntx = (int)c.size() - 1, nty = (int)r.size() - 1;
            if (ntx * nty * npol > kMaxTiles) continue;
            // counters of the largest tile, with its one-cell border
            if ((long long)(max_band(c) + 2) * (max_band(r) + 2) > max_px) continue;
            // fewest tiles, then the squarest
            int score = ntx * nty * 1000 + std::abs(max_band(c) - max_band(r)) % 1000;
            if (best < 0 || score < best) {
                best = score;
                bc = c;
                br = r;
            }
        }
    }
    if (best < 0) return false;
    g.ntx = (int)bc.size() - 1;
    g.nty = (int)br.size() - 1;
    g.nsp = g.ntx * g.nty;
    g.T = g.nsp * npol;
    for (int i = 0; i <= g.ntx; ++i) g.colcut[i] = bc[i];
    for (int i = 0; i <= g.nty; ++i) g.rowcut[i] = br[i];
    g.max_tile_px = max_band(bc) * max_band(br);
    g.ring_px = (max_band(bc) + 2) * (max_band(br) + 2);
    return true;
}

static int check_sensor(ecmd_ctx* c, const ecmd_sensor* s) {
    if (!s) return fail(c, ECMD_EINVAL, "sensor is NULL");
    if (s->width <= 0 || s->height <= 0 || s->width > 32768 || s->height > 32768)
        return fail(c, ECMD_EINVAL, "sensor size %dx%d out of range", s->width, s->height);
    if (!isfinite(s->foe_x) || !isfinite(s->foe_y)) return fail(c, ECMD_EINVAL, "FOE is not finite");
    return ECMD_OK;
}

static int check_search(ecmd_ctx* c, const ecmd_search* s, int* L) {
    if (!s) return fail(c, ECMD_EINVAL, "search is NULL");
    if (!isfinite(s->d_lo) || !isfinite(s->d_hi) || !(s->d_lo >= 0.0f) || !(s->d_lo < s->d_hi))
        return fail(c, ECMD_EINVAL, "need 0 <= d_lo < d_hi (got %g, %g)", s->d_lo, s->d_hi);
    if (!(s->eps > 0.0f) || !isfinite(s->eps)) return fail(c, ECMD_EINVAL, "eps must be > 0");
    *L = grid_depth(s->d_lo, s->d_hi, s->eps);
    if (*L < 1) return fail(c, ECMD_EINVAL, "eps too small for range (depth > 30)");
    if (!(s->gamma >= 0.0) || !isfinite(s->gamma)) return fail(c, ECMD_EINVAL, "gamma must be >= 0");
    if (s->max_nodes < 0) return fail(c, ECMD_EINVAL, "max_nodes must be >= 0");
    if (s->frontier_batch < 0 || s->frontier_batch > 1024)
        return fail(c, ECMD_EINVAL, "frontier_batch must be in [0, 1024]");
    if (s->frontier_capacity < 0) return fail(c, ECMD_EINVAL, "frontier_capacity must be >= 0");
    return ECMD_OK;
}

// Event arrays of a call: device pointers (borrowed) or staged copies.
struct Inputs {
    const float *x = nullptr, *y = nullptr, *t = nullptr, *seeds = nullptr, *tau = nullptr;
    const long long* off = nullptr;
    const signed char* pol = nullptr;  // polarities (device), or NULL: one event image
};

static int stage(ecmd_ctx* c, DevBuf& buf, const void* src, size_t bytes, uint32_t flags,
                 const void** out) {
    if (flags & ECMD_DEVICE_PTR) {
        *out = src;
        return ECMD_OK;
    }
    HIPCHK(c, buf.ensure(bytes));
    if (bytes) HIPCHK(c, hipMemcpyAsync(buf.p, src, bytes, hipMemcpyHostToDevice, c->stream));
    *out = buf.p;
    return ECMD_OK;
}

static double key_to_double(long long hi, unsigned long long lo) {
    __int128 k = (__int128)(((unsigned __int128)(unsigned long long)hi << 64) | (unsigned __int128)lo);
    return (double)k;
}

// --------------------------------------------------------------- pipeline

// Prep of B windows: window params, event binning.  Needs h_off (host copy
// of the offsets) and h_tau.  rebin: keep the window params already on the
// device (binning ranges narrowed to the live search).  copies_out: event
// records written, guest copies included.
static int run_prep(ecmd_ctx* c, const Geometry& g, const Inputs& in, int B, float d_lo, float d_hi,
                    int* nblk_out, long long* copies_out = nullptr) {
    const int T = g.T;
    std::vector<int> blk(B + 1, 0);
    for (int w = 0; w < B; ++w) {
        long long n = c->h_off[w + 1] - c->h_off[w];
        blk[w + 1] = blk[w] + (int)((n + kChunk - 1) / kChunk);
    }
    const int nblk = blk[B];
    HIPCHK(c, c->wp.ensure(sizeof(WinParam) * std::max(B, 1)));
    HIPCHK(c, c->blk.ensure(sizeof(int) * (B + 1)));
    // staging of blk (B + 1 ints) and, later, of the total and B error flags
    HIPCHK(c, c->pinned.ensure(sizeof(int) * B + 72));
    memcpy(c->pinned.p, blk.data(), sizeof(int) * (B + 1));
    HIPCHK(c, hipMemcpyAsync(c->blk.p, c->pinned.p, sizeof(int) * (B + 1), hipMemcpyHostToDevice, c->stream));
    const size_t nctr = prep_counters(B, T);
    HIPCHK(c, c->cnt_own.ensure(sizeof(int) * nctr));
    HIPCHK(c, c->seg_off.ensure(sizeof(long long) * (B * T + 1)));
    HIPCHK(c, c->seg_own.ensure(sizeof(int) * seg_own_words(B, T)));
    HIPCHK(c, c->cursor.ensure(sizeof(unsigned long long) * nctr));
    HIPCHK(c, c->err_flag.ensure(sizeof(int) * B));
    HIPCHK(c, hipMemsetAsync(c->cnt_own.p, 0, sizeof(int) * nctr, c->stream));
    HIPCHK(c, hipMemsetAsync(c->err_flag.p, 0, sizeof(int) * B, c->stream));
    HIPCHK(c, launch_winparam(c->stream, g, in.tau, in.off, B, d_lo, d_hi, c->wp.as<WinParam>()));
    // count + scan (scatter needs the total to size the event store)
    HIPCHK(c, launch_prep(c->stream, 0, g, in.x, in.y, in.t, in.pol, in.off, c->wp.as<WinParam>(), B, c->blk.as<int>(),
                          nblk, kChunk, c->cnt_own.as<int>(), c->seg_off.as<long long>(), c->seg_own.as<int>(),
                          c->cursor.as<unsigned long long>(), nullptr, c->err_flag.as<int>(), -1));
    HIPCHK(c, hipMemcpyAsync(c->pinned.p, c->seg_off.as<long long>() + (size_t)B * T, sizeof(long long),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync((char*)c->pinned.p + 8, c->err_flag.p, sizeof(int) * B, hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const long long total = *(long long*)c->pinned.p;
    const int* errf = (const int*)((char*)c->pinned.p + 8);
    for (int w = 0; w < B; ++w)
        if (errf[w])
            return fail(c, ECMD_EINVAL, "window %d: an event has a non-finite coordinate or t_rel outside [0, tau]",
                        w);
    // padding: the evaluation kernel prefetches up to kEvalPad records past
    // the end of a segment
    HIPCHK(c, c->ev.ensure(sizeof(float4) * (size_t)(total + kEvalPad)));
    HIPCHK(c, launch_prep(c->stream, 1, g, in.x, in.y, in.t, in.pol, in.off, c->wp.as<WinParam>(), B, c->blk.as<int>(),
                          nblk, kChunk, nullptr, nullptr, nullptr, c->cursor.as<unsigned long long>(),
                          c->ev.as<float4>(), nullptr, -1));
    *nblk_out = nblk;
    if (copies_out) *copies_out = total;
    return ECMD_OK;
}

// Bin the events again with the window parameters on the device (binning
// ranges narrowed to the live search), without waiting: the windows and
// their prep blocks are those of the last run_prep, the records cannot
// outnumber its (a narrower range reaches a subset of the tiles), and its
// checks of the events hold.  The scatter writes nothing if the records
// would not fit the store; run_search checks the total afterwards.
static hipError_t enqueue_rebin(ecmd_ctx* c, const Geometry& g, const Inputs& in, int B, int nblk) {
    const size_t nctr = prep_counters(B, g.T);
    hipError_t e = hipMemsetAsync(c->cnt_own.p, 0, sizeof(int) * nctr, c->stream);
    if (e != hipSuccess) return e;
    e = launch_prep(c->stream, 0, g, in.x, in.y, in.t, in.pol, in.off, c->wp.as<WinParam>(), B, c->blk.as<int>(), nblk,
                    kChunk, c->cnt_own.as<int>(), c->seg_off.as<long long>(), c->seg_own.as<int>(),
                    c->cursor.as<unsigned long long>(), nullptr, c->err_flag.as<int>(), -1);
    if (e != hipSuccess) return e;
    const long long cap = (long long)(c->ev.cap / sizeof(float4)) - kEvalPad;
    return launch_prep(c->stream, 1, g, in.x, in.y, in.t, in.pol, in.off, c->wp.as<WinParam>(), B, c->blk.as<int>(),
                       nblk, kChunk, nullptr, c->seg_off.as<long long>(), nullptr, c->cursor.as<unsigned long long>(),
                       c->ev.as<float4>(), nullptr, cap);
}

// Most counters (a tile's pixels and its one-cell border) that the
// evaluation workgroup's LDS holds.
static int tile_budget_for(size_t max_lds) {
    int px = (int)(max_lds / 4);
    while (px > 0 && eval_lds_bytes(px) > max_lds) --px;
    return px;
}

static int tile_budget(ecmd_ctx* c) { return tile_budget_for(c->max_lds); }

// Image tiling and evaluation workgroup size.  Explicit tuning wins
// (tile_px caps the counters per tile, eval_threads sets the workgroup;
// 0 = the whole LDS, 1024).  Otherwise the first of: tiles small enough for
// three 512-thread workgroups per CU, for two, then one 1024-thread
// workgroup on the whole LDS, where the smaller tilings may cut the image
// into at most kMaxSmallTiles tiles.  Measured: several smaller workgroups
// per CU hide latency that one 16-wave workgroup cannot (32 windows of
// 346x260 in 8 tiles: 321 us per evaluation launch against 363 us in 4;
// 64 windows of 640x480 in 24 tiles: 2.33 ms against 2.68 ms in 8), but a
// guest copy walks its whole path in every tile it is copied to, so many
// cuts cost more than they save (256 windows of 1280x720, D up to 2: 2.22 s
// of evaluation in 48 tiles against 1.92 s in 24 with 1024 threads).
constexpr int kMaxSmallTiles = 24;

static bool choose_tiling(size_t max_lds, const ecmd_tuning& tu, int W, int H, float cx, float cy, int npol,
                          Geometry& g, int& nt, int& budget) {
    const int full = tile_budget_for(max_lds);
    if (tu.tile_px > 0 || tu.eval_threads > 0) {
        budget = tu.tile_px > 0 ? std::min(tu.tile_px, full) : full;
        nt = tu.eval_threads > 0 ? tu.eval_threads : 1024;
        return plan_geometry(W, H, cx, cy, budget, npol, g);
    }
    const int divs[] = {3, 2}, nts[] = {512, 512};
    for (int k = 0; k < 2; ++k) {
        budget = tile_budget_for(max_lds / divs[k]);
        nt = nts[k];
        if (plan_geometry(W, H, cx, cy, budget, npol, g) && g.nsp <= kMaxSmallTiles) return true;
    }
    budget = full;
    nt = 1024;
    return plan_geometry(W, H, cx, cy, budget, npol, g);
}

// Persistent workgroup count of the evaluation kernel for `lds` bytes of
// LDS: as many as fit at once, at most 4 per CU.  The kernel's dynamic LDS
// limit is raised to the device maximum once per context, so that every
// context's launches fit whatever another context set.
static hipError_t eval_setup(ecmd_ctx* c, size_t lds, int nt, int* nb) {
    if (c->eval_lds != lds || c->eval_nt != nt) {
        hipError_t e = eval_set_lds(c->max_lds);
        if (e != hipSuccess) return e;
        int per_cu = 0;
        if (eval_occupancy(&per_cu, lds, nt) != hipSuccess || per_cu < 1) per_cu = 1;
        c->eval_lds = lds;
        c->eval_nt = nt;
        c->eval_nb = c->num_cu * std::min(per_cu, 8);
    }
    *nb = c->eval_nb;
    return hipSuccess;
}

// Hypotheses per work item for B windows: two once there are ~48 items per
// CU, else one (measured: 2 is best for 32 windows of 346x260 and for the
// 256-window 1280x720 batch, 1 for 8 windows or fewer; larger groups save
// set-ups but leave launches ending on a few long items), unless the
// context's tuning fixes it.
static int group_for(ecmd_ctx* c, int B, const Search& sp, int T) {
    if (c->tune.group > 0) return std::min(c->tune.group, 64);
    const long long work = (long long)B * sp.HS * T;
    const long long slots = (long long)c->num_cu * 48;
    return (int)std::max(1ll, std::min(2ll, work / std::max(slots, 1ll)));
}

// Group size of the search: the most hypotheses per item (group_for) and,
// unless the tuning fixes it, the per-step rule the frontier applies: the
// first steps of a search have few hypotheses, and groups of one then keep
// more workgroups busy.
static void set_groups(ecmd_ctx* c, int B, Search& sp, int T) {
    sp.G = group_for(c, B, sp, T);
    sp.B = B;
    sp.gslots = c->tune.group > 0 ? 0 : std::max((long long)c->num_cu * 48, 1ll);
}

// Whole batched search on staged inputs; fills out[0..B).
static int run_search(ecmd_ctx* c, const ecmd_sensor* sensor, const Inputs& in, int B,
                      const ecmd_search* search, int L, ecmd_result* out) {
    const int W = sensor->width, H = sensor->height;
    const int npol = in.pol ? 2 : 1;
    const long long M = (long long)W * H * npol;  // cells of the event image(s): the key is M*S - N^2
    Geometry g;
    int nt = 0, budget = 0;
    if (!choose_tiling(c->max_lds, c->tune, W, H, sensor->foe_x, sensor->foe_y, npol, g, nt, budget))
        return fail(c, ECMD_EINVAL, "sensor %dx%d needs more than %d tiles", W, H, kMaxTiles / npol);
    Timers tm(c);
    int nblk = 0;
    long long copies = 0;
    tm.begin();
    int rc = run_prep(c, g, in, B, search->d_lo, search->d_hi, &nblk, &copies);
    if (rc) return rc;
    tm.end(2);
    tm.cut();
    const long long n_events = c->h_off[B] - c->h_off[0];
    int rebins = 0;

    Search sp;
    sp.d_lo = search->d_lo;
    sp.d_hi = search->d_hi;
    sp.L = L;
    sp.F = search->frontier_batch > 0 ? search->frontier_batch
                                      : (c->tune.frontier_batch > 0 ? c->tune.frontier_batch : kDefaultF);
    sp.CAP = search->frontier_capacity > 0 ? search->frontier_capacity : kDefaultCap;
    sp.HS = 3 * sp.F;
    sp.max_nodes = search->max_nodes;
    sp.gamma_key = search->gamma > 0.0 ? (long long)floor(search->gamma * (double)M * (double)M) : -1;
    sp.M = M;
    sp.cert = (search->flags & ECMD_SEARCH_EXACT_BOUNDS) ? 0 : 1;
    sp.pad = 0;
    const int T = g.T;
    set_groups(c, B, sp, T);
    HIPCHK(c, c->state.ensure(sizeof(WinState) * B));
    HIPCHK(c, c->front.ensure(sizeof(Node) * (size_t)B * sp.CAP));
    HIPCHK(c, c->sel.ensure(sizeof(Sel) * (size_t)B * sp.F));
    HIPCHK(c, c->hyps.ensure(sizeof(Hyp) * (size_t)B * sp.HS));
    HIPCHK(c, c->act.ensure(sizeof(int) * (size_t)B * sp.HS));
    const int qcap = ((B + kXcd - 1) / kXcd) * sp.HS * T;  // windows w = r (mod kXcd) share queue r
    HIPCHK(c, c->items.ensure(sizeof(Item) * (size_t)kXcd * qcap));
    HIPCHK(c, c->queues.ensure(sizeof(Queue) * 2 * kXcd));
    HIPCHK(c, c->part.ensure(sizeof(Part) * (size_t)B * sp.HS * T));
    HIPCHK(c, c->n_active.ensure(sizeof(int)));
    HIPCHK(c, hipMemsetAsync(c->queues.p, 0, sizeof(Queue) * 2 * kXcd, c->stream));
    HIPCHK(c, hipMemsetAsync(c->n_active.p, 0, sizeof(int), c->stream));
    Queue* q = c->queues.as<Queue>();
    HIPCHK(c, launch_init(c->stream, sp, c->wp.as<WinParam>(), in.seeds, B, c->state.as<WinState>(),
                          c->sel.as<Sel>(), c->hyps.as<Hyp>(), c->act.as<int>(), c->items.as<Item>(), qcap, &q[0],
                          T, c->seg_off.as<long long>(), InitCheck{nullptr, nullptr, 0}));
    const size_t lds = eval_lds_bytes(g.ring_px);
    int nb = 0;
    HIPCHK(c, eval_setup(c, lds, nt, &nb));
    int active = B;
    auto run_step = [&](bool timed) -> hipError_t {
        // one step: evaluate the step's hypotheses (queue set 0), frontier
        // phase 0 (queues the exact bounds of failed certificates in set 1),
        // evaluate those, frontier phase 1 (queues the next step in set 0)
        for (int parity = 0; parity < 2; ++parity) {
            hipEvent_t a = nullptr, b = nullptr;
            if (timed) tm.pair(0, a, b);
            hipError_t e = launch_eval(c->stream, g, nb, nt, lds, c->ev.as<float4>(), c->seg_off.as<long long>(),
                                       c->seg_own.as<int>(), c->wp.as<WinParam>(), c->hyps.as<Hyp>(), c->act.as<int>(),
                                       c->items.as<Item>(), qcap, &q[parity * kXcd], &q[(1 - parity) * kXcd],
                                       c->part.as<Part>(), sp.HS, nullptr, a, b);
            if (e != hipSuccess) return e;
            if (timed) tm.pair(1, a, b);
            e = launch_frontier(c->stream, parity, sp, c->wp.as<WinParam>(), B, T, c->seg_off.as<long long>(),
                                c->state.as<WinState>(), c->front.as<Node>(), c->sel.as<Sel>(), c->hyps.as<Hyp>(),
                                c->act.as<int>(), c->part.as<Part>(), c->items.as<Item>(), qcap,
                                &q[(1 - parity) * kXcd], c->n_active.as<int>(), a, b);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    const bool graph = c->tune.graph && !c->profiling;
    if (graph) {
        // the captured pair depends on every pointer and by-value argument
        std::vector<unsigned char> key;
        auto put = [&](const void* p, size_t n) {
            const unsigned char* b = (const unsigned char*)p;
            key.insert(key.end(), b, b + n);
        };
        void* ptrs[] = {c->ev.p, c->seg_off.p, c->seg_own.p, c->hyps.p, c->act.p, c->items.p, c->queues.p, c->part.p,
                        c->wp.p, c->state.p, c->front.p, c->sel.p, c->n_active.p, (void*)c->stream};
        put(ptrs, sizeof ptrs);
        put(&g, sizeof g);
        put(&sp, sizeof sp);
        int ints[] = {B, T, nb, (int)lds, qcap};
        put(ints, sizeof ints);
        if (!c->gexec || key != c->gkey) {
            if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
            c->gexec = nullptr;
            hipGraph_t gr = nullptr;
            HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            hipError_t e1 = run_step(false);
            hipError_t e2 = hipStreamEndCapture(c->stream, &gr);
            HIPCHK(c, e1);
            HIPCHK(c, e2);
            hipError_t e3 = hipGraphInstantiate(&c->gexec, gr, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gr);
            HIPCHK(c, e3);
            c->gkey = key;
        }
    }
    // Blocks of four steps.  After each block the host copies the count of
    // finished windows (and the event records) to pinned memory, but waits
    // for block b's copy only once block b + 1 is enqueued, so the device
    // never idles on the host; the block after the last is empty work.
    HIPCHK(c, c->pinned.ensure(64));
    char* const poll = (char*)c->pinned.p;  // two slots: [n_active int][pad][records int64]
    hipEvent_t pev[2] = {pool_event(c), pool_event(c)};
    if (!pev[0] || !pev[1]) return fail(c, ECMD_EDEVICE, "hipEventCreate failed");
    auto enqueue_block = [&](int b) -> hipError_t {
        hipError_t e;
        for (int k = 0; k < 4; ++k) {
            if (graph) {
                if ((e = hipGraphLaunch(c->gexec, c->stream)) != hipSuccess) return e;
            } else if ((e = run_step(true)) != hipSuccess) {
                return e;
            }
        }
        if (!graph) tm.cut();
        char* slot = poll + 16 * (b & 1);
        if ((e = hipMemcpyAsync(slot, c->n_active.p, sizeof(int), hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
            return e;
        if ((e = hipMemcpyAsync(slot + 8, c->seg_off.as<long long>() + (size_t)B * T, sizeof(long long),
                                hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
            return e;
        return hipEventRecord(pev[b & 1], c->stream);
    };
    int blocks = 0;
    HIPCHK(c, enqueue_block(blocks++));
    for (;;) {
        // Events copied to several tiles (guests) are binned by the whole
        // search range; once the frontier has narrowed, bin again with each
        // window's live range (after blocks 1 .. kMaxRebins, while the last
        // binning known here copied more than 1% of the events) to drop
        // copies no longer needed.
        if (rebins < kMaxRebins && copies > n_events + n_events / 100) {
            tm.begin();
            HIPCHK(c, launch_live_range(c->stream, sp, c->state.as<WinState>(), c->front.as<Node>(),
                                        c->sel.as<Sel>(), c->wp.as<WinParam>(), B));
            HIPCHK(c, enqueue_rebin(c, g, in, B, nblk));
            tm.end(2);
            tm.cut();
            ++rebins;
        }
        const bool more = blocks * 4 < kMaxSteps;
        if (more) HIPCHK(c, enqueue_block(blocks++));
        const int done = more ? blocks - 2 : blocks - 1;  // the block whose copy is awaited
        HIPCHK(c, hipEventSynchronize(pev[done & 1]));
        const char* slot = poll + 16 * (done & 1);
        active = B + *(const int*)slot;  // n_active counts finished windows down from zero
        copies = *(const long long*)(slot + 8);
        if (active == 0 || !more) break;
    }
    std::vector<WinState> hs(B);
    HIPCHK(c, hipMemcpyAsync(hs.data(), c->state.p, sizeof(WinState) * B, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(poll, c->seg_off.as<long long>() + (size_t)B * T, sizeof(long long),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    tm.collect();
    if (*(const long long*)poll > (long long)(c->ev.cap / sizeof(float4)) - kEvalPad)
        return fail(c, ECMD_EDEVICE, "re-binned events exceed the event store");
    int first_status = ECMD_OK;
    for (int w = 0; w < B; ++w) {
        const WinState& s = hs[w];
        ecmd_result& r = out[w];
        memset(&r, 0, sizeof r);
        r.status = s.active ? ECMD_EBUDGET : s.status;
        r.j_star = s.j_inc;
        r.L = (uint32_t)L;
        r.d_hat = host_grid_d(search->d_lo, search->d_hi, L, s.j_inc);
        r.K_lo = s.Kinc_lo;
        r.K_hi = s.Kinc_hi;
        const double M2 = (double)M * (double)M;
        r.contrast = key_to_double(s.Kinc_hi, s.Kinc_lo) / M2;
        const double tau = (double)c->h_tau[w];
        r.d_end = (double)r.d_hat / (1.0 - (double)r.d_hat * tau);
        // no finite gap certified: a frontier overflow, or a search cut
        // short while a node kept on its endpoint certificate, with no
        // exactly bounded ancestor, was queued
        if (s.status == ECMD_EFRONTIER || s.gap_hi < 0) r.gap = INFINITY;
        else r.gap = key_to_double(s.gap_hi, s.gap_lo) / M2;
        r.n_events = c->h_off[w + 1] - c->h_off[w];
        r.nodes_expanded = s.nodes_expanded;
        r.nodes_pruned = s.nodes_pruned;
        r.point_evals = s.point_evals;
        r.bound_evals = s.bound_evals;
        r.event_hyp_evals = s.event_hyp;
        r.pixel_updates = s.pixel_updates;
        r.steps = s.steps;
        r.seeded = s.seeded;
        r.bound_certs = s.cert_evals;
        if (r.status != ECMD_OK && first_status == ECMD_OK) first_status = r.status;
    }
    return first_status;
}

static int batched_impl(ecmd_ctx* c, const ecmd_sensor* sensor, const float* x, const float* y,
                        const float* t_rel, const int8_t* pol, const int64_t* offsets, const float* tau, int32_t B,
                        const ecmd_search* search, uint32_t flags, const float* d_seeds, ecmd_result* out) {
    if (!c) return ECMD_EINVAL;
    c->err.clear();
    int rc = check_sensor(c, sensor);
    if (rc) return rc;
    int L = 0;
    rc = check_search(c, search, &L);
    if (rc) return rc;
    if (B < 0 || B > 65535) return fail(c, ECMD_EINVAL, "B = %d out of range", B);
    if (B == 0) return ECMD_OK;
    if (!offsets || !tau || !out) return fail(c, ECMD_EINVAL, "NULL offsets, tau or out");
    HIPCHK(c, hipSetDevice(c->device));
    c->h_off.assign(B + 1, 0);
    c->h_tau.assign(B, 0.0f);
    if (flags & ECMD_DEVICE_PTR) {
        HIPCHK(c, hipMemcpyAsync(c->h_off.data(), offsets, sizeof(long long) * (B + 1), hipMemcpyDeviceToHost,
                                 c->stream));
        HIPCHK(c, hipMemcpyAsync(c->h_tau.data(), tau, sizeof(float) * B, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    } else {
        memcpy(c->h_off.data(), offsets, sizeof(long long) * (B + 1));
        memcpy(c->h_tau.data(), tau, sizeof(float) * B);
    }
    if (c->h_off[0] < 0) return fail(c, ECMD_EINVAL, "offsets[0] < 0");
    for (int w = 0; w < B; ++w) {
        long long n = c->h_off[w + 1] - c->h_off[w];
        if (n < 0) return fail(c, ECMD_EINVAL, "offsets decrease at window %d", w);
        if (n >= kMaxWindowEvents) return fail(c, ECMD_EINVAL, "window %d has too many events (limit 2^28 - 1)", w);
        double bound = (double)n * (double)n * 2.0 * ((double)sensor->width + sensor->height + 3.0);
        if (bound >= 9.0e18) return fail(c, ECMD_EINVAL, "window %d: sums would overflow 64 bits", w);
        float t = c->h_tau[w];
        if (!(t > 0.0f) || !isfinite(t)) return fail(c, ECMD_EINVAL, "tau[%d] must be > 0", w);
        if (!(search->d_hi * t < 1.0f))
            return fail(c, ECMD_EINVAL, "window %d: d_hi * tau must be < 1 (cheirality)", w);
    }
    const long long n_total = c->h_off[B];
    if (n_total > 0 && (!x || !y || !t_rel)) return fail(c, ECMD_EINVAL, "NULL event arrays");
    Inputs in;
    const void* p;
    if ((rc = stage(c, c->sx, x, sizeof(float) * n_total, flags, &p))) return rc;
    in.x = (const float*)p;
    if ((rc = stage(c, c->sy, y, sizeof(float) * n_total, flags, &p))) return rc;
    in.y = (const float*)p;
    if ((rc = stage(c, c->st, t_rel, sizeof(float) * n_total, flags, &p))) return rc;
    in.t = (const float*)p;
    if ((rc = stage(c, c->soff, offsets, sizeof(long long) * (B + 1), flags, &p))) return rc;
    in.off = (const long long*)p;
    if ((rc = stage(c, c->stau, tau, sizeof(float) * B, flags, &p))) return rc;
    in.tau = (const float*)p;
    if (pol) {
        if ((rc = stage(c, c->spol, pol, (size_t)n_total, flags, &p))) return rc;
        in.pol = (const signed char*)p;
    }
    if (d_seeds) {
        if ((rc = stage(c, c->sseed, d_seeds, sizeof(float) * B, flags, &p))) return rc;
        in.seeds = (const float*)p;
    }
    return run_search(c, sensor, in, B, search, L, out);
}


// ------------------------------------------------------- asynchronous plan

// The shape of batched searches up to fixed limits: tiling, search
// parameters and launch sizes (set once, by ecmd_plan_create or by each
// allocation-free call).
struct PlanShape {
    ecmd_plan_limits lim{};
    Geometry g{};
    Search sp{};       // G is set per launch
    int nblk_max = 0;  // prep workgroups of the largest launch
    int qcap = 0;
    size_t lds = 0;
    int nt = 0;        // threads per evaluation workgroup
    int nb = 0;
};

// Device buffers of a plan, in this order.
enum PlanBuf {
    PB_WP, PB_BLK, PB_CNT, PB_SEG_OFF, PB_SEG_OWN, PB_CURSOR, PB_EV, PB_WERR, PB_WSTAT, PB_STATE, PB_FRONT, PB_SEL,
    PB_HYPS, PB_ACT, PB_ITEMS, PB_QUEUES, PB_PART, PB_NACTIVE, PB_COUNT
};

// Bytes of each device buffer for the shape's limits.
static void plan_sizes(const PlanShape& sh, size_t* bytes) {
    const int Bm = sh.lim.max_windows, T = sh.g.T;
    const Search& sp = sh.sp;
    const size_t nctr = prep_counters(Bm, T);
    bytes[PB_WP] = sizeof(WinParam) * Bm;
    bytes[PB_BLK] = sizeof(int) * (Bm + 1);
    bytes[PB_CNT] = sizeof(int) * nctr;
    bytes[PB_SEG_OFF] = sizeof(long long) * ((size_t)Bm * T + 1);
    bytes[PB_SEG_OWN] = sizeof(int) * seg_own_words(Bm, T);
    bytes[PB_CURSOR] = sizeof(unsigned long long) * nctr;
    bytes[PB_EV] = sizeof(float4) * (size_t)(sh.lim.max_records + kEvalPad);  // padded as in the synchronous call
    bytes[PB_WERR] = sizeof(int) * Bm;
    bytes[PB_WSTAT] = sizeof(int) * Bm;
    bytes[PB_STATE] = sizeof(WinState) * Bm;
    bytes[PB_FRONT] = sizeof(Node) * (size_t)Bm * sp.CAP;
    bytes[PB_SEL] = sizeof(Sel) * (size_t)Bm * sp.F;
    bytes[PB_HYPS] = sizeof(Hyp) * (size_t)Bm * sp.HS;
    bytes[PB_ACT] = sizeof(int) * (size_t)Bm * sp.HS;
    bytes[PB_ITEMS] = sizeof(Item) * (size_t)kXcd * sh.qcap;
    bytes[PB_QUEUES] = sizeof(Queue) * 2 * kXcd;
    bytes[PB_PART] = sizeof(Part) * (size_t)Bm * sp.HS * T;
    bytes[PB_NACTIVE] = sizeof(int);
}

// Device buffers of batched searches up to fixed limits; a launch only
// enqueues kernels (no allocation, host copy or wait), so it can be
// captured into a graph and replayed.
struct ecmd_batch_plan {
    ecmd_ctx* ctx = nullptr;  // NULL once the context is destroyed
    ecmd_sensor sensor{};
    ecmd_search search{};
    PlanShape sh;
    DevBuf buf[PB_COUNT];
};

static void plan_release(ecmd_batch_plan* p) {
    for (DevBuf& b : p->buf) b.release();
}

// Validates the sensor, search and limits and fills the shape (zero limits
// replaced by the values used); sets the context's evaluation kernel up.
static int plan_shape(ecmd_ctx* c, const ecmd_sensor* sensor, const ecmd_search* search,
                      const ecmd_plan_limits* lim, PlanShape& sh) {
    int rc = check_sensor(c, sensor);
    if (rc) return rc;
    int L = 0;
    rc = check_search(c, search, &L);
    if (rc) return rc;
    if (!lim) return fail(c, ECMD_EINVAL, "limits is NULL");
    if (lim->max_windows < 1 || lim->max_windows > 65535)
        return fail(c, ECMD_EINVAL, "max_windows = %d out of range 1 .. 65535", lim->max_windows);
    if (lim->max_events < 1 || lim->max_events > (1ll << 40))
        return fail(c, ECMD_EINVAL, "max_events = %lld out of range 1 .. 2^40", (long long)lim->max_events);
    if (lim->max_steps < 0 || lim->max_steps > kMaxSteps)
        return fail(c, ECMD_EINVAL, "max_steps = %d out of range 0 .. %d", lim->max_steps, kMaxSteps);
    if (lim->max_records < 0) return fail(c, ECMD_EINVAL, "max_records must be >= 0");
    HIPCHK(c, hipSetDevice(c->device));
    const int W = sensor->width, H = sensor->height;
    const int npol = lim->polarity ? 2 : 1;
    Geometry& g = sh.g;
    int nt = 0, budget = 0;
    if (!choose_tiling(c->max_lds, c->tune, W, H, sensor->foe_x, sensor->foe_y, npol, g, nt, budget))
        return fail(c, ECMD_EINVAL, "sensor %dx%d needs more than %d tiles", W, H, kMaxTiles / npol);
    ecmd_plan_limits L2 = *lim;
    // default: twice the grid depth and eight more (a level-synchronous
    // search needs about L steps; finished steps still cost two launches)
    if (L2.max_steps == 0) L2.max_steps = min(2 * L + 8, kMaxSteps);
    L2.max_steps = (L2.max_steps + 3) / 4 * 4;  // whole polling blocks of four steps
    if (L2.max_records == 0) {
        // an event's tiles over any range lie in its FOE quadrant (no event
        // crosses an FOE line), so it has at most that many copies
        const bool xcut = sensor->foe_x == floorf(sensor->foe_x) && sensor->foe_x > 0.0f && sensor->foe_x < (float)W;
        const bool ycut = sensor->foe_y == floorf(sensor->foe_y) && sensor->foe_y > 0.0f && sensor->foe_y < (float)H;
        const long long per = (long long)(xcut ? g.ntx / 2 : g.ntx) * (ycut ? g.nty / 2 : g.nty);
        L2.max_records = L2.max_events * per;
    }
    sh.lim = L2;
    Search& sp = sh.sp;
    sp.d_lo = search->d_lo;
    sp.d_hi = search->d_hi;
    sp.L = L;
    sp.F = search->frontier_batch > 0 ? search->frontier_batch
                                      : (c->tune.frontier_batch > 0 ? c->tune.frontier_batch : kDefaultF);
    sp.CAP = search->frontier_capacity > 0 ? search->frontier_capacity : kDefaultCap;
    sp.HS = 3 * sp.F;
    sp.max_nodes = search->max_nodes;
    const long long M = (long long)W * H * npol;
    sp.gamma_key = search->gamma > 0.0 ? (long long)floor(search->gamma * (double)M * (double)M) : -1;
    sp.M = M;
    sp.cert = (search->flags & ECMD_SEARCH_EXACT_BOUNDS) ? 0 : 1;
    sp.pad = 0;
    sp.G = 1;
    sp.B = 1;
    sp.gslots = 0;
    const int Bm = L2.max_windows;
    sh.nblk_max = (int)((L2.max_events + kChunk - 1) / kChunk) + Bm;
    sh.qcap = ((Bm + kXcd - 1) / kXcd) * sp.HS * g.T;
    sh.lds = eval_lds_bytes(g.ring_px);
    sh.nt = nt;
    HIPCHK(c, eval_setup(c, sh.lds, sh.nt, &sh.nb));
    return ECMD_OK;
}

// The prep of a launch: clear the counters, count + scan, scatter (at most
// max_records records).
static hipError_t plan_prep(const PlanShape& sh, void* const* b, hipStream_t s, const float* x, const float* y,
                            const float* t, const signed char* pol, const long long* off, int B) {
    const Geometry& g = sh.g;
    hipError_t e = launch_fill_u32(s, (unsigned*)b[PB_CNT], (long long)prep_counters(B, g.T), 0u);
    if (e != hipSuccess) return e;
    e = launch_prep(s, 0, g, x, y, t, pol, off, (const WinParam*)b[PB_WP], B, (const int*)b[PB_BLK], sh.nblk_max,
                    kChunk, (int*)b[PB_CNT], (long long*)b[PB_SEG_OFF], (int*)b[PB_SEG_OWN],
                    (unsigned long long*)b[PB_CURSOR], nullptr, (int*)b[PB_WERR], -1);
    if (e != hipSuccess) return e;
    return launch_prep(s, 1, g, x, y, t, pol, off, (const WinParam*)b[PB_WP], B, (const int*)b[PB_BLK], sh.nblk_max,
                       kChunk, nullptr, (long long*)b[PB_SEG_OFF], nullptr, (unsigned long long*)b[PB_CURSOR],
                       (float4*)b[PB_EV], nullptr, sh.lim.max_records);
}

// Enqueues a whole batched search of B windows on the context's stream with
// the plan buffers b (device checks, prep, a fixed number of steps, results).
static int plan_enqueue(ecmd_ctx* c, const PlanShape& sh, void* const* b, const float* x, const float* y,
                        const float* t_rel, const int8_t* polarity, const int64_t* offsets, const float* tau, int B,
                        const float* d_seeds, ecmd_result* out) {
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = c->stream;
    const Geometry& g = sh.g;
    const int T = g.T;
    Search sp = sh.sp;
    set_groups(c, B, sp, T);
    const long long* off = (const long long*)offsets;
    const signed char* pol = (const signed char*)polarity;
    WinParam* wp = (WinParam*)b[PB_WP];
    WinState* st = (WinState*)b[PB_STATE];
    Sel* sel = (Sel*)b[PB_SEL];
    Hyp* hyps = (Hyp*)b[PB_HYPS];
    int* act = (int*)b[PB_ACT];
    Item* items = (Item*)b[PB_ITEMS];
    Queue* q = (Queue*)b[PB_QUEUES];
    Part* part = (Part*)b[PB_PART];
    long long* seg_off = (long long*)b[PB_SEG_OFF];
    HIPCHK(c, launch_plan_check(s, off, tau, B, sp.d_hi, g.W, g.H, sh.lim.max_events, kChunk, (int*)b[PB_WSTAT],
                                (int*)b[PB_WERR], (int*)b[PB_BLK], q, (int*)b[PB_NACTIVE]));
    HIPCHK(c, launch_winparam(s, g, tau, off, B, sp.d_lo, sp.d_hi, wp));
    HIPCHK(c, plan_prep(sh, b, s, x, y, t_rel, pol, off, B));
    HIPCHK(c, launch_init(s, sp, wp, d_seeds, B, st, sel, hyps, act, items, sh.qcap, &q[0], T, seg_off,
                          InitCheck{(const int*)b[PB_WSTAT], (const int*)b[PB_WERR], (long long)sh.lim.max_records}));
    for (int step = 0; step < sh.lim.max_steps; step += 4) {
        for (int k = 0; k < 8; ++k) {  // four steps of two phases
            const int parity = k & 1;
            HIPCHK(c, launch_eval(s, g, sh.nb, sh.nt, sh.lds, (const float4*)b[PB_EV], seg_off,
                                  (const int*)b[PB_SEG_OWN], wp, hyps, act, items, sh.qcap, &q[parity * kXcd],
                                  &q[(1 - parity) * kXcd], part, sp.HS, nullptr));
            HIPCHK(c, launch_frontier(s, parity, sp, wp, B, T, seg_off, st, (Node*)b[PB_FRONT], sel, hyps, act, part,
                                      items, sh.qcap, &q[(1 - parity) * kXcd], (int*)b[PB_NACTIVE]));
        }
        // bin again with the live ranges, at the synchronous call's polling
        // points (unconditionally: the host does not see the copy count)
        if (step / 4 < kMaxRebins && step + 4 < sh.lim.max_steps) {
            HIPCHK(c, launch_live_range(s, sp, st, (const Node*)b[PB_FRONT], sel, wp, B));
            HIPCHK(c, plan_prep(sh, b, s, x, y, t_rel, pol, off, B));
        }
    }
    HIPCHK(c, launch_plan_results(s, sp, B, st, off, tau, out));
    return ECMD_OK;
}

// The allocation-free batched search takes its device buffers from this
// array (each device that loads the library holds one copy until the
// process ends).  Its device address is looked up once per device when a
// context is created on it, and only that address is used by host code.
// Calls on one device share the array: calls that overlap (on different
// streams or threads) race.
constexpr size_t kScratchBytes = (size_t)ECMD_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kScratchDevices = 64;
static void* g_scratch_at[kScratchDevices];
static std::mutex g_scratch_mu;

// The scratch array's device address on `device` (the current device),
// looked up on first use.  NULL when the lookup fails.
static void* scratch_address(int device) {
    if (device < 0 || device >= kScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_at[device]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch_at[device] = ptr;
    }
    return g_scratch_at[device];
}

// ------------------------------------------------------------------ ABI

extern "C" {

const char* ecmd_version(void) { return "ecmd-mi355x 0.1"; }

int ecmd_ctx_create(ecmd_ctx** out, int device, void* hip_stream) {
    if (!out) return ECMD_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return ECMD_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return ECMD_EDEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return ECMD_EDEVICE;
    ecmd_ctx* c = new (std::nothrow) ecmd_ctx();
    if (!c) return ECMD_ENOMEM;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    if (!c->stream) {
        // a blocking stream of default priority: ordered with the null stream,
        // and capturable into a graph
        if (hipStreamCreate(&c->own_stream) != hipSuccess) {
            delete c;
            return ECMD_EDEVICE;
        }
        c->stream = c->own_stream;
    }
    c->num_cu = prop.multiProcessorCount;
    c->max_lds = prop.sharedMemPerBlock;
    // the allocation-free call's scratch on this device (device current)
    if (device < kScratchDevices && !scratch_address(device)) {
        if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
        delete c;
        return ECMD_EDEVICE;
    }
    *out = c;
    return ECMD_OK;
}

void ecmd_ctx_destroy(ecmd_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    DevBuf* bufs[] = {&c->sx, &c->sy, &c->st, &c->soff, &c->stau, &c->sseed, &c->spol, &c->wp, &c->blk, &c->cnt_own,
                      &c->cnt_guest, &c->seg_off, &c->seg_own, &c->cursor, &c->ev, &c->err_flag, &c->state,
                      &c->front, &c->sel, &c->hyps, &c->act, &c->items, &c->queues, &c->part, &c->n_active, &c->pix,
                      &c->img, &c->keep, &c->counts, &c->misc};
    for (DevBuf* b : bufs) b->release();
    // networks and plans outlive their context only as empty handles
    for (ecmd_cnn* n : c->nets) {
        cnn_release(n);
        n->ctx = nullptr;
    }
    for (ecmd_batch_plan* p : c->plans) {
        plan_release(p);
        p->ctx = nullptr;
    }
    c->pinned.release();
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    delete c;
}

const char* ecmd_last_error(const ecmd_ctx* c) { return c ? c->err.c_str() : "NULL context"; }

int ecmd_plan(const ecmd_sensor* sensor, const ecmd_search* search, int32_t polarity, int64_t lds_bytes,
              int32_t tile_px, ecmd_plan_info* out) {
    if (!sensor || !search || !out || lds_bytes < 0 || tile_px < 0) return ECMD_EINVAL;
    if (sensor->width <= 0 || sensor->height <= 0 || sensor->width > 32768 || sensor->height > 32768)
        return ECMD_EINVAL;
    if (!isfinite(sensor->foe_x) || !isfinite(sensor->foe_y)) return ECMD_EINVAL;
    if (!(search->eps > 0.0f) || !(search->d_lo >= 0.0f) || !(search->d_lo < search->d_hi)) return ECMD_EINVAL;
    const int L = grid_depth(search->d_lo, search->d_hi, search->eps);
    if (L < 1) return ECMD_EINVAL;
    const int npol = polarity ? 2 : 1;
    ecmd_tuning tu{};
    tu.tile_px = tile_px;
    Geometry g;
    int nt = 0, budget = 0;
    if (!choose_tiling(lds_bytes ? (size_t)lds_bytes : (size_t)160 * 1024, tu, sensor->width, sensor->height,
                       sensor->foe_x, sensor->foe_y, npol, g, nt, budget))
        return ECMD_EINVAL;
    memset(out, 0, sizeof *out);
    out->L = L;
    out->segments = g.T;
    out->ntx = g.ntx;
    out->nty = g.nty;
    out->max_tile_px = g.max_tile_px;
    out->tile_budget_px = budget;
    out->eval_threads = nt;
    for (int i = 0; i <= g.ntx; ++i) out->colcut[i] = g.colcut[i];
    for (int i = 0; i <= g.nty; ++i) out->rowcut[i] = g.rowcut[i];
    return ECMD_OK;
}

int ecmd_measure_peaks(ecmd_ctx* c, int64_t hbm_bytes, double* lds_atomics_per_s, double* hbm_read_bytes_per_s) {
    if (!c || hbm_bytes < 0 || !lds_atomics_per_s || !hbm_read_bytes_per_s) return ECMD_EINVAL;
    c->err.clear();
    HIPCHK(c, hipSetDevice(c->device));
    const long long bytes = (hbm_bytes ? hbm_bytes : (4ll << 30)) & ~255ll;
    if (bytes < (1ll << 20)) return fail(c, ECMD_EINVAL, "hbm_bytes must be at least 1 MiB");
    const int lds_blocks = c->num_cu * 2, iters = 4096;
    const int hbm_blocks = c->num_cu * 8;
    HIPCHK(c, c->misc.ensure(sizeof(float) * (size_t)std::max(lds_blocks, hbm_blocks)));
    DevBuf big;
    hipError_t e = big.ensure((size_t)bytes);
    if (e != hipSuccess) return fail(c, ECMD_ENOMEM, "cannot allocate %lld bytes", bytes);
    e = hipMemsetAsync(big.p, 0, (size_t)bytes, c->stream);  // first touch outside the timing
    hipEvent_t a = nullptr, b = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    double best_lds = 0.0, best_hbm = 0.0;
    for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
        float ms = 0.0f;
        e = hipEventRecord(a, c->stream);
        if (e == hipSuccess) e = launch_lds_atomics(c->stream, lds_blocks, iters, c->misc.as<unsigned>());
        if (e == hipSuccess) e = hipEventRecord(b, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (e == hipSuccess && ms > 0.0f && rep > 0)
            best_lds = std::max(best_lds, (double)lds_blocks * 1024.0 * iters / (ms * 1e-3));
        if (e == hipSuccess) e = hipEventRecord(a, c->stream);
        if (e == hipSuccess) e = launch_stream_read(c->stream, big.p, bytes, hbm_blocks, c->misc.as<float>());
        if (e == hipSuccess) e = hipEventRecord(b, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (e == hipSuccess && ms > 0.0f && rep > 0) best_hbm = std::max(best_hbm, (double)bytes / (ms * 1e-3));
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    (void)hipStreamSynchronize(c->stream);
    big.release();
    HIPCHK(c, e);
    *lds_atomics_per_s = best_lds;
    *hbm_read_bytes_per_s = best_hbm;
    return ECMD_OK;
}

float ecmd_grid_point(float d_lo, float d_hi, uint32_t L, uint32_t j) {
    if (L < 1 || L > 30 || j > (1u << L)) return NAN;
    return host_grid_d(d_lo, d_hi, (int)L, j);
}

int ecmd_ctx_set_tuning(ecmd_ctx* c, const ecmd_tuning* t) {
    if (!c || !t) return ECMD_EINVAL;
    if (t->frontier_batch < 0 || t->frontier_batch > 1024 || t->tile_px < 0 || t->group < 0 || t->group > 64)
        return fail(c, ECMD_EINVAL, "tuning out of range");
    if (t->eval_threads != 0 && t->eval_threads != 256 && t->eval_threads != 512 && t->eval_threads != 1024)
        return fail(c, ECMD_EINVAL, "eval_threads must be 0, 256, 512 or 1024");
    c->tune = *t;
    return ECMD_OK;
}

int ecmd_ctx_get_tuning(const ecmd_ctx* c, ecmd_tuning* out) {
    if (!c || !out) return ECMD_EINVAL;
    *out = c->tune;
    return ECMD_OK;
}

int ecmd_autotune(ecmd_ctx* c, const ecmd_sensor* sensor, const float* x, const float* y, const float* t_rel,
                  const int64_t* offsets, const float* tau, int32_t B, const ecmd_search* search, uint32_t flags,
                  ecmd_tuning* best, double* ms_best) {
    if (!c || !search || !best) return ECMD_EINVAL;
    if (B <= 0) return fail(c, ECMD_EINVAL, "autotune needs windows");
    ecmd_search s = *search;
    s.frontier_batch = 0;
    const ecmd_tuning saved = c->tune;
    const bool prof = c->profiling;
    c->profiling = false;
    std::vector<ecmd_result> out(B);
    const int full = tile_budget(c);
    double best_ms = 1e300;
    ecmd_tuning bt = saved;
    int rc_fail = ECMD_OK;
    // best of two timed calls (after one untimed) for tuning t; keeps the best
    auto trial = [&](const ecmd_tuning& t) {
        if (rc_fail) return;
        c->tune = t;
        double ms = 1e300;
        for (int rep = 0; rep < 3; ++rep) {
            auto t0 = std::chrono::steady_clock::now();
            int rc = batched_impl(c, sensor, x, y, t_rel, nullptr, offsets, tau, B, &s, flags, nullptr, out.data());
            auto t1 = std::chrono::steady_clock::now();
            if (rc < 0 && rc != ECMD_EBUDGET && rc != ECMD_EFRONTIER) {
                rc_fail = rc;
                return;
            }
            if (rep > 0) ms = std::min(ms, std::chrono::duration<double, std::milli>(t1 - t0).count());
        }
        if (ms < best_ms) {
            best_ms = ms;
            bt = t;
        }
    };
    // (1) tile size x workgroup size (smaller tiles let more workgroups share
    // a CU), (2) frontier batch, (3) hypotheses per item and graph replay
    ecmd_tuning t0{};
    t0.frontier_batch = kDefaultF;
    trial(t0);  // the default tiling rule
    const int cands[][2] = {{full, 1024}, {full / 2, 1024}, {full / 2, 512}, {full / 3, 512}, {full / 4, 512},
                            {full / 4, 256}};
    for (const auto& cd : cands) {
        ecmd_tuning t = t0;
        t.tile_px = cd[0];
        t.eval_threads = cd[1];
        Geometry g;
        if (!plan_geometry(sensor->width, sensor->height, sensor->foe_x, sensor->foe_y, cd[0], 1, g)) continue;
        trial(t);
    }
    const ecmd_tuning b1 = bt;
    for (int F : {16, 32, 128, 256}) {
        ecmd_tuning t = b1;
        t.frontier_batch = F;
        trial(t);
    }
    const ecmd_tuning b2 = bt;
    for (int gv = 0; gv < 3; ++gv) {
        ecmd_tuning t = b2;
        if (gv < 2) t.group = gv == 0 ? 1 : 4;
        else t.graph = 1;
        trial(t);
    }
    if (rc_fail) {
        c->tune = saved;
        c->profiling = prof;
        return rc_fail;
    }
    c->tune = bt;
    c->profiling = prof;
    *best = bt;
    if (ms_best) *ms_best = best_ms;
    return ECMD_OK;
}

int ecmd_ctx_set_profiling(ecmd_ctx* c, int enable) {
    if (!c) return ECMD_EINVAL;
    c->profiling = enable != 0;
    return ECMD_OK;
}

int ecmd_ctx_get_profile(ecmd_ctx* c, ecmd_profile* out, int reset) {
    if (!c || !out) return ECMD_EINVAL;
    *out = c->prof;
    if (reset) c->prof = ecmd_profile{};
    return ECMD_OK;
}

int ecmd_estimate_divergence_batched(ecmd_ctx* c, const ecmd_sensor* sensor, const float* x, const float* y,
                                     const float* t_rel, const int64_t* offsets, const float* tau, int32_t B,
                                     const ecmd_search* search, uint32_t flags, const float* d_seeds,
                                     ecmd_result* out) {
    return batched_impl(c, sensor, x, y, t_rel, nullptr, offsets, tau, B, search, flags, d_seeds, out);
}

int ecmd_estimate_divergence_batched_polarity(ecmd_ctx* c, const ecmd_sensor* sensor, const float* x,
                                              const float* y, const float* t_rel, const int8_t* polarity,
                                              const int64_t* offsets, const float* tau, int32_t B,
                                              const ecmd_search* search, uint32_t flags, const float* d_seeds,
                                              ecmd_result* out) {
    if (!c) return ECMD_EINVAL;
    if (!polarity && B > 0) return fail(c, ECMD_EINVAL, "polarity is NULL");
    return batched_impl(c, sensor, x, y, t_rel, polarity, offsets, tau, B, search, flags, d_seeds, out);
}

int ecmd_plan_create(ecmd_ctx* c, const ecmd_sensor* sensor, const ecmd_search* search, ecmd_plan_limits* lim,
                     ecmd_batch_plan** out) {
    if (!c || !out) return ECMD_EINVAL;
    c->err.clear();
    *out = nullptr;
    PlanShape sh;
    int rc = plan_shape(c, sensor, search, lim, sh);
    if (rc) return rc;
    ecmd_batch_plan* p = new (std::nothrow) ecmd_batch_plan();
    if (!p) return fail(c, ECMD_ENOMEM, "host allocation failed");
    p->ctx = c;
    p->sensor = *sensor;
    p->search = *search;
    p->sh = sh;
    size_t bytes[PB_COUNT];
    plan_sizes(sh, bytes);
    hipError_t e = hipSuccess;
    for (int k = 0; k < PB_COUNT && e == hipSuccess; ++k) e = p->buf[k].ensure(bytes[k]);
    if (e != hipSuccess) {
        plan_release(p);
        delete p;
        HIPCHK(c, e);
    }
    c->plans.push_back(p);
    *lim = sh.lim;
    *out = p;
    return ECMD_OK;
}

int ecmd_plan_launch(ecmd_batch_plan* p, const float* x, const float* y, const float* t_rel, const int8_t* polarity,
                     const int64_t* offsets, const float* tau, int32_t B, const float* d_seeds, ecmd_result* out) {
    if (!p) return ECMD_EINVAL;
    ecmd_ctx* c = p->ctx;
    if (!c) return ECMD_EINVAL;  // the context is gone
    c->err.clear();
    if (B < 1 || B > p->sh.lim.max_windows)
        return fail(c, ECMD_EINVAL, "B = %d out of range 1 .. %d", B, p->sh.lim.max_windows);
    if (!x || !y || !t_rel || !offsets || !tau || !out) return fail(c, ECMD_EINVAL, "NULL array argument");
    if ((polarity != nullptr) != (p->sh.lim.polarity != 0))
        return fail(c, ECMD_EINVAL, "polarity must be given exactly when the plan was created for it");
    void* b[PB_COUNT];
    for (int k = 0; k < PB_COUNT; ++k) b[k] = p->buf[k].p;
    return plan_enqueue(c, p->sh, b, x, y, t_rel, polarity, offsets, tau, B, d_seeds, out);
}

void ecmd_plan_destroy(ecmd_batch_plan* p) {
    if (!p) return;
    if (ecmd_ctx* c = p->ctx) {
        (void)hipSetDevice(c->device);
        (void)hipStreamSynchronize(c->stream);
        plan_release(p);
        c->plans.erase(std::remove(c->plans.begin(), c->plans.end(), p), c->plans.end());
    }
    delete p;
}

int ecmd_estimate_divergence_batched_noalloc(ecmd_ctx* c, const ecmd_sensor* sensor, const ecmd_search* search,
                                             const float* x, const float* y, const float* t_rel,
                                             const int64_t* offsets, const float* tau, int32_t B, int64_t max_events,
                                             const float* d_seeds, ecmd_result* out) {
    if (!c) return ECMD_EINVAL;
    c->err.clear();
    if (B < 1 || B > 65535) return fail(c, ECMD_EINVAL, "B = %d out of range 1 .. 65535", B);
    if (!x || !y || !t_rel || !offsets || !tau || !out) return fail(c, ECMD_EINVAL, "NULL array argument");
    ecmd_plan_limits lim{};
    lim.max_windows = B;
    lim.max_events = max_events;
    PlanShape sh;
    int rc = plan_shape(c, sensor, search, &lim, sh);
    if (rc) return rc;
    size_t bytes[PB_COUNT];
    plan_sizes(sh, bytes);
    void* base = scratch_address(c->device);
    if (!base) return fail(c, ECMD_EDEVICE, "no scratch address on device %d", c->device);
    void* b[PB_COUNT];
    size_t used = 0;
    for (int k = 0; k < PB_COUNT; ++k) {
        b[k] = (char*)base + used;
        used += (bytes[k] + 255) / 256 * 256;  // every buffer on a 256-byte boundary
    }
    if (used > kScratchBytes)
        return fail(c, ECMD_ENOMEM,
                    "%d windows of up to %lld events need %zu bytes of scratch, more than the %zu the "
                    "allocation-free call holds",
                    B, (long long)max_events, used, kScratchBytes);
    return plan_enqueue(c, sh, b, x, y, t_rel, nullptr, offsets, tau, B, d_seeds, out);
}

int ecmd_estimate_divergence(ecmd_ctx* c, const ecmd_sensor* sensor, const ecmd_events* events,
                             ecmd_window window, const ecmd_search* search, uint32_t flags, const float* d_seed,
                             ecmd_result* out) {
    if (!c) return ECMD_EINVAL;
    c->err.clear();
    if (!events || !out) return fail(c, ECMD_EINVAL, "NULL events or out");
    if (events->n < 0) return fail(c, ECMD_EINVAL, "n < 0");
    if (!isfinite(window.t0) || !isfinite(window.t1) || !(window.t1 > window.t0))
        return fail(c, ECMD_EINVAL, "window must have t0 < t1");
    const float tau = (float)(window.t1 - window.t0);
    const long long n = events->n;
    if (n > 0 && (!events->x || !events->y || !events->t)) return fail(c, ECMD_EINVAL, "NULL event arrays");
    HIPCHK(c, hipSetDevice(c->device));
    long long m = 0;
    float* dx;
    float* dy;
    float* dt;
    const bool has_pol = events->p != nullptr;
    if (has_pol) HIPCHK(c, c->spol.ensure((size_t)std::max(n, 1ll)));
    if (flags & ECMD_DEVICE_PTR) {
        HIPCHK(c, c->sx.ensure(sizeof(float) * std::max(n, 1ll)));
        HIPCHK(c, c->sy.ensure(sizeof(float) * std::max(n, 1ll)));
        HIPCHK(c, c->st.ensure(sizeof(float) * std::max(n, 1ll)));
        const int nb = (int)((n + 1023) / 1024);
        HIPCHK(c, c->keep.ensure(sizeof(int) * (nb + 1)));
        HIPCHK(c, c->misc.ensure(sizeof(long long)));
        HIPCHK(c, c->err_flag.ensure(sizeof(int)));
        HIPCHK(c, hipMemsetAsync(c->err_flag.p, 0, sizeof(int), c->stream));
        HIPCHK(c, launch_select(c->stream, events->x, events->y, events->t, (const signed char*)events->p, n,
                                window.t0, window.t1, c->sx.as<float>(), c->sy.as<float>(), c->st.as<float>(),
                                has_pol ? c->spol.as<signed char>() : nullptr, c->keep.as<int>(),
                                c->misc.as<long long>()));
        HIPCHK(c, c->pinned.ensure(64));
        HIPCHK(c, hipMemcpyAsync(c->pinned.p, c->misc.p, sizeof(long long), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        m = *(long long*)c->pinned.p;
        dx = c->sx.as<float>();
        dy = c->sy.as<float>();
        dt = c->st.as<float>();
    } else {
        std::vector<float> hx, hy, ht;
        std::vector<signed char> hp;
        hx.reserve(n);
        for (long long i = 0; i < n; ++i) {
            double t = events->t[i];
            if (t >= window.t0 && t <= window.t1) {
                hx.push_back(events->x[i]);
                hy.push_back(events->y[i]);
                ht.push_back((float)(t - window.t0));
                if (has_pol) hp.push_back((signed char)events->p[i]);
            }
        }
        m = (long long)hx.size();
        HIPCHK(c, c->sx.ensure(sizeof(float) * std::max(m, 1ll)));
        HIPCHK(c, c->sy.ensure(sizeof(float) * std::max(m, 1ll)));
        HIPCHK(c, c->st.ensure(sizeof(float) * std::max(m, 1ll)));
        if (m) {
            HIPCHK(c, hipMemcpyAsync(c->sx.p, hx.data(), sizeof(float) * m, hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(c->sy.p, hy.data(), sizeof(float) * m, hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(c->st.p, ht.data(), sizeof(float) * m, hipMemcpyHostToDevice, c->stream));
            if (has_pol) HIPCHK(c, hipMemcpyAsync(c->spol.p, hp.data(), (size_t)m, hipMemcpyHostToDevice, c->stream));
        }
        HIPCHK(c, hipStreamSynchronize(c->stream));  // host vectors die at scope end
        dx = c->sx.as<float>();
        dy = c->sy.as<float>();
        dt = c->st.as<float>();
    }
    long long off[2] = {0, m};
    float seed = d_seed ? *d_seed : NAN;
    // the staged arrays are device memory: run the batched path on them
    int rc;
    {
        // offsets, tau and the seed are tiny: pass them as host values
        int L = 0;
        rc = check_sensor(c, sensor);
        if (rc) return rc;
        rc = check_search(c, search, &L);
        if (rc) return rc;
        c->h_off.assign(off, off + 2);
        c->h_tau.assign(1, tau);
        if (!(tau > 0.0f)) return fail(c, ECMD_EINVAL, "window too short");
        if (!(search->d_hi * tau < 1.0f)) return fail(c, ECMD_EINVAL, "d_hi * tau must be < 1 (cheirality)");
        double bound = (double)m * (double)m * 2.0 * ((double)sensor->width + sensor->height + 3.0);
        if (bound >= 9.0e18 || m >= kMaxWindowEvents) return fail(c, ECMD_EINVAL, "window has too many events");
        Inputs in;
        in.x = dx;
        in.y = dy;
        in.t = dt;
        if (has_pol) in.pol = c->spol.as<signed char>();
        const void* p;
        if ((rc = stage(c, c->soff, off, sizeof off, 0, &p))) return rc;
        in.off = (const long long*)p;
        if ((rc = stage(c, c->stau, &tau, sizeof tau, 0, &p))) return rc;
        in.tau = (const float*)p;
        if (d_seed) {
            if ((rc = stage(c, c->sseed, &seed, sizeof seed, 0, &p))) return rc;
            in.seeds = (const float*)p;
        }
        rc = run_search(c, sensor, in, 1, search, L, out);
    }
    return rc;
}

int ecmd_probe_pixels(ecmd_ctx* c, const ecmd_sensor* sensor, const float* x, const float* y, const float* t_rel,
                      int64_t n, float tau, float d, uint32_t flags, int32_t* pix_out) {
    if (!c) return ECMD_EINVAL;
    c->err.clear();
    int rc = check_sensor(c, sensor);
    if (rc) return rc;
    if (n < 0 || !(tau > 0.0f) || !isfinite(d) || (n > 0 && (!x || !y || !t_rel || !pix_out)))
        return fail(c, ECMD_EINVAL, "bad probe arguments");
    HIPCHK(c, hipSetDevice(c->device));
    const void *px, *py, *pt;
    if ((rc = stage(c, c->sx, x, sizeof(float) * n, flags, &px))) return rc;
    if ((rc = stage(c, c->sy, y, sizeof(float) * n, flags, &py))) return rc;
    if ((rc = stage(c, c->st, t_rel, sizeof(float) * n, flags, &pt))) return rc;
    int* dpix = (int*)pix_out;
    if (!(flags & ECMD_DEVICE_PTR)) {
        HIPCHK(c, c->pix.ensure(sizeof(int) * std::max(n, (int64_t)1)));
        dpix = c->pix.as<int>();
    }
    HIPCHK(c, launch_probe_pixels(c->stream, (const float*)px, (const float*)py, (const float*)pt, n, tau, d,
                                  sensor->width, sensor->height, sensor->foe_x, sensor->foe_y, dpix));
    if (!(flags & ECMD_DEVICE_PTR) && n)
        HIPCHK(c, hipMemcpyAsync(pix_out, dpix, sizeof(int) * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return ECMD_OK;
}

// Evaluate m hypotheses (points if d_b == NULL) on one window.
static int probe_impl(ecmd_ctx* c, const ecmd_sensor* sensor, const float* x, const float* y, const float* t_rel,
                      const int8_t* pol, int64_t n, float tau, float d_lo, float d_hi, const float* d_a, const float* d_b, int32_t m,
                      uint32_t flags, uint64_t* S, int64_t* N, uint32_t* img_out) {
    if (!c) return ECMD_EINVAL;
    c->err.clear();
    int rc = check_sensor(c, sensor);
    if (rc) return rc;
    if (n < 0 || m < 0 || !(tau > 0.0f) || (n > 0 && (!x || !y || !t_rel)) || (m > 0 && (!d_a || !S || !N)))
        return fail(c, ECMD_EINVAL, "bad probe arguments");
    if (m == 0) return ECMD_OK;
    if (!(d_lo >= 0.0f) || !(d_lo <= d_hi) || !(d_hi * tau < 1.0f))
        return fail(c, ECMD_EINVAL, "probe range must satisfy 0 <= d_lo <= d_hi, d_hi * tau < 1");
    HIPCHK(c, hipSetDevice(c->device));
    const int W = sensor->width, H = sensor->height;
    const int npol = pol ? 2 : 1;
    const long long M = (long long)W * H * npol;  // image cells per hypothesis
    Geometry g;
    int nt = 0, budget = 0;
    if (!choose_tiling(c->max_lds, c->tune, W, H, sensor->foe_x, sensor->foe_y, npol, g, nt, budget))
        return fail(c, ECMD_EINVAL, "sensor needs more than %d tiles", kMaxTiles / npol);
    const int T = g.T;
    Inputs in;
    const void* p;
    if ((rc = stage(c, c->sx, x, sizeof(float) * n, flags, &p))) return rc;
    in.x = (const float*)p;
    if ((rc = stage(c, c->sy, y, sizeof(float) * n, flags, &p))) return rc;
    in.y = (const float*)p;
    if ((rc = stage(c, c->st, t_rel, sizeof(float) * n, flags, &p))) return rc;
    in.t = (const float*)p;
    if (pol) {
        if ((rc = stage(c, c->spol, pol, (size_t)n, flags, &p))) return rc;
        in.pol = (const signed char*)p;
    }
    long long off[2] = {0, n};
    if ((rc = stage(c, c->soff, off, sizeof off, 0, &p))) return rc;
    in.off = (const long long*)p;
    if ((rc = stage(c, c->stau, &tau, sizeof tau, 0, &p))) return rc;
    in.tau = (const float*)p;
    c->h_off.assign(off, off + 2);
    c->h_tau.assign(1, tau);
    int nblk = 0;
    rc = run_prep(c, g, in, 1, d_lo, d_hi, &nblk);
    if (rc) return rc;
    const void *pa, *pb = nullptr;
    if ((rc = stage(c, c->sseed, d_a, sizeof(float) * m, flags, &pa))) return rc;
    if (d_b) {
        if ((rc = stage(c, c->misc, d_b, sizeof(float) * m, flags, &pb))) return rc;
    }
    HIPCHK(c, c->hyps.ensure(sizeof(Hyp) * m));
    HIPCHK(c, launch_rates(c->stream, (const float*)pa, (const float*)pb, m, tau, c->hyps.as<Hyp>()));
    // every hypothesis on every tile
    std::vector<Item> items((size_t)m * T);
    for (int h = 0; h < m; ++h)
        for (int t = 0; t < T; ++t) items[(size_t)h * T + t] = Item{0, t, h, 1};
    HIPCHK(c, c->items.ensure(sizeof(Item) * items.size()));
    std::vector<int> ident(m);
    for (int h = 0; h < m; ++h) ident[h] = h;
    HIPCHK(c, c->act.ensure(sizeof(int) * m));
    HIPCHK(c, hipMemcpyAsync(c->act.p, ident.data(), sizeof(int) * m, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->items.p, items.data(), sizeof(Item) * items.size(), hipMemcpyHostToDevice,
                             c->stream));
    Queue hq[2 * kXcd] = {};
    hq[0].n_items = (int)items.size();  // everything in queue 0; the other XCDs steal
    HIPCHK(c, c->queues.ensure(sizeof hq));
    HIPCHK(c, hipMemcpyAsync(c->queues.p, hq, sizeof hq, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, c->part.ensure(sizeof(Part) * items.size()));
    unsigned* dimg = nullptr;
    if (img_out) {
        if (flags & ECMD_DEVICE_PTR) {
            dimg = img_out;
        } else {
            HIPCHK(c, c->img.ensure(sizeof(unsigned) * (size_t)m * M));
            dimg = c->img.as<unsigned>();
        }
    }
    const size_t lds = eval_lds_bytes(g.ring_px);
    int nb = 0;
    HIPCHK(c, eval_setup(c, lds, nt, &nb));
    Queue* q = c->queues.as<Queue>();
    HIPCHK(c, launch_eval(c->stream, g, nb, nt, lds, c->ev.as<float4>(), c->seg_off.as<long long>(),
                          c->seg_own.as<int>(), c->wp.as<WinParam>(), c->hyps.as<Hyp>(), c->act.as<int>(),
                          c->items.as<Item>(), (int)items.size(), &q[0], &q[kXcd], c->part.as<Part>(), m, dimg));
    std::vector<Part> parts(items.size());
    std::vector<long long> seg(T + 1);
    HIPCHK(c, hipMemcpyAsync(parts.data(), c->part.p, sizeof(Part) * parts.size(), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipMemcpyAsync(seg.data(), c->seg_off.p, sizeof(long long) * (T + 1), hipMemcpyDeviceToHost,
                             c->stream));
    if (img_out && !(flags & ECMD_DEVICE_PTR))
        HIPCHK(c, hipMemcpyAsync(img_out, dimg, sizeof(unsigned) * (size_t)m * M, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<uint64_t> hS(m, 0);
    std::vector<int64_t> hN(m, 0);
    for (int h = 0; h < m; ++h) {
        for (int t = 0; t < T; ++t) {
            if (seg[t + 1] == seg[t]) continue;  // empty tile: not evaluated, contributes 0
            hS[h] += parts[(size_t)h * T + t].S;
            hN[h] += parts[(size_t)h * T + t].N;
        }
    }
    if (flags & ECMD_DEVICE_PTR) {
        HIPCHK(c, hipMemcpyAsync(S, hS.data(), sizeof(uint64_t) * m, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(N, hN.data(), sizeof(int64_t) * m, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    } else {
        memcpy(S, hS.data(), sizeof(uint64_t) * m);
        memcpy(N, hN.data(), sizeof(int64_t) * m);
    }
    return ECMD_OK;
}

int ecmd_probe_point(ecmd_ctx* c, const ecmd_sensor* sensor, const float* x, const float* y, const float* t_rel,
                     const int8_t* polarity, int64_t n, float tau, const float* d, int32_t m, uint32_t flags, uint64_t* S, int64_t* N,
                     uint32_t* img_out) {
    if (!c) return ECMD_EINVAL;
    if (m < 0 || (m > 0 && !d)) return fail(c, ECMD_EINVAL, "bad probe arguments");
    // binning range: the span of the probed divergences
    std::vector<float> hd(m);
    if (m) {
        if (flags & ECMD_DEVICE_PTR) {
            HIPCHK(c, hipMemcpy(hd.data(), d, sizeof(float) * m, hipMemcpyDeviceToHost));
        } else {
            memcpy(hd.data(), d, sizeof(float) * m);
        }
    }
    float lo = INFINITY, hi = -INFINITY;
    for (float v : hd) {
        if (!isfinite(v)) return fail(c, ECMD_EINVAL, "non-finite divergence");
        lo = std::min(lo, v);
        hi = std::max(hi, v);
    }
    if (m == 0) lo = hi = 0.0f;
    return probe_impl(c, sensor, x, y, t_rel, polarity, n, tau, lo, hi, d, nullptr, m, flags, S, N, img_out);
}

int ecmd_probe_bound(ecmd_ctx* c, const ecmd_sensor* sensor, const float* x, const float* y, const float* t_rel,
                     const int8_t* polarity, int64_t n, float tau, float d_lo, float d_hi, const float* d_a, const float* d_b, int32_t m,
                     uint32_t flags, uint64_t* S_bar, int64_t* N_low, uint32_t* img_out) {
    if (!c) return ECMD_EINVAL;
    if (m > 0 && (!d_a || !d_b)) return fail(c, ECMD_EINVAL, "NULL interval ends");
    std::vector<float> ha(m), hb(m);
    if (m) {
        if (flags & ECMD_DEVICE_PTR) {
            HIPCHK(c, hipMemcpy(ha.data(), d_a, sizeof(float) * m, hipMemcpyDeviceToHost));
            HIPCHK(c, hipMemcpy(hb.data(), d_b, sizeof(float) * m, hipMemcpyDeviceToHost));
        } else {
            memcpy(ha.data(), d_a, sizeof(float) * m);
            memcpy(hb.data(), d_b, sizeof(float) * m);
        }
    }
    for (int k = 0; k < m; ++k)
        if (!(ha[k] >= d_lo && ha[k] <= hb[k] && hb[k] <= d_hi))
            return fail(c, ECMD_EINVAL, "interval %d not inside [d_lo, d_hi] or reversed", k);
    return probe_impl(c, sensor, x, y, t_rel, polarity, n, tau, d_lo, d_hi, d_a, d_b, m, flags, S_bar, N_low,
                      img_out);
}

int ecmd_downsample(ecmd_ctx* c, const ecmd_sensor* sensor, const float* x, const float* y, const int64_t* offsets,
                    int32_t B, uint32_t flags, uint16_t* out) {
    if (!c) return ECMD_EINVAL;
    c->err.clear();
    int rc = check_sensor(c, sensor);
    if (rc) return rc;
    if (B < 0 || !offsets || !out) return fail(c, ECMD_EINVAL, "bad downsample arguments");
    if (B == 0) return ECMD_OK;
    HIPCHK(c, hipSetDevice(c->device));
    std::vector<long long> off(B + 1);
    if (flags & ECMD_DEVICE_PTR) {
        HIPCHK(c, hipMemcpy(off.data(), offsets, sizeof(long long) * (B + 1), hipMemcpyDeviceToHost));
    } else {
        memcpy(off.data(), offsets, sizeof(long long) * (B + 1));
    }
    std::vector<int> blk(B + 1, 0);
    for (int w = 0; w < B; ++w) {
        long long n = off[w + 1] - off[w];
        if (n < 0 || off[0] < 0) return fail(c, ECMD_EINVAL, "offsets must be non-decreasing and >= 0");
        blk[w + 1] = blk[w] + (int)((n + kChunk - 1) / kChunk);
    }
    const long long n_total = off[B];
    if (n_total > 0 && (!x || !y)) return fail(c, ECMD_EINVAL, "NULL event arrays");
    const void *px, *py, *po;
    if ((rc = stage(c, c->sx, x, sizeof(float) * n_total, flags, &px))) return rc;
    if ((rc = stage(c, c->sy, y, sizeof(float) * n_total, flags, &py))) return rc;
    if ((rc = stage(c, c->soff, offsets, sizeof(long long) * (B + 1), flags, &po))) return rc;
    HIPCHK(c, c->blk.ensure(sizeof(int) * (B + 1)));
    HIPCHK(c, hipMemcpyAsync(c->blk.p, blk.data(), sizeof(int) * (B + 1), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, c->counts.ensure(sizeof(unsigned) * (size_t)B * 4096));
    HIPCHK(c, hipMemsetAsync(c->counts.p, 0, sizeof(unsigned) * (size_t)B * 4096, c->stream));
    uint16_t* dout = out;
    if (!(flags & ECMD_DEVICE_PTR)) {
        HIPCHK(c, c->img.ensure(sizeof(uint16_t) * (size_t)B * 4096));
        dout = c->img.as<uint16_t>();
    }
    HIPCHK(c, launch_downsample(c->stream, (const float*)px, (const float*)py, (const long long*)po, B,
                                sensor->width, sensor->height, c->blk.as<int>(), blk[B], kChunk,
                                c->counts.as<unsigned>(), dout));
    if (!(flags & ECMD_DEVICE_PTR))
        HIPCHK(c, hipMemcpyAsync(out, dout, sizeof(uint16_t) * (size_t)B * 4096, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return ECMD_OK;
}

}  // extern "C"

// ------------------------------------------------------------ preprocessing

// kind 0: hot-pixel removal (max_count); kind 1: resize + resample
static int preproc_impl(ecmd_ctx* c, int kind, const ecmd_sensor* in_s, const ecmd_sensor* out_s, const float* x,
                        const float* y, const float* t_rel, const int64_t* offsets, int32_t B, int32_t max_count,
                        float keep_frac, uint64_t seed, uint32_t flags, float* x_out, float* y_out, float* t_out,
                        int64_t* offsets_out) {
    if (!c) return ECMD_EINVAL;
    c->err.clear();
    int rc = check_sensor(c, in_s);
    if (rc) return rc;
    if (kind == 1 && (rc = check_sensor(c, out_s))) return rc;
    if (B < 0 || !offsets || !offsets_out) return fail(c, ECMD_EINVAL, "bad window arguments");
    if (kind == 0 && max_count < 0) return fail(c, ECMD_EINVAL, "max_count must be >= 0");
    if (kind == 1 && !(keep_frac >= 0.0f && keep_frac <= 1.0f)) return fail(c, ECMD_EINVAL, "keep_frac in [0, 1]");
    HIPCHK(c, hipSetDevice(c->device));
    std::vector<long long> off(B + 1);
    if (flags & ECMD_DEVICE_PTR) {
        HIPCHK(c, hipMemcpy(off.data(), offsets, sizeof(long long) * (B + 1), hipMemcpyDeviceToHost));
    } else {
        memcpy(off.data(), offsets, sizeof(long long) * (B + 1));
    }
    if (off[0] < 0) return fail(c, ECMD_EINVAL, "offsets[0] < 0");
    for (int w = 0; w < B; ++w)
        if (off[w + 1] < off[w]) return fail(c, ECMD_EINVAL, "offsets decrease at window %d", w);
    const long long n = off[B] - off[0];
    if (n > 0 && (!x || !y || !t_rel || !x_out || !y_out || !t_out)) return fail(c, ECMD_EINVAL, "NULL arrays");
    // inputs: device pointers as given, host arrays staged (indexed from offsets[0])
    const float *dx = x, *dy = y, *dt = t_rel;
    const long long* doff = (const long long*)offsets;
    long long base = off[0];
    if (!(flags & ECMD_DEVICE_PTR)) {
        HIPCHK(c, c->sx.ensure(sizeof(float) * std::max(n, 1ll)));
        HIPCHK(c, c->sy.ensure(sizeof(float) * std::max(n, 1ll)));
        HIPCHK(c, c->st.ensure(sizeof(float) * std::max(n, 1ll)));
        if (n) {
            HIPCHK(c, hipMemcpyAsync(c->sx.p, x + base, sizeof(float) * n, hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(c->sy.p, y + base, sizeof(float) * n, hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(c->st.p, t_rel + base, sizeof(float) * n, hipMemcpyHostToDevice, c->stream));
        }
        // staged copies start at index 0: shift the offsets
        std::vector<long long> o0(off);
        for (auto& v : o0) v -= base;
        HIPCHK(c, c->soff.ensure(sizeof(long long) * (B + 1)));
        HIPCHK(c, hipMemcpyAsync(c->soff.p, o0.data(), sizeof(long long) * (B + 1), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        dx = c->sx.as<float>();
        dy = c->sy.as<float>();
        dt = c->st.as<float>();
        doff = c->soff.as<long long>();
        base = 0;
    }
    HIPCHK(c, c->keep.ensure(std::max(n, 1ll)));
    const long long nb = (n + 1023) / 1024;
    HIPCHK(c, c->misc.ensure(sizeof(long long) * (nb + 1)));
    unsigned char* keep = (unsigned char*)c->keep.p;
    const int W = in_s->width, H = in_s->height;
    if (kind == 0) {
        const size_t M = (size_t)W * H;
        HIPCHK(c, c->counts.ensure(sizeof(unsigned) * M * std::max(B, 1)));
        HIPCHK(c, hipMemsetAsync(c->counts.p, 0, sizeof(unsigned) * M * std::max(B, 1), c->stream));
        HIPCHK(c, launch_hot_keep(c->stream, dx, dy, doff, B, n, W, H, c->counts.as<unsigned>(), (unsigned)max_count,
                                  keep));
    } else {
        const double th = floor((double)keep_frac * 16777216.0);
        HIPCHK(c, launch_resample_keep(c->stream, doff, B, n, seed, (unsigned)th, keep));
    }
    const float sx = kind == 1 ? (float)out_s->width / (float)W : 1.0f;
    const float sy = kind == 1 ? (float)out_s->height / (float)H : 1.0f;
    float *ox = x_out, *oy = y_out, *ot = t_out;
    long long* ooff = (long long*)offsets_out;
    if (!(flags & ECMD_DEVICE_PTR)) {
        HIPCHK(c, c->pix.ensure(sizeof(float) * 3 * std::max(n, 1ll) + sizeof(long long) * (B + 1)));
        ox = c->pix.as<float>();
        oy = ox + std::max(n, 1ll);
        ot = oy + std::max(n, 1ll);
        ooff = (long long*)(ot + std::max(n, 1ll));
    }
    HIPCHK(c, launch_compact(c->stream, dx, dy, dt, doff, B, base, n, keep, c->misc.as<long long>(), sx, sy, ox, oy,
                             ot, ooff));
    if (!(flags & ECMD_DEVICE_PTR)) {
        std::vector<long long> ho(B + 1);
        HIPCHK(c, hipMemcpyAsync(ho.data(), ooff, sizeof(long long) * (B + 1), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        const long long m = ho[B];
        if (m) {
            HIPCHK(c, hipMemcpyAsync(x_out, ox, sizeof(float) * m, hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipMemcpyAsync(y_out, oy, sizeof(float) * m, hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipMemcpyAsync(t_out, ot, sizeof(float) * m, hipMemcpyDeviceToHost, c->stream));
        }
        memcpy(offsets_out, ho.data(), sizeof(long long) * (B + 1));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return ECMD_OK;
}

extern "C" {

int ecmd_estimate_stream(ecmd_ctx* c, const ecmd_sensor* sensor, const ecmd_events* events, double t_start,
                         double tau, int32_t K, const ecmd_search* search, uint32_t flags, ecmd_result* out) {
    if (!c) return ECMD_EINVAL;
    c->err.clear();
    if (!events || !out || K < 0 || K > 65535) return fail(c, ECMD_EINVAL, "bad stream arguments");
    if (!isfinite(t_start) || !(tau > 0.0) || !isfinite(tau)) return fail(c, ECMD_EINVAL, "bad t_start or tau");
    if (K == 0) return ECMD_OK;
    const long long n = events->n;
    if (n < 0 || (n > 0 && (!events->x || !events->y || !events->t))) return fail(c, ECMD_EINVAL, "bad events");
    HIPCHK(c, hipSetDevice(c->device));
    // window bounds and offsets on the device
    const double* dt = events->t;
    if (!(flags & ECMD_DEVICE_PTR)) {
        for (long long i = 1; i < n; ++i)
            if (!(events->t[i] >= events->t[i - 1])) return fail(c, ECMD_EINVAL, "stream times must be sorted");
        HIPCHK(c, c->counts.ensure(sizeof(double) * std::max(n, 1ll)));
        if (n) HIPCHK(c, hipMemcpyAsync(c->counts.p, events->t, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
        dt = (const double*)c->counts.p;
    }
    HIPCHK(c, c->misc.ensure(sizeof(long long) * (K + 1)));
    long long* doff = c->misc.as<long long>();
    HIPCHK(c, launch_stream_bounds(c->stream, dt, n, t_start, tau, K, doff));
    std::vector<long long> off(K + 1);
    HIPCHK(c, hipMemcpyAsync(off.data(), doff, sizeof(long long) * (K + 1), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const long long o0 = off[0], m = off[K] - off[0];
    HIPCHK(c, c->keep.ensure(sizeof(float) * std::max(m, 1ll)));
    float* trel = (float*)c->keep.p;
    HIPCHK(c, launch_stream_trel(c->stream, dt, doff, m, K, t_start, tau, trel));
    // batched estimation on the selected range (x, y staged to the device if needed)
    std::vector<long long> rel(K + 1);
    for (int k = 0; k <= K; ++k) rel[k] = off[k] - o0;
    std::vector<float> taus(K, (float)tau);
    const float *dx = events->x + o0, *dy = events->y + o0;
    const signed char* dp = events->p ? (const signed char*)events->p + o0 : nullptr;
    if (events->p && !(flags & ECMD_DEVICE_PTR)) {
        HIPCHK(c, c->spol.ensure((size_t)std::max(m, 1ll)));
        if (m) HIPCHK(c, hipMemcpyAsync(c->spol.p, events->p + o0, (size_t)m, hipMemcpyHostToDevice, c->stream));
        dp = c->spol.as<signed char>();
    }
    if (!(flags & ECMD_DEVICE_PTR)) {
        HIPCHK(c, c->img.ensure(sizeof(float) * 2 * std::max(m, 1ll)));
        float* sxy = c->img.as<float>();
        dx = sxy;
        dy = sxy + std::max(m, 1ll);
        if (m) {
            HIPCHK(c, hipMemcpyAsync((void*)dx, events->x + o0, sizeof(float) * m, hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync((void*)dy, events->y + o0, sizeof(float) * m, hipMemcpyHostToDevice, c->stream));
        }
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // offsets and tau are host values here; the events are on the device
    int L = 0;
    int rc = check_sensor(c, sensor);
    if (rc) return rc;
    if ((rc = check_search(c, search, &L))) return rc;
    if (!(search->d_hi * (float)tau < 1.0f)) return fail(c, ECMD_EINVAL, "d_hi * tau must be < 1 (cheirality)");
    c->h_off = rel;
    c->h_tau = taus;
    Inputs in;
    in.x = dx;
    in.y = dy;
    in.t = trel;
    in.pol = dp;
    const void* p;
    if ((rc = stage(c, c->soff, rel.data(), sizeof(long long) * (K + 1), 0, &p))) return rc;
    in.off = (const long long*)p;
    if ((rc = stage(c, c->stau, taus.data(), sizeof(float) * K, 0, &p))) return rc;
    in.tau = (const float*)p;
    return run_search(c, sensor, in, K, search, L, out);
}

int ecmd_hot_pixel_filter(ecmd_ctx* c, const ecmd_sensor* sensor, const float* x, const float* y, const float* t_rel,
                          const int64_t* offsets, int32_t B, int32_t max_count, uint32_t flags, float* x_out,
                          float* y_out, float* t_out, int64_t* offsets_out) {
    return preproc_impl(c, 0, sensor, nullptr, x, y, t_rel, offsets, B, max_count, 1.0f, 0, flags, x_out, y_out,
                        t_out, offsets_out);
}

int ecmd_resample(ecmd_ctx* c, const ecmd_sensor* in_sensor, const ecmd_sensor* out_sensor, const float* x,
                  const float* y, const float* t_rel, const int64_t* offsets, int32_t B, float keep_frac,
                  uint64_t seed, uint32_t flags, float* x_out, float* y_out, float* t_out, int64_t* offsets_out) {
    return preproc_impl(c, 1, in_sensor, out_sensor, x, y, t_rel, offsets, B, 0, keep_frac, seed, flags, x_out, y_out,
                        t_out, offsets_out);
}

}  // extern "C"

// ------------------------------------------------------------ learned incumbent

// Deterministic parameter initialisation: He-normal weights from a
// splitmix64 stream (Box-Muller), zero biases.
static void cnn_init_params(uint64_t seed, std::vector<float>& p) {
    const int n = cnn_nparam();
    p.assign(n, 0.0f);
    uint64_t st = seed ^ 0x9E3779B97F4A7C15ull;
    auto next = [&]() {
        uint64_t z = (st += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    auto unif = [&]() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); };
    auto normal = [&]() { return sqrt(-2.0 * log(unif())) * cos(6.283185307179586 * unif()); };
    struct Seg { int off, n, fan_in; };
    const Seg segs[] = {{0, 144, 9}, {160, 4608, 144}, {4800, 18432, 288}, {23296, 64, 64}};
    for (const Seg& sg : segs)
        for (int k = 0; k < sg.n; ++k) p[sg.off + k] = (float)(normal() * sqrt(2.0 / sg.fan_in));
}

static int cnn_stage_imgs(ecmd_cnn* n, const uint16_t* imgs, int32_t B, uint32_t flags, const uint16_t** out) {
    ecmd_ctx* c = n->ctx;
    const void* p;
    int rc = stage(c, n->imgs, imgs, sizeof(uint16_t) * (size_t)B * 4096, flags, &p);
    *out = (const uint16_t*)p;
    return rc;
}

// forward (mode 0) or forward + backward with the batch gradient in n->grad
static int cnn_run(ecmd_cnn* n, const uint16_t* imgs, const float* labels, int32_t B, uint32_t flags, int mode) {
    ecmd_ctx* c = n->ctx;
    if (B <= 0 || !imgs || (mode && !labels)) return fail(c, ECMD_EINVAL, "bad network arguments");
    HIPCHK(c, hipSetDevice(c->device));
    const uint16_t* di;
    int rc = cnn_stage_imgs(n, imgs, B, flags, &di);
    if (rc) return rc;
    HIPCHK(c, n->out.ensure(sizeof(float) * B));
    const float* dl = nullptr;
    if (mode) {
        const void* p;
        if ((rc = stage(c, n->labels, labels, sizeof(float) * B, flags, &p))) return rc;
        dl = (const float*)p;
        HIPCHK(c, n->pg.ensure(sizeof(float) * (size_t)B * cnn_nparam()));
        HIPCHK(c, n->lossb.ensure(sizeof(float) * B));
        HIPCHK(c, n->loss.ensure(sizeof(float)));
        HIPCHK(c, n->grad.ensure(sizeof(float) * cnn_nparam()));
    }
    HIPCHK(c, cnn_set_lds());
    HIPCHK(c, launch_cnn(c->stream, n->P.as<float>(), di, B, n->out.as<float>(), mode, dl, n->pg.as<float>(),
                         n->lossb.as<float>()));
    if (mode)
        HIPCHK(c, launch_cnn_reduce(c->stream, n->pg.as<float>(), n->lossb.as<float>(), B, n->grad.as<float>(),
                                    n->loss.as<float>()));
    return ECMD_OK;
}

extern "C" {

int ecmd_cnn_create(ecmd_ctx* c, uint64_t seed, ecmd_cnn** out) {
    if (!c || !out) return ECMD_EINVAL;
    c->err.clear();
    HIPCHK(c, hipSetDevice(c->device));
    ecmd_cnn* n = new (std::nothrow) ecmd_cnn();
    if (!n) return fail(c, ECMD_ENOMEM, "host allocation failed");
    n->ctx = c;
    const int np = cnn_nparam();
    std::vector<float> p;
    cnn_init_params(seed, p);
    std::vector<float> zero(np, 0.0f);
    if (n->P.ensure(sizeof(float) * np) != hipSuccess || n->m.ensure(sizeof(float) * np) != hipSuccess ||
        n->v.ensure(sizeof(float) * np) != hipSuccess) {
        n->P.release(); n->m.release(); n->v.release();
        delete n;
        return fail(c, ECMD_ENOMEM, "device allocation failed");
    }
    HIPCHK(c, hipMemcpy(n->P.p, p.data(), sizeof(float) * np, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(n->m.p, zero.data(), sizeof(float) * np, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(n->v.p, zero.data(), sizeof(float) * np, hipMemcpyHostToDevice));
    c->nets.push_back(n);
    *out = n;
    return ECMD_OK;
}

void ecmd_cnn_destroy(ecmd_cnn* n) {
    if (!n) return;
    if (ecmd_ctx* c = n->ctx) {
        (void)hipSetDevice(c->device);
        (void)hipStreamSynchronize(c->stream);
        cnn_release(n);
        c->nets.erase(std::remove(c->nets.begin(), c->nets.end(), n), c->nets.end());
    }
    delete n;
}

int ecmd_cnn_get_params(ecmd_cnn* n, float* host_params) {
    if (!n || !n->ctx || !host_params) return ECMD_EINVAL;
    ecmd_ctx* c = n->ctx;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipMemcpyAsync(host_params, n->P.p, sizeof(float) * cnn_nparam(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return ECMD_OK;
}

int ecmd_cnn_set_params(ecmd_cnn* n, const float* host_params) {
    if (!n || !n->ctx || !host_params) return ECMD_EINVAL;
    ecmd_ctx* c = n->ctx;
    for (int k = 0; k < cnn_nparam(); ++k)
        if (!isfinite(host_params[k])) return fail(c, ECMD_EINVAL, "parameter %d is not finite", k);
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipMemcpyAsync(n->P.p, host_params, sizeof(float) * cnn_nparam(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return ECMD_OK;
}

static const char kCnnMagic[8] = {'E', 'C', 'M', 'D', 'C', 'N', 'N', '1'};

int ecmd_cnn_save(ecmd_cnn* n, const char* path) {
    if (!n || !n->ctx || !path) return ECMD_EINVAL;
    ecmd_ctx* c = n->ctx;
    c->err.clear();
    const int np = cnn_nparam();
    std::vector<float> buf((size_t)3 * np);
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipMemcpyAsync(buf.data(), n->P.p, sizeof(float) * np, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(buf.data() + np, n->m.p, sizeof(float) * np, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(buf.data() + 2 * np, n->v.p, sizeof(float) * np, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    FILE* f = fopen(path, "wb");
    if (!f) return fail(c, ECMD_EINVAL, "cannot open %s for writing", path);
    const uint32_t count = (uint32_t)np;
    const int32_t step = n->step;
    bool ok = fwrite(kCnnMagic, 1, 8, f) == 8 && fwrite(&count, 4, 1, f) == 1 && fwrite(&step, 4, 1, f) == 1 &&
              fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    ok = (fclose(f) == 0) && ok;
    if (!ok) return fail(c, ECMD_EINVAL, "writing %s failed", path);
    return ECMD_OK;
}

int ecmd_cnn_load(ecmd_cnn* n, const char* path) {
    if (!n || !n->ctx || !path) return ECMD_EINVAL;
    ecmd_ctx* c = n->ctx;
    c->err.clear();
    const int np = cnn_nparam();
    FILE* f = fopen(path, "rb");
    if (!f) return fail(c, ECMD_EINVAL, "cannot open %s", path);
    char magic[8];
    uint32_t count = 0;
    int32_t step = 0;
    std::vector<float> buf((size_t)3 * np);
    bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kCnnMagic, 8) == 0 && fread(&count, 4, 1, f) == 1 &&
              count == (uint32_t)np && fread(&step, 4, 1, f) == 1 && step >= 0 &&
              fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
    char extra;
    ok = ok && fread(&extra, 1, 1, f) == 0;  // nothing after the second moments
    fclose(f);
    if (!ok) return fail(c, ECMD_EINVAL, "%s is not a network checkpoint of %d parameters", path, np);
    for (size_t k = 0; k < buf.size(); ++k)
        if (!isfinite(buf[k])) return fail(c, ECMD_EINVAL, "%s: value %zu is not finite", path, k);
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipMemcpyAsync(n->P.p, buf.data(), sizeof(float) * np, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(n->m.p, buf.data() + np, sizeof(float) * np, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(n->v.p, buf.data() + 2 * np, sizeof(float) * np, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    n->step = step;
    return ECMD_OK;
}

int ecmd_cnn_forward(ecmd_cnn* n, const uint16_t* imgs, int32_t B, uint32_t flags, float* d_out) {
    if (!n || !n->ctx || !d_out) return ECMD_EINVAL;
    ecmd_ctx* c = n->ctx;
    c->err.clear();
    int rc = cnn_run(n, imgs, nullptr, B, flags, 0);
    if (rc) return rc;
    HIPCHK(c, hipMemcpyAsync(d_out, n->out.p, sizeof(float) * B,
                             (flags & ECMD_DEVICE_PTR) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return ECMD_OK;
}

int ecmd_cnn_grads(ecmd_cnn* n, const uint16_t* imgs, const float* labels, int32_t B, uint32_t flags,
                   float* grad_out, float* loss_out) {
    if (!n || !n->ctx || !grad_out || !loss_out) return ECMD_EINVAL;
    ecmd_ctx* c = n->ctx;
    c->err.clear();
    int rc = cnn_run(n, imgs, labels, B, flags, 1);
    if (rc) return rc;
    HIPCHK(c, hipMemcpyAsync(grad_out, n->grad.p, sizeof(float) * cnn_nparam(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(loss_out, n->loss.p, sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return ECMD_OK;
}

int ecmd_cnn_train_step(ecmd_cnn* n, const uint16_t* imgs, const float* labels, int32_t B, float lr, uint32_t flags,
                        float* loss_out) {
    if (!n || !n->ctx) return ECMD_EINVAL;
    ecmd_ctx* c = n->ctx;
    c->err.clear();
    if (!(lr > 0.0f) || !isfinite(lr)) return fail(c, ECMD_EINVAL, "learning rate must be > 0");
    int rc = cnn_run(n, imgs, labels, B, flags, 1);
    if (rc) return rc;
    n->step += 1;
    HIPCHK(c, launch_adam(c->stream, n->P.as<float>(), n->m.as<float>(), n->v.as<float>(), n->grad.as<float>(), lr,
                          n->step));
    if (loss_out) {
        HIPCHK(c, hipMemcpyAsync(loss_out, n->loss.p, sizeof(float), hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return ECMD_OK;
}

int ecmd_estimate_divergence_learned(ecmd_ctx* c, ecmd_cnn* n, const ecmd_sensor* sensor, const float* x,
                                     const float* y, const float* t_rel, const int64_t* offsets, const float* tau,
                                     int32_t B, const ecmd_search* search, uint32_t flags, ecmd_result* out) {
    if (!c || !n || n->ctx != c) return c ? fail(c, ECMD_EINVAL, "network belongs to another context") : ECMD_EINVAL;
    c->err.clear();
    if (B <= 0) return B == 0 ? ECMD_OK : fail(c, ECMD_EINVAL, "B < 0");
    if (!search) return fail(c, ECMD_EINVAL, "search is NULL");
    HIPCHK(c, hipSetDevice(c->device));
    // downsampled images stay on the device
    HIPCHK(c, n->imgs.ensure(sizeof(uint16_t) * (size_t)B * 4096));
    HIPCHK(c, n->seeds.ensure(sizeof(float) * B));
    int rc;
    if (flags & ECMD_DEVICE_PTR) {
        rc = ecmd_downsample(c, sensor, x, y, offsets, B, flags, n->imgs.as<uint16_t>());
    } else {
        std::vector<uint16_t> tmp((size_t)B * 4096);
        rc = ecmd_downsample(c, sensor, x, y, offsets, B, 0, tmp.data());
        if (!rc) {
            HIPCHK(c, hipMemcpyAsync(n->imgs.p, tmp.data(), sizeof(uint16_t) * tmp.size(), hipMemcpyHostToDevice,
                                     c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
        }
    }
    if (rc) return rc;
    rc = cnn_run(n, n->imgs.as<uint16_t>(), nullptr, B, ECMD_DEVICE_PTR, 0);
    if (rc) return rc;
    HIPCHK(c, launch_seed_from_pred(c->stream, n->out.as<float>(), B, search->d_lo, search->d_hi,
                                    n->seeds.as<float>()));
    if (flags & ECMD_DEVICE_PTR)
        return batched_impl(c, sensor, x, y, t_rel, nullptr, offsets, tau, B, search, flags, n->seeds.as<float>(),
                            out);
    std::vector<float> hs(B);
    HIPCHK(c, hipMemcpyAsync(hs.data(), n->seeds.p, sizeof(float) * B, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return batched_impl(c, sensor, x, y, t_rel, nullptr, offsets, tau, B, search, flags, hs.data(), out);
}

}  // extern "C"
