// Internal types and launchers of the MI355X divergence estimator.
//
// Layout in HBM (per batch of B windows sharing one sensor):
//   * events are binned by image tile: segment (w, t) holds the events of
//     window w whose root trajectory (all d in [d_lo, d_hi]) can reach tile
//     t, as float4 (x, y, ax, ay); the events owned by the tile come first
//     (they count towards N_low), guest copies after.  With an integer FOE
//     inside the sensor the tiles split the image at the FOE lines, which no
//     event ever crosses (the warp of eq. (12) only moves events away from
//     the FOE), so there are no guests unless a quadrant is itself split;
//   * hypotheses: per window HS = 3F slots (F centre points, then two child
//     intervals per expanded node), as rates r = d / (1 - d tau);
//   * partial sums per (window, slot, tile), summed by the frontier step;
//   * frontier: up to CAP nodes per window, key K_bar as a signed 128-bit
//     integer, and the incumbent (K, j) per window.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ecmd.h"

namespace ecmd {

typedef __int128 i128;

constexpr int kMaxTiles = 64;    // tiles per sensor
constexpr int kEvalThreads = 1024;  // threads of the largest evaluation workgroup
constexpr int kEvalPad = 2 * kEvalThreads;  // records after the event store: the evaluation kernel prefetches up to two workgroup strides past a segment's end
constexpr int kFrontThreads = 256;  // threads of a frontier workgroup

// HYP_CERT: the endpoint certificate of an interval (owned events only, no
// walk): partial sums S = U (walk pixels of the events inside at both ends),
// N = N_low; K_bar >= U^2 - N_low^2.
enum HypKind : int { HYP_NONE = 0, HYP_POINT = 1, HYP_INTERVAL = 2, HYP_CERT = 3 };

struct Hyp {
    float ra, rb;  // rates of the interval ends (equal for a point)
    int kind;
    int pad;
};

struct Part {
    unsigned long long S;  // sum of squared counts over the tile
    long long N;           // in-image events (point) or N_low (interval)
    unsigned long long U;  // pixel increments
    long long pad;
};

struct Node {
    unsigned long long klo;  // key K_bar, low and high 64-bit words
    long long khi;
    unsigned ja, jb;  // grid interval [ja, jb]; jb carries kNodeCert
    float lc;         // expected endpoint certificate of this node's children
    float ub;         // with kNodeCert: an upper bound of K at every grid point of the node (an
                      // ancestor's exact bound, rounded up; infinity when no ancestor has one)
};

// Set in Node::jb when the key is the endpoint certificate (a lower bound of
// K_bar) rather than K_bar itself (grid indices stay below 2^31).
constexpr unsigned kNodeCert = 0x80000000u;
// Node::khi of a child whose certificate failed, queued in its place until
// its exact bound (hypothesis slot Node::klo) is known later in the step.
constexpr long long kNodeRepair = (long long)(-0x7fffffffffffffffll - 1);

struct Sel {
    unsigned ja, jb, jc, kids;  // expanded node, its centre, 1 if it has children
    float lc;                   // expected endpoint certificate of its children (Node::lc)
    float ub;                   // upper bound of K at the node's grid points (Node::ub)
};

struct Geometry {
    int W, H;
    float cx, cy;
    int T;                        // number of event segments per window: nsp spatial tiles x 1 or 2 polarity images
    int nsp;                      // spatial tiles (ntx * nty); segment t covers tile t % nsp of image t / nsp
    int ntx, nty;                 // tile grid
    int colcut[kMaxTiles + 1];    // column band edges (ntx + 1)
    int rowcut[kMaxTiles + 1];    // row band edges (nty + 1)
    int max_tile_px;              // largest tile area (pixels)
    int ring_px;                  // largest tile's counters with their one-cell border, (w + 2)(h + 2)
};

// Guest copies of a tile segment are split into kGuestBins bins by the
// first of the rates gcut[0] <= ... <= gcut[kGuestBins - 2] at which the
// event has reached the tile (bin m: not reached at gcut[0 .. m-1]), so an
// evaluation at rates up to r reads the bins whose lower cut lies below r.
constexpr int kGuestBins = 4;

struct WinParam {
    float tau;
    float r_lo, r_hi;  // rates at d_lo and d_hi
    float kscale;      // walk-length classes per unit of |ax| + |ay|
    float gcut[kGuestBins - 1];  // guest bin cuts, uniform over [r_lo, r_hi]
    long long n_events;
};

struct Search {
    float d_lo, d_hi;
    int L;
    int F;    // nodes expanded together per step
    int CAP;  // frontier capacity per window
    int HS;   // hypothesis slots per window (3F)
    int G;    // hypotheses per work item (the most; see gslots)
    int B;    // windows of the search
    long long gslots;  // > 0: per step, G = clamp(B * hypotheses * tiles / gslots, 1, G); 0: G fixed
    long long max_nodes;
    long long gamma_key;  // stop when best K_bar - K_inc <= gamma_key (-1: gamma = 0)
    long long M;          // pixels
    int cert;             // endpoint certificates allowed (ECMD_SEARCH_EXACT_BOUNDS not set)
    int pad;
};

struct WinState {
    unsigned long long Kinc_lo;
    long long Kinc_hi;
    unsigned long long gap_lo;  // certified gap key at stop (budget / gamma)
    long long gap_hi;
    unsigned j_inc;
    int status;
    int active;
    int n_front;
    int n_sel;
    int steps;
    int seeded;
    int pad;
    long long nodes_expanded, nodes_pruned, point_evals, bound_evals;
    long long event_hyp, pixel_updates;
    long long cert_evals;  // certificates that kept their node
    int n_repair;          // children whose certificate failed, bounded again this step
    int overflow;          // the frontier outgrew its capacity this step
    int n_front0;          // queued nodes before this step's children
    int pad2;
};

// A work item: tile t of window w for the hypotheses act[w * HS + r0 + k],
// k < cnt (a group of consecutive active slots, evaluated one after another
// by one workgroup so that the item's set-up is paid once per group).
struct Item {
    int w;
    int t;
    int r0;
    int cnt;
};

// Work queues: one per XCD (workgroups are dispatched to the 8 XCDs in
// round-robin order of their index), so that the items of a window are
// evaluated on one XCD and its events stay in that XCD's L2.  Queue r owns
// the item slots [r * qcap, (r + 1) * qcap).
// Events per window stay below 2^28, so every event of a (window, tile)
// segment is reached with a 32-bit byte offset from the segment start.
constexpr long long kMaxWindowEvents = 1ll << 28;
constexpr int kXcd = 8;

struct Queue {
    int n_items;
    int next;
};

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `s` and return the launch status.

hipError_t launch_winparam(hipStream_t s, const Geometry& g, const float* tau, const long long* offsets,
                           int B, float d_lo, float d_hi, WinParam* wp);
// Counters of the prep (per window and tile: owned events by walk class,
// guests by bin and walk class).
size_t prep_counters(int B, int T);
// Ints of seg_own: per window and tile, the owned events, then the end of
// each guest bin, counted from the segment's start.
size_t seg_own_words(int B, int T);
// phase 0: count events per (window, tile, owned/guest, walk class) and scan
// into segments; err_flag[w] is set when window w has an invalid event.
// phase 1: scatter the events into their segments; with cap >= 0, seg_off
// holds the scan of phase 0 and nothing is written when its total exceeds
// cap records.  Blocks at or past blk_start[B] return at once, so nblk may
// be any upper bound of blk_start[B].
hipError_t launch_prep(hipStream_t s, int phase, const Geometry& g, const float* x, const float* y,
                       const float* t_rel, const signed char* pol, const long long* offsets, const WinParam* wp, int B,
                       const int* blk_start, int nblk, int chunk, int* cnt, long long* seg_off, int* seg_own,
                       unsigned long long* cursor, float4* ev, int* err_flag, long long cap);
// Checks made on the device before the search (the asynchronous plan):
// window w starts finished with status wstat[w] when that is non-zero,
// ECMD_EINVAL when werr[w] (an invalid event), ECMD_ENOMEM when the binned
// records exceed cap.  wstat == NULL: no checks.
struct InitCheck {
    const int* wstat;
    const int* werr;
    long long cap;
};
hipError_t launch_init(hipStream_t s, const Search& sp, const WinParam* wp, const float* seeds, int B,
                       WinState* st, Sel* sel, Hyp* hyps, int* act, Item* items, int qcap, Queue* q, int T,
                       const long long* seg_off, InitCheck chk);
// One step of Algorithm 1 in two launches around an evaluation launch:
// phase 0 absorbs the step's evaluations (incumbent, children) and queues
// the exact bound of every child whose endpoint certificate failed (in
// q_fill, usually nothing); phase 1 absorbs those bounds, prunes, stops or
// selects the next nodes and queues their hypotheses in q_fill.
// t0, t1 (nullable): events that take the kernel's own start and end times
hipError_t launch_frontier(hipStream_t s, int phase, const Search& sp, const WinParam* wp, int B, int T,
                           const long long* seg_off, WinState* st, Node* front, Sel* sel, Hyp* hyps, int* act,
                           const Part* part, Item* items, int qcap, Queue* q_fill, int* n_active,
                           hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
// q, q_reset: kXcd queues each; nt: threads per workgroup (256, 512 or 1024)
hipError_t launch_eval(hipStream_t s, const Geometry& g, int nblocks, int nt, size_t lds_bytes,
                       const float4* ev, const long long* seg_off, const int* seg_own, const WinParam* wp,
                       const Hyp* hyps, const int* act, const Item* items, int qcap, Queue* q, Queue* q_reset,
                       Part* part, int HS, unsigned* img_out, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
hipError_t launch_rates(hipStream_t s, const float* d_a, const float* d_b, int m, float tau, Hyp* hyps);
hipError_t launch_probe_pixels(hipStream_t s, const float* x, const float* y, const float* t_rel,
                               long long n, float tau, float d, int W, int H, float cx, float cy,
                               int* pix);
hipError_t launch_downsample(hipStream_t s, const float* x, const float* y, const long long* offsets,
                             int B, int W, int H, const int* blk_start, int nblk, int chunk,
                             unsigned* counts, uint16_t* out);
hipError_t eval_set_lds(size_t bytes);
// LDS bytes of the evaluation kernel for tiles of up to ring_px counters
// (a tile of w x h pixels has (w + 2)(h + 2), its one-cell border included).
size_t eval_lds_bytes(int ring_px);
hipError_t eval_occupancy(int* blocks_per_cu, size_t lds_bytes, int nt);
// Events with t in [t0, t1], compacted in order, t_rel = float(t - t0);
// their polarities too when p is not NULL.
hipError_t launch_select(hipStream_t s, const float* x, const float* y, const double* t, const signed char* p,
                         long long n, double t0, double t1, float* xo, float* yo, float* to, signed char* po,
                         int* blk_cnt, long long* total);

// preprocessing (ecmd_preproc.hip)
hipError_t launch_compact(hipStream_t s, const float* x, const float* y, const float* t, const long long* offsets,
                          int B, long long off0, long long n, const unsigned char* keep, long long* blk, float sx,
                          float sy, float* xo, float* yo, float* to, long long* off_out);
hipError_t launch_resample_keep(hipStream_t s, const long long* offsets, int B, long long n, unsigned long long seed,
                                unsigned thresh24, unsigned char* keep);
hipError_t launch_hot_keep(hipStream_t s, const float* x, const float* y, const long long* offsets, int B, long long n,
                           int W, int H, unsigned* counts, unsigned max_count, unsigned char* keep);

hipError_t launch_stream_bounds(hipStream_t s, const double* t, long long n, double t_start, double tau, int K,
                                long long* offsets);
hipError_t launch_stream_trel(hipStream_t s, const double* t, const long long* offsets, long long n_sel, int K,
                              double t_start, double tau, float* t_rel);

// learned incumbent (ecmd_cnn.hip)
size_t cnn_lds_bytes();
int cnn_nparam();
hipError_t cnn_set_lds();
hipError_t launch_cnn(hipStream_t s, const float* P, const uint16_t* imgs, int B, float* out, int mode,
                      const float* labels, float* pg, float* lossb);
hipError_t launch_cnn_reduce(hipStream_t s, const float* pg, const float* lossb, int B, float* grad, float* loss);
hipError_t launch_adam(hipStream_t s, float* P, float* m, float* v, const float* grad, float lr, int step);
hipError_t launch_seed_from_pred(hipStream_t s, const float* pred, int B, float d_lo, float d_hi, float* seeds);

// the live grid range of every active window (queued and selected nodes)
// as its binning range r_lo, r_hi
hipError_t launch_live_range(hipStream_t s, const Search& sp, const WinState* st, const Node* front, const Sel* sel,
                             WinParam* wp, int B);

// asynchronous plan: device-side window checks and prep block prefix (one
// workgroup), a fill, and the per-window results
hipError_t launch_plan_check(hipStream_t s, const long long* off, const float* tau, int B, float d_hi, int W, int H,
                             long long max_events, int chunk, int* wstat, int* werr, int* blk, Queue* q,
                             int* n_active);
hipError_t launch_fill_u32(hipStream_t s, unsigned* p, long long n, unsigned v);
hipError_t launch_plan_results(hipStream_t s, const Search& sp, int B, const WinState* st, const long long* off,
                               const float* tau, ecmd_result* out);

// calibration (roofline denominators measured on the device)
hipError_t launch_lds_atomics(hipStream_t s, int blocks, int iters, unsigned* sink);
hipError_t launch_stream_read(hipStream_t s, const void* a, long long bytes, int blocks, float* partial);

}  // namespace ecmd
