/*
 * ECMD oracle: a plain, slow CPU statement of what the exact divergence
 * estimator computes.  TEST INFRASTRUCTURE ONLY: the tests, the smoke check
 * and the benchmark's CPU-baseline leg call it; the product path (the HIP
 * library) never links, includes or calls anything here, and nothing here
 * comes from the product path.
 *
 * Everything follows "Globally Optimal Event-Based Divergence Estimation for
 * Ventral Landing" (McLeod, Chin, et al., arXiv 2209.13168):
 *
 *   - radial warp f_i(nu) of Sec. 4.2, eq. (12), with Z0 = 1 and the search
 *     variable d = -nu >= 0 (Sec. 4.1, eq. (11): nu <= 0, 1 + nu*tau > 0);
 *   - event image H(u; nu), eq. (13), and contrast C(nu), eq. (14), kept as
 *     the exact integer key K = M*S - N^2 = M^2 * C (S = sum H^2, N = sum H;
 *     the variance rewrite is the supplement's eq. for C = S/M - mu^2);
 *   - upper bound C_bar(V) = S_bar/M - mu_low^2, eqs. (15)-(20), from the
 *     upper-bound image H_bar (pixels crossed by the segment joining the
 *     warped endpoints, eq. (17)) and mu_low (segments fully in the image,
 *     eq. (20)), kept as K_bar = M*S_bar - N_low^2;
 *   - Algorithm 1 (best-first branch and bound) over a dyadic grid of d;
 *   - optionally, the event image kept per polarity (the *_pol functions),
 *     with the contrast taken over both images together.
 *
 * Readings where the paper is silent (fixed so that results are exactly
 * checkable):
 *   - fp32 arithmetic for every value that decides a pixel, in this order:
 *       ux = x - cx, uy = y - cy, delta = tau - t', ax = ux*delta,
 *       ay = uy*delta (per event); den = 1 - d*tau, r = d/den (per
 *       hypothesis); xw = fmaf(ax, r, x), yw = fmaf(ay, r, y).
 *     Algebraically this is eq. (12): u*(1 - d t)/(1 - d tau) =
 *     u + u*(tau - t)*d/(1 - d tau).  Each step is monotone in d, so the
 *     pixel coordinates of an event are monotone in d;
 *   - pixel k covers [k, k+1); an event is in the image iff 0 <= xw < W and
 *     0 <= yw < H; pixel index ky*W + kx;
 *   - the segment/pixel intersection of eq. (17) is a monotone staircase
 *     walk between the endpoint pixels (endpoint coordinates clamped to
 *     [-1, W] x [-1, H]) that, at each corner ahead, steps across whichever
 *     pixel edge the event's ray (through (x, y), direction (ax, ay)) meets
 *     first, decided in fp64 from e = |X - x|*|ay| - |Y - y|*|ax|; when the
 *     ray passes within 2^-8 px of the corner (|e| <= 2^-8 (|ax| + |ay|))
 *     both side pixels are counted.  The slack covers fp32 rounding off the
 *     exact ray, so H_bar >= H holds for every fp32 d in the interval;
 *   - "fully lies in the image plane" (eq. (20)): both fp32 endpoints are in
 *     the image;
 *   - grid: L = smallest L >= 1 with (d_hi - d_lo) 2^-L <= eps;
 *     d_j = float(d_lo + (d_hi - d_lo) j 2^-L) (fp64, then fp32); the
 *     candidates are j = 1 .. 2^L - 1, the centres of the dyadic nodes;
 *   - ties: the canonical optimum is the smallest j among the maximisers
 *     of K (Algorithm 1's ">=" is replaced by this lexicographic order).
 *
 * Build: cc -O2 -ffp-contract=off -fno-fast-math -std=gnu11 -shared -fPIC
 * (no contraction, so every product and sum is rounded exactly as written).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_EBUDGET = -4 };

/* ------------------------------------------------------------------ grid */

/* Depth of the dyadic grid: smallest L >= 1 with (d_hi - d_lo) 2^-L <= eps. */
int orc_depth(float d_lo, float d_hi, float eps)
{
    double span = (double)d_hi - (double)d_lo;
    for (int L = 1; L <= 30; ++L)
        if (ldexp(span, -L) <= (double)eps) return L;
    return -1;
}

/* Grid point j of depth L (the candidate divergence values). */
float orc_grid_d(float d_lo, float d_hi, int L, int64_t j)
{
    double span = (double)d_hi - (double)d_lo;
    double v = (double)d_lo + span * ldexp((double)j, -L);
    return (float)v;
}

/* Per-hypothesis rate r = d / (1 - d tau): with it eq. (12) moves an event
 * by (ax, ay) * r.  Evaluated in fp32 as written. */
float orc_rate(float d, float tau)
{
    float a = d * tau;
    float den = 1.0f - a;
    return d / den;
}

/* --------------------------------------------------------- event warping */

typedef struct {
    float x, y;   /* event position (pixel coordinates) */
    float ax, ay; /* (x - cx)(tau - t'), (y - cy)(tau - t') in fp32 */
} ev32_t;

static ev32_t *prep32(const float *x, const float *y, const float *t_rel,
                      int64_t n, float tau, float cx, float cy)
{
    ev32_t *e = (ev32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(ev32_t));
    if (!e) return NULL;
    for (int64_t i = 0; i < n; ++i) {
        float ux = x[i] - cx;
        float uy = y[i] - cy;
        float delta = tau - t_rel[i];
        e[i].x = x[i];
        e[i].y = y[i];
        e[i].ax = ux * delta;
        e[i].ay = uy * delta;
    }
    return e;
}

/* Warped position of event e at rate r: eq. (12). */
static void warp32(const ev32_t *e, float r, float *xw, float *yw)
{
    *xw = fmaf(e->ax, r, e->x);
    *yw = fmaf(e->ay, r, e->y);
}

static int inside32(float xw, float yw, int W, int H)
{
    return xw >= 0.0f && xw < (float)W && yw >= 0.0f && yw < (float)H;
}

/* Pixel index of every event at hypothesis d (-1 = outside the image). */
void orc_pixels(const float *x, const float *y, const float *t_rel, int64_t n,
                int W, int H, float cx, float cy, float tau, float d,
                int32_t *pix)
{
    ev32_t *e = prep32(x, y, t_rel, n, tau, cx, cy);
    float r = orc_rate(d, tau);
    for (int64_t i = 0; i < n; ++i) {
        float xw, yw;
        warp32(&e[i], r, &xw, &yw);
        if (inside32(xw, yw, W, H)) {
            int kx = (int)floorf(xw), ky = (int)floorf(yw);
            pix[i] = ky * W + kx;
        } else {
            pix[i] = -1;
        }
    }
    free(e);
}

/* --------------------------------------------------------- point value */

/* S = sum_u H(u)^2 and N = sum_u H(u) of the event image, eqs. (13)-(14). */
static void image_moments(const uint32_t *img, int64_t M, uint64_t *S, int64_t *N)
{
    uint64_t s = 0;
    int64_t nn = 0;
    for (int64_t p = 0; p < M; ++p) {
        s += (uint64_t)img[p] * (uint64_t)img[p];
        nn += img[p];
    }
    *S = s;
    *N = nn;
}

/* Event image H(u; d), eq. (13). */
static void point_image32(const ev32_t *e, int64_t n, int W, int H, float r,
                          uint32_t *img)
{
    memset(img, 0, (size_t)W * (size_t)H * sizeof(uint32_t));
    for (int64_t i = 0; i < n; ++i) {
        float xw, yw;
        warp32(&e[i], r, &xw, &yw);
        if (inside32(xw, yw, W, H)) {
            int kx = (int)floorf(xw), ky = (int)floorf(yw);
            img[(int64_t)ky * W + kx] += 1;
        }
    }
}

/* Point value of hypothesis d: (S, N) and optionally the image H. */
int orc_point(const float *x, const float *y, const float *t_rel, int64_t n,
              int W, int H, float cx, float cy, float tau, float d,
              uint64_t *S, int64_t *N, uint32_t *img_out)
{
    int64_t M = (int64_t)W * H;
    ev32_t *e = prep32(x, y, t_rel, n, tau, cx, cy);
    uint32_t *img = img_out ? img_out : (uint32_t *)malloc((size_t)M * sizeof(uint32_t));
    if (!e || !img) { free(e); if (!img_out) free(img); return ORC_ENOMEM; }
    point_image32(e, n, W, H, orc_rate(d, tau), img);
    image_moments(img, M, S, N);
    free(e);
    if (!img_out) free(img);
    return ORC_OK;
}

/* --------------------------------------------------------- interval value */

static void visit(uint32_t *img, int W, int H, int kx, int ky)
{
    if (kx >= 0 && kx < W && ky >= 0 && ky < H) img[(int64_t)ky * W + kx] += 1;
}

/* Add one to every pixel that the segment from pixel (kxa, kya) to pixel
 * (kxb, kyb) crosses (eq. (17)), following the event's ray through (x, y)
 * with direction (ax, ay).  Pixels outside the image are not counted. */
static void walk(uint32_t *img, int W, int H, int kxa, int kya, int kxb, int kyb,
                 double x, double y, double ax, double ay)
{
    int sx = (kxb > kxa) - (kxb < kxa);
    int sy = (kyb > kya) - (kyb < kya);
    double thr = ldexp(fabs(ax) + fabs(ay), -8);
    int kx = kxa, ky = kya;
    visit(img, W, H, kx, ky);
    while (kx != kxb || ky != kyb) {
        if (kx == kxb) {
            ky += sy;
        } else if (ky == kyb) {
            kx += sx;
        } else {
            /* corner shared with the diagonal neighbour ahead */
            double X = (double)(kx + (sx > 0));
            double Y = (double)(ky + (sy > 0));
            double ex = fabs(X - x) * fabs(ay); /* |ax||ay| * (ray parameter at x = X) */
            double ey = fabs(Y - y) * fabs(ax); /* |ax||ay| * (ray parameter at y = Y) */
            double e = ex - ey;
            if (e < -thr) {
                kx += sx;
            } else if (e > thr) {
                ky += sy;
            } else {
                visit(img, W, H, kx + sx, ky);
                visit(img, W, H, kx, ky + sy);
                kx += sx;
                ky += sy;
            }
        }
        visit(img, W, H, kx, ky);
    }
}

static int clamp_floor32(float v, int hi)
{
    float c = v < -1.0f ? -1.0f : v;
    c = c > (float)hi ? (float)hi : c;
    return (int)floorf(c);
}

/* Upper-bound image H_bar and N_low for the interval [r_a, r_b] of rates. */
static int64_t bound_image32(const ev32_t *e, int64_t n, int W, int H,
                             float ra, float rb, uint32_t *img)
{
    int64_t n_low = 0;
    memset(img, 0, (size_t)W * (size_t)H * sizeof(uint32_t));
    for (int64_t i = 0; i < n; ++i) {
        float xa, ya, xb, yb;
        warp32(&e[i], ra, &xa, &ya);
        warp32(&e[i], rb, &xb, &yb);
        if (inside32(xa, ya, W, H) && inside32(xb, yb, W, H)) n_low += 1;
        walk(img, W, H, clamp_floor32(xa, W), clamp_floor32(ya, H),
             clamp_floor32(xb, W), clamp_floor32(yb, H),
             (double)e[i].x, (double)e[i].y, (double)e[i].ax, (double)e[i].ay);
    }
    return n_low;
}

/* Interval value of [d_a, d_b]: (S_bar, N_low) and optionally H_bar. */
int orc_bound(const float *x, const float *y, const float *t_rel, int64_t n,
              int W, int H, float cx, float cy, float tau, float d_a, float d_b,
              uint64_t *S_bar, int64_t *N_low, uint32_t *img_out)
{
    int64_t M = (int64_t)W * H, dummy;
    if (!(d_a <= d_b)) return ORC_EINVAL;
    ev32_t *e = prep32(x, y, t_rel, n, tau, cx, cy);
    uint32_t *img = img_out ? img_out : (uint32_t *)malloc((size_t)M * sizeof(uint32_t));
    if (!e || !img) { free(e); if (!img_out) free(img); return ORC_ENOMEM; }
    *N_low = bound_image32(e, n, W, H, orc_rate(d_a, tau), orc_rate(d_b, tau), img);
    image_moments(img, M, S_bar, &dummy);
    free(e);
    if (!img_out) free(img);
    return ORC_OK;
}

/* --------------------------------------------------------- branch and bound */

typedef struct {
    int32_t status;
    uint32_t j_star, L;
    float d_hat;
    double contrast, d_end, gap;
    int64_t nodes_expanded, nodes_pruned, point_evals, bound_evals;
    uint64_t K_lo; /* low and high words of the exact key K = M*S - N^2 */
    int64_t K_hi;
} orc_result_t;

typedef struct {
    i128 key;
    uint32_t ja, jb;
} node_t;

/* a is popped before b: larger key first, then smaller left end */
static int before(const node_t *a, const node_t *b)
{
    return a->key > b->key || (a->key == b->key && a->ja < b->ja);
}

typedef struct {
    node_t *v;
    int64_t n, cap;
} heap_t;

static int heap_push(heap_t *h, node_t x)
{
    if (h->n == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 1024;
        node_t *nv = (node_t *)realloc(h->v, (size_t)nc * sizeof(node_t));
        if (!nv) return ORC_ENOMEM;
        h->v = nv;
        h->cap = nc;
    }
    int64_t i = h->n++;
    h->v[i] = x;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!before(&h->v[i], &h->v[p])) break;
        node_t t = h->v[i]; h->v[i] = h->v[p]; h->v[p] = t;
        i = p;
    }
    return ORC_OK;
}

static node_t heap_pop(heap_t *h)
{
    node_t top = h->v[0];
    h->v[0] = h->v[--h->n];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < h->n && before(&h->v[l], &h->v[m])) m = l;
        if (r < h->n && before(&h->v[r], &h->v[m])) m = r;
        if (m == i) break;
        node_t t = h->v[i]; h->v[i] = h->v[m]; h->v[m] = t;
        i = m;
    }
    return top;
}

/* A node [ja, jb] can still hold a candidate that beats the incumbent
 * (K_inc, j_inc) in the order (larger K, then smaller j). */
static int improvable(i128 key, uint32_t ja, i128 K_inc, uint32_t j_inc)
{
    return key > K_inc || (key == K_inc && (uint64_t)ja + 1 < (uint64_t)j_inc);
}

static i128 key_of(int64_t M, uint64_t S, int64_t N)
{
    return (i128)M * (i128)S - (i128)N * (i128)N;
}

/* Shared driver for the fp32 and fp64 statements: `pt` evaluates the key of
 * candidate j, `bd` the key of the node [ja, jb]. */
typedef i128 (*point_fn)(void *ctx, uint32_t j);
typedef i128 (*bound_fn)(void *ctx, uint32_t ja, uint32_t jb);

static int bnb_run(void *ctx, point_fn pt, bound_fn bd, int L, int64_t M,
                   double gamma, int64_t max_nodes, orc_result_t *res)
{
    heap_t h = {0};
    uint32_t top = 1u << L;
    uint32_t j_inc = top / 2; /* Algorithm 1: the incumbent starts at the centre */
    i128 K_inc = pt(ctx, j_inc);
    double M2 = (double)M * (double)M;
    res->point_evals = 1;
    res->bound_evals = 1;
    res->nodes_expanded = res->nodes_pruned = 0;
    res->status = ORC_OK;
    res->gap = 0.0;
    node_t root = {bd(ctx, 0, top), 0, top};
    if (heap_push(&h, root)) return ORC_ENOMEM;
    while (h.n > 0) {
        node_t nd = heap_pop(&h);
        if (gamma > 0.0) {
            /* paper mode: stop once the best bound is within gamma */
            double diff = (double)(nd.key - K_inc);
            if (diff <= gamma * M2) {
                res->gap = diff > 0 ? diff / M2 : 0.0;
                res->nodes_pruned += 1 + h.n;
                break;
            }
        } else if (!improvable(nd.key, nd.ja, K_inc, j_inc)) {
            /* every queued node ranks no higher: none can beat the incumbent */
            res->nodes_pruned += 1 + h.n;
            break;
        }
        if (max_nodes > 0 && res->nodes_expanded >= max_nodes) {
            double diff = (double)(nd.key - K_inc);
            res->gap = diff > 0 ? diff / M2 : 0.0;
            res->status = ORC_EBUDGET;
            break;
        }
        uint32_t jc = (nd.ja + nd.jb) / 2;
        i128 Kc = pt(ctx, jc);
        res->point_evals += 1;
        res->nodes_expanded += 1;
        if (Kc > K_inc || (Kc == K_inc && jc < j_inc)) {
            K_inc = Kc;
            j_inc = jc;
        }
        if (nd.jb - nd.ja >= 4) {
            node_t kids[2] = {{0, nd.ja, jc}, {0, jc, nd.jb}};
            for (int s = 0; s < 2; ++s) {
                kids[s].key = bd(ctx, kids[s].ja, kids[s].jb);
                res->bound_evals += 1;
                if (improvable(kids[s].key, kids[s].ja, K_inc, j_inc)) {
                    if (heap_push(&h, kids[s])) { free(h.v); return ORC_ENOMEM; }
                } else {
                    res->nodes_pruned += 1;
                }
            }
        }
    }
    free(h.v);
    res->j_star = j_inc;
    res->L = (uint32_t)L;
    res->K_lo = (uint64_t)K_inc;
    res->K_hi = (int64_t)(K_inc >> 64);
    res->contrast = (double)K_inc / M2;
    return res->status;
}

/* fp32 statement */
typedef struct {
    ev32_t *e;
    int64_t n, M;
    int W, H;
    float *r; /* rate of every grid point */
    uint32_t *img;
} ctx32_t;

static i128 pt32(void *c, uint32_t j)
{
    ctx32_t *k = (ctx32_t *)c;
    uint64_t S;
    int64_t N;
    point_image32(k->e, k->n, k->W, k->H, k->r[j], k->img);
    image_moments(k->img, k->M, &S, &N);
    return key_of(k->M, S, N);
}

static i128 bd32(void *c, uint32_t ja, uint32_t jb)
{
    ctx32_t *k = (ctx32_t *)c;
    uint64_t S;
    int64_t N;
    int64_t n_low = bound_image32(k->e, k->n, k->W, k->H, k->r[ja], k->r[jb], k->img);
    image_moments(k->img, k->M, &S, &N);
    return key_of(k->M, S, n_low);
}

static int validate(int64_t n, int W, int H, float tau, float d_lo, float d_hi, float eps)
{
    if (n < 0 || W <= 0 || H <= 0) return ORC_EINVAL;
    if (!(tau > 0.0f) || !(eps > 0.0f) || !(d_lo >= 0.0f) || !(d_lo < d_hi)) return ORC_EINVAL;
    if (!(d_hi * tau < 1.0f)) return ORC_EINVAL; /* cheirality: 1 + nu tau > 0 */
    if (orc_depth(d_lo, d_hi, eps) < 1) return ORC_EINVAL;
    return ORC_OK;
}

/* Canonical branch and bound (Algorithm 1) on the fp32 statement. */
int orc_bnb(const float *x, const float *y, const float *t_rel, int64_t n,
            int W, int H, float cx, float cy, float tau,
            float d_lo, float d_hi, float eps, double gamma, int64_t max_nodes,
            orc_result_t *res)
{
    int rc = validate(n, W, H, tau, d_lo, d_hi, eps);
    if (rc) { res->status = rc; return rc; }
    int L = orc_depth(d_lo, d_hi, eps);
    ctx32_t k = {0};
    k.n = n; k.W = W; k.H = H; k.M = (int64_t)W * H;
    k.e = prep32(x, y, t_rel, n, tau, cx, cy);
    k.r = (float *)malloc(((size_t)1 << L) * sizeof(float) + sizeof(float));
    k.img = (uint32_t *)malloc((size_t)k.M * sizeof(uint32_t));
    if (!k.e || !k.r || !k.img) { free(k.e); free(k.r); free(k.img); res->status = ORC_ENOMEM; return ORC_ENOMEM; }
    for (int64_t j = 0; j <= ((int64_t)1 << L); ++j) k.r[j] = orc_rate(orc_grid_d(d_lo, d_hi, L, j), tau);
    rc = bnb_run(&k, pt32, bd32, L, k.M, gamma, max_nodes, res);
    res->d_hat = orc_grid_d(d_lo, d_hi, L, res->j_star);
    res->d_end = (double)res->d_hat / (1.0 - (double)res->d_hat * (double)tau);
    free(k.e); free(k.r); free(k.img);
    return rc;
}

/* ------------------------------------------------ polarity-aware contrast */

/* The event image of eq. (13) kept per polarity (the paper notes after
 * eq. (14) that polarity can be accommodated): H_-(u) counts the events with
 * p <= 0 and H_+(u) those with p > 0.  The contrast of eq. (14) is then the
 * variance over all 2M cells (u, polarity), kept as K = 2M*S - N^2 with S
 * and N summed over both images.  Each image gets the upper bound of
 * eqs. (15)-(20) unchanged: the bound image is H_bar_- next to H_bar_+ and
 * N_low sums over both. */
typedef struct {
    ev32_t *e[2]; /* [0]: p <= 0, [1]: p > 0 */
    int64_t n[2];
} split32_t;

static void split_free(split32_t *s)
{
    free(s->e[0]);
    free(s->e[1]);
}

static int split_pol(const float *x, const float *y, const float *t_rel, const int8_t *pol,
                     int64_t n, float tau, float cx, float cy, split32_t *s)
{
    memset(s, 0, sizeof(*s));
    for (int l = 0; l < 2; ++l) {
        int64_t m = 0;
        for (int64_t i = 0; i < n; ++i) m += ((pol[i] > 0) == l);
        size_t bytes = (size_t)(m > 0 ? m : 1) * sizeof(float);
        float *bx = (float *)malloc(bytes), *by = (float *)malloc(bytes), *bt = (float *)malloc(bytes);
        if (!bx || !by || !bt) { free(bx); free(by); free(bt); split_free(s); return ORC_ENOMEM; }
        m = 0;
        for (int64_t i = 0; i < n; ++i) {
            if ((pol[i] > 0) != l) continue;
            bx[m] = x[i]; by[m] = y[i]; bt[m] = t_rel[i];
            ++m;
        }
        s->e[l] = prep32(bx, by, bt, m, tau, cx, cy);
        s->n[l] = m;
        free(bx); free(by); free(bt);
        if (!s->e[l]) { split_free(s); return ORC_ENOMEM; }
    }
    return ORC_OK;
}

/* Point value with polarity: (S, N) over both images; img_out (nullable)
 * receives H_- in its first W*H cells and H_+ in the next W*H. */
int orc_point_pol(const float *x, const float *y, const float *t_rel, const int8_t *pol, int64_t n,
                  int W, int H, float cx, float cy, float tau, float d,
                  uint64_t *S, int64_t *N, uint32_t *img_out)
{
    int64_t M = (int64_t)W * H;
    split32_t s;
    if (split_pol(x, y, t_rel, pol, n, tau, cx, cy, &s)) return ORC_ENOMEM;
    uint32_t *img = img_out ? img_out : (uint32_t *)malloc((size_t)(2 * M) * sizeof(uint32_t));
    if (!img) { split_free(&s); return ORC_ENOMEM; }
    float r = orc_rate(d, tau);
    point_image32(s.e[0], s.n[0], W, H, r, img);
    point_image32(s.e[1], s.n[1], W, H, r, img + M);
    image_moments(img, 2 * M, S, N);
    split_free(&s);
    if (!img_out) free(img);
    return ORC_OK;
}

/* Interval value with polarity: (S_bar, N_low) over both bound images. */
int orc_bound_pol(const float *x, const float *y, const float *t_rel, const int8_t *pol, int64_t n,
                  int W, int H, float cx, float cy, float tau, float d_a, float d_b,
                  uint64_t *S_bar, int64_t *N_low, uint32_t *img_out)
{
    int64_t M = (int64_t)W * H, dummy;
    if (!(d_a <= d_b)) return ORC_EINVAL;
    split32_t s;
    if (split_pol(x, y, t_rel, pol, n, tau, cx, cy, &s)) return ORC_ENOMEM;
    uint32_t *img = img_out ? img_out : (uint32_t *)malloc((size_t)(2 * M) * sizeof(uint32_t));
    if (!img) { split_free(&s); return ORC_ENOMEM; }
    float ra = orc_rate(d_a, tau), rb = orc_rate(d_b, tau);
    *N_low = bound_image32(s.e[0], s.n[0], W, H, ra, rb, img)
           + bound_image32(s.e[1], s.n[1], W, H, ra, rb, img + M);
    image_moments(img, 2 * M, S_bar, &dummy);
    split_free(&s);
    if (!img_out) free(img);
    return ORC_OK;
}

typedef struct {
    split32_t s;
    int W, H;
    int64_t M; /* W*H: cells per image */
    float *r;
    uint32_t *img; /* 2M cells */
} ctxpol_t;

static i128 ptpol(void *c, uint32_t j)
{
    ctxpol_t *k = (ctxpol_t *)c;
    uint64_t S;
    int64_t N;
    point_image32(k->s.e[0], k->s.n[0], k->W, k->H, k->r[j], k->img);
    point_image32(k->s.e[1], k->s.n[1], k->W, k->H, k->r[j], k->img + k->M);
    image_moments(k->img, 2 * k->M, &S, &N);
    return key_of(2 * k->M, S, N);
}

static i128 bdpol(void *c, uint32_t ja, uint32_t jb)
{
    ctxpol_t *k = (ctxpol_t *)c;
    uint64_t S;
    int64_t N;
    int64_t n_low = bound_image32(k->s.e[0], k->s.n[0], k->W, k->H, k->r[ja], k->r[jb], k->img)
                  + bound_image32(k->s.e[1], k->s.n[1], k->W, k->H, k->r[ja], k->r[jb], k->img + k->M);
    image_moments(k->img, 2 * k->M, &S, &N);
    return key_of(2 * k->M, S, n_low);
}

/* Canonical branch and bound (Algorithm 1) on the polarity-aware contrast. */
int orc_bnb_pol(const float *x, const float *y, const float *t_rel, const int8_t *pol, int64_t n,
                int W, int H, float cx, float cy, float tau,
                float d_lo, float d_hi, float eps, double gamma, int64_t max_nodes,
                orc_result_t *res)
{
    int rc = validate(n, W, H, tau, d_lo, d_hi, eps);
    if (rc) { res->status = rc; return rc; }
    int L = orc_depth(d_lo, d_hi, eps);
    ctxpol_t k;
    memset(&k, 0, sizeof k);
    k.W = W; k.H = H; k.M = (int64_t)W * H;
    if (split_pol(x, y, t_rel, pol, n, tau, cx, cy, &k.s)) { res->status = ORC_ENOMEM; return ORC_ENOMEM; }
    k.r = (float *)malloc(((size_t)1 << L) * sizeof(float) + sizeof(float));
    k.img = (uint32_t *)malloc((size_t)(2 * k.M) * sizeof(uint32_t));
    if (!k.r || !k.img) { split_free(&k.s); free(k.r); free(k.img); res->status = ORC_ENOMEM; return ORC_ENOMEM; }
    for (int64_t j = 0; j <= ((int64_t)1 << L); ++j) k.r[j] = orc_rate(orc_grid_d(d_lo, d_hi, L, j), tau);
    rc = bnb_run(&k, ptpol, bdpol, L, 2 * k.M, gamma, max_nodes, res);
    res->d_hat = orc_grid_d(d_lo, d_hi, L, res->j_star);
    res->d_end = (double)res->d_hat / (1.0 - (double)res->d_hat * (double)tau);
    split_free(&k.s); free(k.r); free(k.img);
    return rc;
}

/* Dense sweep: the plain definition of the canonical optimum, the
 * lexicographic maximum of (K_j, -j) over j = 1 .. 2^L - 1.  Optionally
 * writes S_j and N_j for every j = 0 .. 2^L. */
int orc_dense(const float *x, const float *y, const float *t_rel, int64_t n,
              int W, int H, float cx, float cy, float tau,
              float d_lo, float d_hi, float eps, orc_result_t *res,
              uint64_t *S_all, int64_t *N_all)
{
    int rc = validate(n, W, H, tau, d_lo, d_hi, eps);
    if (rc) { res->status = rc; return rc; }
    int L = orc_depth(d_lo, d_hi, eps);
    int64_t M = (int64_t)W * H, top = (int64_t)1 << L;
    ev32_t *e = prep32(x, y, t_rel, n, tau, cx, cy);
    uint32_t *img = (uint32_t *)malloc((size_t)M * sizeof(uint32_t));
    if (!e || !img) { free(e); free(img); res->status = ORC_ENOMEM; return ORC_ENOMEM; }
    i128 best = -1;
    uint32_t jbest = 0;
    memset(res, 0, sizeof(*res));
    for (int64_t j = 0; j <= top; ++j) {
        if (!S_all && (j == 0 || j == top)) continue;
        uint64_t S;
        int64_t N;
        point_image32(e, n, W, H, orc_rate(orc_grid_d(d_lo, d_hi, L, j), tau), img);
        image_moments(img, M, &S, &N);
        if (S_all) { S_all[j] = S; N_all[j] = N; }
        if (j == 0 || j == top) continue;
        i128 K = key_of(M, S, N);
        res->point_evals += 1;
        if (K > best) { best = K; jbest = (uint32_t)j; }
    }
    res->status = ORC_OK;
    res->j_star = jbest;
    res->L = (uint32_t)L;
    res->d_hat = orc_grid_d(d_lo, d_hi, L, jbest);
    res->d_end = (double)res->d_hat / (1.0 - (double)res->d_hat * (double)tau);
    res->K_lo = (uint64_t)best;
    res->K_hi = (int64_t)(best >> 64);
    res->contrast = (double)best / ((double)M * (double)M);
    free(e); free(img);
    return ORC_OK;
}

/* ------------------------------------------------------------ fp64 statement */

/* The same method with every value in fp64 and grid points not rounded to
 * fp32; reported beside the fp32 result (|d_hat32 - d_hat64|). */
typedef struct {
    double x, y, ax, ay;
} ev64_t;

typedef struct {
    ev64_t *e;
    int64_t n, M;
    int W, H;
    double *r;
    uint32_t *img;
} ctx64_t;

static ev64_t *prep64(const float *x, const float *y, const float *t_rel, int64_t n,
                      float tau, float cx, float cy)
{
    ev64_t *e = (ev64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(ev64_t));
    if (!e) return NULL;
    for (int64_t i = 0; i < n; ++i) {
        double delta = (double)tau - (double)t_rel[i];
        e[i].x = x[i];
        e[i].y = y[i];
        e[i].ax = ((double)x[i] - (double)cx) * delta;
        e[i].ay = ((double)y[i] - (double)cy) * delta;
    }
    return e;
}

static int inside64(double xw, double yw, int W, int H)
{
    return xw >= 0.0 && xw < (double)W && yw >= 0.0 && yw < (double)H;
}

static int clamp_floor64(double v, int hi)
{
    double c = v < -1.0 ? -1.0 : v;
    c = c > (double)hi ? (double)hi : c;
    return (int)floor(c);
}

static void point_image64(const ev64_t *e, int64_t n, int W, int H, double r, uint32_t *img)
{
    memset(img, 0, (size_t)W * (size_t)H * sizeof(uint32_t));
    for (int64_t i = 0; i < n; ++i) {
        double xw = e[i].x + e[i].ax * r, yw = e[i].y + e[i].ay * r;
        if (inside64(xw, yw, W, H)) img[(int64_t)floor(yw) * W + (int64_t)floor(xw)] += 1;
    }
}

static i128 pt64(void *c, uint32_t j)
{
    ctx64_t *k = (ctx64_t *)c;
    uint64_t S;
    int64_t N;
    point_image64(k->e, k->n, k->W, k->H, k->r[j], k->img);
    image_moments(k->img, k->M, &S, &N);
    return key_of(k->M, S, N);
}

static i128 bd64(void *c, uint32_t ja, uint32_t jb)
{
    ctx64_t *k = (ctx64_t *)c;
    uint64_t S;
    int64_t N;
    int64_t n_low = 0;
    memset(k->img, 0, (size_t)k->M * sizeof(uint32_t));
    for (int64_t i = 0; i < k->n; ++i) {
        const ev64_t *e = &k->e[i];
        double xa = e->x + e->ax * k->r[ja], ya = e->y + e->ay * k->r[ja];
        double xb = e->x + e->ax * k->r[jb], yb = e->y + e->ay * k->r[jb];
        if (inside64(xa, ya, k->W, k->H) && inside64(xb, yb, k->W, k->H)) n_low += 1;
        walk(k->img, k->W, k->H, clamp_floor64(xa, k->W), clamp_floor64(ya, k->H),
             clamp_floor64(xb, k->W), clamp_floor64(yb, k->H), e->x, e->y, e->ax, e->ay);
    }
    image_moments(k->img, k->M, &S, &N);
    return key_of(k->M, S, n_low);
}

int orc_bnb64(const float *x, const float *y, const float *t_rel, int64_t n,
              int W, int H, float cx, float cy, float tau,
              float d_lo, float d_hi, float eps, double gamma, int64_t max_nodes,
              orc_result_t *res, double *d_hat64)
{
    int rc = validate(n, W, H, tau, d_lo, d_hi, eps);
    if (rc) { res->status = rc; return rc; }
    int L = orc_depth(d_lo, d_hi, eps);
    ctx64_t k = {0};
    k.n = n; k.W = W; k.H = H; k.M = (int64_t)W * H;
    k.e = prep64(x, y, t_rel, n, tau, cx, cy);
    k.r = (double *)malloc(((size_t)1 << L) * sizeof(double) + sizeof(double));
    k.img = (uint32_t *)malloc((size_t)k.M * sizeof(uint32_t));
    if (!k.e || !k.r || !k.img) { free(k.e); free(k.r); free(k.img); res->status = ORC_ENOMEM; return ORC_ENOMEM; }
    double span = (double)d_hi - (double)d_lo;
    for (int64_t j = 0; j <= ((int64_t)1 << L); ++j) {
        double d = (double)d_lo + span * ldexp((double)j, -L);
        k.r[j] = d / (1.0 - d * (double)tau);
    }
    rc = bnb_run(&k, pt64, bd64, L, k.M, gamma, max_nodes, res);
    *d_hat64 = (double)d_lo + span * ldexp((double)res->j_star, -L);
    res->d_hat = (float)*d_hat64;
    res->d_end = *d_hat64 / (1.0 - *d_hat64 * (double)tau);
    free(k.e); free(k.r); free(k.img);
    return rc;
}

/* fp64 point value at an arbitrary fp64 d (used by the continuum sweep). */
int orc_point64(const float *x, const float *y, const float *t_rel, int64_t n,
                int W, int H, float cx, float cy, float tau, double d,
                uint64_t *S, int64_t *N)
{
    int64_t M = (int64_t)W * H;
    ev64_t *e = prep64(x, y, t_rel, n, tau, cx, cy);
    uint32_t *img = (uint32_t *)malloc((size_t)M * sizeof(uint32_t));
    if (!e || !img) { free(e); free(img); return ORC_ENOMEM; }
    point_image64(e, n, W, H, d / (1.0 - d * (double)tau), img);
    image_moments(img, M, S, N);
    free(e); free(img);
    return ORC_OK;
}

/* ------------------------------------------------------------ window prep */

/* Events of the window [t0, t1] (closed) with offsets t' = float(t - t0);
 * returns the count, writes the selected indices and offsets. */
int64_t orc_select(const double *t, int64_t n, double t0, double t1,
                   int64_t *idx, float *t_rel)
{
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (t[i] >= t0 && t[i] <= t1) {
            idx[m] = i;
            t_rel[m] = (float)(t[i] - t0);
            ++m;
        }
    }
    return m;
}

/* ------------------------------------------------ learned-incumbent input */

/* Unwarped event-count image binned to G x G cells, scaled by G*G/N and
 * rounded to bfloat16 (round to nearest even): the network's input.
 * Cell of an event: floor(float(x*G)/W) (fp32, clamped to G-1). */
static uint16_t to_bf16(float v)
{
    uint32_t u;
    memcpy(&u, &v, 4);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return (uint16_t)(u >> 16);
}

int orc_downsample(const float *x, const float *y, int64_t n, int W, int H, int G,
                   uint16_t *out)
{
    uint32_t *cnt = (uint32_t *)calloc((size_t)G * G, sizeof(uint32_t));
    if (!cnt) return ORC_ENOMEM;
    for (int64_t i = 0; i < n; ++i) {
        float fx = (x[i] * (float)G) / (float)W;
        float fy = (y[i] * (float)G) / (float)H;
        int bx = (int)floorf(fx), by = (int)floorf(fy);
        if (bx > G - 1) bx = G - 1;
        if (by > G - 1) by = G - 1;
        if (bx < 0) bx = 0;
        if (by < 0) by = 0;
        cnt[by * G + bx] += 1;
    }
    float scale = n > 0 ? (float)(G * G) / (float)n : 0.0f;
    for (int i = 0; i < G * G; ++i) out[i] = to_bf16((float)cnt[i] * scale);
    free(cnt);
    return ORC_OK;
}
