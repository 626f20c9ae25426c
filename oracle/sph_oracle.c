/*
 * sph_oracle.c -- plain CPU reference for the SPH density path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or helper with the GPU library; both are fed the same
 * seeded inputs and nothing else.
 *
 * Everything is IEEE binary64, built with -ffp-contract=off (no fused
 * multiply-add), so pair distances are computed exactly as written here.
 *
 * What it computes (paper: Baruffa et al., "Performance Optimisation of SPH
 * Algorithms for Multi/Many-Core Architectures", arXiv:1612.06090):
 *   - the SPH density sum of Eq. (1), in gather form with the particle's own
 *     smoothing length h_i, over all j with |r_ij| < h_i (the "within a
 *     smoothing length" test of Listing 1), self term included;
 *   - the per-particle recompute loop of Sec. IV-A (Listings 2/3): h_i is
 *     adjusted and the density re-evaluated until the particle's neighbour
 *     criterion holds.  The paper does not give the update rule; the rule
 *     below is a safeguarded Newton step on the weighted neighbour count with
 *     doubling / halving / bisection fall-backs;
 *   - the lockless work sharing of Listing 3 (OpenMP dynamic schedule over
 *     the particles still to compute);
 *   - Morton keys, a stable key sort and a cell table (inputs of the GPU
 *     path's spatial sort; no counterpart in the paper, whose tree is given);
 *   - the analytic adjoint of the density with h held on its implicit root.
 *
 * Kernels (cfg.kernel), both with compact support h, W(r,h) = sigma/h^3 f(r/h):
 *   0  M4 cubic spline (the Gadget-2 convention), sigma = 8/pi:
 *      f = 1 - 6q^2 + 6q^3 (q <= 1/2), 2(1-q)^3 (1/2 < q <= 1);
 *   1  Wendland C6, the kernel of the paper's runs (Sec. II-B), in its 3D
 *      normalisation, sigma = 1365/(64 pi):  f = (1-q)^8 (1 + 8q + 25q^2 + 32q^3).
 * The weighted neighbour count is n = (4 pi/3) h^3 sum_j W = C sum_j f with
 * C = (4 pi/3) sigma (32/3 and 1365/48).
 *
 * Parity pins for every function here live in the CPU test-suite
 * (normalisation integral, brute force vs k-d tree, lattice sums, closed-form
 * two-particle roots, finite differences and invariants of the adjoint).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* status word: low 16 bits = number of h updates, high bits = flags */
#define ORC_NOCONV      (1 << 16)
#define ORC_HTOOLARGE   (1 << 17)
#define ORC_BADINPUT    (1 << 18)
#define ORC_UNREACHABLE (1 << 19)

typedef struct {
    int32_t periodic;       /* 1: periodic cube [0,box)^3 ; 0: isolated groups */
    double box;
    int32_t ngroups;        /* 0: one set; else number of groups (offsets has ngroups+1) */
    const int64_t *offsets; /* group CSR in caller order, or NULL */
    double n_target;
    double n_tol;
    int32_t mode;           /* 0: band |n-Nt| <= dN ; 1: root |n-Nt| <= root_tol*Nt */
    double root_tol;
    int32_t max_iter;       /* 0: evaluate at h_init only */
    int32_t search;         /* 0: brute force ; 1: k-d tree */
    int32_t nthreads;       /* <= 0: OpenMP default */
    int32_t kernel;         /* 0: M4 cubic spline ; 1: Wendland C6 */
} orc_cfg;

/* ------------------------------------------------------------------ kernel */

/* f(q) of the M4 cubic spline with support q < 1. */
double oracle_kernel_f(double q)
{
    if (q < 0.0) q = -q;
    if (q <= 0.5) return 1.0 - 6.0 * q * q + 6.0 * q * q * q;
    if (q <= 1.0) {
        double t = 1.0 - q;
        return 2.0 * t * t * t;
    }
    return 0.0;
}

/* df/dq of the same spline. */
double oracle_kernel_dfdq(double q)
{
    if (q <= 0.5) return -12.0 * q + 18.0 * q * q;
    if (q <= 1.0) {
        double t = 1.0 - q;
        return -6.0 * t * t;
    }
    return 0.0;
}

/* W(r,h) = 8/(pi h^3) f(r/h) */
double oracle_kernel_W(double r, double h)
{
    return 8.0 / (ORC_PI * h * h * h) * oracle_kernel_f(r / h);
}

/* f(q) of the Wendland C6 function with support q < 1. */
double oracle_wendland6_f(double q)
{
    if (q < 0.0) q = -q;
    if (q >= 1.0) return 0.0;
    double t = 1.0 - q;
    double t2 = t * t, t4 = t2 * t2, t8 = t4 * t4;
    return t8 * (1.0 + 8.0 * q + 25.0 * q * q + 32.0 * q * q * q);
}

/* df/dq of the same function: -22 q (1-q)^7 (1 + 7q + 16q^2). */
double oracle_wendland6_dfdq(double q)
{
    if (q >= 1.0) return 0.0;
    double t = 1.0 - q;
    double t2 = t * t, t4 = t2 * t2, t7 = t4 * t2 * t;
    return -22.0 * q * t7 * (1.0 + 7.0 * q + 16.0 * q * q);
}

/* Kernel selected by id: shape, normalisation sigma and count constant C. */
double oracle_f(int32_t kernel, double q)
{
    return kernel == 1 ? oracle_wendland6_f(q) : oracle_kernel_f(q);
}

double oracle_dfdq(int32_t kernel, double q)
{
    return kernel == 1 ? oracle_wendland6_dfdq(q) : oracle_kernel_dfdq(q);
}

double oracle_sigma(int32_t kernel)
{
    return kernel == 1 ? 1365.0 / (64.0 * ORC_PI) : 8.0 / ORC_PI;
}

double oracle_count_const(int32_t kernel)
{
    return kernel == 1 ? 1365.0 / 48.0 : 32.0 / 3.0;
}

/* ---------------------------------------------------------------- geometry */

/* Minimum-image component: d = xj - xi, wrapped once into [-L/2, L/2]. */
static double mi(double d, double L, int *wcode)
{
    *wcode = 0;
    if (d > 0.5 * L) { *wcode = -1; return d - L; }
    if (d < -0.5 * L) { *wcode = 1; return d + L; }
    return d;
}

/* r^2 = (dx*dx + dy*dy) + dz*dz, evaluated in that order. wc receives the
 * wrap applied on each axis (for the k-d tree's image bookkeeping). */
static double pair_r2(const orc_cfg *c, double xi, double yi, double zi,
                      double xj, double yj, double zj, double *d, int *wc)
{
    double dx = xj - xi, dy = yj - yi, dz = zj - zi;
    wc[0] = wc[1] = wc[2] = 0;
    if (c->periodic) {
        dx = mi(dx, c->box, &wc[0]);
        dy = mi(dy, c->box, &wc[1]);
        dz = mi(dz, c->box, &wc[2]);
    }
    if (d) { d[0] = dx; d[1] = dy; d[2] = dz; }
    return (dx * dx + dy * dy) + dz * dz;
}

static int valid_particle(const orc_cfg *c, double x, double y, double z, double m, double h)
{
    if (!isfinite(x) || !isfinite(y) || !isfinite(z) || !isfinite(m) || !isfinite(h)) return 0;
    if (!(h > 0.0)) return 0;
    if (c->periodic) {
        if (!(x >= 0.0 && x < c->box)) return 0;
        if (!(y >= 0.0 && y < c->box)) return 0;
        if (!(z >= 0.0 && z < c->box)) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------ Morton keys */

/* Spread the low `bits` bits of v so that bit b lands on bit 3b. */
static uint64_t spread_bits(uint64_t v, int bits)
{
    uint64_t r = 0;
    for (int b = 0; b < bits; ++b) r |= ((v >> b) & 1ull) << (3 * b);
    return r;
}

static uint64_t quantise(double t, uint64_t nmax)
{
    /* floor(t) clamped to [0, nmax-1]; NaN -> 0 */
    if (!(t >= 0.0)) return 0;
    if (t >= (double)nmax) return nmax - 1;
    return (uint64_t)floor(t);
}

/* Periodic set: q = floor(x * (2^21/L)) per axis, key bit 3k+2 <- x bit k,
 * 3k+1 <- y bit k, 3k <- z bit k. */
void oracle_morton_periodic(int64_t n, const double *x, const double *y, const double *z,
                            double box, uint64_t *keys)
{
    const double s = 2097152.0 / box;
    for (int64_t i = 0; i < n; ++i) {
        uint64_t qx = quantise(x[i] * s, 1ull << 21);
        uint64_t qy = quantise(y[i] * s, 1ull << 21);
        uint64_t qz = quantise(z[i] * s, 1ull << 21);
        keys[i] = (spread_bits(qx, 21) << 2) | (spread_bits(qy, 21) << 1) | spread_bits(qz, 21);
    }
}

/* Group bounding cube: lower corner and scale 2^16 / (largest extent). */
void oracle_group_frames(int32_t ngroups, const int64_t *offsets, const double *x,
                         const double *y, const double *z, double *origin /*3G*/,
                         double *scale /*G*/)
{
    for (int32_t g = 0; g < ngroups; ++g) {
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int64_t i = offsets[g]; i < offsets[g + 1]; ++i) {
            const double p[3] = {x[i], y[i], z[i]};
            for (int a = 0; a < 3; ++a) {
                if (!isfinite(p[a])) continue;
                if (p[a] < lo[a]) lo[a] = p[a];
                if (p[a] > hi[a]) hi[a] = p[a];
            }
        }
        double ext = 0.0;
        for (int a = 0; a < 3; ++a) {
            if (!(lo[a] <= hi[a])) { lo[a] = 0.0; hi[a] = 0.0; }
            double e = hi[a] - lo[a];
            if (e > ext) ext = e;
        }
        if (!(ext > 0.0)) ext = 1.0;
        origin[3 * g + 0] = lo[0];
        origin[3 * g + 1] = lo[1];
        origin[3 * g + 2] = lo[2];
        scale[g] = 65536.0 / ext;
    }
}

/* Isolated groups: key = (g << 48) | 16-bit-per-axis Morton code on the
 * group's bounding cube, q = floor((x - lo) * (2^16/extent)). */
void oracle_morton_groups(int64_t n, int32_t ngroups, const int64_t *offsets,
                          const double *x, const double *y, const double *z, uint64_t *keys)
{
    (void)n;
    double *org = (double *)malloc(sizeof(double) * 3 * (size_t)(ngroups > 0 ? ngroups : 1));
    double *sc = (double *)malloc(sizeof(double) * (size_t)(ngroups > 0 ? ngroups : 1));
    oracle_group_frames(ngroups, offsets, x, y, z, org, sc);
    for (int32_t g = 0; g < ngroups; ++g) {
        for (int64_t i = offsets[g]; i < offsets[g + 1]; ++i) {
            uint64_t qx = quantise((x[i] - org[3 * g + 0]) * sc[g], 1ull << 16);
            uint64_t qy = quantise((y[i] - org[3 * g + 1]) * sc[g], 1ull << 16);
            uint64_t qz = quantise((z[i] - org[3 * g + 2]) * sc[g], 1ull << 16);
            keys[i] = ((uint64_t)g << 48) |
                      (spread_bits(qx, 16) << 2) | (spread_bits(qy, 16) << 1) | spread_bits(qz, 16);
        }
    }
    free(org);
    free(sc);
}

/* ------------------------------------------------------------ stable sort */

typedef struct { uint64_t key; int64_t idx; } kv_t;

static int kv_cmp(const void *a, const void *b)
{
    const kv_t *p = (const kv_t *)a, *q = (const kv_t *)b;
    if (p->key < q->key) return -1;
    if (p->key > q->key) return 1;
    return (p->idx > q->idx) - (p->idx < q->idx);
}

/* Ascending by key; equal keys keep the caller's order. perm[s] = original index. */
void oracle_stable_sort(int64_t n, const uint64_t *keys, uint64_t *sorted, int32_t *perm)
{
    kv_t *t = (kv_t *)malloc(sizeof(kv_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) { t[i].key = keys[i]; t[i].idx = i; }
    qsort(t, (size_t)n, sizeof(kv_t), kv_cmp);
    for (int64_t i = 0; i < n; ++i) { sorted[i] = t[i].key; perm[i] = (int32_t)t[i].idx; }
    free(t);
}

/* Contract cell level: max(1, ceil((ceil(log2 n) - 3) / 3)), capped at `cap`. */
int32_t oracle_cell_level(int64_t n, int32_t cap)
{
    int lg = 0;
    while (lg < 62 && ((int64_t)1 << lg) < n) ++lg;
    int t = lg - 3;
    int lc = t <= 0 ? 1 : (t + 2) / 3;
    if (lc < 1) lc = 1;
    if (lc > cap) lc = cap;
    return lc;
}

/* Occupied cells of sorted keys at `shift`: (key >> shift, first index, count). */
int64_t oracle_cell_table(int64_t n, const uint64_t *sorted, int32_t shift,
                          uint64_t *cell_id, int32_t *start, int32_t *count)
{
    int64_t nc = 0;
    for (int64_t s = 0; s < n; ++s) {
        uint64_t c = sorted[s] >> shift;
        if (s == 0 || c != (sorted[s - 1] >> shift)) {
            cell_id[nc] = c;
            start[nc] = (int32_t)s;
            count[nc] = 0;
            ++nc;
        }
        count[nc - 1] += 1;
    }
    return nc;
}

/* --------------------------------------------------------------- k-d tree */

typedef struct {
    double lo[3], hi[3];
    int64_t begin, end;   /* range of kd->idx */
    int32_t left, right;  /* -1 for a leaf */
} kdnode;

typedef struct {
    kdnode *nodes;
    int64_t nnodes, cap;
    int64_t *idx;
    const double *p[3];
} kdtree;

#define KD_LEAF 16

static double coord(const kdtree *t, int64_t j, int a) { return t->p[a][j]; }

/* Partition idx[b,e) so that position k holds the k-th smallest along axis a
 * (ties broken by particle index, which keeps the build deterministic). */
static int kd_less(const kdtree *t, int64_t u, int64_t v, int a)
{
    double cu = coord(t, u, a), cv = coord(t, v, a);
    if (cu < cv) return 1;
    if (cu > cv) return 0;
    return u < v;
}

static void kd_select(kdtree *t, int64_t b, int64_t e, int64_t k, int a)
{
    int64_t *ix = t->idx;
    while (e - b > 1) {
        int64_t mid = b + (e - b) / 2;
        /* median of three as pivot */
        int64_t i0 = ix[b], i1 = ix[mid], i2 = ix[e - 1], pv;
        if (kd_less(t, i0, i1, a)) {
            if (kd_less(t, i1, i2, a)) pv = i1;
            else if (kd_less(t, i0, i2, a)) pv = i2;
            else pv = i0;
        } else {
            if (kd_less(t, i0, i2, a)) pv = i0;
            else if (kd_less(t, i1, i2, a)) pv = i2;
            else pv = i1;
        }
        /* three-way partition around pv */
        int64_t lt = b, i = b, gt = e;
        while (i < gt) {
            int64_t v = ix[i];
            if (kd_less(t, v, pv, a)) { ix[i] = ix[lt]; ix[lt] = v; ++lt; ++i; }
            else if (kd_less(t, pv, v, a)) { --gt; ix[i] = ix[gt]; ix[gt] = v; }
            else ++i;
        }
        if (k < lt) e = lt;
        else if (k >= gt) b = gt;
        else return;
    }
}

static int32_t kd_build_rec(kdtree *t, int64_t b, int64_t e)
{
    if (t->nnodes == t->cap) {
        t->cap = t->cap ? 2 * t->cap : 64;
        t->nodes = (kdnode *)realloc(t->nodes, sizeof(kdnode) * (size_t)t->cap);
    }
    int32_t id = (int32_t)t->nnodes++;
    kdnode nd;
    for (int a = 0; a < 3; ++a) { nd.lo[a] = INFINITY; nd.hi[a] = -INFINITY; }
    for (int64_t s = b; s < e; ++s) {
        for (int a = 0; a < 3; ++a) {
            double v = coord(t, t->idx[s], a);
            if (v < nd.lo[a]) nd.lo[a] = v;
            if (v > nd.hi[a]) nd.hi[a] = v;
        }
    }
    nd.begin = b;
    nd.end = e;
    nd.left = nd.right = -1;
    if (e - b > KD_LEAF) {
        int ax = 0;
        double ext = nd.hi[0] - nd.lo[0];
        for (int a = 1; a < 3; ++a)
            if (nd.hi[a] - nd.lo[a] > ext) { ext = nd.hi[a] - nd.lo[a]; ax = a; }
        int64_t mid = b + (e - b) / 2;
        kd_select(t, b, e, mid, ax);
        nd.left = kd_build_rec(t, b, mid);
        nd.right = kd_build_rec(t, mid, e);
    }
    t->nodes[id] = nd;
    return id;
}

/* Tree over the valid particles among [b, e). */
static void kd_build(kdtree *t, const orc_cfg *c, const double *x, const double *y,
                     const double *z, const double *m, const double *h0, int64_t b, int64_t e)
{
    memset(t, 0, sizeof(*t));
    t->p[0] = x; t->p[1] = y; t->p[2] = z;
    t->idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(e - b > 0 ? e - b : 1));
    int64_t k = 0;
    for (int64_t j = b; j < e; ++j)
        if (valid_particle(c, x[j], y[j], z[j], m[j], h0 ? h0[j] : 1.0)) t->idx[k++] = j;
    if (k > 0) kd_build_rec(t, 0, k);
}

static void kd_free(kdtree *t)
{
    free(t->nodes);
    free(t->idx);
    memset(t, 0, sizeof(*t));
}

/* ---------------------------------------------------------- density sums */

typedef struct {
    double S0;  /* sum f(q)               */
    double S1;  /* sum q f'(q)            */
    double R;   /* sum m_j f(q)           */
    double A;   /* sum m_j (3 f + q f')   */
    int64_t N;  /* pairs with r^2 < h^2   */
} sums_t;

static void add_pair(sums_t *s, int32_t kernel, double r2, double h, double mj)
{
    double q = sqrt(r2) / h;
    double f = oracle_f(kernel, q);
    double fp = oracle_dfdq(kernel, q);
    s->S0 += f;
    s->S1 += q * fp;
    s->R += mj * f;
    s->A += mj * (3.0 * f + q * fp);
    s->N += 1;
}

typedef struct {
    const orc_cfg *c;
    int64_t n;
    const double *x, *y, *z, *m, *h0;
    unsigned char *valid;
    int64_t *dom;       /* domain (group) of each particle, or NULL */
    kdtree *trees;      /* one per domain when search == 1 */
    int32_t ndom;
} ctx_t;

static void dom_range(const ctx_t *k, int64_t i, int64_t *b, int64_t *e, int32_t *d)
{
    if (k->c->ngroups > 0) {
        int64_t g = k->dom[i];
        *b = k->c->offsets[g];
        *e = k->c->offsets[g + 1];
        *d = (int32_t)g;
    } else {
        *b = 0;
        *e = k->n;
        *d = 0;
    }
}

/* Visitor called once per neighbour j of i: r^2 and the min-image
 * displacement d = x_j - x_i. */
typedef void (*visit_fn)(void *u, int64_t j, double r2, const double *d);

/* All j of i's domain with r_ij^2 < h^2, by direct enumeration (definition). */
static void visit_brute(const ctx_t *k, int64_t i, double h, visit_fn fn, void *u)
{
    int64_t b, e;
    int32_t d;
    dom_range(k, i, &b, &e, &d);
    const double h2 = h * h;
    int wc[3];
    double dv[3];
    for (int64_t j = b; j < e; ++j) {
        if (!k->valid[j]) continue;
        double r2 = pair_r2(k->c, k->x[i], k->y[i], k->z[i], k->x[j], k->y[j], k->z[j], dv, wc);
        if (r2 < h2) fn(u, j, r2, dv);
    }
}

/* Same set via the k-d tree: query each periodic image of x_i that the ball
 * can reach, and accept j only from the image that is its minimum image, so
 * that no pair is visited twice.  r^2 is the same expression as above. */
static void visit_kd(const ctx_t *k, int64_t i, double h, visit_fn fn, void *u)
{
    int64_t b, e;
    int32_t d;
    dom_range(k, i, &b, &e, &d);
    const kdtree *t = &k->trees[d];
    if (t->nnodes == 0) return;
    const double h2 = h * h;
    const double slack = h * (1.0 + 1e-9);
    const double L = k->c->box;
    const double pi3[3] = {k->x[i], k->y[i], k->z[i]};
    int codes[3][3], nc[3];
    for (int a = 0; a < 3; ++a) {
        nc[a] = 0;
        codes[a][nc[a]++] = 0;
        if (k->c->periodic) {
            if (pi3[a] - slack < 0.0) codes[a][nc[a]++] = 1;
            if (pi3[a] + slack >= L) codes[a][nc[a]++] = -1;
        }
    }
    int32_t stack[256];
    for (int ia = 0; ia < nc[0]; ++ia)
    for (int ib = 0; ib < nc[1]; ++ib)
    for (int ic = 0; ic < nc[2]; ++ic) {
        const int sc[3] = {codes[0][ia], codes[1][ib], codes[2][ic]};
        const double p[3] = {pi3[0] + sc[0] * L, pi3[1] + sc[1] * L, pi3[2] + sc[2] * L};
        int sp = 0;
        stack[sp++] = 0;
        while (sp > 0) {
            const kdnode *nd = &t->nodes[stack[--sp]];
            double d2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                double g = 0.0;
                if (p[a] < nd->lo[a]) g = nd->lo[a] - p[a];
                else if (p[a] > nd->hi[a]) g = p[a] - nd->hi[a];
                d2 += g * g;
            }
            if (d2 > slack * slack) continue;
            if (nd->left >= 0) {
                stack[sp++] = nd->left;
                stack[sp++] = nd->right;
                continue;
            }
            for (int64_t s = nd->begin; s < nd->end; ++s) {
                int64_t j = t->idx[s];
                int wc[3];
                double dv[3];
                double r2 = pair_r2(k->c, pi3[0], pi3[1], pi3[2], k->x[j], k->y[j], k->z[j], dv, wc);
                if (!(r2 < h2)) continue;
                if (wc[0] != -sc[0] || wc[1] != -sc[1] || wc[2] != -sc[2]) continue;
                fn(u, j, r2, dv);
            }
        }
    }
}

static void visit(const ctx_t *k, int64_t i, double h, visit_fn fn, void *u)
{
    if (k->c->search == 1) visit_kd(k, i, h, fn, u);
    else visit_brute(k, i, h, fn, u);
}

typedef struct { sums_t s; double h; const double *m; int32_t kernel; } sum_acc;

static void sum_visit(void *u, int64_t j, double r2, const double *d)
{
    (void)d;
    sum_acc *a = (sum_acc *)u;
    add_pair(&a->s, a->kernel, r2, a->h, a->m[j]);
}

static sums_t eval_sums(const ctx_t *k, int64_t i, double h)
{
    sum_acc a;
    memset(&a, 0, sizeof(a));
    a.h = h;
    a.m = k->m;
    a.kernel = k->c->kernel;
    visit(k, i, h, sum_visit, &a);
    return a.s;
}

static void ctx_init(ctx_t *k, const orc_cfg *c, int64_t n, const double *x, const double *y,
                     const double *z, const double *m, const double *h0)
{
    memset(k, 0, sizeof(*k));
    k->c = c; k->n = n; k->x = x; k->y = y; k->z = z; k->m = m; k->h0 = h0;
    k->valid = (unsigned char *)malloc((size_t)(n > 0 ? n : 1));
    for (int64_t j = 0; j < n; ++j)
        k->valid[j] = (unsigned char)valid_particle(c, x[j], y[j], z[j], m[j], h0 ? h0[j] : 1.0);
    if (c->ngroups > 0) {
        k->dom = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        for (int32_t g = 0; g < c->ngroups; ++g)
            for (int64_t j = c->offsets[g]; j < c->offsets[g + 1]; ++j) k->dom[j] = g;
    }
    k->ndom = c->ngroups > 0 ? c->ngroups : 1;
    if (c->search == 1) {
        k->trees = (kdtree *)calloc((size_t)k->ndom, sizeof(kdtree));
        if (c->ngroups > 0) {
#pragma omp parallel for schedule(dynamic)
            for (int32_t g = 0; g < c->ngroups; ++g)
                kd_build(&k->trees[g], c, x, y, z, m, h0, c->offsets[g], c->offsets[g + 1]);
        } else {
            kd_build(&k->trees[0], c, x, y, z, m, h0, 0, n);
        }
    }
}

static void ctx_free(ctx_t *k)
{
    if (k->trees) {
        for (int32_t d = 0; d < k->ndom; ++d) kd_free(&k->trees[d]);
        free(k->trees);
    }
    free(k->valid);
    free(k->dom);
}

static void set_threads(const orc_cfg *c)
{
#ifdef _OPENMP
    if (c->nthreads > 0) omp_set_num_threads(c->nthreads);
#else
    (void)c;
#endif
}

int32_t oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Density and its h-derivatives at given smoothing lengths (no iteration).
 * rho = sigma R/h^3, n = C S0, dn/dh = -C S1/h, drho/dh = -sigma A/h^4
 * (M4: sigma = 8/pi, C = 32/3). Any output pointer may be NULL. */
void oracle_eval_at_h(const orc_cfg *c, int64_t n, const double *x, const double *y,
                      const double *z, const double *m, const double *h, double *rho,
                      double *nw, double *dndh, double *drhodh, int64_t *nngb)
{
    ctx_t k;
    set_threads(c);
    ctx_init(&k, c, n, x, y, z, m, h);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        if (!k.valid[i]) {
            if (rho) rho[i] = NAN;
            if (nw) nw[i] = NAN;
            if (dndh) dndh[i] = NAN;
            if (drhodh) drhodh[i] = NAN;
            if (nngb) nngb[i] = 0;
            continue;
        }
        double hi = h[i];
        sums_t s = eval_sums(&k, i, hi);
        const double sg = oracle_sigma(c->kernel), cc = oracle_count_const(c->kernel);
        if (rho) rho[i] = sg * s.R / (hi * hi * hi);
        if (nw) nw[i] = cc * s.S0;
        if (dndh) dndh[i] = -cc * s.S1 / hi;
        if (drhodh) drhodh[i] = -sg * s.A / (hi * hi * hi * hi);
        if (nngb) nngb[i] = s.N;
    }
    ctx_free(&k);
}

/* ulp of a positive finite double */
static double ulp_of(double h)
{
    return nextafter(h, INFINITY) - h;
}

typedef struct {
    double rho, h, nw, dndh;
    int32_t nngb, status;
    int64_t pairs;   /* in-range pairs evaluated over all trial h */
} solve_out;

/* The recompute loop for one particle (independent of all others). */
static solve_out solve_one(const ctx_t *k, int64_t i)
{
    const orc_cfg *c = k->c;
    solve_out o;
    memset(&o, 0, sizeof(o));
    double h = k->h0[i];
    if (!k->valid[i] || !(h > 0.0)) {
        o.rho = NAN; o.h = h; o.nw = NAN; o.dndh = NAN; o.nngb = 0;
        o.status = ORC_BADINPUT;
        return o;
    }
    const double Nt = c->n_target, dN = c->n_tol;
    const double hmax = c->periodic ? 0.5 * c->box * (1.0 - 0x1p-20) : INFINITY;
    int32_t flags = 0;
    int fixed = c->max_iter == 0;
    if (c->ngroups > 0) {
        int64_t g = k->dom[i];
        double nmax = oracle_count_const(c->kernel) * (double)(c->offsets[g + 1] - c->offsets[g]);
        if (nmax < Nt - dN) { flags |= ORC_UNREACHABLE; fixed = 1; }
    }
    if (h > hmax) h = hmax;
    double lo = 0.0, hi = INFINITY;
    int32_t it = 0;
    sums_t s;
    double nwv, dndh;
    for (;;) {
        s = eval_sums(k, i, h);
        o.pairs += s.N;
        nwv = oracle_count_const(c->kernel) * s.S0;
        dndh = -oracle_count_const(c->kernel) * s.S1 / h;
        if (fixed) break;
        int conv;
        if (c->mode == 0) {
            conv = fabs(nwv - Nt) <= dN;
        } else {
            conv = fabs(nwv - Nt) <= c->root_tol * Nt;
            if (!conv && lo > 0.0 && hi < INFINITY && hi - lo <= 4.0 * ulp_of(h)) conv = 1;
        }
        if (conv) break;
        if (it >= c->max_iter) { flags |= ORC_NOCONV; break; }
        if (nwv < Nt) lo = h; else hi = h;
        double hn = 0.0;
        int ok = 0;
        if (dndh > 0.0) {
            hn = h + (Nt - nwv) / dndh;
            ok = hn > lo && hn < hi && hn >= 0.5 * h && hn <= 2.0 * h;
        }
        if (!ok) {
            if (hi == INFINITY) hn = 2.0 * h;
            else if (lo == 0.0) hn = 0.5 * h;
            else hn = 0.5 * (lo + hi);
        }
        if (hn >= hmax) {
            if (h == hmax) { flags |= ORC_HTOOLARGE; break; }
            hn = hmax;
        }
        h = hn;
        ++it;
    }
    o.h = h;
    o.rho = oracle_sigma(c->kernel) * s.R / (h * h * h);
    o.nw = nwv;
    o.dndh = dndh;
    o.nngb = (int32_t)s.N;
    o.status = flags | (it & 0xffff);
    return o;
}

/* Solve every particle (subset == NULL: outputs indexed by particle) or the
 * listed ones (outputs indexed by position in subset).  OpenMP dynamic
 * schedule over particles: each is independent, as in Listing 3. */
void oracle_solve(const orc_cfg *c, int64_t n, const double *x, const double *y,
                  const double *z, const double *m, const double *h_init,
                  const int64_t *subset, int64_t nsub, double *rho, double *h, double *nw,
                  double *dndh, int32_t *nngb, int32_t *status, int64_t *pairs)
{
    ctx_t k;
    set_threads(c);
    ctx_init(&k, c, n, x, y, z, m, h_init);
    int64_t cnt = subset ? nsub : n;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t u = 0; u < cnt; ++u) {
        int64_t i = subset ? subset[u] : u;
        solve_out o = solve_one(&k, i);
        if (rho) rho[u] = o.rho;
        if (h) h[u] = o.h;
        if (nw) nw[u] = o.nw;
        if (dndh) dndh[u] = o.dndh;
        if (nngb) nngb[u] = o.nngb;
        if (status) status[u] = o.status;
        if (pairs) pairs[u] = o.pairs;
    }
    ctx_free(&k);
}

/* --------------------------------------------- exact K nearest neighbours */

/* The K-nearest criterion of Sec. IV-D: particle i's smoothing length is the
 * distance of the K-th nearest particle of its domain, counting i itself as
 * the first (the paper sorts the neighbour list, or selects with QUICKSELECT,
 * and keeps the first K); the density is Eq. (1) at that h, where the K-th
 * neighbour sits at q = 1 and contributes W = 0, so ties at the K-th
 * distance do not change rho.  Done the plain way: every squared distance
 * inside a ball that doubles from h_init until it holds at least K particles
 * is collected, the list is sorted (qsort), and entry K-1 is taken.
 * Flags: UNREACHABLE for a group with fewer than K valid particles (h stays
 * h_init, rho evaluated there); H_TOO_LARGE when the periodic ball reaches the
 * cap L/2 (1 - 2^-20) before holding K (h = the cap).  The low 16 status bits
 * are 0 (no iteration here).  subset == NULL: every particle, outputs indexed
 * by particle; else the listed ones, outputs indexed by position in subset. */
typedef struct { double *d2; int64_t cnt, cap; } d2_list;

static void d2_visit(void *u, int64_t j, double r2, const double *d)
{
    (void)j; (void)d;
    d2_list *L = (d2_list *)u;
    if (L->cnt == L->cap) {
        L->cap = L->cap ? 2 * L->cap : 1024;
        L->d2 = (double *)realloc(L->d2, sizeof(double) * (size_t)L->cap);
    }
    L->d2[L->cnt++] = r2;
}

static int cmp_double(const void *a, const void *b)
{
    const double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

void oracle_knn(const orc_cfg *c, int64_t n, const double *x, const double *y,
                const double *z, const double *m, const double *h_init, int32_t K,
                const int64_t *subset, int64_t nsub,
                double *rho, double *h, double *nw, int32_t *nngb, int32_t *status)
{
    ctx_t k;
    set_threads(c);
    ctx_init(&k, c, n, x, y, z, m, h_init);
    const double hmax = c->periodic ? 0.5 * c->box * (1.0 - 0x1p-20) : INFINITY;
    const double sg = oracle_sigma(c->kernel), cc = oracle_count_const(c->kernel);
    const int64_t cnt = subset ? nsub : n;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t u = 0; u < cnt; ++u) {
        const int64_t i = subset ? subset[u] : u;
        double hi = h_init[i];
        int32_t flags = 0;
        if (!k.valid[i]) {
            rho[u] = NAN; h[u] = hi; nw[u] = NAN; nngb[u] = 0; status[u] = ORC_BADINPUT;
            continue;
        }
        int64_t b, e;
        int32_t dm;
        dom_range(&k, i, &b, &e, &dm);
        int64_t nvalid = 0;
        for (int64_t j = b; j < e; ++j) nvalid += k.valid[j];
        if (hi > hmax) hi = hmax;
        if (!c->periodic && nvalid < K) {
            flags |= ORC_UNREACHABLE;
        } else {
            d2_list L = {NULL, 0, 0};
            double r = hi;
            for (;;) {
                L.cnt = 0;
                visit(&k, i, r, d2_visit, &L);
                if (L.cnt >= K) break;
                if (r >= hmax) { flags |= ORC_HTOOLARGE; break; }
                r = 2.0 * r < hmax ? 2.0 * r : hmax;
            }
            if (flags & ORC_HTOOLARGE) {
                hi = hmax;
            } else {
                qsort(L.d2, (size_t)L.cnt, sizeof(double), cmp_double);
                hi = sqrt(L.d2[K - 1]);
                if (hi >= hmax) { hi = hmax; flags |= ORC_HTOOLARGE; }
            }
            free(L.d2);
        }
        sums_t s = eval_sums(&k, i, hi);
        h[u] = hi;
        rho[u] = sg * s.R / (hi * hi * hi);
        nw[u] = cc * s.S0;
        nngb[u] = (int32_t)s.N;
        status[u] = flags;
    }
    ctx_free(&k);
}

/* ------------------------------------------------ scatter and symmetric form */

/* Eq. (1) as printed: rho_i = sum_j m_j W(r_ij, h_j), every particle j
 * spreading its mass over its own sphere r < h_j (the particle itself
 * included, r = 0).  Done the plain way: a serial loop over j that visits
 * every i inside j's sphere and adds m_j W(r_ij, h_j) to rho_s[i].  The
 * symmetric form averages it with the gather form at i's own h:
 * rho_sym_i = (rho_g_i + rho_s_i) / 2, rho_g_i = sum_j m_j W(r_ij, h_i).
 * Invalid particles get NaN and are nobody's neighbour; nngb_s[i] counts the
 * j whose sphere holds i. */
typedef struct { double mj, hj; int32_t kernel; double *rho; int64_t *cnt; } scat_acc;

static void scat_visit(void *u, int64_t i, double r2, const double *d)
{
    (void)d;
    scat_acc *a = (scat_acc *)u;
    const double hj = a->hj;
    const double q = sqrt(r2) / hj;
    a->rho[i] += a->mj * oracle_sigma(a->kernel) / (hj * hj * hj) * oracle_f(a->kernel, q);
    a->cnt[i] += 1;
}

void oracle_scatter(const orc_cfg *c, int64_t n, const double *x, const double *y,
                    const double *z, const double *m, const double *h, double *rho_s,
                    double *rho_sym, int64_t *nngb_s)
{
    ctx_t k;
    set_threads(c);
    ctx_init(&k, c, n, x, y, z, m, h);
    int64_t *cnt = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) rho_s[i] = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        if (!k.valid[j]) continue;
        scat_acc a = {m[j], h[j], c->kernel, rho_s, cnt};
        visit(&k, j, h[j], scat_visit, &a);
    }
    const double sg = oracle_sigma(c->kernel);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        if (!k.valid[i]) {
            rho_s[i] = NAN;
            if (rho_sym) rho_sym[i] = NAN;
            if (nngb_s) nngb_s[i] = 0;
            continue;
        }
        if (rho_sym) {
            const double hi = h[i];
            sums_t sg_i = eval_sums(&k, i, hi);
            rho_sym[i] = 0.5 * (sg * sg_i.R / (hi * hi * hi) + rho_s[i]);
        }
        if (nngb_s) nngb_s[i] = cnt[i];
    }
    free(cnt);
    ctx_free(&k);
}

typedef struct {
    int64_t i;
    double h, gr, lam;
    const double *m;
    double *gx, *gy, *gz, *gm;
    int32_t kernel;
} bw_acc;

static void bw_visit(void *u, int64_t j, double r2, const double *d)
{
    bw_acc *a = (bw_acc *)u;
    const double hi = a->h;
    const double cW = oracle_sigma(a->kernel) / (hi * hi * hi);
    double r = sqrt(r2);
    double q = r / hi;
    a->gm[j] += a->gr * cW * oracle_f(a->kernel, q);
    if (j == a->i || r == 0.0) return;
    double fp = oracle_dfdq(a->kernel, q);
    double cij = a->gr * a->m[j] * cW / hi * fp
               + a->lam * oracle_count_const(a->kernel) * fp / hi;
    /* unit vector u = (x_i - x_j)/r = -d/r */
    double ux = -d[0] / r, uy = -d[1] / r, uz = -d[2] / r;
    a->gx[a->i] += cij * ux; a->gy[a->i] += cij * uy; a->gz[a->i] += cij * uz;
    a->gx[j] -= cij * ux; a->gy[j] -= cij * uy; a->gz[j] -= cij * uz;
}

/* Analytic adjoint of rho (and optionally h) with h_i held on the implicit
 * root n_i(h_i, x) = n_i(achieved).  For a cotangent (gr, gh):
 *   lambda_i = -(gr_i drho_i/dh_i + gh_i) / (dn_i/dh_i)      (0 if dn/dh = 0)
 *   pair (i, j in N(i), j != i), q = r_ij/h_i, u = (x_i - x_j)/r_ij:
 *     c_ij = gr_i m_j sigma/h_i^4 f'(q) + lambda_i C f'(q) / h_i
 *     gx_i += c_ij u ;  gx_j -= c_ij u
 *   mass: gm_j += gr_i W(r_ij, h_i)   (self term included; n is number-
 *   weighted, so h does not depend on the masses).
 * Plain serial scatter over the brute-force (or k-d tree) neighbour sets. */
void oracle_backward(const orc_cfg *c, int64_t n, const double *x, const double *y,
                     const double *z, const double *m, const double *h, const double *grad_rho,
                     const double *grad_h, double *gx, double *gy, double *gz, double *gm)
{
    ctx_t k;
    set_threads(c);
    ctx_init(&k, c, n, x, y, z, m, h);
    double *lam = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        lam[i] = 0.0;
        if (!k.valid[i]) continue;
        double hi = h[i];
        sums_t s = eval_sums(&k, i, hi);
        double drhodh = -oracle_sigma(c->kernel) * s.A / (hi * hi * hi * hi);
        double dndh = -oracle_count_const(c->kernel) * s.S1 / hi;
        double gh = grad_h ? grad_h[i] : 0.0;
        if (dndh > 0.0) lam[i] = -(grad_rho[i] * drhodh + gh) / dndh;
    }
    for (int64_t j = 0; j < n; ++j) { gx[j] = 0.0; gy[j] = 0.0; gz[j] = 0.0; gm[j] = 0.0; }
    for (int64_t i = 0; i < n; ++i) {
        if (!k.valid[i]) continue;
        bw_acc a;
        a.i = i; a.h = h[i]; a.gr = grad_rho[i]; a.lam = lam[i]; a.m = m;
        a.kernel = c->kernel;
        a.gx = gx; a.gy = gy; a.gz = gz; a.gm = gm;
        visit(&k, i, h[i], bw_visit, &a);
    }
    free(lam);
    ctx_free(&k);
}
