// Density and smoothing-length solve: Eq. (1) of the paper evaluated in
// gather form with each particle's own h, inside the per-particle recompute
// loop of Sec. IV-A (Listings 2 and 3).
//
// GPU design (one wavefront = one tile of up to 64 Morton-consecutive
// particles, one particle per lane):
//  * Work sharing: a persistent grid pulls tiles from a device work queue
//    with one atomic per tile -- the lock-free dynamic schedule of Listing 3,
//    without the single hot lock of Listing 2.
//  * Neighbour search: instead of the paper's tree walk (Sec. IV-B), the
//    tile's active particles define a region; the Morton cells covering it at
//    a level whose cell side is at least the tile's largest h are culled
//    against every active particle's sphere, and the surviving cells'
//    contiguous runs of the sorted arrays are streamed in coalesced load
//    rounds of 64 candidates.  Each candidate is tested once against the
//    region of the (sub-)tile -- its particles' bounding box widened by their
//    largest h -- and the ones inside are appended (ballot slots) to a staging
//    buffer in LDS; whenever 64 are staged, every lane reads them by broadcast
//    and tests them against its own particle and h.  Tiles that straddle a
//    large jump of the Morton curve are split in halves until the region is
//    small.
//  * The in-support test of Listing 1 is an exact r^2 < h^2 compare;
//    the kernel sums run only on in-range pairs.
//  * h iteration: after each pass every lane updates its own h (safeguarded
//    Newton on the weighted count, FP64); a ballot gives the lanes still
//    iterating and only they define the next pass's region.  This replaces the
//    "todo" list of Sec. IV-A: converged lanes drop out of the region.
//
// Precision forms:
//  FP64  -- positions, distances and sums in binary64; r^2 is evaluated as
//           (dx*dx + dy*dy) + dz*dz without contraction, so neighbour sets at a
//           given h are bit-identical to a plain CPU evaluation.
//  FP32C -- positions held as integer Morton-grid coordinates plus binary32
//           fractions; each tile works relative to an integer origin, so
//           pair differences carry the precision of the local separation, not
//           of the box.  Kernel sums in binary32 with Kahan compensation; the
//           convergence test and the h update stay binary64.
#include "sph_internal.h"

#include <type_traits>

namespace sph {

constexpr int kMaxRegionCells = 512;  // split tiles whose region needs more cells

struct SolveArgs {
    int64_t n;
    int32_t G;
    const int64_t *goff;
    const uint64_t *skeys;
    const int32_t *perm;
    const double4 *sp;  // FP64: x, y, z, m
    const double *sh0;
    const int4 *qp;     // FP32C: grid cell, mass bits
    const float4 *fp;   // FP32C: fraction
    const int32_t *table;
    int32_t Ld;
    const double *frame;
    const int32_t *gitems;
    const int32_t *gorder;
    int64_t n_items;
    int32_t seg;
    double box;
    int32_t bits;
    double Nt, dN, root_tol;
    int32_t mode, max_iter, cell_exp;
    int32_t out_f32;
    void *rho, *h, *nw;
    int32_t *nngb, *status;
    int64_t ost, ost_i;  // byte strides of the floating and the int32 outputs
    int32_t *queue;
    uint64_t *stats;
    // exact-K stages: the count stage's h and status, the selected h
    double *knn_h;
    int32_t sel_cap;  // entries of the selection heap (16, 32 or 64)
    int32_t *knn_st;
    int32_t *knn_items;
    double *sh_out;
};

// Values every lane of the wave already holds (results of a full-wave
// reduction or broadcast), moved to scalar registers.
__device__ inline double uniform_d(double v) {
    int2 b = __builtin_bit_cast(int2, v);
    b.x = __builtin_amdgcn_readfirstlane(b.x);
    b.y = __builtin_amdgcn_readfirstlane(b.y);
    return __builtin_bit_cast(double, b);
}

__device__ inline int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ inline uint64_t uniform_u64(uint64_t v) {
    return __builtin_bit_cast(uint64_t, uniform_d(__builtin_bit_cast(double, v)));
}

struct HState {
    double h, lo, hi;
    int it, flags;
    bool fixed;
    // exact-K count stage: counts at the bracket ends, bracket width before
    // the last step
    int nlo, nhi;
    double wprev;
};


// One update of the h iteration.  Returns true when the particle is finished.
// Exact-K mode iterates on the integer count N = #(r < h) towards the band
// [K, K + dK].  Until both ends are bracketed it takes the volume-ratio step
// h (K' / N)^(1/3) (K' the band centre) within [h/8, 2h] (a count far above
// the band is a reliable measure of how much to shrink; growing is capped
// harder, a sphere that reaches a clump can overshoot), or, where the count
// has grown (or fallen) more slowly than h^(3/2) since the previous step on
// the same side, the step of that local power law; once bracketed it
// interpolates log N linearly in log h between the ends (the count's local
// power law, which is steep where the sphere reaches a clump and makes the
// plain volume step oscillate), kept 5% inside the bracket, and bisects
// whenever the previous step did not halve the bracket.  Any h whose count
// lies in [K, K + sel_cap - 1] lets the selection stage find the K-th
// distance, so the upper end is handed over once the bracket is narrower than
// 2^-10 h and its count within reach of the selection heap (ties: the count
// jumps over the band), or when the updates run out; the
// path does not affect what is returned.
template <bool KNN>
__device__ inline bool h_step(HState &s, double nwv, double dndh, int32_t ncount,
                              const SolveArgs &a, double hmax) {
    if (s.fixed) return true;
    if (KNN) {
        const double N = (double)ncount;
        if (N >= a.Nt && N <= a.Nt + a.dN) return true;
        // the previous end on this side (the count's local power law, below)
        const double h_pv = N < a.Nt ? s.lo : s.hi;
        const int32_t n_pv = N < a.Nt ? s.nlo : s.nhi;
        if (N < a.Nt) { s.lo = s.h; s.nlo = ncount; } else { s.hi = s.h; s.nhi = ncount; }
        const bool br = s.lo > 0.0 && s.hi < INFINITY;
        const bool narrow = br && s.hi - s.lo <= 0x1p-10 * s.hi &&
                            (double)s.nhi - a.Nt < (double)a.sel_cap;
        const bool closed = br && s.hi - s.lo <= 4.0 * (nextafter(s.hi, INFINITY) - s.hi);
        if (narrow || closed || s.it >= a.max_iter) {
            if (s.hi < INFINITY) s.h = s.hi;
            else s.flags |= SPH_ST_NOCONV;
            return true;
        }
        const double Kc = a.Nt + 0.5 * a.dN + 0.5;
        double hn;
        if (br) {
            const double w = s.hi - s.lo;
            if (w > 0.5 * s.wprev || s.nlo < 1) {
                hn = 0.5 * (s.lo + s.hi);
            } else {
                // binary32 is ample for a step that is checked against the bracket
                const float lnlo = __logf((float)s.nlo);
                float t = (__logf((float)Kc) - lnlo) / (__logf((float)s.nhi) - lnlo);
                t = fminf(fmaxf(t, 0.05f), 0.95f);
                hn = s.lo * (double)__expf(t * __logf((float)(s.hi / s.lo)));
                if (!(hn > s.lo && hn < s.hi)) hn = 0.5 * (s.lo + s.hi);
            }
            s.wprev = w;
        } else {
            // where the count follows the volume less than as h^(3/2) since
            // the previous step on this side (a sphere inside a dense clump
            // that must reach past it), the volume step would creep: the
            // step follows that local power law instead (exponent >= 1/4)
            // (binary32 is ample for a step that is clamped and checked)
            float ex = 3.f;
            if (h_pv > 0.0 && h_pv < INFINITY && n_pv > 0 && h_pv != s.h) {
                const float lr = __logf((float)(N / (double)n_pv)) / __logf((float)(s.h / h_pv));
                if (lr < 1.5f) ex = fmaxf(lr, 0.25f);
            }
            hn = ex == 3.f ? s.h * cbrt(Kc / fmax(N, 1.0))
                           : s.h * (double)__expf(__logf((float)(Kc / fmax(N, 1.0))) / ex);
            hn = fmin(fmax(hn, 0.125 * s.h), 2.0 * s.h);
        }
        if (hn >= hmax) {
            if (s.h == hmax) {
                s.flags |= SPH_ST_HTOOLARGE;
                return true;
            }
            hn = hmax;
        }
        s.h = hn;
        s.it += 1;
        return false;
    }
    bool conv;
    if (a.mode == SPH_BAND) {
        conv = fabs(nwv - a.Nt) <= a.dN;
    } else {
        conv = fabs(nwv - a.Nt) <= a.root_tol * a.Nt;
        if (!conv && s.lo > 0.0 && s.hi < INFINITY &&
            s.hi - s.lo <= 4.0 * (nextafter(s.h, INFINITY) - s.h))
            conv = true;
    }
    if (conv) return true;
    if (s.it >= a.max_iter) {
        s.flags |= SPH_ST_NOCONV;
        return true;
    }
    if (nwv < a.Nt) s.lo = s.h; else s.hi = s.h;
    double hn = 0.0;
    bool ok = false;
    if (dndh > 0.0) {
        hn = s.h + (a.Nt - nwv) / dndh;
        ok = hn > s.lo && hn < s.hi && hn >= 0.5 * s.h && hn <= 2.0 * s.h;
    }
    if (!ok) {
        if (s.hi == INFINITY) hn = 2.0 * s.h;
        else if (s.lo == 0.0) hn = 0.5 * s.h;
        else hn = 0.5 * (s.lo + s.hi);
    }
    if (hn >= hmax) {
        if (s.h == hmax) {
            s.flags |= SPH_ST_HTOOLARGE;
            return true;
        }
        hn = hmax;
    }
    s.h = hn;
    s.it += 1;
    return false;
}

__device__ inline void write_out(const SolveArgs &a, int64_t i, double rho, double h, double nw,
                                 int32_t nngb, int32_t status) {
    if (a.out_f32) {
        st<float>(a.rho, i, rho, a.ost);
        st<float>(a.h, i, h, a.ost);
        if (a.nw) st<float>(a.nw, i, nw, a.ost);
    } else {
        st<double>(a.rho, i, rho, a.ost);
        st<double>(a.h, i, h, a.ost);
        if (a.nw) st<double>(a.nw, i, nw, a.ost);
    }
    if (a.nngb) st_i32(a.nngb, i, nngb, a.ost_i);
    if (a.status) st_i32(a.status, i, status, a.ost_i);
}

// Smallest level-L cell side 2^e (grid units) with 2^e >= v, e >= 0.
__device__ inline int ceil_log2_pos(double v) {
    if (!(v > 1.0)) return 0;
    int ex;
    const double m = frexp(v, &ex);  // v = m 2^ex, m in [0.5, 1)
    return m == 0.5 ? ex - 1 : ex;
}

// Sorted-slot range of the level-L cell with Morton code cm (periodic set).
__device__ inline void cell_range_periodic(const SolveArgs &a, uint64_t cm, int L, int32_t &st_,
                                           int32_t &en_) {
    const int Ld = a.Ld;
    if (L <= Ld) {
        const int sh = 3 * (Ld - L);
        st_ = a.table[cm << sh];
        en_ = a.table[(cm + 1) << sh];
        return;
    }
    const uint64_t anc = cm >> (3 * (L - Ld));
    int32_t lo = a.table[anc], hi = a.table[anc + 1];
    const int ks = 3 * (a.bits - L);
    const uint64_t k0 = cm << ks, k1 = (cm + 1) << ks;
    // lower_bound(k0) and lower_bound(k1) inside [lo, hi)
    int32_t b = lo, e = hi;
    while (b < e) {
        const int32_t mid = (b + e) >> 1;
        if (a.skeys[mid] < k0) b = mid + 1; else e = mid;
    }
    st_ = b;
    e = hi;
    while (b < e) {
        const int32_t mid = (b + e) >> 1;
        if (a.skeys[mid] < k1) b = mid + 1; else e = mid;
    }
    en_ = b;
}

// Same for a cell of group g: binary search inside the group's sorted range.
__device__ inline void cell_range_group(const SolveArgs &a, int32_t g, uint64_t cm, int L,
                                        int32_t &st_, int32_t &en_) {
    const int ks = 3 * (a.bits - L);
    const uint64_t gb = (uint64_t)(uint32_t)g << 48;
    const uint64_t k0 = gb + (cm << ks), k1 = gb + ((cm + 1) << ks);
    int32_t lo = (int32_t)a.goff[g], hi = (int32_t)a.goff[g + 1];
    int32_t b = lo, e = hi;
    while (b < e) {
        const int32_t mid = (b + e) >> 1;
        if (a.skeys[mid] < k0) b = mid + 1; else e = mid;
    }
    st_ = b;
    e = hi;
    while (b < e) {
        const int32_t mid = (b + e) >> 1;
        if (a.skeys[mid] < k1) b = mid + 1; else e = mid;
    }
    en_ = b;
}

template <int PREC>
struct CandLDS;

// Staging buffer of the candidate stream: the candidates that passed the
// sub-tile's region test and wait to be tested by its particles.  Up to 63
// wait between test rounds and a load round adds up to 64, so 127 entries.
constexpr int kStage = 128;

template <>
struct CandLDS<SPH_FP64> {
    double x[kStage], y[kStage], z[kStage], m[kStage], shx[kStage], shy[kStage], shz[kStage];
};

template <>
struct CandLDS<SPH_FP32C> {
    float4 c[kStage];  // x, y, z relative to the tile origin (grid units), m
};

struct Sums {
    // FP64: s0, s1, r.  FP32C: float sums with Kahan compensations.
    double d0, d1, dr;
    float f0, f1, fr, c0, c1, cr;
    int32_t n;
};

__device__ inline void kahan(float &s, float &c, float x) {
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// P particles per wave tile; each particle is held by S = 64/P lanes, and
// lane copy kk of a particle tests chunk candidates kk, kk + S, ...; the
// copies' sums are combined before the (replicated) h update.  Smaller P
// means a smaller tile region (fewer candidates per particle) and a shorter
// sequential stream per wave, at the price of more tiles.
// Exact-K selection: status bit of a particle that stage 2 leaves to stage 4,
// and the control word (after the work queue's) that counts the tiles holding
// one (their items listed in knn_items)
constexpr int32_t kSelRetry = 1 << 30;
constexpr int kSelRetrySlot = 8;

// Selection heap of the exact-K mode: per lane, a min-heap of the CAP largest
// squared distances inside h (binary64 for FP64, binary32 for FP32C: rounding
// is monotone, so the order is kept and only the selected value is rounded),
// slot i of lane l at [i * 64 + l].  `hmin` mirrors the root in a register, so
// a candidate below it costs one compare.
template <int CAP, typename T>
__device__ inline void sel_insert(T *H, int l, int &hc, T x, T &hmin) {
    if (hc < CAP) {
        int i = hc++;
        while (i > 0) {
            const int q = (i - 1) >> 1;
            const T pv = H[q * 64 + l];
            if (pv <= x) break;
            H[i * 64 + l] = pv;
            i = q;
        }
        H[i * 64 + l] = x;
        hmin = H[l];
    } else if (x > hmin) {
        int i = 0;
        for (;;) {
            int c = 2 * i + 1;
            if (c >= CAP) break;
            T cv = H[c * 64 + l];
            if (c + 1 < CAP && H[(c + 1) * 64 + l] < cv) { ++c; cv = H[c * 64 + l]; }
            if (cv >= x) break;
            H[i * 64 + l] = cv;
            i = c;
        }
        H[i * 64 + l] = x;
        hmin = H[l];
    }
}

// Remove the heap minimum (heap of size hc > 0).
template <typename T>
__device__ inline void sel_pop(T *H, int l, int &hc) {
    const T x = H[(hc - 1) * 64 + l];
    --hc;
    int i = 0;
    for (;;) {
        int c = 2 * i + 1;
        if (c >= hc) break;
        T cv = H[c * 64 + l];
        if (c + 1 < hc && H[(c + 1) * 64 + l] < cv) { ++c; cv = H[c * 64 + l]; }
        if (cv >= x) break;
        H[i * 64 + l] = cv;
        i = c;
    }
    if (hc > 0) H[i * 64 + l] = x;
}

// STAGE 0: the density solve of the band and root modes.  Exact K runs three
// launches: 1 iterates h on the integer count into the band [K, K + dK]
// (writes knn_h, knn_st); 2 selects (16-particle tiles, 4 lanes per
// particle): at the count-stage h of each particle the squared distances
// inside h are ranked and the K-th smallest becomes the particle's h (writes
// sh_out, knn_st); 3 evaluates at that h with the status of knn_st.  The
// stage is a template argument so that the band-mode kernel carries none of
// it.
//
// Selection.  The K-th smallest of the c distances inside h is their
// (c - K + 1)-th largest, and the count stage hands over only an h whose rank
// is at most CAP.  Stage 2 keeps, per lane, only the distances of an outer
// shell r^2 > tau^2 (a volume fraction of the sphere expected to hold about
// CAP + 8 particles at uniform density) in a list of at most CAP (a full
// list keeps the CAP largest met), and ranks the union of a particle's lists
// once at the end of the pass by counting.  Where the shell holds fewer than
// the rank, it marks the particle (kSelRetry) and counts it; stage 4 then
// passes over the
// marked particles only (it returns at once when none is marked), with every
// distance inside h going through a per-lane heap of the CAP largest, merged
// by copy 0.  Both return the same element of the same set, so the result
// does not depend on which one found it.
template <int PREC, bool GROUPED, int P, int KERNEL, int STAGE = 0, int CAP = 64>
__global__ __launch_bounds__(64) void k_solve(SolveArgs a) {
    using KT = Kern<KERNEL>;
    constexpr bool SEL = STAGE == 2 || STAGE == 4;
    constexpr bool SEL_LIST = STAGE == 2;
    using HeapT = typename std::conditional<PREC == SPH_FP64, double, float>::type;
    // per lane: the shell list (stage 2) or the heap (stage 4)
    __shared__ HeapT selheap[SEL ? 64 * CAP : 1];
    // the selection reads four candidates per copy at a time, up to three
    // rounds of S slots past the last full one
    static_assert(!SEL || 64 + 3 * (64 / P) <= kStage, "selection reads past the staging buffer");
    // stage 4 visits only the tiles stage 2 listed
    const int32_t n_retry = STAGE == 4 ? uniform_i(a.queue[kSelRetrySlot]) : 0;
    if (STAGE == 4 && n_retry == 0) return;
    constexpr int S = 64 / P;
    __shared__ double act_t[3][P];
    __shared__ double act_H[P];
    // candidate ranges of the current cell batch: (sorted slot minus the
    // range's first stream position, image code) and the stream positions at
    // which ranges start; rg_mark maps a load round's slots to range starts
    __shared__ int2 rg_so[64];
    __shared__ int32_t rg_mark[64];
    __shared__ CandLDS<PREC> cd;
    __shared__ float4 regbox[2];  // FP32C region of the current sub-tile
    __shared__ double4 regbox_d[1];  // FP64 region: the box centre
    // Per particle of the tile, in LDS rather than registers (the kernel
    // stays within 128 VGPRs): its position (FP64: x, y, z; FP32C: grid cell
    // and fraction), the h iteration's bracket and counters while a pass runs
    // (only h is needed there), and the pass's sums
    __shared__ double4 own_x[PREC == SPH_FP64 ? P : 1];
    __shared__ int4 own_q[PREC == SPH_FP32C ? P : 1];
    __shared__ float4 own_f[PREC == SPH_FP32C ? P : 1];
    __shared__ double park_d[4][P];
    __shared__ int32_t park_i[4][P];
    __shared__ double acc_d[3][P];
    __shared__ int32_t acc_n[P];

    const int l = threadIdx.x;
    const int p = l & (P - 1);   // particle slot in the tile
    const int kk = l / P;        // copy index of this lane
    const int B = a.bits;
    // selection shell: r^2 > sel_g h^2 is the outer volume fraction sel_f of
    // the sphere (sel_g < 0: the whole sphere)
    const double sel_f = SEL ? (CAP + 8.0) / a.Nt : 1.0;
    const double sel_g = sel_f < 1.0 ? cbrt((1.0 - sel_f) * (1.0 - sel_f)) : -1.0;
    constexpr uint64_t kTileMask = P == 64 ? ~0ull : ((1ull << P) - 1ull);
    uint64_t cnt_pairs = 0, cnt_cands = 0, cnt_passes = 0, cnt_region = 0;  // wave totals

    for (;;) {
        int item = 0;
        if (l == 0) item = atomicAdd(a.queue, 1);
        item = uniform_i(__shfl(item, 0, 64));
        const int64_t n_items = STAGE == 4 ? (int64_t)n_retry
                                : GROUPED ? (int64_t)a.gitems[a.G] : a.n_items;
        if (item >= n_items) break;
        if (STAGE == 4) item = uniform_i(a.knn_items[item]);

        int64_t b, e;
        int32_t g = 0;
        double org0 = 0.0, org1 = 0.0, org2 = 0.0, sc;
        if (!GROUPED) {
            b = (int64_t)item * a.seg;
            e = b + a.seg < a.n ? b + a.seg : a.n;
            sc = 2097152.0 / a.box;
        } else {
            int32_t lo = 0, hi = a.G - 1;
            while (lo < hi) {
                const int32_t mid = (lo + hi + 1) >> 1;
                if (a.gitems[mid] <= item) lo = mid; else hi = mid - 1;
            }
            g = a.gorder[lo];  // position lo of the largest-first order
            b = a.goff[g] + (int64_t)(item - a.gitems[lo]) * a.seg;
            e = b + a.seg < a.goff[g + 1] ? b + a.seg : a.goff[g + 1];
            const double *f = a.frame + 8 * (int64_t)g;
            org0 = uniform_d(f[0]); org1 = uniform_d(f[1]); org2 = uniform_d(f[2]);
            sc = uniform_d(f[6]);
        }
        const double hmax = GROUPED ? INFINITY : 0.5 * a.box * (1.0 - 0x1p-20);

        const int64_t s = b + p;
        const bool mine = s < e;
        // this lane's particle
        HState hs;
        hs.h = mine ? (SEL ? a.knn_h[s] : a.sh0[s]) : 1.0;
        hs.lo = 0.0;
        hs.hi = INFINITY;
        hs.it = 0;
        hs.flags = 0;
        hs.nlo = hs.nhi = 0;
        hs.wprev = INFINITY;
        hs.fixed = a.max_iter == 0 || STAGE >= 2;
        // exact-K stages 2 and 3 carry the count stage's status
        int32_t st_in = (STAGE >= 2 && mine) ? a.knn_st[s] : 0;
        // stage 4: particles stage 2 settled are left as they are
        const bool skip = STAGE == 4 && (st_in & kSelRetry) == 0;
        st_in &= ~kSelRetry;
        if (STAGE == 3) {
            hs.flags = st_in & ~0xFFFF;
            hs.it = st_in & 0xFFFF;
        }
        int sel_n = 0, sel_hc = 0;  // selection: in-range count, heap size
        HeapT sel_min = 0;          // selection: the heap's root
        int sel_cnt = 0;            // selection: shell members met (list length)
        bool valid = false;
        if (mine) {
            if (PREC == SPH_FP64) {
                const double4 p4 = a.sp[s];
                if (kk == 0) own_x[p] = p4;
                valid = !isnan(p4.x);
            } else {
                const int4 q4 = a.qp[s];
                const float4 f4 = a.fp[s];
                if (kk == 0) {
                    own_q[p] = q4;
                    own_f[p] = f4;
                }
                valid = !isnan(f4.x);
            }
        }
        // grid-unit position (culling), recomputed where needed
        auto grid_pos = [&](double &tx, double &ty, double &tz) {
            if (PREC == SPH_FP64) {
                const double4 o4 = own_x[p];
                tx = (o4.x - org0) * sc; ty = (o4.y - org1) * sc; tz = (o4.z - org2) * sc;
            } else {
                const int4 q4 = own_q[p];
                const float4 f4 = own_f[p];
                tx = (double)q4.x + (double)f4.x;
                ty = (double)q4.y + (double)f4.y;
                tz = (double)q4.z + (double)f4.z;
            }
        };
        if (mine && !valid && kk == 0 && STAGE != 4) {
            if (SEL) a.sh_out[s] = hs.h;
            else write_out(a, a.perm[s], NAN, hs.h, NAN, 0, SPH_ST_BADINPUT);
            if (STAGE == 1) { a.knn_h[s] = hs.h; a.knn_st[s] = SPH_ST_BADINPUT; }
        }
        if (GROUPED && mine && valid && STAGE <= 1) {
            const double ng = (double)(a.goff[g + 1] - a.goff[g]);
            if (STAGE == 1 ? ng < a.Nt : KT::count * ng < a.Nt - a.dN) {
                hs.flags |= SPH_ST_UNREACHABLE;
                hs.fixed = true;
            }
        }
        if (hs.h > hmax) hs.h = hmax;
        bool done = !(mine && valid) || skip;
        if (SEL && !done && (st_in >> 16) != 0) {
            // flagged by the count stage: h passes through unchanged
            a.sh_out[s] = hs.h;
            done = true;
        }

        for (;;) {
            // active particles (bits 0..P-1: the lanes of copy 0)
            const uint64_t am = __ballot(!done) & kTileMask;
            if (am == 0) break;
            const double hq = hs.h * sc;  // h in grid units
            const double Hs = hq * (1.0 + 0x1p-20) + 0x1p-20;
            if (kk == 0) {
                double tx, ty, tz;
                grid_pos(tx, ty, tz);
                act_t[0][p] = tx;
                act_t[1][p] = ty;
                act_t[2][p] = tz;
                act_H[p] = done ? -1.0 : Hs;
            }
            uint64_t pass_cands = 0;   // wave total: candidates tested x particles
            uint64_t pass_region = 0;  // wave total: candidates tested against a region
            if (kk == 0) {
                park_d[0][p] = hs.lo; park_d[1][p] = hs.hi; park_d[2][p] = hs.wprev;
                park_d[3][p] = hs.h;
                park_i[0][p] = hs.it; park_i[1][p] = hs.flags;
                park_i[2][p] = hs.nlo; park_i[3][p] = hs.nhi;
                acc_d[0][p] = 0.0; acc_d[1][p] = 0.0; acc_d[2][p] = 0.0;
                acc_n[p] = 0;
            }
            __syncthreads();

            // sub-tiles: lane ranges [la, lb) of the active set, split in halves
            // depth first.  The pending ranges always tile [la, P) in order, so
            // the stack is the bit set of their first lanes.
            uint64_t starts = 1;
            while (starts) {
                const int la = __builtin_ctzll(starts);
                starts &= starts - 1;
                const int lb = starts ? __builtin_ctzll(starts) : P;
                const uint64_t rmask = (lb == 64 ? ~0ull : ((1ull << lb) - 1ull)) &
                                       ~((1ull << la) - 1ull);
                const uint64_t sub = am & rmask;
                if (sub == 0) continue;
                const bool in_sub = ((sub >> p) & 1ull) != 0;
                double tx, ty, tz;
                grid_pos(tx, ty, tz);
                const double mn0 = uniform_d(wave_min(in_sub ? tx : INFINITY));
                const double mn1 = uniform_d(wave_min(in_sub ? ty : INFINITY));
                const double mn2 = uniform_d(wave_min(in_sub ? tz : INFINITY));
                const double mx0 = uniform_d(wave_max(in_sub ? tx : -INFINITY));
                const double mx1 = uniform_d(wave_max(in_sub ? ty : -INFINITY));
                const double mx2 = uniform_d(wave_max(in_sub ? tz : -INFINITY));
                const double Hm = uniform_d(wave_max(in_sub ? Hs : 0.0));
                int ex = ceil_log2_pos(ldexp(Hm, a.cell_exp));
                int L = B - ex;
                const int Lmin = GROUPED ? 0 : 1;
                if (L < Lmin) { L = Lmin; ex = B - L; }
                const double side = ldexp(1.0, ex);
                const double inv = ldexp(1.0, -ex);
                // cell coordinates stay within [-2^22, 2^23): 32 bits suffice
                int32_t clo0 = (int32_t)floor((mn0 - Hm) * inv), chi0 = (int32_t)floor((mx0 + Hm) * inv);
                int32_t clo1 = (int32_t)floor((mn1 - Hm) * inv), chi1 = (int32_t)floor((mx1 + Hm) * inv);
                int32_t clo2 = (int32_t)floor((mn2 - Hm) * inv), chi2 = (int32_t)floor((mx2 + Hm) * inv);
                const int32_t ncell = (int32_t)1 << L;
                if (GROUPED) {
                    clo0 = clo0 < 0 ? 0 : clo0; clo1 = clo1 < 0 ? 0 : clo1; clo2 = clo2 < 0 ? 0 : clo2;
                    chi0 = chi0 >= ncell ? ncell - 1 : chi0;
                    chi1 = chi1 >= ncell ? ncell - 1 : chi1;
                    chi2 = chi2 >= ncell ? ncell - 1 : chi2;
                }
                const int32_t nx = chi0 - clo0 + 1, ny = chi1 - clo1 + 1, nz = chi2 - clo2 + 1;
                if (nx <= 0 || ny <= 0 || nz <= 0) continue;
                const int64_t K = (int64_t)nx * ny * nz;
                if (K > kMaxRegionCells && __popcll(sub) > 1) {
                    // split the active lanes of this range into two halves
                    int cnt = __popcll(sub) / 2;
                    uint64_t t = sub;
                    for (int k = 0; k < cnt; ++k) t &= t - 1;  // drop the lowest cnt lanes
                    const int mid = __ffsll((unsigned long long)t) - 1;
                    starts |= (1ull << la) | (1ull << mid);
                    continue;
                }
                // FP32C origin: the grid point at the centre of the sub-tile's box, so
                // that the binary32 coordinates of the region are as small as they can be
                const int32_t o0 = (int32_t)floor(0.5 * (mn0 + mx0));
                const int32_t o1 = (int32_t)floor(0.5 * (mn1 + mx1));
                const int32_t o2 = (int32_t)floor(0.5 * (mn2 + mx2));
                // lanes of the sub-tile: its A particles get all 64 lanes, Sp
                // copies each (Pp = A rounded up to a power of two particle
                // slots; lane l serves slot l mod Pp, copy l / Pp), so lanes
                // of converged particles or of other sub-tiles never idle.
                // The selection stage keeps the tile's own mapping (its heaps
                // are per lane).
                const int A = __popcll(sub);
                int lgPp = 0;
                while ((1 << lgPp) < A) ++lgPp;
                if (SEL) lgPp = __builtin_ctz(P);
                const int Pp = 1 << lgPp, Sp = 64 >> lgPp;
                if (!SEL && kk == 0 && in_sub)
                    rg_mark[__popcll(sub & ((1ull << p) - 1ull))] = p;  // slot of own particle
                __builtin_amdgcn_wave_barrier();
                const int slot = l & (Pp - 1);
                const int kk2 = l >> lgPp;
                const bool in2 = SEL ? in_sub : slot < A;
                const int pv = SEL ? p : (in2 ? rg_mark[slot] : p);
                // the served particle's h and position (its copy-0 lane holds them)
                const double h_l = park_d[3][pv];
                const double hq_l = h_l * sc;
                const double h2 = h_l * h_l;
                const float ih2 = (float)(1.0 / (hq_l * hq_l));
                const float h2f = (float)(hq_l * hq_l);
                double x2 = 0.0, y2 = 0.0, z2 = 0.0;
                float pix = 0.f, piy = 0.f, piz = 0.f;
                if (PREC == SPH_FP64) {
                    const double4 o4 = own_x[pv];
                    x2 = o4.x; y2 = o4.y; z2 = o4.z;
                } else {
                    const int4 q4 = own_q[pv];
                    const float4 f4 = own_f[pv];
                    pix = (float)(q4.x - o0) + f4.x;
                    piy = (float)(q4.y - o1) + f4.y;
                    piz = (float)(q4.z - o2) + f4.z;
                }
                Sums sm;
                sm.d0 = sm.d1 = sm.dr = 0.0;
                sm.f0 = sm.f1 = sm.fr = sm.c0 = sm.c1 = sm.cr = 0.f;
                sm.n = 0;
                float pa0 = 0.f, pa1 = 0.f, par = 0.f;  // FP32C plain partial sums
                int pterms = 0;                         // terms per lane since the last fold

                // region of the sub-tile: its particles' bounding box (exactly
                // the coordinates its pair tests use) widened by Hm.  A
                // candidate farther than that from the box is out of every
                // sphere: the margin 2^-16 of Hm^2 on top of Hm's own covers
                // the rounding of both tests
                const int nsub = __popcll(sub);
                // (kept in LDS: the scalar registers are taken by the cell
                // enumeration, and these are read once per load round)
                if (PREC == SPH_FP64) {
                    const double a0 = wave_min(in2 ? x2 : INFINITY);
                    const double a1 = wave_min(in2 ? y2 : INFINITY);
                    const double a2 = wave_min(in2 ? z2 : INFINITY);
                    const double b0 = wave_max(in2 ? x2 : -INFINITY);
                    const double b1 = wave_max(in2 ? y2 : -INFINITY);
                    const double b2 = wave_max(in2 ? z2 : -INFINITY);
                    // tested in binary32 relative to the box centre: the
                    // half-extents rounded up and a relative margin of 2^-8 on
                    // Hm^2 cover the binary32 rounding of the offsets (at most
                    // 2^-24 of an offset no larger than ~600 Hm within the
                    // split limit on the region's cells)
                    const double Ha = Hm / sc;
                    if (l == 0) {
                        regbox_d[0] = make_double4(0.5 * (a0 + b0), 0.5 * (a1 + b1), 0.5 * (a2 + b2), 0.0);
                        regbox[0] = make_float4((float)(0.5 * (b0 - a0) * (1.0 + 0x1p-20)),
                                                (float)(0.5 * (b1 - a1) * (1.0 + 0x1p-20)),
                                                (float)(0.5 * (b2 - a2) * (1.0 + 0x1p-20)),
                                                (float)(Ha * Ha * (1.0 + 0x1p-8)));
                    }
                } else {
                    const float a0 = wave_min(in2 ? pix : INFINITY);
                    const float a1 = wave_min(in2 ? piy : INFINITY);
                    const float a2 = wave_min(in2 ? piz : INFINITY);
                    const float b0 = wave_max(in2 ? pix : -INFINITY);
                    const float b1 = wave_max(in2 ? piy : -INFINITY);
                    const float b2 = wave_max(in2 ? piz : -INFINITY);
                    if (l == 0) {
                        regbox[0] = make_float4(a0, a1, a2, (float)(Hm * Hm * (1.0 + 0x1p-16)));
                        regbox[1] = make_float4(b0, b1, b2, 0.f);
                    }
                }
                int staged = 0;  // candidates in the staging buffer (wave-uniform)

                // one test round: every particle of the sub-tile against the
                // first mc staged candidates (mc <= 64; slots mc..63 padded)
                auto test_round = [&](const int mc) {
                        // candidates per copy: the slots past mc hold padding, and
                        // ceil(mc / Sp) * Sp <= 64 (Sp divides 64)
                        const int nu = (mc + Sp - 1) >> (6 - lgPp);
                        if (PREC == SPH_FP32C && pterms + nu > 64) {
                            kahan(sm.f0, sm.c0, pa0);
                            kahan(sm.f1, sm.c1, pa1);
                            kahan(sm.fr, sm.cr, par);
                            pa0 = pa1 = par = 0.f;
                            pterms = 0;
                        }
                        pterms += nu;
                        if (SEL && in_sub) {
                            // selection: squared distances inside h into the
                            // shell list (first pass) or the heap (second)
                            // (the shell test in binary32: rounding is monotone,
                            // so the shell stays a top set of the distances)
                            auto scan = [&](auto heap) {
                                auto keep = [&](HeapT r2, float tau2) {
                                    if (heap) {
                                        sel_insert<CAP>(selheap, l, sel_hc, r2, sel_min);
                                    } else if ((float)r2 > tau2) {
                                        if (sel_cnt < CAP) {
                                            selheap[sel_cnt * 64 + l] = r2;
                                            sel_min = sel_cnt == 0 || r2 < sel_min ? r2 : sel_min;
                                            ++sel_cnt;
                                        } else if (r2 > sel_min) {
                                            // a full list keeps the CAP largest
                                            // met: the new one replaces (one copy
                                            // of) its minimum
                                            bool put = false;
                                            HeapT nm = r2;
#pragma unroll 1
                                            for (int i = 0; i < CAP; ++i) {
                                                const HeapT w = selheap[i * 64 + l];
                                                if (!put && w == sel_min) {
                                                    selheap[i * 64 + l] = r2;
                                                    put = true;
                                                } else {
                                                    nm = w < nm ? w : nm;
                                                }
                                            }
                                            sel_min = nm;
                                            ++sel_cnt;
                                        }
                                    }
                                };
                                // four candidates per copy at a time: their
                                // LDS reads and distances issue together, the
                                // list or heap work follows (slot u * S + kk of
                                // the round; slots past mc hold padding, and
                                // the reads stay inside the 128-slot buffer)
                                if (PREC == SPH_FP64) {
                                    auto &c = reinterpret_cast<CandLDS<SPH_FP64> &>(cd);
                                    const float tau2 = (float)(h2 * sel_g);
                                    for (int u0 = 0; u0 < nu; u0 += 4) {
                                        HeapT v[4];
                                        bool in[4];
#pragma unroll
                                        for (int q = 0; q < 4; ++q) {
                                            const int t = (u0 + q) * S + kk;
                                            const double dx = (c.x[t] - x2) + c.shx[t];
                                            const double dy = (c.y[t] - y2) + c.shy[t];
                                            const double dz = (c.z[t] - z2) + c.shz[t];
                                            const double r2 = (dx * dx + dy * dy) + dz * dz;
                                            in[q] = r2 < h2 && u0 + q < nu;
                                            v[q] = (HeapT)r2;
                                        }
#pragma unroll
                                        for (int q = 0; q < 4; ++q)
                                            if (in[q]) {
                                                ++sel_n;
                                                keep(v[q], tau2);
                                            }
                                    }
                                } else {
                                    // binary32 coordinates, differences and squares
                                    // (grid units), as in the count stage but about
                                    // another origin.  The sphere is widened by a
                                    // relative 2^-18 so that it holds every particle
                                    // the count stage's test counted inside h (each
                                    // test's rounding stays below 2^-21 of r^2): the
                                    // list then holds at least K
                                    auto &c = reinterpret_cast<CandLDS<SPH_FP32C> &>(cd);
                                    const float hq2 = (float)(hq_l * hq_l * (1.0 + 0x1p-18));
                                    const float tau2 = (float)(hq_l * hq_l * sel_g);
                                    for (int u0 = 0; u0 < nu; u0 += 4) {
                                        HeapT v[4];
                                        bool in[4];
#pragma unroll
                                        for (int q = 0; q < 4; ++q) {
                                            const float4 cj = c.c[(u0 + q) * S + kk];
                                            const float dx = cj.x - pix;
                                            const float dy = cj.y - piy;
                                            const float dz = cj.z - piz;
                                            const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
                                            in[q] = r2 < hq2 && u0 + q < nu;
                                            v[q] = r2;
                                        }
#pragma unroll
                                        for (int q = 0; q < 4; ++q)
                                            if (in[q]) {
                                                ++sel_n;
                                                keep(v[q], tau2);
                                            }
                                    }
                                }
                            };
                            scan(std::integral_constant<bool, !SEL_LIST>{});
                        } else if (in2) {
                            // binary32: branch free.  With one particle-candidate
                            // pair per lane a wave almost always holds an in-range
                            // pair, so a branch would not skip the pair terms, only
                            // keep the compiler from issuing the unrolled LDS reads
                            // together.  An out-of-range pair is evaluated at q = 1,
                            // where every term is exactly zero; staged candidates
                            // have finite masses (invalid particles never pass the
                            // region test), so it adds exact zeros
                            if (PREC == SPH_FP64) {
                                // binary64 keeps the branch: its pair terms (a
                                // binary64 square root among them) need more
                                // registers than a branch-free unrolled loop leaves
                                auto &c = reinterpret_cast<CandLDS<SPH_FP64> &>(cd);
                                const double hinv = 1.0 / h_l;
#pragma unroll 4
                                for (int u = 0; u < nu; ++u) {
                                    const int t = u * Sp + kk2;
                                    const double dx = (c.x[t] - x2) + c.shx[t];
                                    const double dy = (c.y[t] - y2) + c.shy[t];
                                    const double dz = (c.z[t] - z2) + c.shz[t];
                                    const double r2 = (dx * dx + dy * dy) + dz * dz;
                                    if (r2 < h2) {
                                        // the exact-K count stage needs the count only
                                        if (STAGE != 1) {
                                            // scaled pair terms (factors applied to the totals)
                                            const double q = sqrt_pos(r2) * hinv;
                                            double fh, gs;
                                            KT::template terms<double>(q, q * q, fh, gs);
                                            sm.d0 += fh;
                                            sm.d1 += gs;
                                            sm.dr += c.m[t] * fh;
                                        }
                                        sm.n += 1;
                                    }
                                }
                            } else {
                                auto &c = reinterpret_cast<CandLDS<SPH_FP32C> &>(cd);
                                // cascade summation: up to 64 terms per lane in plain
                                // binary32, then Kahan-compensated into the totals.
                                // The stride between a copy's candidates is Sp; when
                                // the sub-tile fills the tile it is the constant S,
                                // and the LDS offsets become immediates
                                auto eval32 = [&](auto stride) {
#pragma unroll 4
                                    for (int u = 0; u < nu; ++u) {
                                        const float4 cj = c.c[u * stride + kk2];
                                        const float dx = cj.x - pix;
                                        const float dy = cj.y - piy;
                                        const float dz = cj.z - piz;
                                        const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
                                        const bool in = r2 < h2f;
                                        if (STAGE != 1) {
                                            // scaled pair terms (factors applied to the
                                            // totals), q^2 clamped to 1: out of range, or
                                            // within rounding of the edge, every term is 0
                                            const float q2 = __builtin_fminf(__builtin_fmaxf(r2 * ih2, 0.0f), 1.0f);
                                            const float q = __builtin_amdgcn_sqrtf(q2);  // 1 ulp
                                            KT::accum(q, q2, cj.w, pa0, pa1, par);
                                        }
                                        sm.n += in ? 1 : 0;
                                    }
                                };
                                if (Sp == S) eval32(std::integral_constant<int, S>{});
                                else eval32(Sp);
                            }
                        }
                };

                for (int64_t kb = 0; kb < K; kb += 64) {
                    const int64_t k = kb + l;
                    bool pass = false;
                    int32_t c_st = 0, c_en = 0, code = 0;
                    if (k < K) {
                        const int32_t kq = (int32_t)k;
                        const int32_t c0 = clo0 + kq % nx;
                        const int32_t c1 = clo1 + (kq / nx) % ny;
                        const int32_t c2 = clo2 + kq / (nx * ny);
                        const double lo0 = (double)c0 * side - 0x1p-20, hi0 = (double)(c0 + 1) * side + 0x1p-20;
                        const double lo1 = (double)c1 * side - 0x1p-20, hi1 = (double)(c1 + 1) * side + 0x1p-20;
                        const double lo2 = (double)c2 * side - 0x1p-20, hi2 = (double)(c2 + 1) * side + 0x1p-20;
                        uint64_t it = sub;
                        while (it) {
                            const int q = __ffsll((unsigned long long)it) - 1;
                            it &= it - 1;
                            const double p0 = act_t[0][q], p1 = act_t[1][q], p2 = act_t[2][q];
                            const double H = act_H[q];
                            const double g0 = fmax(0.0, fmax(lo0 - p0, p0 - hi0));
                            const double g1 = fmax(0.0, fmax(lo1 - p1, p1 - hi1));
                            const double g2 = fmax(0.0, fmax(lo2 - p2, p2 - hi2));
                            if (g0 * g0 + g1 * g1 + g2 * g2 <= H * H) { pass = true; break; }
                        }
                        if (pass) {
                            int64_t w0 = c0, w1 = c1, w2 = c2;
                            int s0 = 0, s1 = 0, s2 = 0;
                            if (!GROUPED) {
                                s0 = (int)(c0 >> L); s1 = (int)(c1 >> L); s2 = (int)(c2 >> L);
                                w0 = c0 & (ncell - 1); w1 = c1 & (ncell - 1); w2 = c2 & (ncell - 1);
                            }
                            const uint64_t cm = morton3((uint64_t)w0, (uint64_t)w1, (uint64_t)w2);
                            if (!GROUPED) cell_range_periodic(a, cm, L, c_st, c_en);
                            else cell_range_group(a, g, cm, L, c_st, c_en);
                            code = (s0 + 1) | ((s1 + 1) << 2) | ((s2 + 1) << 4);
                            pass = c_en > c_st;
                        }
                    }
                    const uint64_t pm = __ballot(pass);
                    if (pm == 0) continue;
                    const int cnt = pass ? c_en - c_st : 0;
                    const int incl = wave_incl_scan(cnt);
                    const int total = __builtin_amdgcn_readlane(incl, 63);
                    const int nr = __popcll(pm);
                    __syncthreads();
                    if (pass) {
                        const int slot = (int)mbcnt(pm);
                        rg_so[slot] = make_int2(c_st - (incl - cnt), code);
                        rg_mark[slot] = l;  // the lane that found range `slot`
                    }
                    __syncthreads();
                    // stream position at which range l starts (past the end for l >= nr)
                    const int rsrc = l < nr ? rg_mark[l] : 0;
                    const int rstart0 = __shfl(incl - cnt, rsrc, 64);
                    const int rstart = l < nr ? rstart0 : INT_MAX;
                    int rcarry = 0;  // range of the stream position before the round
                    for (int cbase = 0; cbase < total; cbase += 64) {
                        // load round: each lane takes one candidate of the
                        // region's cells and keeps it if it lies within Hm of
                        // the sub-tile's bounding box; the kept ones are
                        // appended to the staging buffer (ballot slots)
                        const int gidx = cbase + l;
                        // range of each slot: the ranges starting inside the round
                        // mark their first slot, a wave max-scan carries each mark
                        // forward, and slots before the first mark keep the range
                        // running at the end of the previous round
                        rg_mark[l] = -1;
                        const int pos = rstart - cbase;
                        if (pos >= 0 && pos < 64) rg_mark[pos] = l;
                        __builtin_amdgcn_wave_barrier();
                        int rr = wave_max_scan(rg_mark[l]);
                        rr = rr > rcarry ? rr : rcarry;
                        rcarry = __builtin_amdgcn_readlane(rr, 63);
                        bool keep = false;
                        float4 cf = make_float4(0.f, 0.f, 0.f, 0.f);
                        double4 cdv = make_double4(0.0, 0.0, 0.0, 0.0);
                        double csx = 0.0, csy = 0.0, csz = 0.0;
                        if (gidx < total) {
                            const int2 so = rg_so[rr];
                            const int64_t j = (int64_t)(so.x + gidx);
                            const int cc = so.y;
                            const int sh0 = (cc & 3) - 1, sh1 = ((cc >> 2) & 3) - 1,
                                      sh2 = ((cc >> 4) & 3) - 1;
                            if (PREC == SPH_FP64) {
                                cdv = a.sp[j];
                                csx = (double)sh0 * a.box;
                                csy = (double)sh1 * a.box;
                                csz = (double)sh2 * a.box;
                                const double4 rc = regbox_d[0];
                                const float4 rh = regbox[0];
                                const float ex = __builtin_fmaxf(__builtin_fabsf((float)((cdv.x + csx) - rc.x)) - rh.x, 0.0f);
                                const float ey = __builtin_fmaxf(__builtin_fabsf((float)((cdv.y + csy) - rc.y)) - rh.y, 0.0f);
                                const float ez = __builtin_fmaxf(__builtin_fabsf((float)((cdv.z + csz) - rc.z)) - rh.z, 0.0f);
                                keep = __builtin_fmaf(ex, ex, __builtin_fmaf(ey, ey, ez * ez)) <= rh.w;
                            } else {
                                const int32_t W = 1 << B;
                                const int4 q4 = a.qp[j];
                                const float4 f4 = a.fp[j];
                                cf = make_float4((float)(q4.x + sh0 * W - o0) + f4.x,
                                                 (float)(q4.y + sh1 * W - o1) + f4.y,
                                                 (float)(q4.z + sh2 * W - o2) + f4.z,
                                                 __int_as_float(q4.w));
                                const float4 rl = regbox[0], rh = regbox[1];
                                const float ex = cf.x - fminf(fmaxf(cf.x, rl.x), rh.x);
                                const float ey = cf.y - fminf(fmaxf(cf.y, rl.y), rh.y);
                                const float ez = cf.z - fminf(fmaxf(cf.z, rl.z), rh.z);
                                keep = __builtin_fmaf(ex, ex, __builtin_fmaf(ey, ey, ez * ez)) <= rl.w;
                            }
                        }
                        const uint64_t km = __ballot(keep);
                        const int nk = __popcll(km);
                        if (keep) {
                            const int slot = staged + (int)mbcnt(km);
                            if (PREC == SPH_FP64) {
                                auto &c = reinterpret_cast<CandLDS<SPH_FP64> &>(cd);
                                c.x[slot] = cdv.x; c.y[slot] = cdv.y; c.z[slot] = cdv.z;
                                c.m[slot] = cdv.w;
                                c.shx[slot] = csx; c.shy[slot] = csy; c.shz[slot] = csz;
                            } else {
                                auto &c = reinterpret_cast<CandLDS<SPH_FP32C> &>(cd);
                                c.c[slot] = cf;
                            }
                        }
                        staged += nk;
                        pass_cands += (uint64_t)nk * (uint64_t)nsub;
                        pass_region += (uint64_t)(total - cbase < 64 ? total - cbase : 64);
                        if (staged >= 64) {
                            __syncthreads();
                            test_round(64);
                            __syncthreads();
                            // the entries past the round move to the front
                            if (l < staged - 64) {
                                if (PREC == SPH_FP64) {
                                    auto &c = reinterpret_cast<CandLDS<SPH_FP64> &>(cd);
                                    const double t0 = c.x[64 + l], t1 = c.y[64 + l], t2 = c.z[64 + l];
                                    const double t3 = c.m[64 + l], t4 = c.shx[64 + l];
                                    const double t5 = c.shy[64 + l], t6 = c.shz[64 + l];
                                    c.x[l] = t0; c.y[l] = t1; c.z[l] = t2; c.m[l] = t3;
                                    c.shx[l] = t4; c.shy[l] = t5; c.shz[l] = t6;
                                } else {
                                    auto &c = reinterpret_cast<CandLDS<SPH_FP32C> &>(cd);
                                    const float4 t = c.c[64 + l];
                                    c.c[l] = t;
                                }
                            }
                            staged -= 64;
                            __syncthreads();
                        }
                    }
                }
                // the sub-tile's last, partial round (its origin and lanes are
                // its own): slots past the staged candidates hold padding, a
                // candidate at infinite distance that is never in range
                if (staged > 0) {
                    if (l >= staged) {
                        if (PREC == SPH_FP64) {
                            auto &c = reinterpret_cast<CandLDS<SPH_FP64> &>(cd);
                            c.x[l] = INFINITY; c.y[l] = INFINITY; c.z[l] = INFINITY;
                            c.m[l] = 0.0;
                            c.shx[l] = 0.0; c.shy[l] = 0.0; c.shz[l] = 0.0;
                        } else {
                            auto &c = reinterpret_cast<CandLDS<SPH_FP32C> &>(cd);
                            c.c[l] = make_float4(INFINITY, INFINITY, INFINITY, 0.f);
                        }
                    }
                    __syncthreads();
                    test_round(staged);
                    __syncthreads();
                    staged = 0;
                }
                if (!SEL) {
                    // the sub-tile's sums: each served slot's copies combined by a
                    // butterfly of commutative adds (every copy ends with the same
                    // bits), then moved to the lanes that hold that particle
                    double v0, v1, vr;
                    if (PREC == SPH_FP64) {
                        v0 = sm.d0; v1 = sm.d1; vr = sm.dr;
                    } else {
                        kahan(sm.f0, sm.c0, pa0);
                        kahan(sm.f1, sm.c1, pa1);
                        kahan(sm.fr, sm.cr, par);
                        v0 = (double)sm.f0 - (double)sm.c0;
                        v1 = (double)sm.f1 - (double)sm.c1;
                        vr = (double)sm.fr - (double)sm.cr;
                    }
                    int32_t vn = sm.n;
                    for (int o = Pp; o < 64; o <<= 1) {
                        v0 += __shfl_xor(v0, o, 64);
                        v1 += __shfl_xor(v1, o, 64);
                        vr += __shfl_xor(vr, o, 64);
                        vn += __shfl_xor(vn, o, 64);
                    }
                    if (in2 && kk2 == 0) {
                        acc_d[0][pv] += v0; acc_d[1][pv] += v1; acc_d[2][pv] += vr;
                        acc_n[pv] += vn;
                    }
                }
            }

            __builtin_amdgcn_wave_barrier();
            const double S0 = KT::fscale * acc_d[0][p], S1 = KT::gscale * acc_d[1][p];
            const double R = KT::fscale * acc_d[2][p];
            const int32_t npair = acc_n[p];
            if (a.stats) {
                cnt_pairs += uniform_u64(wave_sum<uint64_t>(!done && kk == 0 ? (uint64_t)npair : 0));
                cnt_cands += pass_cands;
                cnt_region += pass_region;
                cnt_passes += (uint64_t)__popcll(am);
            }
            if (SEL_LIST) {
                // each copy's list holds the CAP largest of its share of the
                // m shell members (all of them when it met no more than CAP).
                // When rank <= m the rank-th largest v of the distances inside
                // h is a shell member, and counting over the union of the
                // lists, v is the one element e with #(> e) < rank <= #(>= e):
                // every member above v is in its copy's CAP largest (fewer
                // than rank <= CAP of them exist), and the lists hold at least
                // min(CAP, #(>= v)) >= rank members >= v.  Each lane checks
                // its own list against the union
                int seln = sel_n;
#pragma unroll
                for (int o = P; o < 64; o <<= 1) seln += __shfl_xor(seln, o, 64);
                // list lengths through LDS (the lane-map words are free now)
                rg_mark[l] = sel_cnt;
                __syncthreads();
                int m = 0;  // shell members met by the copies
#pragma unroll
                for (int k = 0; k < S; ++k) m += rg_mark[p + k * P];
                const int rank = seln - (int)a.Nt + 1;
                const int own = sel_cnt < CAP ? sel_cnt : CAP;
                int found = 0;
                HeapT ans = 0;
                if (!done && rank >= 1 && rank <= CAP && rank <= m) {
                    // four own elements at a time against each union element
                    // (read once per four); counts packed as #(>) + 2^16 #(>=)
#pragma unroll 1
                    for (int i0 = 0; i0 < own; i0 += 4) {
                        HeapT e[4];
                        int cn[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int i = i0 + q < CAP ? i0 + q : CAP - 1;
                            e[q] = selheap[i * 64 + l];
                            cn[q] = 0;
                        }
#pragma unroll 1
                        for (int k = 0; k < S; ++k) {
                            const int ckr = rg_mark[p + k * P];
                            const int ck = ckr < CAP ? ckr : CAP;
                            const HeapT *col = selheap + p + k * P;
#pragma unroll 2
                            for (int j = 0; j < ck; ++j) {
                                const HeapT v = col[j * 64];
#pragma unroll
                                for (int q = 0; q < 4; ++q)
                                    cn[q] += (v > e[q] ? 1 : 0) + (v >= e[q] ? 0x10000 : 0);
                            }
                        }
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int gt = cn[q] & 0xFFFF, ge = cn[q] >> 16;
                            if (i0 + q < own && gt < rank && rank <= ge) { found = 1; ans = e[q]; }
                        }
                    }
                }
                // copy 0 takes the element found by any copy (equal values
                // where several are found)
                HeapT ans0 = ans;
                int found0 = found;
#pragma unroll
                for (int k = 1; k < S; ++k) {
                    const int fk = __shfl(found, p + k * P, 64);
                    const HeapT ak = __shfl(ans, p + k * P, 64);
                    if (fk && !found0) { found0 = 1; ans0 = ak; }
                }
                int retry = 0;
                if (!done && kk == 0) {
                    if (found0) {
                        const double d2 = (double)ans0;
                        a.sh_out[b + p] = PREC == SPH_FP64 ? sqrt(d2) : sqrt(d2) / sc;
                        a.knn_st[b + p] = st_in;
                    } else if (rank < 1 || rank > CAP) {
                        // the count stage's h did not hold K within reach
                        a.sh_out[b + p] = hs.h;
                        a.knn_st[b + p] = st_in | SPH_ST_NOCONV;
                    } else {
                        // shell too thin: stage 4
                        a.knn_st[b + p] = st_in | kSelRetry;
                        retry = 1;
                    }
                }
                if (__ballot(retry != 0) != 0 && l == 0)
                    a.knn_items[atomicAdd(&a.queue[kSelRetrySlot], 1)] = item;
                done = true;
            } else if (SEL) {
                // second pass: each copy kept the CAP largest of its share of
                // the distances inside h; copy 0 takes in the other copies'
                // heaps (the union's CAP largest contain its rank-th largest
                // for any rank <= CAP)
                int seln = sel_n;
                int hco[S > 1 ? S - 1 : 1];
#pragma unroll
                for (int o = P; o < 64; o <<= 1) seln += __shfl_xor(seln, o, 64);
#pragma unroll
                for (int k = 1; k < S; ++k) hco[k - 1] = __shfl(sel_hc, p + k * P, 64);
                __syncthreads();
                if (!done && kk == 0) {
#pragma unroll
                    for (int k = 1; k < S; ++k) {
                        const int lo = p + k * P;
                        for (int i = 0; i < hco[k - 1]; ++i)
                            sel_insert<CAP>(selheap, l, sel_hc, selheap[i * 64 + lo], sel_min);
                    }
                    // the K-th smallest of the seln distances inside h is the
                    // (seln - K + 1)-th largest: pop the heap down to that rank
                    const int rank = seln - (int)a.Nt + 1;
                    double hk = hs.h;
                    int32_t stt = st_in;
                    if (rank >= 1 && rank <= sel_hc) {
                        while (sel_hc > rank) sel_pop(selheap, l, sel_hc);
                        const double d2 = (double)selheap[l];
                        hk = PREC == SPH_FP64 ? sqrt(d2) : sqrt(d2) / sc;
                    } else {
                        stt |= SPH_ST_NOCONV;  // the count stage's h did not hold K
                    }
                    a.sh_out[b + p] = hk;
                    a.knn_st[b + p] = stt;
                }
                done = true;
            }
            hs.lo = park_d[0][p]; hs.hi = park_d[1][p]; hs.wprev = park_d[2][p];
            hs.h = park_d[3][p];
            hs.it = park_i[0][p]; hs.flags = park_i[1][p];
            hs.nlo = park_i[2][p]; hs.nhi = park_i[3][p];
            if (!SEL && !done) {
                const double nwv = KT::count * S0;
                const double dndh = -KT::count * S1 / hs.h;
                const double hcur = hs.h;
                if (h_step<STAGE == 1>(hs, nwv, dndh, npair, a, hmax)) {
                    const double rho = KT::sigma * R / (hcur * hcur * hcur);
                    const int32_t stout = hs.flags | (hs.it & 0xFFFF);
                    if (kk == 0) {
                        // The FP32C exact-K count stage writes no outputs (the
                        // evaluation stage writes every particle's), which
                        // brings it to 4 waves per SIMD (5.5 -> 5.2 ms at
                        // K = 295); the binary64 one measured slower at 4
                        // waves than at 3 (9.8 against 8.7 ms) and keeps them
                        if (STAGE != 1 || PREC == SPH_FP64)
                            write_out(a, a.perm[b + p], rho, hcur, nwv, npair, stout);
                        if (STAGE == 1) {
                            // hs.h differs from hcur only where the count
                            // stage hands its upper bracket to the selection
                            a.knn_h[b + p] = hs.h;
                            a.knn_st[b + p] = stout;
                        }
                    }
                    done = true;
                }
            }
        }
    }
    if (a.stats && l == 0) {
        atomicAdd((unsigned long long *)&a.stats[0], (unsigned long long)cnt_pairs);
        atomicAdd((unsigned long long *)&a.stats[1], (unsigned long long)cnt_cands);
        atomicAdd((unsigned long long *)&a.stats[2], (unsigned long long)cnt_passes);
        atomicAdd((unsigned long long *)&a.stats[3], (unsigned long long)cnt_region);
    }
}

// One launch of the density kernel with the arguments in `a`; the grid and
// tile size come from the plan (`seg` particles per work item); `stage` as the
// kernel's STAGE.
template <int STAGE>
static void launch_stage(const Plan &pl, const SolveArgs &a, int P, const dim3 grid,
                         hipStream_t st) {
    const dim3 block(64);
    const bool f32c = pl.prm.precision == SPH_FP32C;
    const bool wc6 = pl.prm.kernel == SPH_KERNEL_WENDLAND_C6;
#define SPH_LAUNCH_K(PR, GR, PP, KK) \
    hipLaunchKernelGGL((k_solve<PR, GR, PP, KK, STAGE>), grid, block, 0, st, a)
#define SPH_LAUNCH(PR, GR, PP)                                             \
    do {                                                                  \
        if (wc6) SPH_LAUNCH_K(PR, GR, PP, SPH_KERNEL_WENDLAND_C6);        \
        else SPH_LAUNCH_K(PR, GR, PP, SPH_KERNEL_M4);                     \
    } while (0)
#define SPH_LAUNCH_P(PR, GR)                                   \
    do {                                                      \
        if (P == 8) SPH_LAUNCH(PR, GR, 8);                    \
        else if (P == 16) SPH_LAUNCH(PR, GR, 16);             \
        else if (P == 32) SPH_LAUNCH(PR, GR, 32);             \
        else SPH_LAUNCH(PR, GR, 64);                          \
    } while (0)
    if (!pl.grouped) {
        if (f32c) SPH_LAUNCH_P(SPH_FP32C, false);
        else SPH_LAUNCH_P(SPH_FP64, false);
    } else {
        if (f32c) SPH_LAUNCH_P(SPH_FP32C, true);
        else SPH_LAUNCH_P(SPH_FP64, true);
    }
#undef SPH_LAUNCH_P
#undef SPH_LAUNCH
#undef SPH_LAUNCH_K
}

static hipError_t launch_solve(const Plan &pl, SolveArgs &a, int seg, int64_t grid_n, int stage,
                               hipStream_t st) {
    hipError_t e = run_zero_i32(pl.ctrl, 4, st);
    if (e != hipSuccess) return e;
    a.queue = pl.ctrl;
    a.seg = seg;
    const dim3 grid((unsigned)grid_n), block(64);
    const bool f32c = pl.prm.precision == SPH_FP32C;
    if (stage == 2 || stage == 4) {
        // the selection passes need distances only: one kernel shape per
        // precision and list/heap size
        if (stage == 2) {
            e = run_zero_i32(pl.ctrl + kSelRetrySlot, 1, st);
            if (e != hipSuccess) return e;
        }
#define SPH_SEL(PR, GR, CP)                                                                   \
    do {                                                                                      \
        if (stage == 2)                                                                       \
            hipLaunchKernelGGL((k_solve<PR, GR, kSelTile, SPH_KERNEL_M4, 2, CP>), grid, block, \
                               0, st, a);                                                     \
        else                                                                                  \
            hipLaunchKernelGGL((k_solve<PR, GR, kSelTile, SPH_KERNEL_M4, 4, CP>), grid, block, \
                               0, st, a);                                                     \
    } while (0)
#define SPH_SEL_CAP(PR, GR)                                  \
    do {                                                    \
        if (a.sel_cap == 16) SPH_SEL(PR, GR, 16);           \
        else if (a.sel_cap == 32) SPH_SEL(PR, GR, 32);      \
        else SPH_SEL(PR, GR, 64);                           \
    } while (0)
        if (!pl.grouped) {
            if (f32c) SPH_SEL_CAP(SPH_FP32C, false);
            else SPH_SEL_CAP(SPH_FP64, false);
        } else {
            if (f32c) SPH_SEL_CAP(SPH_FP32C, true);
            else SPH_SEL_CAP(SPH_FP64, true);
        }
#undef SPH_SEL_CAP
#undef SPH_SEL
    } else if (stage == 1) {
        launch_stage<1>(pl, a, seg, grid, st);
    } else if (stage == 3) {
        launch_stage<3>(pl, a, seg, grid, st);
    } else {
        launch_stage<0>(pl, a, seg, grid, st);
    }
    return hipGetLastError();
}

// Exact K, periodic set: the count stage's starting h.  The K-th distance does
// not depend on where the iteration starts, so the caller's h_init is moved to
// within a factor 1.25 of a local estimate: the occupancy of the particle's
// Morton cell, from the dense-table level upwards until the cell holds at
// least K/8 particles, taken as a number density, gives h = (3K/(4 pi n))^(1/3).
// A uniform h_init is far too large inside clusters; this saves the count
// stage its largest passes.
__global__ void k_knn_start(int64_t n, const uint64_t *skeys, const int32_t *table, int Ld,
                            int bits, double box, double K, const double4 *sp,
                            const float4 *fp, double *sh0) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    // invalid particles (NaN position after the permute) keep their h_init
    if (sp ? isnan(sp[s].x) : isnan(fp[s].x)) return;
    const double h = sh0[s];
    const uint64_t c = skeys[s] >> (3 * (bits - Ld));
    int L = Ld;
    int32_t cnt = 0;
    for (;;) {
        const int sh = 3 * (Ld - L);
        const uint64_t a0 = (c >> sh) << sh;
        cnt = table[a0 + ((uint64_t)1 << sh)] - table[a0];
        if ((double)cnt >= 0.125 * K || L == 1) break;
        --L;
    }
    const double side = ldexp(box, -L);
    const double dens = (double)(cnt > 0 ? cnt : 1) / (side * side * side);
    const double he = cbrt(3.0 * K / (4.0 * kPi * dens));
    sh0[s] = fmin(fmax(h, 0.8 * he), 1.25 * he);
}

hipError_t run_solve(Plan &pl, const int64_t *goff, void *rho, void *h, void *nw,
                     int32_t *nngb, int32_t *status, uint64_t *stats, hipStream_t st) {
    SolveArgs a;
    a.n = pl.n;
    a.G = pl.G;
    a.goff = goff;
    a.skeys = pl.skeys;
    a.perm = pl.perm;
    a.sp = pl.sp; a.sh0 = pl.sh0;
    a.qp = pl.qp;
    a.fp = pl.fp;
    a.table = pl.table;
    a.Ld = pl.Ld;
    a.frame = pl.frame;
    a.gitems = pl.gitems;
    a.gorder = pl.gorder;
    a.n_items = pl.n_items;
    a.box = pl.prm.box;
    a.bits = pl.bits;
    a.Nt = pl.prm.n_target;
    a.dN = pl.prm.n_tol;
    a.root_tol = pl.prm.root_tol;
    a.mode = pl.prm.mode;
    a.max_iter = pl.prm.max_iter;
    a.cell_exp = pl.prm.tile_cell;
    a.out_f32 = pl.prm.io_dtype == SPH_F32;
    a.rho = rho; a.h = h; a.nw = nw;
    a.nngb = nngb; a.status = status;
    a.ost = pl.out_stride;
    a.ost_i = pl.out_stride_i;
    a.stats = stats;
    a.knn_h = pl.knn_h;
    // the selection ranks up to dK + 1 (one more where FP32C's widened sphere
    // takes in a particle at the edge); a narrow count-stage bracket is handed
    // over only while its count stays within the heap
    a.sel_cap = pl.prm.n_tol + 2.0 <= 16.0 ? 16 : (pl.prm.n_tol + 2.0 <= 32.0 ? 32 : 64);
    a.knn_st = pl.knn_st;
    a.knn_items = pl.knn_items;
    a.sh_out = pl.sh0;
    hipError_t e = hipSuccess;
    if (stats) {
        e = run_zero_u64(stats, 4, st);
        if (e != hipSuccess) return e;
    }
    if (pl.prm.prof_events[0]) {
        e = hipEventRecord((hipEvent_t)pl.prm.prof_events[0], st);
        if (e != hipSuccess) return e;
    }
    const int seg = pl.prm.segment;
    if (pl.prm.mode != SPH_KNN) {
        e = launch_solve(pl, a, seg, pl.grid, 0, st);
    } else {
        // exact K: count band, selection of the K-th distance (its own tile
        // size), evaluation at that distance
        const int64_t full = (int64_t)256 * pl.prm.waves_per_cu;
        if (!pl.grouped) {
            hipLaunchKernelGGL(k_knn_start, dim3((unsigned)ceil_div(pl.n, 256)), dim3(256), 0, st,
                               pl.n, pl.skeys, pl.table, pl.Ld, pl.bits, pl.prm.box,
                               pl.prm.n_target,
                               pl.prm.precision == SPH_FP32C ? nullptr : pl.sp,
                               pl.prm.precision == SPH_FP32C ? pl.fp : nullptr, pl.sh0);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = launch_solve(pl, a, seg, pl.grid, 1, st);
        if (e == hipSuccess && pl.grouped) {
            pl.prm.segment = kSelTile;
            e = run_group_items(pl, goff, st);
        }
        if (e == hipSuccess) {
            a.n_items = ceil_div(pl.n, kSelTile);
            const int64_t g2 = pl.grouped ? full : (a.n_items < full ? a.n_items : full);
            e = launch_solve(pl, a, kSelTile, g2 > 0 ? g2 : 1, 2, st);
            if (e == hipSuccess) e = launch_solve(pl, a, kSelTile, g2 > 0 ? g2 : 1, 4, st);
        }
        if (e == hipSuccess && pl.grouped) {
            pl.prm.segment = seg;
            e = run_group_items(pl, goff, st);
        }
        if (e == hipSuccess) {
            a.n_items = pl.n_items;
            e = launch_solve(pl, a, seg, pl.grid, 3, st);
        }
    }
    if (e != hipSuccess) return e;
    if (pl.prm.prof_events[1]) e = hipEventRecord((hipEvent_t)pl.prm.prof_events[1], st);
    return e;
}

}  // namespace sph
