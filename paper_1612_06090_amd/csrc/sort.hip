// Spatial sort of the particles: Morton keys, LSD radix sort of (key, index),
// gather into sorted structure-of-arrays, and the cell tables.
//
// The paper's kernel walks a pre-built Barnes-Hut tree (Sec. II-A); on the
// GPU the particles are instead ordered along a Morton curve, whose key
// prefixes are exactly the nodes of an octree: a cell at level L is a
// contiguous run of the sorted array.  The gather into structure-of-arrays
// follows the SoA redesign of Sec. IV-B (only the fields the density loop
// reads: positions, mass, smoothing length).
//
// Radix sort: least-significant-digit first, 8-bit digits, stable scatter
// passes.  Inside a tile each wave ranks 64 consecutive keys per round with 8
// ballots (lanes sharing a digit), keeping one running count per digit in
// LDS, so equal digits keep their input order and every pass is stable.  The
// particle keys of sets above 2^21 take a single sweep per pass: one
// histogram pass counts the digits of all passes at once, and a tile finds
// the output offset of each digit from the counts that the tiles before it
// publish (decoupled look-back).  Smaller sets and the group-order sort keep
// reduce-then-scan (per-tile histograms, a digit-major scan of them, then
// the scatter).
#include "sph_internal.h"

#include <limits.h>

namespace sph {

// ------------------------------------------------------------------- keys

template <typename T>
__global__ void k_keys_periodic(int64_t n, const void *x, const void *y, const void *z,
                                int64_t ins, double box, uint64_t *keys, int32_t *vals) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double s = 2097152.0 / box;
    const uint32_t qx = quantise(ld<T>(x, i, ins) * s, 1u << 21);
    const uint32_t qy = quantise(ld<T>(y, i, ins) * s, 1u << 21);
    const uint32_t qz = quantise(ld<T>(z, i, ins) * s, 1u << 21);
    keys[i] = morton3(qx, qy, qz);
    vals[i] = (int32_t)i;
}

// The periodic keys of the single-sweep sort, with the digit counts of its
// eight passes taken while the keys are in registers: gh[p * 256 + d] +=
// number of keys whose digit p is d.  Grid-stride over batches of four
// keys per thread, their coordinates loaded together.
template <typename T>
__global__ __launch_bounds__(kSortThreads) void k_keys_periodic_hist(int64_t n, const void *x,
                                                                    const void *y,
                                                                    const void *z, int64_t ins,
                                                                    double box, uint64_t *keys,
                                                                    int32_t *vals,
                                                                    uint32_t *gh) {
    __shared__ uint32_t h[8][256];
    const int tid = threadIdx.x;
    for (int k = tid; k < 8 * 256; k += kSortThreads) (&h[0][0])[k] = 0u;
    __syncthreads();
    const double s = 2097152.0 / box;
    const int64_t step = (int64_t)gridDim.x * kSortThreads * 4;
    for (int64_t i0 = (int64_t)blockIdx.x * kSortThreads * 4 + tid; i0 < n; i0 += step) {
        double px[4], py[4], pz[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = i0 + (int64_t)u * kSortThreads;
            if (i < n) {
                px[u] = ld<T>(x, i, ins);
                py[u] = ld<T>(y, i, ins);
                pz[u] = ld<T>(z, i, ins);
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = i0 + (int64_t)u * kSortThreads;
            if (i < n) {
                const uint64_t k = morton3(quantise(px[u] * s, 1u << 21),
                                           quantise(py[u] * s, 1u << 21),
                                           quantise(pz[u] * s, 1u << 21));
                keys[i] = k;
                vals[i] = (int32_t)i;
#pragma unroll
                for (int p = 0; p < 8; ++p)
                    atomicAdd(&h[p][(uint32_t)(k >> (8 * p)) & 255u], 1u);
            }
        }
    }
    __syncthreads();
    for (int k = tid; k < 8 * 256; k += kSortThreads) {
        const uint32_t v = (&h[0][0])[k];
        if (v) atomicAdd(&gh[k], v);
    }
}

// One block per group: bounding box of the group's finite coordinates.
// frame[8g + 0..2] = lower corner, [3..5] = extents, [6] = 2^16 / largest
// extent (largest extent 1 when it is 0), [7] = largest extent.
template <typename T>
__global__ __launch_bounds__(256) void k_group_frames(int32_t G, const int64_t *goff,
                                                      const void *x, const void *y,
                                                      const void *z, int64_t ins,
                                                      double *frame) {
    const int g = blockIdx.x;
    if (g >= G) return;
    const int64_t b = goff[g], e = goff[g + 1];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
        const double p[3] = {ld<T>(x, i, ins), ld<T>(y, i, ins), ld<T>(z, i, ins)};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (!isfinite(p[a])) continue;
            lo[a] = fmin(lo[a], p[a]);
            hi[a] = fmax(hi[a], p[a]);
        }
    }
    __shared__ double red[6][4];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double vl = wave_min(lo[a]);
        double vh = wave_max(hi[a]);
        if (l == 0) { red[a][w] = vl; red[3 + a][w] = vh; }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ext = 0.0;
        double L[3], E[3];
        for (int a = 0; a < 3; ++a) {
            double vl = red[a][0], vh = red[3 + a][0];
            for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
                vl = fmin(vl, red[a][k]);
                vh = fmax(vh, red[3 + a][k]);
            }
            if (!(vl <= vh)) { vl = 0.0; vh = 0.0; }
            L[a] = vl;
            E[a] = vh - vl;
            if (E[a] > ext) ext = E[a];
        }
        if (!(ext > 0.0)) ext = 1.0;
        double *f = frame + 8 * (int64_t)g;
        f[0] = L[0]; f[1] = L[1]; f[2] = L[2];
        f[3] = E[0]; f[4] = E[1]; f[5] = E[2];
        f[6] = 65536.0 / ext;
        f[7] = ext;
    }
}

// Group of particle i: the largest g with goff[g] <= i.
__device__ inline int32_t group_of(const int64_t *goff, int32_t G, int64_t i) {
    int32_t lo = 0, hi = G - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (goff[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <typename T>
__global__ void k_keys_groups(int64_t n, int32_t G, const int64_t *goff, const void *x,
                              const void *y, const void *z, int64_t ins, const double *frame,
                              uint64_t *keys, int32_t *vals) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t g = group_of(goff, G, i);
    const double *f = frame + 8 * (int64_t)g;
    const double sc = f[6];
    const uint32_t qx = quantise((ld<T>(x, i, ins) - f[0]) * sc, 1u << 16);
    const uint32_t qy = quantise((ld<T>(y, i, ins) - f[1]) * sc, 1u << 16);
    const uint32_t qz = quantise((ld<T>(z, i, ins) - f[2]) * sc, 1u << 16);
    keys[i] = ((uint64_t)(uint32_t)g << 48) | morton3(qx, qy, qz);
    vals[i] = (int32_t)i;
}

// ------------------------------------------------------------- radix sort

template <int ROUNDS>
__global__ __launch_bounds__(kSortThreads) void k_radix_up(int64_t n, const uint64_t *keys,
                                                          int shift, uint32_t *hist,
                                                          int64_t nb) {
    __shared__ uint32_t h[4][256];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    for (int k = tid; k < 4 * 256; k += kSortThreads) (&h[0][0])[k] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * (256 * ROUNDS) + (int64_t)w * 64 * ROUNDS;
    // all loads first, so that they are in flight together
    uint32_t dg[ROUNDS];
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const int64_t idx = base + r * 64 + l;
        dg[r] = idx < n ? (uint32_t)(keys[idx] >> shift) & 255u : 256u;
    }
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r)
        if (dg[r] < 256u) atomicAdd(&h[w][dg[r]], 1u);
    __syncthreads();
    hist[(int64_t)tid * nb + blockIdx.x] = h[0][tid] + h[1][tid] + h[2][tid] + h[3][tid];
}

// Exclusive scan of 256 per-thread values across a 256-thread block.
__device__ inline uint32_t block_excl_scan_256(uint32_t v, uint32_t *total) {
    __shared__ uint32_t wt[4];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(inc, o, 64);
        if (l >= o) inc += t;
    }
    if (l == 63) wt[w] = inc;
    __syncthreads();
    uint32_t off = 0;
    for (int k = 0; k < w; ++k) off += wt[k];
    if (total) *total = wt[0] + wt[1] + wt[2] + wt[3];
    __syncthreads();
    return off + inc - v;
}

// One block per digit: exclusive scan of that digit's per-tile counts.
__global__ __launch_bounds__(kSortThreads) void k_radix_scan(uint32_t *hist, int64_t nb,
                                                            uint32_t *digit_tot) {
    uint32_t *row = hist + (int64_t)blockIdx.x * nb;
    const int tid = threadIdx.x;
    const int64_t per = (nb + kSortThreads - 1) / kSortThreads;
    const int64_t b = tid * per;
    const int64_t e = b + per < nb ? b + per : nb;
    uint32_t s = 0;
    for (int64_t k = b; k < e; ++k) s += row[k];
    uint32_t tot;
    uint32_t run = block_excl_scan_256(s, &tot);
    for (int64_t k = b; k < e; ++k) {
        const uint32_t v = row[k];
        row[k] = run;
        run += v;
    }
    if (tid == 0) digit_tot[blockIdx.x] = tot;
}

// Scatter of one pass.  Each block ranks its 256 * ROUNDS keys stably by the
// pass digit (waves in index order, rounds in order within a wave, lanes in
// order within a round), places them in LDS in that order, and then writes
// them out from LDS: consecutive threads write consecutive slots of each
// digit's run in the output, so the stores coalesce.
template <int ROUNDS>
__global__ __launch_bounds__(kSortThreads) void k_radix_down(int64_t n, const uint64_t *kin,
                                                            const int32_t *vin, uint64_t *kout,
                                                            int32_t *vout, int shift,
                                                            const uint32_t *hist,
                                                            const uint32_t *digit_tot,
                                                            int64_t nb) {
    constexpr int TILE = 256 * ROUNDS;
    __shared__ uint32_t wcnt[4][256];
    __shared__ uint32_t dbase[256];   // output start of each digit's run of this block
    __shared__ uint32_t lbase[256];   // LDS start of each digit's run
    __shared__ uint64_t skey[TILE];
    __shared__ int32_t sval[TILE];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    for (int k = tid; k < 4 * 256; k += kSortThreads) (&wcnt[0][0])[k] = 0u;
    {
        const uint32_t tot = digit_tot[tid];
        const uint32_t pre = block_excl_scan_256(tot, nullptr);
        dbase[tid] = pre + hist[(int64_t)tid * nb + blockIdx.x];
    }
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * TILE + (int64_t)w * 64 * ROUNDS;
    uint64_t key[ROUNDS];
    int32_t val[ROUNDS];
    uint32_t rank[ROUNDS];
    // all loads first, so that they are in flight together
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const int64_t idx = base + r * 64 + l;
        const bool valid = idx < n;
        key[r] = valid ? kin[idx] : ~0ull;
        val[r] = valid ? vin[idx] : 0;
    }
    volatile uint32_t *wc = wcnt[w];
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const int64_t idx = base + r * 64 + l;
        const bool valid = idx < n;
        const uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bal = __ballot(bit);
            m &= bit ? bal : ~bal;
        }
        const uint32_t before = mbcnt(m);
        const uint32_t cnt0 = wc[d];
        rank[r] = cnt0 + before;
        __builtin_amdgcn_wave_barrier();
        if (valid && before == 0) wc[d] = cnt0 + (uint32_t)__popcll(m);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    {
        // per digit: the waves' counts become offsets, their total the run
        // length, and the runs are laid out in digit order in LDS
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t t = wcnt[k][tid];
            wcnt[k][tid] = s;
            s += t;
        }
        const uint32_t lb = block_excl_scan_256(s, nullptr);
        lbase[tid] = lb;
        // output slot of LDS slot j of this digit: dbase + (j - lbase)
        dbase[tid] = dbase[tid] - lb;
    }
    __syncthreads();
    const int64_t blk0 = (int64_t)blockIdx.x * TILE;
    const int cnt = n - blk0 < TILE ? (int)(n - blk0) : TILE;
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const int64_t idx = base + r * 64 + l;
        if (idx < n) {
            const uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
            const uint32_t j = lbase[d] + wcnt[w][d] + rank[r];
            skey[j] = key[r];
            sval[j] = val[r];
        }
    }
    __syncthreads();
    for (int j = tid; j < cnt; j += kSortThreads) {
        const uint64_t k = skey[j];
        const uint32_t d = (uint32_t)(k >> shift) & 255u;
        const uint32_t pos = dbase[d] + (uint32_t)j;
        kout[pos] = k;
        vout[pos] = sval[j];
    }
}

// ------------------------------------------------- single-sweep passes
//
// Tiles take their index from a counter in the order their blocks start, so
// a tile waits only on tiles that started before it.  Each tile first
// publishes its own count per digit (flag A), then looks back over the
// tiles before it, adding their counts, until it meets an inclusive prefix
// (flag P), and publishes its own inclusive prefix.  Since every tile
// publishes its counts before it waits and the tiles it waits on have
// started, every wait ends; each one is still bounded (kLookbackSpin loads
// of descriptors not yet published), and a wait that reaches the bound is
// counted in sort_wait_faults, which the host reads back.
//
// Descriptors: 256 per tile (tile-major), 64 bits: flag in the high half,
// count in the low half.  Within one sort the flags of pass p are 2p + 1 (A)
// and 2p + 2 (P), so what earlier passes left reads as not yet published;
// the descriptors are cleared once per sort.

constexpr uint32_t kLookbackSpin = 1u << 22;
constexpr int kLookbackWin = 2;
constexpr int kDigitHistBlocks = 1024;

__device__ uint32_t sort_wait_faults;

// Digit counts of all `passes` passes in one read of the keys:
// gh[p * 256 + d] += number of keys whose digit p is d.
__global__ __launch_bounds__(kSortThreads) void k_digit_hist(int64_t n, const uint64_t *keys,
                                                            int passes, uint32_t *gh) {
    __shared__ uint32_t h[8][256];
    const int tid = threadIdx.x;
    for (int k = tid; k < 8 * 256; k += kSortThreads) (&h[0][0])[k] = 0u;
    __syncthreads();
    const int64_t step = (int64_t)gridDim.x * kSortThreads;
    for (int64_t i = (int64_t)blockIdx.x * kSortThreads + tid; i < n; i += step) {
        const uint64_t k = keys[i];
        for (int p = 0; p < passes; ++p) atomicAdd(&h[p][(uint32_t)(k >> (8 * p)) & 255u], 1u);
    }
    __syncthreads();
    for (int k = tid; k < passes * 256; k += kSortThreads) {
        const uint32_t v = (&h[0][0])[k];
        if (v) atomicAdd(&gh[k], v);
    }
}

// Exclusive scan of 256 per-thread values across a 256-thread block, with
// its four wave totals in caller-provided LDS.
__device__ inline uint32_t block_excl_scan_256_at(uint32_t v, uint32_t *wt) {
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(inc, o, 64);
        if (l >= o) inc += t;
    }
    if (l == 63) wt[w] = inc;
    __syncthreads();
    uint32_t off = 0;
    for (int k = 0; k < w; ++k) off += wt[k];
    __syncthreads();
    return off + inc - v;
}

// One scatter pass: the ranking and the LDS-staged write of k_radix_down,
// with the tile's output offsets from the global digit counts gh (scanned
// here) and the look-back over the descriptors.  LDS is held to 52 KiB (the
// wave counts, the staged keys and values; the scan's wave totals and the
// tile index live in the value buffer before it is filled) so that three
// blocks fit on a CU, whose tiles hide each other's look-back.
template <int ROUNDS>
__global__ __launch_bounds__(kSortThreads) void k_radix_sweep(int64_t n, const uint64_t *kin,
                                                             const int32_t *vin, uint64_t *kout,
                                                             int32_t *vout, int pass,
                                                             const uint32_t *gh,
                                                             uint64_t *desc, int32_t *tile_ctr) {
    constexpr int TILE = 256 * ROUNDS;
    __shared__ uint32_t wcnt[4][256];
    __shared__ uint64_t skey[TILE];
    __shared__ int32_t sval[TILE];
    uint32_t *wt = reinterpret_cast<uint32_t *>(sval);   // until the values are staged
    int32_t *s_tile = sval + 4;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int shift = 8 * pass;
    for (int k = tid; k < 4 * 256; k += kSortThreads) (&wcnt[0][0])[k] = 0u;
    if (tid == 0) *s_tile = atomicAdd(tile_ctr + pass, 1);
    const uint32_t gpre = block_excl_scan_256_at(gh[pass * 256 + tid], wt);
    const int64_t tile = *s_tile;
    const int64_t blk0 = tile * TILE;
    const int64_t base = blk0 + (int64_t)w * 64 * ROUNDS;
    uint64_t key[ROUNDS];
    int32_t val[ROUNDS];
    uint32_t rank[ROUNDS];
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const int64_t idx = base + r * 64 + l;
        const bool valid = idx < n;
        key[r] = valid ? kin[idx] : ~0ull;
        val[r] = valid ? vin[idx] : 0;
    }
    volatile uint32_t *wc = wcnt[w];
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const int64_t idx = base + r * 64 + l;
        const bool valid = idx < n;
        const uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
        uint64_t m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bal = __ballot(bit);
            m &= bit ? bal : ~bal;
        }
        const uint32_t before = mbcnt(m);
        const uint32_t cnt0 = wc[d];
        rank[r] = cnt0 + before;
        __builtin_amdgcn_wave_barrier();
        if (valid && before == 0) wc[d] = cnt0 + (uint32_t)__popcll(m);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // thread tid owns digit tid: its count s over the tile, published at
    // once; the waves' counts become LDS slots (digit runs in digit order)
    uint32_t s = 0;
    uint32_t wv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        wv[k] = s;
        s += wcnt[k][tid];
    }
    const uint64_t flag_a = (uint64_t)(2 * pass + 1) << 32;
    const uint64_t flag_p = (uint64_t)(2 * pass + 2) << 32;
    uint64_t *mine = desc + tile * 256 + tid;
    __hip_atomic_store(mine, (tile == 0 ? flag_p : flag_a) | s, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t lb = block_excl_scan_256_at(s, wt);
#pragma unroll
    for (int k = 0; k < 4; ++k) wcnt[k][tid] = lb + wv[k];
    __syncthreads();
    const int cnt = n - blk0 < TILE ? (int)(n - blk0) : TILE;
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const int64_t idx = base + r * 64 + l;
        if (idx < n) {
            const uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
            const uint32_t j = wcnt[w][d] + rank[r];
            skey[j] = key[r];
            sval[j] = val[r];
        }
    }
    __syncthreads();
    // look back kLookbackWin tiles at a time: add the counts (A) in order up
    // to the first inclusive prefix (P); at a tile not yet published, load
    // again from there
    uint32_t excl = 0;
    if (tile > 0) {
        int64_t k = tile - 1;
        uint32_t spins = 0;
        for (;;) {
            uint64_t v[kLookbackWin];
#pragma unroll
            for (int u = 0; u < kLookbackWin; ++u)
                v[u] = k - u >= 0 ? __hip_atomic_load(desc + (k - u) * 256 + tid, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT)
                                  : 0ull;
            int used = kLookbackWin;
            bool done = false;
#pragma unroll
            for (int u = 0; u < kLookbackWin; ++u) {
                if (used != kLookbackWin || done) continue;
                const uint32_t f = (uint32_t)(v[u] >> 32);
                if (k - u < 0 || f < (uint32_t)(2 * pass + 1)) {
                    used = u;
                    continue;
                }
                excl += (uint32_t)v[u];
                done = f == (uint32_t)(2 * pass + 2);
            }
            if (done) break;
            k -= used;
            if (used == 0) {
                if (++spins >= kLookbackSpin) {
                    atomicAdd(&sort_wait_faults, 1u);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __hip_atomic_store(mine, flag_p | (uint64_t)(excl + s), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    // output slot of LDS slot j of digit d: gpre + excl + (j - lb), kept in
    // the first row of the wave counts, which the staging no longer needs
    uint32_t *dbase = wcnt[0];
    dbase[tid] = gpre + excl - lb;
    __syncthreads();
    // the bound on pos matters only after a wait reached its bound: offsets
    // are then wrong, and no store may leave the arrays
    for (int j = tid; j < cnt; j += kSortThreads) {
        const uint64_t k = skey[j];
        const uint32_t d = (uint32_t)(k >> shift) & 255u;
        const uint32_t pos = dbase[d] + (uint32_t)j;
        if ((int64_t)pos < n) {
            kout[pos] = k;
            vout[pos] = sval[j];
        }
    }
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t cnt);

// All `passes` passes over the particle keys in (keysA, valsA); the result
// ends in the A buffers after an even number of passes, or in (kfin, vfin)
// when given.
// With `counted` the sweep run was cleared and the digit counts taken
// before the keys were written (k_keys_periodic_hist).
template <int ROUNDS>
static hipError_t sweep_passes(Plan &pl, int passes, hipStream_t st, uint64_t *kfin,
                               int32_t *vfin, bool counted) {
    if (passes < 1 || passes > 8) return hipErrorInvalidValue;
    const int64_t n = pl.n, nb = pl.nb_sort;
    if (!counted) {
        hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)ceil_div(pl.sweep_words, 256)), dim3(256),
                           0, st, pl.sweep, 0, pl.sweep_words);
        const int64_t hb = nb < kDigitHistBlocks ? nb : kDigitHistBlocks;
        hipLaunchKernelGGL(k_digit_hist, dim3((unsigned)hb), dim3(kSortThreads), 0, st, n,
                           pl.keysA, passes, pl.sweep_gh);
    }
    uint64_t *ka = pl.keysA, *kb = pl.keysB;
    int32_t *va = pl.valsA, *vb = pl.valsB;
    for (int p = 0; p < passes; ++p) {
        if (p == passes - 1 && kfin) { kb = kfin; vb = vfin; }
        hipLaunchKernelGGL(k_radix_sweep<ROUNDS>, dim3((unsigned)nb), dim3(kSortThreads), 0, st,
                           n, ka, va, kb, vb, p, pl.sweep_gh, pl.sweep_desc, pl.sweep_ctr);
        uint64_t *tk = ka; ka = kb; kb = tk;
        int32_t *tv = va; va = vb; vb = tv;
    }
    pl.skeys = ka;
    pl.perm = va;
    return hipGetLastError();
}

hipError_t read_sort_wait_faults(uint32_t *count) {
    uint32_t v = 0;
    hipError_t e = hipMemcpyFromSymbol(&v, HIP_SYMBOL(sort_wait_faults), sizeof(v), 0,
                                       hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    const uint32_t zero = 0;
    e = hipMemcpyToSymbol(HIP_SYMBOL(sort_wait_faults), &zero, sizeof(zero), 0,
                          hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    *count = v;
    return hipSuccess;
}

// LSD radix sort of (key, value) pairs over `passes` 8-bit digits; the result
// ends in the A buffers after an even number of passes, or in (kfin, vfin)
// when given (the last pass writes there).
template <int ROUNDS>
static hipError_t radix_passes(int64_t n, int64_t nb, int passes, uint64_t *ka, uint64_t *kb,
                               int32_t *va, int32_t *vb, uint32_t *hist, uint32_t *digit_tot,
                               hipStream_t st, uint64_t **kout, int32_t **vout,
                               uint64_t *kfin = nullptr, int32_t *vfin = nullptr) {
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        if (p == passes - 1 && kfin) { kb = kfin; vb = vfin; }
        hipLaunchKernelGGL(k_radix_up<ROUNDS>, dim3((unsigned)nb), dim3(kSortThreads), 0, st, n,
                           ka, shift, hist, nb);
        hipLaunchKernelGGL(k_radix_scan, dim3(256), dim3(kSortThreads), 0, st, hist, nb,
                           digit_tot);
        hipLaunchKernelGGL(k_radix_down<ROUNDS>, dim3((unsigned)nb), dim3(kSortThreads), 0, st,
                           n, ka, va, kb, vb, shift, hist, digit_tot, nb);
        uint64_t *tk = ka; ka = kb; kb = tk;
        int32_t *tv = va; va = vb; vb = tv;
    }
    *kout = ka;
    *vout = va;
    return hipGetLastError();
}

// Sets above 2^21 keys take the single sweep.  Smaller ones (1024-key
// tiles) keep reduce-then-scan: all their tiles are resident at once, so a
// look-back would cross most of them in every pass (measured at 2^20: 0.38
// ms per sort against 0.26); their per-tile histograms use the start of the
// sweep run, which holds twice as many words.
static hipError_t radix_sort(Plan &pl, int passes, hipStream_t st, uint64_t *kfin,
                             int32_t *vfin, bool counted) {
    if (pl.sort_rounds == 16) return sweep_passes<16>(pl, passes, st, kfin, vfin, counted);
    return radix_passes<4>(pl.n, pl.nb_sort, passes, pl.keysA, pl.keysB, pl.valsA, pl.valsB,
                           reinterpret_cast<uint32_t *>(pl.sweep), pl.digit_tot, st, &pl.skeys,
                           &pl.perm, kfin, vfin);
}

hipError_t run_keys_and_sort(Plan &pl, const int64_t *goff, const void *x, const void *y,
                             const void *z, hipStream_t st, uint64_t *keys_out,
                             int32_t *perm_out) {
    const int64_t n = pl.n;
    const unsigned nbk = (unsigned)ceil_div(n, 256);
    const bool f32 = pl.prm.io_dtype == SPH_F32;
    // periodic sets of the single sweep: clear its run, then keys and digit
    // counts in one kernel
    const bool counted = !pl.grouped && pl.sort_rounds == 16;
    if (counted) {
        hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)ceil_div(pl.sweep_words, 256)), dim3(256),
                           0, st, pl.sweep, 0, pl.sweep_words);
        const int64_t hb = pl.nb_sort < kDigitHistBlocks ? pl.nb_sort : kDigitHistBlocks;
        if (f32)
            hipLaunchKernelGGL(k_keys_periodic_hist<float>, dim3((unsigned)hb),
                               dim3(kSortThreads), 0, st, n, x, y, z, pl.in_stride, pl.prm.box,
                               pl.keysA, pl.valsA, pl.sweep_gh);
        else
            hipLaunchKernelGGL(k_keys_periodic_hist<double>, dim3((unsigned)hb),
                               dim3(kSortThreads), 0, st, n, x, y, z, pl.in_stride, pl.prm.box,
                               pl.keysA, pl.valsA, pl.sweep_gh);
    } else if (!pl.grouped) {
        if (f32)
            hipLaunchKernelGGL(k_keys_periodic<float>, dim3(nbk), dim3(256), 0, st, n, x, y, z,
                               pl.in_stride, pl.prm.box, pl.keysA, pl.valsA);
        else
            hipLaunchKernelGGL(k_keys_periodic<double>, dim3(nbk), dim3(256), 0, st, n, x, y, z,
                               pl.in_stride, pl.prm.box, pl.keysA, pl.valsA);
    } else {
        if (f32) {
            hipLaunchKernelGGL(k_group_frames<float>, dim3(pl.G), dim3(256), 0, st, pl.G, goff,
                               x, y, z, pl.in_stride, pl.frame);
            hipLaunchKernelGGL(k_keys_groups<float>, dim3(nbk), dim3(256), 0, st, n, pl.G, goff,
                               x, y, z, pl.in_stride, pl.frame, pl.keysA, pl.valsA);
        } else {
            hipLaunchKernelGGL(k_group_frames<double>, dim3(pl.G), dim3(256), 0, st, pl.G, goff,
                               x, y, z, pl.in_stride, pl.frame);
            hipLaunchKernelGGL(k_keys_groups<double>, dim3(nbk), dim3(256), 0, st, n, pl.G,
                               goff, x, y, z, pl.in_stride, pl.frame, pl.keysA, pl.valsA);
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return radix_sort(pl, 8, st, keys_out, perm_out, counted);
}

// ------------------------------------------------------- sorted SoA gather

// Default initial smoothing length 2 (V / n)^(1/3): V = box^3, or the group's
// bounding-box volume with every extent at least 2^-16 of the largest.
__device__ inline double default_h(bool grouped, double box, int64_t n, const double *frame,
                                   const int64_t *goff, uint64_t key) {
    if (!grouped) return 2.0 * cbrt(box * box * box / (double)n);
    const uint32_t g = (uint32_t)(key >> 48);
    const double *f = frame + 8 * (int64_t)g;
    const double emin = f[7] * 0x1p-16;
    const double V = fmax(f[3], emin) * fmax(f[4], emin) * fmax(f[5], emin);
    const double ng = (double)(goff[g + 1] - goff[g]);
    return 2.0 * cbrt(V / ng);
}

__device__ inline bool valid_input(bool periodic, double box, double x, double y, double z,
                                   double m, double h) {
    if (!isfinite(x) || !isfinite(y) || !isfinite(z) || !isfinite(m) || !isfinite(h)) return false;
    if (!(h > 0.0)) return false;
    if (periodic) {
        if (!(x >= 0.0 && x < box) || !(y >= 0.0 && y < box) || !(z >= 0.0 && z < box))
            return false;
    }
    return true;
}

template <typename T>
__global__ void k_permute64(int64_t n, const int32_t *perm, const uint64_t *skeys,
                            const void *x, const void *y, const void *z, const void *m,
                            const void *h0, int64_t ins, bool grouped, double box, const double *frame,
                            const int64_t *goff, double4 *sp, double *sh0) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t i = perm[s];
    double xv = ld<T>(x, i, ins), yv = ld<T>(y, i, ins), zv = ld<T>(z, i, ins), mv = ld<T>(m, i, ins);
    const double hv = h0 ? ld<T>(h0, i, ins) : default_h(grouped, box, n, frame, goff, skeys[s]);
    if (!valid_input(!grouped, box, xv, yv, zv, mv, hv)) {
        xv = NAN; yv = NAN; zv = NAN;
    }
    sp[s] = make_double4(xv, yv, zv, mv);
    sh0[s] = hv;
}

// Positions as integer Morton-grid coordinates q (units of the grid spacing:
// box / 2^21, or the group cube / 2^16) plus a binary32 fraction in [0, 1],
// packed per particle as (q, mass bits) and (fraction, 0): a candidate is two
// 16-byte loads.
template <typename T>
__global__ void k_permute32(int64_t n, const int32_t *perm, const uint64_t *skeys,
                            const void *x, const void *y, const void *z, const void *m,
                            const void *h0, int64_t ins, bool grouped, double box, const double *frame,
                            const int64_t *goff, int4 *qp, float4 *fp, double *sh0) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t i = perm[s];
    const double xv = ld<T>(x, i, ins), yv = ld<T>(y, i, ins), zv = ld<T>(z, i, ins), mv = ld<T>(m, i, ins);
    const double hv = h0 ? ld<T>(h0, i, ins) : default_h(grouped, box, n, frame, goff, skeys[s]);
    double tx, ty, tz;
    uint32_t nmax;
    if (!grouped) {
        const double sc = 2097152.0 / box;
        tx = xv * sc; ty = yv * sc; tz = zv * sc;
        nmax = 1u << 21;
    } else {
        const double *f = frame + 8 * (int64_t)(uint32_t)(skeys[s] >> 48);
        tx = (xv - f[0]) * f[6]; ty = (yv - f[1]) * f[6]; tz = (zv - f[2]) * f[6];
        nmax = 1u << 16;
    }
    const uint32_t ux = quantise(tx, nmax), uy = quantise(ty, nmax), uz = quantise(tz, nmax);
    float ax = (float)(tx - (double)ux), ay = (float)(ty - (double)uy), az = (float)(tz - (double)uz);
    if (!valid_input(!grouped, box, xv, yv, zv, mv, hv)) { ax = NAN; ay = NAN; az = NAN; }
    qp[s] = make_int4((int32_t)ux, (int32_t)uy, (int32_t)uz, __float_as_int((float)mv));
    fp[s] = make_float4(ax, ay, az, 0.f);
    sh0[s] = hv;
}

hipError_t run_permute(Plan &pl, const int64_t *goff, const void *x, const void *y,
                       const void *z, const void *m, const void *h0, bool fp32c,
                       hipStream_t st) {
    const int64_t n = pl.n;
    const unsigned nbk = (unsigned)ceil_div(n, 256);
    const bool f32 = pl.prm.io_dtype == SPH_F32;
    if (!fp32c) {
        if (f32)
            hipLaunchKernelGGL(k_permute64<float>, dim3(nbk), dim3(256), 0, st, n, pl.perm,
                               pl.skeys, x, y, z, m, h0, pl.in_stride, pl.grouped, pl.prm.box, pl.frame, goff,
                               pl.sp, pl.sh0);
        else
            hipLaunchKernelGGL(k_permute64<double>, dim3(nbk), dim3(256), 0, st, n, pl.perm,
                               pl.skeys, x, y, z, m, h0, pl.in_stride, pl.grouped, pl.prm.box, pl.frame, goff,
                               pl.sp, pl.sh0);
    } else {
        if (f32)
            hipLaunchKernelGGL(k_permute32<float>, dim3(nbk), dim3(256), 0, st, n, pl.perm,
                               pl.skeys, x, y, z, m, h0, pl.in_stride, pl.grouped, pl.prm.box, pl.frame, goff,
                               pl.qp, pl.fp, pl.sh0);
        else
            hipLaunchKernelGGL(k_permute32<double>, dim3(nbk), dim3(256), 0, st, n, pl.perm,
                               pl.skeys, x, y, z, m, h0, pl.in_stride, pl.grouped, pl.prm.box, pl.frame, goff,
                               pl.qp, pl.fp, pl.sh0);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ scans
//
// Device-wide scans of int32 arrays in three launches: per-tile reductions,
// a scan of the tile totals in one block, then per-tile scans plus carry.
// OP 0 = sum, 1 = min.  REV scans from the end of the array backwards.

template <int OP>
__device__ inline int32_t sop(int32_t a, int32_t b) {
    if (OP == 0) return a + b;
    return a < b ? a : b;
}

template <int OP>
__device__ inline int32_t sid() {
    return OP == 0 ? 0 : INT_MAX;
}

// Exclusive block scan of one value per thread (blockDim.x = kScanThreads or 1024).
template <int OP, int NT>
__device__ inline int32_t block_excl(int32_t v, int32_t *total) {
    __shared__ int32_t wt[NT / 64];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    int32_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int32_t t = __shfl_up(inc, o, 64);
        if (l >= o) inc = sop<OP>(inc, t);
    }
    if (l == 63) wt[w] = inc;
    __syncthreads();
    int32_t off = sid<OP>();
    for (int k = 0; k < w; ++k) off = sop<OP>(off, wt[k]);
    if (total) {
        int32_t t = sid<OP>();
        for (int k = 0; k < NT / 64; ++k) t = sop<OP>(t, wt[k]);
        *total = t;
    }
    __syncthreads();
    int32_t ex = __shfl_up(inc, 1, 64);
    if (l == 0) ex = sid<OP>();
    return sop<OP>(off, ex);
}

template <int OP, bool REV>
__device__ inline int64_t phys(int64_t li, int64_t cnt) {
    return REV ? cnt - 1 - li : li;
}

template <int OP, bool REV>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int32_t *in, int64_t cnt,
                                                             int32_t *bsum) {
    const int64_t b0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t acc = sid<OP>();
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t li = b0 + k;
        if (li < cnt) acc = sop<OP>(acc, in[phys<OP, REV>(li, cnt)]);
    }
    int32_t tot;
    block_excl<OP, kScanThreads>(acc, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

template <int OP>
__global__ __launch_bounds__(1024) void k_scan_bsum(int32_t *bsum, int64_t nb) {
    __shared__ int32_t carry_s;
    int32_t carry = sid<OP>();
    for (int64_t c0 = 0; c0 < nb; c0 += 1024 * 8) {
        const int64_t b0 = c0 + (int64_t)threadIdx.x * 8;
        int32_t v[8];
        int32_t acc = sid<OP>();
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            v[k] = b0 + k < nb ? bsum[b0 + k] : sid<OP>();
            acc = sop<OP>(acc, v[k]);
        }
        int32_t tot;
        int32_t ex = block_excl<OP, 1024>(acc, &tot);
        ex = sop<OP>(carry, ex);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (b0 + k < nb) bsum[b0 + k] = ex;
            ex = sop<OP>(ex, v[k]);
        }
        if (threadIdx.x == 0) carry_s = sop<OP>(carry, tot);
        __syncthreads();
        carry = carry_s;
        __syncthreads();
    }
}

template <int OP, bool REV, bool INCL>
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const int32_t *in, int32_t *out,
                                                            int64_t cnt, const int32_t *bsum) {
    const int64_t b0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    int32_t acc = sid<OP>();
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t li = b0 + k;
        v[k] = li < cnt ? in[phys<OP, REV>(li, cnt)] : sid<OP>();
        acc = sop<OP>(acc, v[k]);
    }
    int32_t ex = block_excl<OP, kScanThreads>(acc, nullptr);
    ex = sop<OP>(bsum[blockIdx.x], ex);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t li = b0 + k;
        const int32_t nx = sop<OP>(ex, v[k]);
        if (li < cnt) out[phys<OP, REV>(li, cnt)] = INCL ? nx : ex;
        ex = nx;
    }
}

template <int OP, bool REV, bool INCL>
static hipError_t scan(const int32_t *in, int32_t *out, int64_t cnt, int32_t *bsum,
                       hipStream_t st) {
    if (cnt <= 0) return hipSuccess;
    const int64_t nb = ceil_div(cnt, kScanTile);
    hipLaunchKernelGGL((k_scan_reduce<OP, REV>), dim3((unsigned)nb), dim3(kScanThreads), 0, st,
                       in, cnt, bsum);
    hipLaunchKernelGGL(k_scan_bsum<OP>, dim3(1), dim3(1024), 0, st, bsum, nb);
    hipLaunchKernelGGL((k_scan_apply<OP, REV, INCL>), dim3((unsigned)nb), dim3(kScanThreads), 0,
                       st, in, out, cnt, bsum);
    return hipGetLastError();
}

// ------------------------------------------------------------- cell tables

// Slot s of the sorted keys starts a cell of the level (cell = key >> shift)
// when it is the first slot or its cell differs from the previous slot's.
__device__ inline int32_t cell_start_flag(const uint64_t *skeys, int64_t s, int shift) {
    return (s == 0 || (skeys[s] >> shift) != (skeys[s - 1] >> shift)) ? 1 : 0;
}

// Per scan tile: the number of cell starts (the flags are computed from the
// keys here and again in k_cell_emit rather than stored).  Slots are taken in
// rounds of kScanThreads consecutive ones, so that the loads coalesce.
__global__ __launch_bounds__(kScanThreads) void k_cell_reduce(int64_t n, const uint64_t *skeys,
                                                             int shift, int32_t *bsum) {
    const int64_t t0 = (int64_t)blockIdx.x * kScanTile;
    int32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t li = t0 + (int64_t)k * kScanThreads + threadIdx.x;
        if (li < n) acc += cell_start_flag(skeys, li, shift);
    }
    int32_t tot;
    block_excl<0, kScanThreads>(acc, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// With bsum holding the exclusive scan of the tiles' counts, the cell starting
// at slot s has index ci = the number of starts before s: records its id and
// first slot (tmp gets the first slots); the last slot stores the number of
// cells in *nc (and the caller's *n_cells).  The tile is taken in rounds of
// kScanThreads consecutive slots: a start's index within its round comes from
// the wave ballots, the rounds' counts are carried.
__global__ __launch_bounds__(kScanThreads) void k_cell_emit(int64_t n, const uint64_t *skeys,
                                                           int shift, const int32_t *bsum,
                                                           uint64_t *cell_id, int32_t *cell_start,
                                                           int32_t *tmp, int32_t *nc,
                                                           int32_t *n_cells) {
    constexpr int NW = kScanThreads / 64;
    __shared__ int32_t wcnt[kScanItems][NW];
    const int tid = threadIdx.x, w = tid >> 6;
    const int64_t t0 = (int64_t)blockIdx.x * kScanTile;
    int32_t f[kScanItems];
    uint64_t bm[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t li = t0 + (int64_t)k * kScanThreads + tid;
        f[k] = li < n ? cell_start_flag(skeys, li, shift) : 0;
        bm[k] = __ballot(f[k] != 0);
        if ((tid & 63) == 0) wcnt[k][w] = __popcll(bm[k]);
    }
    __syncthreads();
    int32_t carry = bsum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t li = t0 + (int64_t)k * kScanThreads + tid;
        int32_t before = carry;
        for (int v = 0; v < w; ++v) before += wcnt[k][v];
        const int32_t ci = before + (int32_t)mbcnt(bm[k]);
        if (f[k]) {
            tmp[ci] = (int32_t)li;
            if (cell_id) cell_id[ci] = skeys[li] >> shift;
            if (cell_start) cell_start[ci] = (int32_t)li;
        }
        for (int v = 0; v < NW; ++v) carry += wcnt[k][v];
        if (li == n - 1) {
            *nc = ci + f[k];
            if (n_cells) *n_cells = ci + f[k];
        }
    }
}

// Grid-stride over the cells, whose number is known only on the device: a
// grid sized for n would mostly launch blocks with nothing to do.
constexpr int kCellCountBlocks = 2048;

__global__ void k_cell_counts(int64_t n, const int32_t *nc_p, const int32_t *tmp,
                              int32_t *cell_count) {
    const int32_t nc = *nc_p;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nc; c += step) {
        const int32_t e = c + 1 < nc ? tmp[c + 1] : (int32_t)n;
        cell_count[c] = e - tmp[c];
    }
}

hipError_t run_contract_cells(Plan &pl, uint64_t *cell_id, int32_t *cell_start,
                              int32_t *cell_count, int32_t *n_cells, hipStream_t st) {
    const int64_t n = pl.n;
    const int shift = 3 * (pl.bits - pl.Lc);
    const unsigned nbk = (unsigned)ceil_div(n, 256);
    const int64_t nb = ceil_div(n, kScanTile);
    // the radix sort's second value buffer is free once the sort is done; the
    // control word 12 holds the number of cells
    int32_t *tmp = pl.perm == pl.valsA ? pl.valsB : pl.valsA;
    int32_t *nc = pl.ctrl + 12;
    hipLaunchKernelGGL(k_cell_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, st, n, pl.skeys,
                       shift, pl.bsum);
    hipLaunchKernelGGL(k_scan_bsum<0>, dim3(1), dim3(1024), 0, st, pl.bsum, nb);
    hipLaunchKernelGGL(k_cell_emit, dim3((unsigned)nb), dim3(kScanThreads), 0, st, n, pl.skeys,
                       shift, pl.bsum, cell_id, cell_start, tmp, nc, n_cells);
    if (cell_count)
        hipLaunchKernelGGL(k_cell_counts,
                           dim3(nbk < (unsigned)kCellCountBlocks ? nbk : (unsigned)kCellCountBlocks),
                           dim3(256), 0, st, n, nc, tmp, cell_count);
    return hipGetLastError();
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t cnt) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < cnt) p[i] = v;
}

__global__ void k_fill_u64(uint64_t *p, uint64_t v, int64_t cnt) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < cnt) p[i] = v;
}

__global__ void k_table_bounds(int64_t n, const uint64_t *skeys, int shift, int32_t *table) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint64_t c = skeys[s] >> shift;
    if (s == 0 || c != (skeys[s - 1] >> shift)) table[c] = (int32_t)s;
}

// table[c] = first sorted slot whose level-Ld cell is >= c (c = 0 .. 8^Ld).
hipError_t run_dense_table(Plan &pl, hipStream_t st) {
    const int64_t tn = pl.table_n;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)ceil_div(tn, 256)), dim3(256), 0, st, pl.table,
                       (int32_t)pl.n, tn);
    const int shift = 3 * (pl.bits - pl.Ld);
    hipLaunchKernelGGL(k_table_bounds, dim3((unsigned)ceil_div(pl.n, 256)), dim3(256), 0, st, pl.n,
                       pl.skeys, shift, pl.table);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return scan<1, true, true>(pl.table, pl.table, tn, pl.bsum, st);
}

// Largest group first: sort key (2^31 - 1 - size) << 16 | g, so that the
// ascending sort lists groups by decreasing size, ties by group id.
__global__ void k_group_lpt_keys(int32_t G, const int64_t *goff, uint64_t *keys, int32_t *vals) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= G) return;
    const int64_t ng = goff[g + 1] - goff[g];
    keys[g] = ((uint64_t)(0x7FFFFFFFll - ng) << 16) | (uint64_t)g;
    vals[g] = (int32_t)g;
}

// Work items of the batched form: the group at position k of the
// largest-first order (gorder[k]) owns items [gitems[k], gitems[k+1]), one per
// `segment` particles; gitems[G] = total.
__global__ void k_group_ntiles(int32_t G, const int64_t *goff, const int32_t *gorder,
                               int32_t seg, int32_t *cnt) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k > G) return;
    if (k == G) { cnt[k] = 0; return; }
    const int32_t g = gorder[k];
    const int64_t ng = goff[g + 1] - goff[g];
    cnt[k] = (int32_t)((ng + seg - 1) / seg);
}

hipError_t run_group_items(Plan &pl, const int64_t *goff, hipStream_t st) {
    const int64_t G = pl.G;
    hipLaunchKernelGGL(k_group_lpt_keys, dim3((unsigned)ceil_div(G, 256)), dim3(256), 0, st,
                       pl.G, goff, pl.gkeysA, pl.gvalsA);
    uint64_t *ko = nullptr;
    int32_t *vo = nullptr;
    // sizes < 2^31 and ids < 2^16: 47 key bits, 6 digit passes
    hipError_t e = radix_passes<4>(G, pl.nb_gsort, 6, pl.gkeysA, pl.gkeysB, pl.gvalsA,
                                   pl.gvalsB, pl.ghist, pl.digit_tot, st, &ko, &vo);
    if (e != hipSuccess) return e;
    pl.gorder = vo;
    const int64_t cnt = G + 1;
    hipLaunchKernelGGL(k_group_ntiles, dim3((unsigned)ceil_div(cnt, 256)), dim3(256), 0, st,
                       pl.G, goff, pl.gorder, pl.prm.segment, pl.gitems);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return scan<0, false, false>(pl.gitems, pl.gitems, cnt, pl.bsum, st);
}

hipError_t run_zero_u64(uint64_t *p, int64_t cnt, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)ceil_div(cnt, 256)), dim3(256), 0, st, p, 0ull,
                       cnt);
    return hipGetLastError();
}

hipError_t run_zero_i32(int32_t *p, int64_t cnt, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)ceil_div(cnt, 256)), dim3(256), 0, st, p, 0, cnt);
    return hipGetLastError();
}

}  // namespace sph
