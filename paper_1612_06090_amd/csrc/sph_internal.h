// Internal declarations of libsph (HIP, gfx950).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sph.h"

namespace sph {

constexpr double kPi = 3.14159265358979323846;
constexpr int kWave = 64;
// Particles per wave tile of the exact-K selection passes (4 lanes per
// particle, each with its own list or heap)
constexpr int kSelTile = 16;

// Radix sort geometry: one 256-thread block = 4 waves; a wave ranks ROUNDS
// rounds of 64 consecutive keys, so a block tile holds 4*64*ROUNDS keys.
constexpr int kSortThreads = 256;

// Smoothing kernels, W(r, h) = sigma/h^3 f(q), q = r/h < 1, weighted count
// n = count * sum f.  Pair terms are produced in a scaled form that needs no
// branch: f = fscale * fh and q f'(q) = gscale * gs.
template <int K>
struct Kern;

template <>
struct Kern<SPH_KERNEL_M4> {
    static constexpr double sigma = 8.0 / kPi;
    static constexpr double count = 32.0 / 3.0;
    static constexpr double fscale = 2.0, gscale = 6.0;
    // f = 2 (u^3 - 4 v^3), q f' = 6 q (4 v^2 - u^2), u = 1 - q, v = max(1/2 - q, 0):
    // one form for both pieces of the spline (beyond q = 1 both vanish to rounding)
    template <typename T>
    __device__ static void terms(T q, T /*q2*/, T &fh, T &gs) {
        const T u = T(1) - q;
        const T v = fmin(fmax(T(0.5) - q, T(0)), T(1));
        const T u2 = u * u, v2 = v * v;
        fh = fma(T(-4) * v, v2, u2 * u);
        gs = q * fma(T(4), v2, -u2);
    }
    // Binary32 sums of the scaled terms, added in place: s0 += f/2, s1 += q f'/6,
    // sr += m f/2, for q in [0, 1] (q = 1 gives exact zeros).  With
    // w = 4^(1/3) v, 4 v^3 = w^3 and 4 v^2 = 4^(1/3) w^2, so the factor 4 costs
    // no instruction, and q f'/6 = q (4^(1/3) w^2 - u^2) is fused into its sum.
    __device__ static void accum(float q, float /*q2*/, float m, float &s0, float &s1,
                                 float &sr) {
        constexpr float c = 1.587401051968199f;  // 4^(1/3)
        const float u = 1.0f - q;
        const float w = __builtin_fminf(__builtin_fmaxf(__builtin_fmaf(-c, q, 0.5f * c), 0.0f), 1.0f);
        const float u2 = u * u, w2 = w * w;
        const float fh = __builtin_fmaf(-w2, w, u2 * u);
        s0 += fh;
        s1 = __builtin_fmaf(q, __builtin_fmaf(c, w2, -u2), s1);
        sr = __builtin_fmaf(m, fh, sr);
    }
    // f and f'
    template <typename T>
    __device__ static void fd(T q, T &f, T &fp) {
        const T u = T(1) - q;
        const T v = fmin(fmax(T(0.5) - q, T(0)), T(1));
        const T u2 = u * u, v2 = v * v;
        f = T(2) * (u2 * u - T(4) * v * v2);
        fp = T(6) * (T(4) * v2 - u2);
    }
};

template <>
struct Kern<SPH_KERNEL_WENDLAND_C6> {
    static constexpr double sigma = 1365.0 / (64.0 * kPi);
    static constexpr double count = 1365.0 / 48.0;
    static constexpr double fscale = 1.0, gscale = -22.0;
    // f = u^8 (1 + 8q + 25q^2 + 32q^3), q f' = -22 q^2 u^7 (1 + 7q + 16q^2)
    template <typename T>
    __device__ static void terms(T q, T q2, T &fh, T &gs) {
        const T u = T(1) - q;
        const T u2 = u * u, u4 = u2 * u2;
        const T u7 = u4 * (u2 * u);
        const T P = fma(q, fma(q, fma(T(32), q, T(25)), T(8)), T(1));
        const T Q = fma(q, fma(T(16), q, T(7)), T(1));
        fh = (u7 * u) * P;
        gs = (q2 * u7) * Q;
    }
    // binary32 sums of the scaled terms, added in place (q = 1 gives zeros)
    __device__ static void accum(float q, float q2, float m, float &s0, float &s1,
                                 float &sr) {
        const float u = 1.0f - q;
        const float u2 = u * u, u4 = u2 * u2;
        const float u7 = u4 * (u2 * u);
        const float P = __builtin_fmaf(q, __builtin_fmaf(q, __builtin_fmaf(32.0f, q, 25.0f), 8.0f), 1.0f);
        const float Q = __builtin_fmaf(q, __builtin_fmaf(16.0f, q, 7.0f), 1.0f);
        const float fh = (u7 * u) * P;
        s0 += fh;
        s1 = __builtin_fmaf(q2 * u7, Q, s1);
        sr = __builtin_fmaf(m, fh, sr);
    }
    template <typename T>
    __device__ static void fd(T q, T &f, T &fp) {
        const T u = T(1) - q;
        const T u2 = u * u, u4 = u2 * u2;
        const T u7 = u4 * (u2 * u);
        f = (u7 * u) * (T(1) + q * (T(8) + q * (T(25) + T(32) * q)));
        fp = T(-22) * q * u7 * (T(1) + q * (T(7) + T(16) * q));
    }
};

// Particles per wave tile of the adjoint kernels.
constexpr int kAdjTile = 16;

// Scan geometry: 256 threads x 8 items per block.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

// Everything the host computes once per call: sizes, levels and the carved-up
// workspace.  Pointers are device addresses inside the caller's workspace.
struct Plan {
    sph_params prm;
    int64_t n = 0;
    int32_t G = 0;            // groups (0: one periodic set)
    bool grouped = false;
    int bits = 21;            // bits per axis of the Morton key
    int Lc = 1;               // cell level of the sort's cell table
    int Ld = 0;               // level of the dense start table (periodic only)
    int64_t table_n = 0;      // 8^Ld + 1 entries
    int sort_rounds = 4;      // radix rounds per wave
    int64_t sort_tile = 0;    // keys per radix block
    int64_t nb_sort = 0;      // radix blocks
    int64_t nb_scan_n = 0;    // scan blocks over n
    int64_t nb_scan_t = 0;    // scan blocks over table_n
    int64_t n_items = 0;      // work items of the density kernel (periodic)
    int grid = 0;             // persistent grid size
    // byte strides of the caller's per-particle arrays: inputs (x, y, z, m,
    // h_init, cotangents), floating outputs, int32 outputs
    int64_t in_stride = 8, out_stride = 8, out_stride_i = 4;

    uint64_t *keysA = nullptr, *keysB = nullptr;
    int32_t *valsA = nullptr, *valsB = nullptr;
    uint32_t *digit_tot = nullptr;  // digit totals of the group-order sort
    // single-sweep particle sort, one run cleared by one fill per sort:
    // look-back descriptors (256 per radix block), the digit counts of the
    // eight passes and the passes' tile counters (reduce-then-scan sorts of
    // small sets keep their per-tile histograms at its start)
    int32_t *sweep = nullptr;
    int64_t sweep_words = 0;     // int32 words of that run
    uint64_t *sweep_desc = nullptr;
    uint32_t *sweep_gh = nullptr;
    int32_t *sweep_ctr = nullptr;
    // sorted structure-of-arrays
    double4 *sp = nullptr;       // FP64: x, y, z, m per particle (one 32-byte record)
    double *sh0 = nullptr;
    // FP32C: per particle (qx, qy, qz, bits of the binary32 mass) and (fx, fy,
    // fz, 0): the integer grid cell and the binary32 fraction, 2 x 16 bytes
    int4 *qp = nullptr;
    float4 *fp = nullptr;
    int32_t *table = nullptr;
    int32_t *bsum = nullptr;     // block sums of scans
    double *frame = nullptr;     // per group: lo xyz, ext xyz, scale, pad (8 doubles)
    int32_t *gitems = nullptr;   // per group: first work item (G+1)
    int32_t *gorder = nullptr;   // groups in processing order, largest first (G)
    uint64_t *gkeysA = nullptr, *gkeysB = nullptr;  // group-order sort (G each)
    int32_t *gvalsA = nullptr, *gvalsB = nullptr;
    uint32_t *ghist = nullptr;
    int64_t nb_gsort = 0;        // radix blocks of the group-order sort
    int64_t *goff = nullptr;     // groups: the caller's offsets made well formed (G+1)
    int32_t *ctrl = nullptr;     // [0] work queue head, [8] exact-K tiles left, [12] cell count
                                 // of the sort's cell list, others reserved
    uint64_t *stats = nullptr;   // 4 x uint64 device counters
    double *adj = nullptr;       // adjoint, sorted order: alpha, beta, gamma, grad_rho, grad_h (5 x n)
    float4 *adj_rec = nullptr;   // adjoint, binary32 form: h, 1/h (grid units), alpha, beta (n)
    float *adj_g = nullptr;      //   and gamma (n)
    float *rmq = nullptr;        // adjoint: range-max table of h (grid units), rmq_levels x n
    int rmq_levels = 0;
    double *knn_h = nullptr;     // exact-K mode: count-stage h and status, sorted order
    int32_t *knn_st = nullptr;
    int32_t *knn_items = nullptr;  // exact-K mode: selection tiles left to the heap pass

    // after sorting
    uint64_t *skeys = nullptr;
    int32_t *perm = nullptr;
    size_t total = 0;
};

// Fills plan sizes and, when ws != nullptr, the pointers.  Returns SPH_OK or
// an error code (does not touch the device).
int make_plan(const sph_params *p, int64_t n, int32_t G, void *ws, Plan *out);

// sort.hip
// keys_out, perm_out: where the sorted keys and permutation end (the last
// radix pass writes there), else in the workspace
hipError_t run_keys_and_sort(Plan &pl, const int64_t *goff, const void *x, const void *y,
                             const void *z, hipStream_t st, uint64_t *keys_out = nullptr,
                             int32_t *perm_out = nullptr);
hipError_t run_permute(Plan &pl, const int64_t *goff, const void *x, const void *y,
                       const void *z, const void *m, const void *h0, bool fp32c,
                       hipStream_t st);
hipError_t run_contract_cells(Plan &pl, uint64_t *cell_id, int32_t *cell_start,
                              int32_t *cell_count, int32_t *n_cells, hipStream_t st);
hipError_t run_dense_table(Plan &pl, hipStream_t st);
hipError_t run_group_items(Plan &pl, const int64_t *goff, hipStream_t st);
hipError_t run_zero_u64(uint64_t *p, int64_t cnt, hipStream_t st);
hipError_t run_zero_i32(int32_t *p, int64_t cnt, hipStream_t st);
// Reads and clears the device's count of sort look-back waits that reached
// their bound (synchronous).
hipError_t read_sort_wait_faults(uint32_t *count);
hipError_t run_clean_offsets(const Plan &pl, const int64_t *goff, hipStream_t st);

// solve.hip
hipError_t run_solve(Plan &pl, const int64_t *goff, void *rho, void *h, void *nw,
                     int32_t *nngb, int32_t *status, uint64_t *stats, hipStream_t st);

// backward.hip
hipError_t run_backward(Plan &pl, const int64_t *goff, const void *h, const void *grad_rho,
                        const void *grad_h, void *gx, void *gy, void *gz, void *gm,
                        hipStream_t st);
hipError_t run_scatter(Plan &pl, const int64_t *goff, void *rho_s, void *rho_sym,
                       int32_t *nngb_s, hipStream_t st);
hipError_t run_backward_sorted(Plan &pl, const int64_t *goff, void *gx, void *gy, void *gz,
                               void *gm, hipStream_t st);
hipError_t run_force(Plan &pl, const int64_t *goff, const void *m, const void *rho,
                     const void *P, void *ax, void *ay, void *az, hipStream_t st);

// ---------------------------------------------------------------- helpers

// Interleave: bit k of v goes to bit 3k (21-bit input).
__host__ __device__ inline uint64_t spread3_21(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x001f00000000ffffull;
    v = (v | (v << 16)) & 0x001f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__host__ __device__ inline uint64_t morton3(uint64_t qx, uint64_t qy, uint64_t qz) {
    return (spread3_21(qx) << 2) | (spread3_21(qy) << 1) | spread3_21(qz);
}

// floor(t) clamped to [0, nmax - 1]; NaN -> 0.
__device__ inline uint32_t quantise(double t, uint32_t nmax) {
    if (!(t >= 0.0)) return 0u;
    if (t >= (double)nmax) return nmax - 1u;
    return (uint32_t)floor(t);
}

// Caller arrays: element i of p sits at byte i * stride (the packed stride is
// the element size; an array of particle structs gives the struct size, with
// p pointing at the field).
template <typename T>
__device__ inline double ld(const void *p, int64_t i, int64_t stride) {
    return (double)*reinterpret_cast<const T *>(static_cast<const char *>(p) + i * stride);
}

template <typename T>
__device__ inline void st(void *p, int64_t i, double v, int64_t stride) {
    *reinterpret_cast<T *>(static_cast<char *>(p) + i * stride) = (T)v;
}

__device__ inline void st_i32(int32_t *p, int64_t i, int32_t v, int64_t stride) {
    *reinterpret_cast<int32_t *>(reinterpret_cast<char *>(p) + i * stride) = v;
}

__device__ inline int lane_id() { return __lane_id(); }

__device__ inline uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ inline int readlane_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

// Values every lane of the wave already holds (results of a full-wave
// reduction or broadcast), moved to scalar registers.
__device__ inline float uniform_f(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}

__device__ inline double uniform_dbl(double v) {
    int2 b = __builtin_bit_cast(int2, v);
    b.x = __builtin_amdgcn_readfirstlane(b.x);
    b.y = __builtin_amdgcn_readfirstlane(b.y);
    return __builtin_bit_cast(double, b);
}

__device__ inline double readlane_d(double v, int l) {
    int2 a = __builtin_bit_cast(int2, v);
    a.x = __builtin_amdgcn_readlane(a.x, l);
    a.y = __builtin_amdgcn_readlane(a.y, l);
    return __builtin_bit_cast(double, a);
}

__device__ inline float readlane_f(float v, int l) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

// Value of v in lane `src` (a per-lane index), by bpermute.
// Square root of x > 0 (0 for x = 0) to within about an ulp: Goldschmidt's
// iteration for g ~ sqrt(x) and h ~ 1/(2 sqrt(x)) started from the hardware
// reciprocal square root (about binary32 accuracy), then one Newton
// correction of g.  For the pair terms of the binary64 sums, whose bound is
// 1e-12 relative; values that must match exactly keep sqrt().  x must be 0 or
// a normal number (squared distances of distinct particles are).
__device__ inline double sqrt_pos(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y;
    double h = 0.5 * y;
    const double r = __builtin_fma(-h, g, 0.5);
    g = __builtin_fma(g, r, g);
    h = __builtin_fma(h, r, h);
    const double d = __builtin_fma(-g, g, x);
    g = __builtin_fma(d, h, g);
    return x > 0.0 ? g : 0.0;
}

__device__ inline double readlane_bperm_d(double v, int src) {
    int2 a = __builtin_bit_cast(int2, v);
    a.x = __shfl(a.x, src, 64);
    a.y = __shfl(a.y, src, 64);
    return __builtin_bit_cast(double, a);
}

template <typename T>
__device__ inline T wave_max(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}

template <typename T>
__device__ inline T wave_min(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        T w = __shfl_xor(v, o, 64);
        v = w < v ? w : v;
    }
    return v;
}

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Inclusive prefix sum across the wave.
__device__ inline int wave_incl_scan(int v) {
    const int l = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int w = __shfl_up(v, o, 64);
        if (l >= o) v += w;
    }
    return v;
}

// Index of the last entry of excl[0..nr) that is <= g, for ascending excl
// with excl[0] <= g and a wave-uniform nr in [1, 64]: a branch-free binary
// descent over power-of-two steps (the steps not below nr are skipped by the
// whole wave).
__device__ inline int range_of(const int32_t *excl, int nr, int g) {
    int r = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
        if (step < nr) {
            const int t = r + step;
            const int ts = t < nr ? t : nr - 1;
            r = (t < nr && excl[ts] <= g) ? t : r;
        }
    }
    return r;
}

// Inclusive max-scan across the wave: Hillis-Steele within each row of 16
// lanes by DPP row shifts of 1, 2, 4 and 8, then the GFX9 row broadcasts of
// lane 15 (into rows 1 and 3) and lane 31 (into rows 2 and 3).  Lanes without
// a DPP source take INT_MIN.
__device__ inline int wave_max_scan(int v) {
    int t;
    t = __builtin_amdgcn_update_dpp(INT_MIN, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v = v > t ? v : t;
    t = __builtin_amdgcn_update_dpp(INT_MIN, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v = v > t ? v : t;
    t = __builtin_amdgcn_update_dpp(INT_MIN, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v = v > t ? v : t;
    t = __builtin_amdgcn_update_dpp(INT_MIN, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v = v > t ? v : t;
    t = __builtin_amdgcn_update_dpp(INT_MIN, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v = v > t ? v : t;
    t = __builtin_amdgcn_update_dpp(INT_MIN, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    v = v > t ? v : t;
    return v;
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace sph
