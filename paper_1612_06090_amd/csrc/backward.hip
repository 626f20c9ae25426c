// Adjoint of the density solve, with each smoothing length held on its
// implicit root n_i(h_i, x) = n_i(achieved) (the derivative of the converged
// recompute loop of Sec. IV-A, Listings 2/3, through Eq. 1).
//
// For a cotangent (gr, gh) on (rho, h):
//   lambda_i = -(gr_i drho_i/dh_i + gh_i) / (dn_i/dh_i)          (0 if dn/dh = 0)
//   alpha_i = gr_i sigma/h_i^4, beta_i = lambda_i C/h_i, gamma_i = gr_i sigma/h_i^3
//   (W = sigma/h^3 f(r/h), n = C sum f: M4 8/pi and 32/3, Wendland C6
//   1365/(64 pi) and 1365/48)
//   pair (i, j in N(i)): c_ij = f'(r/h_i) (alpha_i m_j + beta_i)
//   dL/dx_k = sum_{j: r < h_k} c_kj (x_k - x_j)/r + sum_{i: r < h_i} c_ik (x_k - x_i)/r
//   dL/dm_k = sum_{i: r < h_i} gamma_i f(r/h_i)          (self term included)
//
// Gather form, no atomics: phase 1 computes lambda and the coefficients of
// every particle; phase 2 gives each particle both its own neighbours
// (r < h_k) and its reverse neighbours (particles i whose own sphere reaches
// it, r < h_i, h_i != h_k).  The reverse set is found by a walk over the
// implicit octree of the Morton-sorted array: a node (key prefix = a
// contiguous range) is opened only if it comes within max(h_k, h_max(node))
// of some particle k of the tile, with h_max of any range read in O(1) from a
// range-max table.  Every candidate is visited once and tested against both
// radii.
//
// The pressure force of the variational (grad-h) SPH equations is the same
// adjoint: with h held on its count constraint, m_k a_k = -dE/dx_k for the
// thermal energy E = sum_i m_i u_i(rho_i), du/drho = P/rho^2, i.e. the
// position gradient for the cotangent gr_i = m_i P_i/rho_i^2, scaled by
// -1/m_k.
//
// A wave holds a tile of 16 consecutive sorted particles, each on 4 lanes
// that split every 64-candidate chunk between them (partial sums are folded
// across the 4 copies at the end).  The next chunk's candidates are loaded
// while the current one is evaluated.
#include "sph_internal.h"

namespace sph {

constexpr int kLeafMax = 32;   // a walk node with at most this many particles is a leaf
// walk stack capacity (overflowing nodes become leaves); the binary32 form
// gives half of it to the candidate staging buffer
template <int PREC>
constexpr int kWorkCap = PREC == SPH_FP32C ? 128 : 256;
constexpr float kSplitExtent = 4.0f;  // split particle ranges wider than this many radii
constexpr int kAdjP = kAdjTile;       // particles per wave tile
constexpr int kAdjS = 64 / kAdjP;     // lanes per particle
constexpr int kAdjWavesPerCU = 16;    // persistent waves per compute unit
static_assert(kAdjP * kAdjS == 64, "tile shape");

struct AdjArgs {
    int64_t n;
    int32_t G;
    const int64_t *goff;
    const uint64_t *skeys;
    const int32_t *perm;
    const double4 *sp;  // FP64: x, y, z, m
    const double *sh;
    const int4 *qp;     // FP32C: grid cell, mass bits
    const float4 *fp;   // FP32C: fraction
    const int32_t *table;
    int32_t Ld;
    const double *frame;
    const int32_t *gitems;
    const int32_t *gorder;
    int64_t n_items;
    const float *rmq;
    int32_t rmq_levels;
    double box;
    int32_t bits;
    double *alpha, *beta, *gamma;
    // binary32 form, written by pass 1 for pass 2: each particle's h and 1/h
    // in grid units, alpha, beta, and gamma, rounded as pass 2 uses them
    float4 *rec;
    float *recg;
    const double *grs, *ghs;
    int32_t phase;
    int32_t out_f32;
    void *gx, *gy, *gz, *gm;
    int64_t ost, ost_i;  // byte strides of the floating and int32 outputs
    int32_t *queue;
};

// max of rmq level 0 over [st, en), en > st
__device__ inline float range_hmax(const AdjArgs &a, int32_t st, int32_t en) {
    const int32_t len = en - st;
    const int k = 31 - __builtin_clz((unsigned)len);
    const float *t = a.rmq + (int64_t)k * a.n;
    const float u = t[st], v = t[en - (1 << k)];
    return u > v ? u : v;
}

// first slot in [b, e) whose key is >= k
__device__ inline int32_t lower_bound_key(const uint64_t *keys, int32_t b, int32_t e, uint64_t k) {
    while (b < e) {
        const int32_t mid = (b + e) >> 1;
        if (keys[mid] < k) b = mid + 1; else e = mid;
    }
    return b;
}

template <int PREC>
struct AdjCand;

template <>
struct AdjCand<SPH_FP64> {
    double4 p;     // x, y, z (absolute), m
    double4 s;     // image shift (absolute), unused
    double4 h;     // h, 1/h, alpha, beta
    double g;      // gamma
};

template <>
struct AdjCand<SPH_FP32C> {
    float4 p;      // x, y, z relative to the tile origin (grid units), m
    float4 h;      // h (grid units), 1/h (grid units), alpha, beta (absolute)
    float g;       // gamma
};

// Candidates waiting to be evaluated.  Binary64: one chunk of 64 as streamed.
// Binary32: the candidates that passed the range's region test (its box
// widened by the larger of the range's radius and the candidate's own),
// appended in load rounds of 64 and evaluated 64 at a time, so up to 127 wait.
template <int PREC>
struct AdjStage {
    AdjCand<PREC> cand[64];
};

template <>
struct AdjStage<SPH_FP32C> {
    float4 p[128];  // x, y, z (grid units, range origin), m
    float4 h[128];  // h, 1/h (grid units), alpha, beta
    float g[128];   // gamma
};

template <int PREC>
struct AdjLDS {
    int32_t wk_st[kWorkCap<PREC>], wk_en[kWorkCap<PREC>], wk_c[kWorkCap<PREC>][3],
        wk_L[kWorkCap<PREC>];
    int32_t rg_start[64], rg_excl[64], rg_code[64], rg_mark[64];
    // the range's spheres: x, y, z (grid units, range origin), radius; slots
    // of particles outside the range hold a sphere that reaches nothing
    float4 sp[kAdjP];
    // each particle of the tile: grid cell and radius bits, fraction (read
    // once per range rather than held in registers through the walk)
    int4 oq[kAdjP];
    float4 of[kAdjP];
    float4 box[2];        // binary32: the range's box (min, max) and Ht^2
    AdjStage<PREC> st;
};

// PHASE 1 and 2: the two passes of the adjoint; 3: the scatter form
template <int PREC, bool GROUPED, int KERNEL, int PHASE>
__global__ __launch_bounds__(64) void k_adjoint(AdjArgs a) {
    using KT = Kern<KERNEL>;
    __shared__ AdjLDS<PREC> S;
    const int l = threadIdx.x;
    const int p = l & (kAdjP - 1);  // particle slot of this lane
    const int kk = l / kAdjP;       // copy: this lane's share of each chunk
    constexpr uint64_t kTileMask = (1ull << kAdjP) - 1ull;
    const int B = a.bits;

    for (;;) {
        int item = 0;
        if (l == 0) item = atomicAdd(a.queue, 1);
        item = __builtin_amdgcn_readlane(item, 0);
        const int64_t n_items = GROUPED ? (int64_t)a.gitems[a.G] : a.n_items;
        if (item >= n_items) break;

        int64_t b, e;
        int32_t g = 0;
        double org0 = 0.0, org1 = 0.0, org2 = 0.0, sc;
        if (!GROUPED) {
            b = (int64_t)item * kAdjP;
            e = b + kAdjP < a.n ? b + kAdjP : a.n;
            sc = 2097152.0 / a.box;
        } else {
            int32_t lo = 0, hi = a.G - 1;
            while (lo < hi) {
                const int32_t mid = (lo + hi + 1) >> 1;
                if (a.gitems[mid] <= item) lo = mid; else hi = mid - 1;
            }
            g = a.gorder[lo];  // position lo of the largest-first order
            b = a.goff[g] + (int64_t)(item - a.gitems[lo]) * kAdjP;
            e = b + kAdjP < a.goff[g + 1] ? b + kAdjP : a.goff[g + 1];
            const double *f = a.frame + 8 * (int64_t)g;
            org0 = uniform_dbl(f[0]); org1 = uniform_dbl(f[1]); org2 = uniform_dbl(f[2]);
            sc = uniform_dbl(f[6]);
        }
        const int64_t s = b + p;
        const bool mine = s < e;
        double xk = 0.0, yk = 0.0, zk = 0.0, mk = 0.0, hk = 1.0;
        int32_t qxk = 0, qyk = 0, qzk = 0;
        float fxk = 0.f, fyk = 0.f, fzk = 0.f;
        bool valid = false;
        if (mine) {
            hk = a.sh[s];
            if constexpr (PREC == SPH_FP64) {
                const double4 p4 = a.sp[s];
                xk = p4.x; yk = p4.y; zk = p4.z; mk = p4.w;
                valid = !isnan(xk);
                const double tx = (xk - org0) * sc, ty = (yk - org1) * sc, tz = (zk - org2) * sc;
                qxk = valid ? (int32_t)floor(tx) : 0;
                qyk = valid ? (int32_t)floor(ty) : 0;
                qzk = valid ? (int32_t)floor(tz) : 0;
                fxk = (float)(tx - (double)qxk);
                fyk = (float)(ty - (double)qyk);
                fzk = (float)(tz - (double)qzk);
            } else {
                const int4 q4 = a.qp[s];
                const float4 f4 = a.fp[s];
                qxk = q4.x; qyk = q4.y; qzk = q4.z;
                fxk = f4.x; fyk = f4.y; fzk = f4.z;
                mk = (double)__int_as_float(q4.w);
                valid = !isnan(fxk);
            }
        }
        const uint64_t vm = __ballot(valid) & kTileMask;
        double ak = 0.0, bk = 0.0;  // own alpha, beta (phase 2)
        float akf = 0.f, bkf = 0.f;
        if constexpr (PREC == SPH_FP32C) {
            if (PHASE == 2 && valid) {
                const float4 r4 = a.rec[s];
                akf = r4.z;
                bkf = r4.w;
            }
        } else {
            if (PHASE == 2 && valid) { ak = a.alpha[s]; bk = a.beta[s]; }
        }
        const float mkf = (float)mk;

        // per-lane partial sums: phase 1 -> S1, R, T ; phase 2 -> gx, gy, gz, gm
        double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;

        const double hq = hk * sc;  // own h in grid units
        const float Hk = (float)(hq * (1.0 + 0x1p-16)) + 0x1p-10f;
        const float hk2f = (float)(hq * hq);
        const float hkinvf = (float)(1.0 / hq);
        const double hk2 = hk * hk, hkinv = 1.0 / hk;
        if (kk == 0) {
            S.oq[p] = make_int4(qxk, qyk, qzk, __float_as_int(Hk));
            S.of[p] = make_float4(fxk, fyk, fzk, 0.f);
        }
        __builtin_amdgcn_wave_barrier();
        const int64_t gbase = GROUPED ? a.goff[g] : 0;
        const int64_t gend = GROUPED ? a.goff[g + 1] : a.n;
        float hall = 0.f;  // largest h of the set (phase 2: any sphere may reach)
        if (PHASE >= 2 && vm != 0)
            hall = uniform_f(range_hmax(a, (int32_t)gbase, (int32_t)gend));

        // Particle ranges of the tile, each walked on its own.  A range whose
        // bounding box is wide compared with its radius (it straddles distant
        // parts of the Morton order) is split in halves of its valid
        // particles: the walk region stays compact and the binary32
        // coordinates relative to the range's origin keep the precision of the
        // local separation.
        // The ranges still pending always tile [la, kAdjP) in order (depth
        // first, lower half first), so they are kept as the bit set of their
        // first slots.
        uint32_t starts = vm != 0 ? 1u : 0u;
        while (starts) {
            const int la = __builtin_ctz(starts);
            starts &= starts - 1;
            const int lb = starts ? __builtin_ctz(starts) : kAdjP;
            const bool in_sub = valid && p >= la && p < lb;
            const uint64_t sm = __ballot(in_sub) & kTileMask;
            if (sm == 0) continue;
            const int first = __ffsll((unsigned long long)sm) - 1;
            const int4 oq = S.oq[p];
            const float4 of = S.of[p];
            const float Hk = __int_as_float(oq.w);
            const int32_t t0 = readlane_i(oq.x, first), t1 = readlane_i(oq.y, first),
                          t2 = readlane_i(oq.z, first);
            const float pk0 = (float)(oq.x - t0) + of.x;
            const float pk1 = (float)(oq.y - t1) + of.y;
            const float pk2 = (float)(oq.z - t2) + of.z;
            const float mn0 = uniform_f(wave_min(in_sub ? pk0 : INFINITY));
            const float mx0 = uniform_f(wave_max(in_sub ? pk0 : -INFINITY));
            const float mn1 = uniform_f(wave_min(in_sub ? pk1 : INFINITY));
            const float mx1 = uniform_f(wave_max(in_sub ? pk1 : -INFINITY));
            const float mn2 = uniform_f(wave_min(in_sub ? pk2 : INFINITY));
            const float mx2 = uniform_f(wave_max(in_sub ? pk2 : -INFINITY));
            const float Ht = uniform_f(wave_max(in_sub ? Hk : 0.f));
            const float ext = fmaxf(mx0 - mn0, fmaxf(mx1 - mn1, mx2 - mn2));
            if (ext > kSplitExtent * Ht && __popcll(sm) > 1) {
                // lower half of the valid particles, then the upper half
                uint64_t t = sm;
                for (int k = __popcll(sm) / 2; k > 0; --k) t &= t - 1;
                const int mid = __ffsll((unsigned long long)t) - 1;
                starts |= (1u << la) | (1u << mid);
                continue;
            }
            __syncthreads();
            if (kk == 0)
                S.sp[p] = in_sub ? make_float4(pk0, pk1, pk2, Hk) : make_float4(1e30f, 1e30f, 1e30f, 0.f);
            if (l == 0) {
                S.box[0] = make_float4(mn0, mn1, mn2, Ht * Ht);
                S.box[1] = make_float4(mx0, mx1, mx2, 0.f);
            }
            __syncthreads();

            int wsz = 0;   // work stack size (uniform)
            int nl = 0;    // leaves collected (uniform)
            float Rroot = PHASE >= 2 && hall > Ht ? hall : Ht;
            Rroot = Rroot * (1.0f + 0x1p-12f) + 1.0f;

            // one candidate of the leaf list (flat index gidx) into registers
            auto load_cand = [&](int gidx, int total, int nleaf, AdjCand<PREC> &c) {
                if (gidx < total) {
                    const int lo = range_of(S.rg_excl, nleaf, gidx);
                    const int64_t j = (int64_t)S.rg_start[lo] + (gidx - S.rg_excl[lo]);
                    const int cc = S.rg_code[lo];
                    const int sh0 = (cc & 3) - 1, sh1 = ((cc >> 2) & 3) - 1, sh2 = ((cc >> 4) & 3) - 1;
                    const double hj = a.sh[j];
                    const double aj = PHASE == 2 ? a.alpha[j] : 0.0;
                    const double bj = PHASE == 2 ? a.beta[j] : 0.0;
                    const double gj = PHASE >= 2 ? a.gamma[j] : 0.0;
                    if constexpr (PREC == SPH_FP64) {
                        c.p = a.sp[j];
                        c.s = make_double4((double)sh0 * a.box, (double)sh1 * a.box,
                                           (double)sh2 * a.box, 0.0);
                        c.h = make_double4(hj, 1.0 / hj, aj, bj);
                        c.g = gj;
                    } else {
                        const int32_t W = 1 << B;
                        const double hqj = hj * sc;
                        const int4 q4 = a.qp[j];
                        const float4 f4 = a.fp[j];
                        c.p = make_float4((float)(q4.x + sh0 * W - t0) + f4.x,
                                          (float)(q4.y + sh1 * W - t1) + f4.y,
                                          (float)(q4.z + sh2 * W - t2) + f4.z,
                                          __int_as_float(q4.w));
                        c.h = make_float4((float)hqj, (float)(1.0 / hqj), (float)aj, (float)bj);
                        c.g = (float)gj;
                    }
                } else {
                    if constexpr (PREC == SPH_FP64) {
                        c.p = make_double4(INFINITY, INFINITY, INFINITY, 0.0);
                        c.s = make_double4(0.0, 0.0, 0.0, 0.0);
                        c.h = make_double4(1.0, 1.0, 0.0, 0.0);
                        c.g = 0.0;
                    } else {
                        c.p = make_float4(INFINITY, INFINITY, INFINITY, 0.f);
                        c.h = make_float4(1.f, 1.f, 0.f, 0.f);
                        c.g = 0.f;
                    }
                }
            };

            // binary32 candidate at stream position gidx of range rr
            auto load_cand_r = [&](int gidx, int rr, AdjCand<PREC> &c) {
                const int64_t j = (int64_t)S.rg_start[rr] + (gidx - S.rg_excl[rr]);
                const int cc = S.rg_code[rr];
                const int sh0 = (cc & 3) - 1, sh1 = ((cc >> 2) & 3) - 1, sh2 = ((cc >> 4) & 3) - 1;
                if constexpr (PREC == SPH_FP32C) {
                    const int32_t W = 1 << B;
                    const int4 q4 = a.qp[j];
                    const float4 f4 = a.fp[j];
                    c.p = make_float4((float)(q4.x + sh0 * W - t0) + f4.x,
                                      (float)(q4.y + sh1 * W - t1) + f4.y,
                                      (float)(q4.z + sh2 * W - t2) + f4.z,
                                      __int_as_float(q4.w));
                    if (PHASE == 2) {
                        const float4 hr = a.rec[j];
                        c.h = make_float4(hr.x, hr.y, hr.z, hr.w);
                        c.g = a.recg[j];
                    } else if (PHASE == 3) {
                        const double hqj = a.sh[j] * sc;
                        c.h = make_float4((float)hqj, (float)(1.0 / hqj), 0.f, 0.f);
                        c.g = (float)a.gamma[j];
                    } else {
                        c.h = make_float4(1.f, 1.f, 0.f, 0.f);
                        c.g = 0.f;
                    }
                }
            };

            // the pair terms of one LDS chunk for this lane's share of it
            auto eval_chunk = [&](int mc) {
                const int nu = (mc + kAdjS - 1) / kAdjS;
                if constexpr (PREC == SPH_FP64) {
                    for (int u = 0; u < nu; ++u) {
                        const AdjCand<SPH_FP64> c = S.st.cand[u * kAdjS + kk];
                        const double dx = (c.p.x - xk) + c.s.x;
                        const double dy = (c.p.y - yk) + c.s.y;
                        const double dz = (c.p.z - zk) + c.s.z;
                        const double r2 = (dx * dx + dy * dy) + dz * dz;
                        const bool in1 = r2 < hk2;
                        if (PHASE == 1) {
                            if (in1) {
                                const double q = sqrt(r2) * hkinv;
                                double f, fp;
                                KT::template fd<double>(q, f, fp);
                                acc0 += q * fp;
                                acc1 += c.p.w * f;
                                acc2 += c.p.w * q * fp;
                            }
                        } else if (PHASE == 3) {
                            // scatter form: gather sum at h_k, spread sum at h_j
                            const bool in2 = r2 < c.h.x * c.h.x;
                            if (in1 || in2) {
                                const double r = sqrt(r2);
                                double f1, fp1, f2, fp2;
                                KT::template fd<double>(fmin(r * hkinv, 1.0), f1, fp1);
                                KT::template fd<double>(fmin(r * c.h.y, 1.0), f2, fp2);
                                acc0 += in1 ? c.p.w * f1 : 0.0;
                                acc1 += in2 ? c.g * f2 : 0.0;
                                acc2 += in2 ? 1.0 : 0.0;
                            }
                        } else {
                            const bool in2 = r2 < c.h.x * c.h.x;
                            if (in1 || in2) {
                                const double r = sqrt(r2);
                                double f1, fp1, f2, fp2;
                                KT::template fd<double>(fmin(r * hkinv, 1.0), f1, fp1);
                                KT::template fd<double>(fmin(r * c.h.y, 1.0), f2, fp2);
                                const double c1 = in1 ? fp1 * (ak * c.p.w + bk) : 0.0;
                                const double c2 = in2 ? fp2 * (c.h.z * mk + c.h.w) : 0.0;
                                acc3 += in2 ? c.g * f2 : 0.0;
                                const double w = r > 0.0 ? (c1 + c2) / r : 0.0;
                                acc0 -= w * dx;
                                acc1 -= w * dy;
                                acc2 -= w * dz;
                            }
                        }
                    }
                } else {
                    // round partial sums in binary32 (at most 16 terms per lane),
                    // folded into binary64.  Branch free: with one particle-candidate
                    // pair per lane a wave almost always holds an in-range pair, so
                    // a branch would skip nothing; out of range, q is clamped to 1,
                    // where f and f' vanish, and the selects give exact zeros
                    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
                    if (PHASE == 1) {
#pragma unroll 4
                        for (int u = 0; u < nu; ++u) {
                            const float4 cp = S.st.p[u * kAdjS + kk];
                            const float dx = cp.x - pk0, dy = cp.y - pk1, dz = cp.z - pk2;
                            const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
                            const bool in1 = r2 < hk2f;
                            const float q = fminf(__builtin_amdgcn_sqrtf(r2) * hkinvf, 1.0f);
                            float f, fp;
                            KT::template fd<float>(q, f, fp);
                            const float qfp = in1 ? q * fp : 0.f;
                            const float fs = in1 ? f : 0.f;
                            s0 += qfp;
                            s1 = __builtin_fmaf(cp.w, fs, s1);
                            s2 = __builtin_fmaf(cp.w, qfp, s2);
                        }
                    } else if (PHASE == 3) {
#pragma unroll 2
                        for (int u = 0; u < nu; ++u) {
                            const int t = u * kAdjS + kk;
                            const float4 cp = S.st.p[t];
                            const float4 ch = S.st.h[t];
                            const float cg = S.st.g[t];
                            const float dx = cp.x - pk0, dy = cp.y - pk1, dz = cp.z - pk2;
                            const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
                            const bool in1 = r2 < hk2f;
                            const bool in2 = r2 < ch.x * ch.x;
                            const float r = __builtin_amdgcn_sqrtf(r2);
                            float f1, fp1, f2, fp2;
                            KT::template fd<float>(fminf(r * hkinvf, 1.0f), f1, fp1);
                            KT::template fd<float>(fminf(r * ch.y, 1.0f), f2, fp2);
                            s0 = __builtin_fmaf(in1 ? cp.w : 0.f, f1, s0);
                            s1 = __builtin_fmaf(in2 ? cg : 0.f, f2, s1);
                            s2 += in2 ? 1.f : 0.f;
                        }
                    } else {
#pragma unroll 1
                        for (int u = 0; u < nu; ++u) {
                            const int t = u * kAdjS + kk;
                            const float4 cp = S.st.p[t];
                            const float4 ch = S.st.h[t];
                            const float cg = S.st.g[t];
                            const float dx = cp.x - pk0, dy = cp.y - pk1, dz = cp.z - pk2;
                            const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
                            const bool in1 = r2 < hk2f;
                            const bool in2 = r2 < ch.x * ch.x;
                            const float r = __builtin_amdgcn_sqrtf(r2);
                            const float rinv = r > 0.f ? __builtin_amdgcn_rcpf(r) : 0.f;
                            float f1, fp1, f2, fp2;
                            KT::template fd<float>(fminf(r * hkinvf, 1.0f), f1, fp1);
                            KT::template fd<float>(fminf(r * ch.y, 1.0f), f2, fp2);
                            const float c1 = in1 ? fp1 * __builtin_fmaf(akf, cp.w, bkf) : 0.f;
                            const float c2 = in2 ? fp2 * __builtin_fmaf(ch.z, mkf, ch.w) : 0.f;
                            s3 = __builtin_fmaf(in2 ? cg : 0.f, f2, s3);
                            const float w = (c1 + c2) * rinv;
                            s0 = __builtin_fmaf(-w, dx, s0);
                            s1 = __builtin_fmaf(-w, dy, s1);
                            s2 = __builtin_fmaf(-w, dz, s2);
                        }
                    }
                    acc0 += (double)s0;
                    acc1 += (double)s1;
                    acc2 += (double)s2;
                    acc3 += (double)s3;
                }
            };

            // stream the collected leaves (ranges) through LDS.  Binary64: one
            // chunk of 64 candidates ahead in registers.  Binary32: load rounds of
            // 64; a candidate farther than max(Ht, its own h) from the range's
            // box (the exact binary32 coordinates of its spheres) reaches no
            // sphere of the range and no sphere of the range reaches it, so only
            // the others are staged (ballot slots) and evaluated 64 at a time
            int staged = 0;  // binary32: candidates waiting in the staging buffer
            auto eval_staged = [&]() {
                __syncthreads();
                if (in_sub) eval_chunk(64);
                __syncthreads();
                // the entries past the round move to the front
                if constexpr (PREC == SPH_FP32C) {
                    if (l < staged - 64) {
                        const float4 tp = S.st.p[64 + l], th = S.st.h[64 + l];
                        const float tg = S.st.g[64 + l];
                        S.st.p[l] = tp; S.st.h[l] = th; S.st.g[l] = tg;
                    }
                }
                staged -= 64;
                __syncthreads();
            };
            auto stream_leaves = [&](int nleaf) {
                const int cnt = l < nleaf ? S.rg_excl[l] : 0;  // rg_excl holds counts here
                const int incl = wave_incl_scan(cnt);
                const int total = __builtin_amdgcn_readlane(incl, 63);
                __syncthreads();
                if (l < nleaf) S.rg_excl[l] = incl - cnt;
                __syncthreads();
                if constexpr (PREC == SPH_FP64) {
                    AdjCand<PREC> nxt;
                    load_cand(l, total, nleaf, nxt);
                    for (int cbase = 0; cbase < total; cbase += 64) {
                        __syncthreads();
                        S.st.cand[l] = nxt;
                        __syncthreads();
                        if (cbase + 64 < total) load_cand(cbase + 64 + l, total, nleaf, nxt);
                        const int mc = total - cbase < 64 ? total - cbase : 64;
                        if (in_sub) eval_chunk(mc);
                    }
                } else {
                    const int rstart = l < nleaf ? S.rg_excl[l] : INT_MAX;
                    int rcarry = 0;
                    for (int cbase = 0; cbase < total; cbase += 64) {
                        // the range of each slot: marks at range starts, carried
                        // forward by a wave max-scan
                        S.rg_mark[l] = -1;
                        const int pos = rstart - cbase;
                        if (pos >= 0 && pos < 64) S.rg_mark[pos] = l;
                        __builtin_amdgcn_wave_barrier();
                        int rr = wave_max_scan(S.rg_mark[l]);
                        rr = rr > rcarry ? rr : rcarry;
                        rcarry = __builtin_amdgcn_readlane(rr, 63);
                        const int gidx = cbase + l;
                        bool keep = false;
                        AdjCand<PREC> c{};
                        if (gidx < total) {
                            load_cand_r(gidx, rr, c);
                            const float4 bl = S.box[0], bh = S.box[1];
                            const float ex = c.p.x - fminf(fmaxf(c.p.x, bl.x), bh.x);
                            const float ey = c.p.y - fminf(fmaxf(c.p.y, bl.y), bh.y);
                            const float ez = c.p.z - fminf(fmaxf(c.p.z, bl.z), bh.z);
                            const float R2 = PHASE >= 2 ? fmaxf(bl.w, c.h.x * c.h.x) : bl.w;
                            keep = __builtin_fmaf(ex, ex, __builtin_fmaf(ey, ey, ez * ez)) <=
                                   R2 * (1.0f + 0x1p-12f);
                        }
                        const uint64_t km = __ballot(keep);
                        if (keep) {
                            const int slot = staged + (int)mbcnt(km);
                            S.st.p[slot] = c.p;
                            S.st.h[slot] = c.h;
                            S.st.g[slot] = c.g;
                        }
                        staged += __popcll(km);
                        if (staged >= 64) eval_staged();
                    }
                }
            };
            // the range's last, partial round: slots past the staged candidates
            // hold padding, a candidate so far away (finite, so that the zero
            // pair weight times its offset stays zero; its r^2 overflows to
            // infinity) that it is never in range
            auto flush_staged = [&]() {
                if (staged > 0) {
                    if constexpr (PREC == SPH_FP32C) {
                        if (l >= staged) {
                            S.st.p[l] = make_float4(1e30f, 1e30f, 1e30f, 0.f);
                            S.st.h[l] = make_float4(1.f, 1.f, 0.f, 0.f);
                            S.st.g[l] = 0.f;
                        }
                    }
                    __syncthreads();
                    if (in_sub) eval_chunk(staged);
                    __syncthreads();
                    staged = 0;
                }
            };

            // node test: does the node box (grid units, relative to the range
            // origin) come within the radius of some sphere of the range -- its
            // own h (phase 1), or max(h, the node's largest h) (phase 2)?
            // (cell coordinates at level L, images included, and their corners
            // in grid units stay within [-2^22, 2^23): 32 bits suffice)
            auto node_pass = [&](int32_t c0, int32_t c1, int32_t c2, int L, int32_t st, int32_t en) {
                const int ex = B - L;
                const int32_t sd = 1 << ex;
                const float side = (float)sd;
                const float lo0 = (float)(c0 * sd - t0), lo1 = (float)(c1 * sd - t1),
                            lo2 = (float)(c2 * sd - t2);
                const float hm = PHASE >= 2 ? range_hmax(a, st, en) : 0.f;
                // slack covers the binary32 rounding of tile coordinates (up to
                // 2^-3 grid units at 2^21) and of the node corners
                const float slack = side * 0x1p-12f + 1.0f;
                // every slot, unrolled, so that the sphere reads issue together
                // (a far slot's distance squares to infinity and never passes)
                bool pass = false;
#pragma unroll
                for (int i = 0; i < kAdjP; ++i) {
                    const float4 q = S.sp[i];
                    const float H = fmaxf(q.w, hm) * (1.0f + 0x1p-12f) + slack;
                    const float g0 = fmaxf(0.f, fmaxf(lo0 - q.x, q.x - (lo0 + side)));
                    const float g1 = fmaxf(0.f, fmaxf(lo1 - q.y, q.y - (lo1 + side)));
                    const float g2 = fmaxf(0.f, fmaxf(lo2 - q.z, q.z - (lo2 + side)));
                    pass = pass | (g0 * g0 + g1 * g1 + g2 * g2 <= H * H);
                }
                return pass;
            };

            // append passing nodes of this round: leaves to the leaf list, the rest
            // to the work stack (a full stack turns them into leaves)
            auto place = [&](bool pass, bool leaf, int32_t st, int32_t en, int32_t c0, int32_t c1,
                             int32_t c2, int L) {
                uint64_t wm = __ballot(pass && !leaf);
                const int nw = __popcll(wm);
                if (wsz + nw > kWorkCap<PREC>) {
                    leaf = leaf || pass;
                    wm = 0;
                }
                const uint64_t lm = __ballot(pass && leaf);
                const int nlf = __popcll(lm);
                if (nl + nlf > 64) {
                    stream_leaves(nl);
                    nl = 0;
                }
                __syncthreads();
                if ((wm >> l) & 1ull) {
                    const int k = wsz + (int)mbcnt(wm);
                    S.wk_st[k] = st;
                    S.wk_en[k] = en;
                    S.wk_c[k][0] = c0;
                    S.wk_c[k][1] = c1;
                    S.wk_c[k][2] = c2;
                    S.wk_L[k] = L;
                }
                if ((lm >> l) & 1ull) {
                    const int k = nl + (int)mbcnt(lm);
                    int code = 0;
                    if (!GROUPED) {
                        const int s0 = (int)(c0 >> L), s1 = (int)(c1 >> L), s2 = (int)(c2 >> L);
                        code = (s0 + 1) | ((s1 + 1) << 2) | ((s2 + 1) << 4);
                    } else {
                        code = 1 | (1 << 2) | (1 << 4);
                    }
                    S.rg_start[k] = st;
                    S.rg_excl[k] = en - st;  // counts; turned into prefix sums on streaming
                    S.rg_code[k] = code;
                }
                __syncthreads();
                wsz += __popcll(wm);
                nl += nlf;
            };

            // expand the work stack: pop up to 8 nodes, one lane per child
            auto expand_all = [&]() {
                while (wsz > 0) {
                    const int n8 = wsz < 8 ? wsz : 8;
                    const int base = wsz - n8;
                    const int nd = l >> 3, ch = l & 7;
                    bool pass = false, leaf = false;
                    int32_t st = 0, en = 0, pen = 0;
                    int32_t c0 = 0, c1 = 0, c2 = 0;
                    int L = 0;
                    if (nd < n8) {
                        const int k = base + nd;
                        const int32_t pst = S.wk_st[k];
                        pen = S.wk_en[k];
                        const int pL = S.wk_L[k];
                        const int32_t p0 = S.wk_c[k][0], p1 = S.wk_c[k][1], p2 = S.wk_c[k][2];
                        L = pL + 1;
                        c0 = 2 * p0 + ((ch >> 2) & 1);
                        c1 = 2 * p1 + ((ch >> 1) & 1);
                        c2 = 2 * p2 + (ch & 1);
                        // key range of the child: its Morton prefix (wrapped) at level L
                        const int32_t m = (int32_t)((1u << L) - 1u);
                        const uint64_t cm = morton3((uint64_t)(c0 & m), (uint64_t)(c1 & m),
                                                    (uint64_t)(c2 & m));
                        if (!GROUPED && L <= a.Ld) {
                            const int sh = 3 * (a.Ld - L);
                            st = a.table[cm << sh];
                            en = a.table[(cm + 1) << sh];
                        } else {
                            const int ks = 3 * (B - L);
                            const uint64_t gb = GROUPED ? ((uint64_t)(uint32_t)g << 48) : 0ull;
                            st = lower_bound_key(a.skeys, pst, pen, gb + (cm << ks));
                        }
                    }
                    if (GROUPED || a.Ld < B) {
                        // searched children end where the next sibling starts
                        const int32_t nst = __shfl_down(st, 1, 64);
                        if (nd < n8 && (GROUPED || L > a.Ld)) en = ch == 7 ? pen : nst;
                    }
                    if (nd < n8) {
                        pass = en > st && node_pass(c0, c1, c2, L, st, en);
                        leaf = en - st <= kLeafMax || L >= B;
                    }
                    __syncthreads();
                    wsz = base;
                    place(pass, leaf, st, en, c0, c1, c2, L);
                }
            };

            // roots: periodic -- the cell images at level Lr meeting the region
            // (range box +- Rroot), Lr the finest level (at most that of the
            // dense table) whose cells cover the region's width in 6; groups --
            // the group itself (level 0).  Each batch of 64 roots is walked in turn.
            if (!GROUPED) {
                const float wdt = fmaxf(mx0 - mn0, fmaxf(mx1 - mn1, mx2 - mn2)) + 2.0f * Rroot;
                int ex = 0;
                while (ex < B - 1 && 6.0f * (float)(1 << ex) < wdt) ++ex;
                int Lr = B - ex;
                if (Lr > a.Ld) Lr = a.Ld;
                if (Lr < 1) Lr = 1;
                ex = B - Lr;
                // (grid coordinates of the region stay within [-2^22, 2^23))
                const int32_t lo0 = (t0 + (int32_t)floorf(mn0 - Rroot) - 1) >> ex;
                const int32_t lo1 = (t1 + (int32_t)floorf(mn1 - Rroot) - 1) >> ex;
                const int32_t lo2 = (t2 + (int32_t)floorf(mn2 - Rroot) - 1) >> ex;
                const int32_t hi0 = (t0 + (int32_t)floorf(mx0 + Rroot) + 1) >> ex;
                const int32_t hi1 = (t1 + (int32_t)floorf(mx1 + Rroot) + 1) >> ex;
                const int32_t hi2 = (t2 + (int32_t)floorf(mx2 + Rroot) + 1) >> ex;
                const int32_t nx = hi0 - lo0 + 1, ny = hi1 - lo1 + 1, nz = hi2 - lo2 + 1;
                const int32_t nroot = nx * ny * nz;  // at most 9^3 (6^3 at level 1)
                const int32_t msk = (int32_t)((1u << Lr) - 1u);
                const int sh = 3 * (a.Ld - Lr);
                for (int32_t rb = 0; rb < nroot; rb += 64) {
                    const int32_t r = rb + l;
                    bool pass = false, leaf = false;
                    int32_t st = 0, en = 0;
                    int32_t c0 = 0, c1 = 0, c2 = 0;
                    if (r < nroot) {
                        c0 = lo0 + r % nx;
                        c1 = lo1 + (r / nx) % ny;
                        c2 = lo2 + r / (nx * ny);
                        const uint64_t cm = morton3((uint64_t)(c0 & msk), (uint64_t)(c1 & msk),
                                                    (uint64_t)(c2 & msk));
                        st = a.table[cm << sh];
                        en = a.table[(cm + 1) << sh];
                        pass = en > st && node_pass(c0, c1, c2, Lr, st, en);
                        leaf = en - st <= kLeafMax || Lr >= B;
                    }
                    place(pass, leaf, st, en, c0, c1, c2, Lr);
                    expand_all();
                }
            } else {
                bool pass = false, leaf = false;
                int32_t st = 0, en = 0;
                if (l == 0) {
                    st = (int32_t)gbase;
                    en = (int32_t)gend;
                    pass = en > st && node_pass(0, 0, 0, 0, st, en);
                    leaf = en - st <= kLeafMax;
                }
                place(pass, leaf, st, en, 0, 0, 0, 0);
                expand_all();
            }
            if (nl > 0) stream_leaves(nl);
            if constexpr (PREC == SPH_FP32C) flush_staged();
        }

        // fold the copies' partial sums (lanes p, p + 16, p + 32, p + 48)
        for (int o = kAdjP; o < 64; o <<= 1) {
            acc0 += __shfl_xor(acc0, o, 64);
            acc1 += __shfl_xor(acc1, o, 64);
            acc2 += __shfl_xor(acc2, o, 64);
            acc3 += __shfl_xor(acc3, o, 64);
        }

        // ---- per-particle results (copy 0 writes)
        if (PHASE == 1) {
            if (mine && kk == 0) {
                double al = 0.0, be = 0.0, ga = 0.0;
                if (valid) {
                    const double gr = a.grs[s], gh = a.ghs[s];
                    const double h4 = hk * hk * hk * hk;
                    const double drhodh = -KT::sigma * (3.0 * acc1 + acc2) / h4;
                    const double dndh = -KT::count * acc0 / hk;
                    const double lam = dndh > 0.0 ? -(gr * drhodh + gh) / dndh : 0.0;
                    al = gr * KT::sigma / h4;
                    be = lam * KT::count / hk;
                    ga = gr * KT::sigma / (hk * hk * hk);
                }
                if constexpr (PREC == SPH_FP32C) {
                    const double hqs = hk * sc;
                    a.rec[s] = make_float4((float)hqs, (float)(1.0 / hqs), (float)al, (float)be);
                    a.recg[s] = (float)ga;
                } else {
                    a.alpha[s] = al;
                    a.beta[s] = be;
                    a.gamma[s] = ga;
                }
            }
        } else if (PHASE == 3) {
            if (mine && kk == 0) {
                // gx: rho_s, gy: rho_sym (optional), gz: int32 count (optional)
                const int64_t oi = a.perm[s];
                double rs = NAN, rsym = NAN;
                int32_t cnt = 0;
                if (valid) {
                    rs = acc1;
                    rsym = 0.5 * (KT::sigma * acc0 / (hk * hk * hk) + acc1);
                    cnt = (int32_t)acc2;
                }
                if (a.out_f32) {
                    st<float>(a.gx, oi, rs, a.ost);
                    if (a.gy) st<float>(a.gy, oi, rsym, a.ost);
                } else {
                    st<double>(a.gx, oi, rs, a.ost);
                    if (a.gy) st<double>(a.gy, oi, rsym, a.ost);
                }
                if (a.gz) st_i32(static_cast<int32_t *>(a.gz), oi, cnt, a.ost_i);
            }
        } else if (mine && kk == 0) {
            const int64_t oi = a.perm[s];
            double g0 = 0.0, g1 = 0.0, g2 = 0.0, g3 = 0.0;
            // the sums hold c (x_k - x_j)/r: unit vectors, the same in grid units
            if (valid) { g0 = acc0; g1 = acc1; g2 = acc2; g3 = acc3; }
            if (a.out_f32) {
                st<float>(a.gx, oi, g0, a.ost); st<float>(a.gy, oi, g1, a.ost);
                st<float>(a.gz, oi, g2, a.ost);
                if (a.gm) st<float>(a.gm, oi, g3, a.ost);
            } else {
                st<double>(a.gx, oi, g0, a.ost); st<double>(a.gy, oi, g1, a.ost);
                st<double>(a.gz, oi, g2, a.ost);
                if (a.gm) st<double>(a.gm, oi, g3, a.ost);
            }
        }
    }
}

// sorted-order cotangents
template <typename T>
__global__ void k_adj_gather(int64_t n, const int32_t *perm, const void *gr, const void *gh,
                             int64_t ins, double *grs, double *ghs) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t i = perm[s];
    grs[s] = ld<T>(gr, i, ins);
    ghs[s] = gh ? ld<T>(gh, i, ins) : 0.0;
}

// level 0 of the range-max table at slot s: h in grid units, rounded up to
// binary32
__device__ inline float rmq_h0(int64_t s, const double *sh, const uint64_t *skeys, bool grouped,
                               double box, const double *frame) {
    const double sc = grouped ? frame[8 * (int64_t)(uint32_t)(skeys[s] >> 48) + 6] : 2097152.0 / box;
    const double hq = sh[s] * sc;
    float f = (float)hq;
    if (!(hq > 0.0) || !isfinite(hq)) f = 0.f;
    else if ((double)f < hq) f = nextafterf(f, INFINITY);
    return f;
}

// Levels 0 .. kRmqLow in one pass.  Level k at slot s is the largest level-0
// value over [s, min(s + 2^k - 1, n - 1)], so a block that stages level 0 of
// 512 slots (past n: slot n - 1 again) derives levels 1 .. 8 of its first
// 256 slots in LDS.
constexpr int kRmqLow = 8;

__global__ __launch_bounds__(256) void k_rmq_low(int64_t n, int levels, const double *sh,
                                                 const uint64_t *skeys, bool grouped, double box,
                                                 const double *frame, float *t) {
    __shared__ float w[512];
    const int tid = threadIdx.x;
    const int64_t b0 = (int64_t)blockIdx.x * 256;
    for (int j = tid; j < 512; j += 256) {
        const int64_t s = b0 + j;
        w[j] = rmq_h0(s < n ? s : n - 1, sh, skeys, grouped, box, frame);
    }
    __syncthreads();
    const int64_t s = b0 + tid;
    if (s < n) t[s] = w[tid];
    const int top = levels - 1 < kRmqLow ? levels - 1 : kRmqLow;
    for (int k = 1; k <= top; ++k) {
        // w[j] holds level k - 1 wherever j + 2^(k-1) <= 512
        const int h = 1 << (k - 1);
        const float a0 = fmaxf(w[tid], w[tid + h]);
        const float a1 = tid + 256 + h < 512 ? fmaxf(w[tid + 256], w[tid + 256 + h]) : w[tid + 256];
        __syncthreads();
        w[tid] = a0;
        w[tid + 256] = a1;
        __syncthreads();
        if (s < n) t[(int64_t)k * n + s] = a0;
    }
}

__global__ void k_rmq_level(int64_t n, int k, float *t) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    const float *p = t + (int64_t)(k - 1) * n;
    const int64_t o = s + ((int64_t)1 << (k - 1));
    const float u = p[s], v = p[o < n ? o : n - 1];
    t[(int64_t)k * n + s] = u > v ? u : v;
}

// the range-max table of h over the sorted order (all levels)
static hipError_t build_rmq(Plan &pl, hipStream_t st) {
    const int64_t n = pl.n;
    const unsigned nbk = (unsigned)ceil_div(n, 256);
    hipLaunchKernelGGL(k_rmq_low, dim3(nbk), dim3(256), 0, st, n, pl.rmq_levels, pl.sh0, pl.skeys,
                       pl.grouped, pl.prm.box, pl.frame, pl.rmq);
    for (int k = kRmqLow + 1; k < pl.rmq_levels; ++k)
        hipLaunchKernelGGL(k_rmq_level, dim3(nbk), dim3(256), 0, st, n, k, pl.rmq);
    return hipGetLastError();
}

static void adj_args(const Plan &pl, const int64_t *goff, AdjArgs &a) {
    const int64_t n = pl.n;
    a.n = n;
    a.G = pl.G;
    a.goff = goff;
    a.skeys = pl.skeys;
    a.perm = pl.perm;
    a.sp = pl.sp; a.sh = pl.sh0;
    a.qp = pl.qp;
    a.fp = pl.fp;
    a.table = pl.table;
    a.Ld = pl.Ld;
    a.frame = pl.frame;
    a.gitems = pl.gitems;
    a.gorder = pl.gorder;
    a.n_items = ceil_div(n, kAdjP);
    a.rmq = pl.rmq;
    a.rmq_levels = pl.rmq_levels;
    a.box = pl.prm.box;
    a.bits = pl.bits;
    a.alpha = pl.adj; a.beta = pl.adj + n; a.gamma = pl.adj + 2 * n;
    a.rec = pl.adj_rec; a.recg = pl.adj_g;
    a.grs = pl.adj + 3 * n; a.ghs = pl.adj + 4 * n;
    a.out_f32 = pl.prm.io_dtype == SPH_F32;
    a.ost = pl.out_stride;
    a.ost_i = pl.out_stride_i;
    a.queue = pl.ctrl;
}

// one launch of the walk kernel for phase a.phase
static hipError_t launch_adjoint(const Plan &pl, AdjArgs &a, hipStream_t st) {
    hipError_t e = run_zero_i32(pl.ctrl, 4, st);
    if (e != hipSuccess) return e;
    const int64_t full = (int64_t)256 * kAdjWavesPerCU;
    const dim3 grid((unsigned)(pl.grouped ? full : (a.n_items < full ? a.n_items : full)));
    const bool f32c = pl.prm.precision == SPH_FP32C;
    const bool wc6 = pl.prm.kernel == SPH_KERNEL_WENDLAND_C6;
#define SPH_ADJ_K(PR, GR, K)                                                              \
    do {                                                                                  \
        if (a.phase == 1)                                                                 \
            hipLaunchKernelGGL((k_adjoint<PR, GR, K, 1>), grid, dim3(64), 0, st, a);      \
        else if (a.phase == 2)                                                            \
            hipLaunchKernelGGL((k_adjoint<PR, GR, K, 2>), grid, dim3(64), 0, st, a);      \
        else                                                                              \
            hipLaunchKernelGGL((k_adjoint<PR, GR, K, 3>), grid, dim3(64), 0, st, a);      \
    } while (0)
#define SPH_ADJ(PR, GR)                                                 \
    do {                                                                \
        if (wc6) SPH_ADJ_K(PR, GR, SPH_KERNEL_WENDLAND_C6);             \
        else SPH_ADJ_K(PR, GR, SPH_KERNEL_M4);                          \
    } while (0)
    if (!pl.grouped) {
        if (f32c) SPH_ADJ(SPH_FP32C, false);
        else SPH_ADJ(SPH_FP64, false);
    } else {
        if (f32c) SPH_ADJ(SPH_FP32C, true);
        else SPH_ADJ(SPH_FP64, true);
    }
#undef SPH_ADJ
#undef SPH_ADJ_K
    return hipGetLastError();
}

hipError_t run_backward(Plan &pl, const int64_t *goff, const void *h, const void *grad_rho,
                        const void *grad_h, void *gx, void *gy, void *gz, void *gm,
                        hipStream_t st) {
    (void)h;
    const int64_t n = pl.n;
    const unsigned nbk = (unsigned)ceil_div(n, 256);
    double *grs = pl.adj + 3 * n, *ghs = pl.adj + 4 * n;
    if (pl.prm.io_dtype == SPH_F32)
        hipLaunchKernelGGL(k_adj_gather<float>, dim3(nbk), dim3(256), 0, st, n, pl.perm, grad_rho,
                           grad_h, pl.in_stride, grs, ghs);
    else
        hipLaunchKernelGGL(k_adj_gather<double>, dim3(nbk), dim3(256), 0, st, n, pl.perm, grad_rho,
                           grad_h, pl.in_stride, grs, ghs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return run_backward_sorted(pl, goff, gx, gy, gz, gm, st);
}

// both passes of the adjoint with the sorted-order cotangents already in place
hipError_t run_backward_sorted(Plan &pl, const int64_t *goff, void *gx, void *gy, void *gz,
                               void *gm, hipStream_t st) {
    hipError_t e = build_rmq(pl, st);
    if (e != hipSuccess) return e;
    AdjArgs a;
    adj_args(pl, goff, a);
    a.gx = gx; a.gy = gy; a.gz = gz; a.gm = gm;
    if (pl.prm.prof_events[0]) {
        e = hipEventRecord((hipEvent_t)pl.prm.prof_events[0], st);
        if (e != hipSuccess) return e;
    }
    for (int phase = 1; phase <= 2 && e == hipSuccess; ++phase) {
        a.phase = phase;
        e = launch_adjoint(pl, a, st);
    }
    if (e != hipSuccess) return e;
    if (pl.prm.prof_events[1]) e = hipEventRecord((hipEvent_t)pl.prm.prof_events[1], st);
    return e;
}

// Pressure force cotangent m_i P_i / rho_i^2 in sorted order (caller arrays,
// strided), grad_h = 0.
template <typename T>
__global__ void k_force_coef(int64_t n, const int32_t *perm, const void *m, const void *P,
                             const void *rho, int64_t ins, double *grs, double *ghs) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t i = perm[s];
    const double r = ld<T>(rho, i, ins);
    grs[s] = ld<T>(m, i, ins) * ld<T>(P, i, ins) / (r * r);
    ghs[s] = 0.0;
}

// a_k = -dE/dx_k / m_k, in place on the adjoint's position gradient
template <typename T>
__global__ void k_force_scale(int64_t n, const void *m, int64_t ins, void *ax, void *ay,
                              void *az, int64_t ost) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double w = -1.0 / ld<T>(m, i, ins);
    st<T>(ax, i, ld<T>(ax, i, ost) * w, ost);
    st<T>(ay, i, ld<T>(ay, i, ost) * w, ost);
    st<T>(az, i, ld<T>(az, i, ost) * w, ost);
}

hipError_t run_force(Plan &pl, const int64_t *goff, const void *m, const void *rho,
                     const void *P, void *ax, void *ay, void *az, hipStream_t st) {
    const int64_t n = pl.n;
    const unsigned nbk = (unsigned)ceil_div(n, 256);
    double *grs = pl.adj + 3 * n, *ghs = pl.adj + 4 * n;
    const bool f32 = pl.prm.io_dtype == SPH_F32;
    if (f32)
        hipLaunchKernelGGL(k_force_coef<float>, dim3(nbk), dim3(256), 0, st, n, pl.perm, m, P,
                           rho, pl.in_stride, grs, ghs);
    else
        hipLaunchKernelGGL(k_force_coef<double>, dim3(nbk), dim3(256), 0, st, n, pl.perm, m, P,
                           rho, pl.in_stride, grs, ghs);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = run_backward_sorted(pl, goff, ax, ay, az, nullptr, st);
    if (e != hipSuccess) return e;
    if (f32)
        hipLaunchKernelGGL(k_force_scale<float>, dim3(nbk), dim3(256), 0, st, n, m,
                           pl.in_stride, ax, ay, az, pl.out_stride);
    else
        hipLaunchKernelGGL(k_force_scale<double>, dim3(nbk), dim3(256), 0, st, n, m,
                           pl.in_stride, ax, ay, az, pl.out_stride);
    return hipGetLastError();
}

// gamma_j = m_j sigma / h_j^3 (sorted order; 0 for invalid particles), from the
// masses the walk itself uses (binary32 in FP32C)
template <int KERNEL>
__global__ void k_scatter_coef(int64_t n, const double4 *sp, const int4 *qp, const double *sh,
                               const float4 *fp, double *gamma) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    const double h = sh[s];
    const bool valid = sp ? !isnan(sp[s].x) : !isnan(fp[s].x);
    const double m = sp ? sp[s].w : (double)__int_as_float(qp[s].w);
    gamma[s] = valid ? m * Kern<KERNEL>::sigma / (h * h * h) : 0.0;
}

hipError_t run_scatter(Plan &pl, const int64_t *goff, void *rho_s, void *rho_sym,
                       int32_t *nngb_s, hipStream_t st) {
    const int64_t n = pl.n;
    const unsigned nbk = (unsigned)ceil_div(n, 256);
    const bool f32c = pl.prm.precision == SPH_FP32C;
    double *gamma = pl.adj + 2 * n;
    const double4 *sp = f32c ? nullptr : pl.sp;
    if (pl.prm.kernel == SPH_KERNEL_WENDLAND_C6)
        hipLaunchKernelGGL(k_scatter_coef<SPH_KERNEL_WENDLAND_C6>, dim3(nbk), dim3(256), 0, st,
                           n, sp, pl.qp, pl.sh0, pl.fp, gamma);
    else
        hipLaunchKernelGGL(k_scatter_coef<SPH_KERNEL_M4>, dim3(nbk), dim3(256), 0, st, n, sp,
                           pl.qp, pl.sh0, pl.fp, gamma);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = build_rmq(pl, st);
    if (e != hipSuccess) return e;
    AdjArgs a;
    adj_args(pl, goff, a);
    a.gx = rho_s; a.gy = rho_sym; a.gz = nngb_s; a.gm = nullptr;
    a.phase = 3;
    if (pl.prm.prof_events[0]) {
        e = hipEventRecord((hipEvent_t)pl.prm.prof_events[0], st);
        if (e != hipSuccess) return e;
    }
    e = launch_adjoint(pl, a, st);
    if (e != hipSuccess) return e;
    if (pl.prm.prof_events[1]) e = hipEventRecord((hipEvent_t)pl.prm.prof_events[1], st);
    return e;
}

}  // namespace sph
