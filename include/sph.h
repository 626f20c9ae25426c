/*
 * sph.h -- C ABI of the MI355X (gfx950) SPH density library, libsph.so.
 *
 * The library computes, for every particle i, the SPH density
 *     rho_i = sum_j m_j W(|r_i - r_j|, h_i)
 * (Baruffa et al., arXiv:1612.06090, Sec. II-B, Eq. 1, evaluated in gather
 * form with the particle's own smoothing length, over the neighbours "within
 * a smoothing length" of Listing 1, self term included) together with the
 * smoothing length h_i, which is adjusted per particle until its weighted
 * neighbour count n_i = (4 pi/3) h_i^3 sum_j W(r_ij, h_i) reaches the target
 * (the recompute loop of Sec. IV-A, Listings 2 and 3).  W = sigma/h^3 f(r/h)
 * has compact support h: by default the M4 cubic spline (sigma = 8/pi,
 * f(q) = 1 - 6q^2 + 6q^3 (q <= 1/2), 2(1-q)^3 (1/2 < q <= 1), 0 beyond), or
 * the paper's Wendland C6 (params->kernel).  With C = (4 pi/3) sigma the
 * weighted count is n = C sum_j f (C = 32/3 for M4, 1365/48 for Wendland C6).
 *
 * Conventions shared by every entry point:
 *  - All array arguments are DEVICE pointers on the current HIP device,
 *    except `params` and `bytes`, which are host pointers.
 *  - Particle arrays are structure-of-arrays (the SoA layout of Sec. IV-B):
 *    x[n], y[n], z[n], m[n], ... of element type io_dtype (double or float).
 *  - The caller owns every buffer, including the workspace `ws` of at least
 *    sph_workspace_size() bytes (256-byte aligned).  No call allocates or
 *    frees device memory, synchronises the host, or prints.
 *  - Calls are asynchronous on `stream` (a hipStream_t; NULL = the null
 *    stream).  Argument errors are detected on the host and returned
 *    synchronously before anything is enqueued.  Per-particle conditions
 *    detected on the device never fail the call: they set bits of
 *    status_out[i] (below), readable after the stream completes.
 *  - Outputs of sph_density_solve / sph_density_backward are in the
 *    caller's original particle order.  sph_sort returns sorted order.
 *  - One workspace must not be used by two calls that may run concurrently.
 *    Besides the scratch of sph_density_solve_noalloc, the library holds one
 *    other piece of state: a per-device count of the sort's bounded waits
 *    that reached their bound (sph_sort_wait_faults).  Calls on different
 *    workspaces are thread-safe.
 */
#ifndef SPH_H
#define SPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPH_ABI_VERSION 1u

/* return codes */
#define SPH_OK            0
#define SPH_E_INVALID    (-1)  /* bad argument: null pointer, n out of range, bad enum, ... */
#define SPH_E_WORKSPACE  (-2)  /* ws_bytes smaller than sph_workspace_size() */
#define SPH_E_HIP        (-3)  /* a HIP launch failed; see sph_last_hip_error() */
#define SPH_E_UNSUPPORTED (-4) /* valid but not supported combination */

/* precision: arithmetic of the pair loop */
#define SPH_FP64   0   /* IEEE binary64 throughout; pair distances bit-identical to a
                          plain (dx*dx + dy*dy) + dz*dz evaluation without FMA */
#define SPH_FP32C  1   /* pair distances and kernel sums in binary32 from positions
                          stored relative to Morton-cell origins, compensated (Kahan)
                          sums; h iteration and convergence test in binary64 */

/* kernel: the smoothing function (both with compact support h; the weighted
 * count is n = (4 pi/3) h^3 sum_j W = C sum_j f, C = (4 pi/3) sigma) */
#define SPH_KERNEL_M4          0  /* M4 cubic spline (Gadget-2 convention), sigma = 8/pi:
                                     f = 1 - 6q^2 + 6q^3 (q <= 1/2), 2(1-q)^3 (q <= 1) */
#define SPH_KERNEL_WENDLAND_C6 1  /* Wendland C6, the kernel of the paper's runs
                                     (Sec. II-B), sigma = 1365/(64 pi):
                                     f = (1-q)^8 (1 + 8q + 25q^2 + 32q^3) */

/* io_dtype: element type of caller arrays x, y, z, m, h_init, rho, h, nw, grads */
#define SPH_F64    0
#define SPH_F32    1

/* mode: stopping rule of the h iteration */
#define SPH_BAND   0   /* stop when |n - n_target| <= n_tol */
#define SPH_ROOT   1   /* stop when |n - n_target| <= root_tol * n_target, or when the
                          bracket [lo, hi] has shrunk to 4 ulp(h) */
#define SPH_KNN    2   /* exact K nearest (Sec. IV-D): h = the distance of the K-th
                          nearest particle of the particle's set, the particle itself
                          counted first, K = n_target (an integer in [2, 2^20]); rho,
                          nw and nngb are evaluated at that h (where the K-th neighbour
                          has W = 0).  If K particles coincide, h = 0 and rho is not
                          finite.  Found by iterating h on the integer count
                          N = #(r < h) into [K, K + n_tol] (n_tol an integer in
                          [0, 48]) and selecting the K-th smallest distance among
                          those N.  FP32C selects from binary32 coordinates with
                          binary64 differences.  On a periodic set the count stage
                          starts from h_init moved to within a factor 1.25 of a local
                          estimate from the occupancy of the particle's Morton cell
                          (the result does not depend on the start); isolated groups
                          start from h_init.  The selection keeps the 16, 32 or
                          64 largest distances inside the count-stage h (for n_tol
                          up to 14, 30, 48); where ties make the count jump over the
                          band, the count stage hands over a bracket end holding up
                          to that many more than K.  The low status bits count the
                          count-stage updates; NOCONV also marks a particle whose
                          selection could not rank the K-th distance (the count
                          stage ran out of updates away from the band, or more
                          particles tie at the K-th distance than the heap holds).
                          sph_density_backward rejects this mode (SPH_E_UNSUPPORTED):
                          h is not a smooth function of the positions. */

/* status_out[i]: low 16 bits = number of h updates made, high bits = flags */
#define SPH_ST_ITER_MASK   0xFFFF
#define SPH_ST_NOCONV      (1 << 16)  /* max_iter updates without meeting the stopping rule */
#define SPH_ST_HTOOLARGE   (1 << 17)  /* periodic: h needed >= box/2 (h is left at
                                         box/2 (1 - 2^-20), the largest allowed) */
#define SPH_ST_BADINPUT    (1 << 18)  /* non-finite x, y, z, m or h_init, h_init <= 0, or
                                         (periodic) a coordinate outside [0, box).  Such a
                                         particle is never anyone's neighbour; its rho and
                                         nw are NaN, h = h_init, nngb = 0. */
#define SPH_ST_UNREACHABLE (1 << 19)  /* isolated group of n_g particles with
                                         C n_g < n_target - n_tol: evaluated at
                                         h_init only */

/* Parameters.  Initialise with sph_default_params() and override fields. */
typedef struct {
    uint32_t abi_version;   /* must be SPH_ABI_VERSION */
    int32_t  precision;     /* SPH_FP64 | SPH_FP32C */
    int32_t  io_dtype;      /* SPH_F64 | SPH_F32 */
    int32_t  mode;          /* SPH_BAND | SPH_ROOT | SPH_KNN */
    int32_t  periodic;      /* 1: one periodic cube [0, box)^3 (n_groups must be 0);
                               0: isolated groups given by group_offsets */
    int32_t  max_iter;      /* h updates allowed per particle, 0..65535 (default 64);
                               0 = evaluate at h_init only */
    double   box;           /* periodic box side L > 0 */
    double   n_target;      /* N_t > 0: target weighted neighbour count (e.g. 64) */
    double   n_tol;         /* dN >= 0: band half-width (e.g. 2) */
    double   root_tol;      /* SPH_ROOT relative tolerance (default 1e-12) */
    int32_t  cell_level;    /* level of the cell table returned by sph_sort;
                               -1 = max(1, ceil((ceil(log2 n) - 3) / 3)) */
    int32_t  tile_cell;     /* tuning: neighbour-cell side in units of the tile's largest
                               h, as a power of two exponent in {-2, -1, 0} (default -1);
                               results do not depend on it */
    int32_t  waves_per_cu;  /* tuning: persistent grid = 256 CUs x this (default 16) */
    int32_t  segment;       /* tuning: particles per wavefront tile, 8/16/32/64 (default
                               16); each particle is held by 64/segment lanes that split
                               its candidate stream; results do not depend on it beyond
                               summation order */
    void    *prof_events[2];/* optional hipEvent_t pair recorded on `stream` immediately
                               before and after the density kernel (sph_density_solve)
                               or the two adjoint kernels (sph_density_backward);
                               NULL: none */
    int32_t  kernel;        /* smoothing kernel, W(r, h) = sigma/h^3 f(r/h), support r < h:
                               SPH_KERNEL_M4 (default) or SPH_KERNEL_WENDLAND_C6 */
    int32_t  in_stride;     /* bytes from particle i to i + 1 in every per-particle input
                               (x, y, z, m, h_init; h, grad_rho, grad_h of the backward);
                               0 = packed arrays (the element size).  A caller that keeps
                               an array of particle structs (Sec. IV-B) passes the struct
                               size and points each input at its field: the library's
                               own gather into sorted arrays reads the structs directly.
                               A multiple of the element size (8 for SPH_F64, 4 for
                               SPH_F32), at most 65536 */
    int32_t  out_stride;    /* the same for every per-particle output (rho, h, nw, nngb,
                               status; grad_x .. grad_m), which are written through the
                               sort permutation straight into the caller's structs.
                               0 = packed (floating outputs at the element size, nngb
                               and status at 4 bytes); else a multiple of the element
                               size (and of 4), at most 65536, shared by all outputs */
    int32_t  reserved[5];   /* must be zero */
} sph_params;

/* Fill *p with the defaults: FP64 compute and io, band mode, periodic unit
 * box, n_target 64, n_tol 2, root_tol 1e-12, max_iter 64, cell_level -1. */
void sph_default_params(sph_params *p);

/* Host only.  Bytes of workspace needed by sph_sort, sph_density_solve and
 * sph_density_backward for n particles in n_groups groups (0 = one periodic
 * set).  The size is monotone in n.  Every entry point accepts 0 <= n <
 * 2^31 - 1 (sorted indices are 32-bit) and 1 <= n_groups <= 65535 for
 * isolated groups (n_groups = 0 for a periodic set); other sizes give
 * SPH_E_INVALID.  Returns SPH_OK or SPH_E_INVALID. */
int sph_workspace_size(const sph_params *params, int64_t n, int32_t n_groups, size_t *bytes);

/* The spatial sort that precedes the density loop (no counterpart in the
 * paper, whose Barnes-Hut tree is given; Sec. II-A).
 *   Keys: periodic -- q = floor(x * (2^21/box)) per axis clamped to
 *   [0, 2^21 - 1]; key bit 3k+2 = bit k of qx, 3k+1 of qy, 3k of qz.
 *   Groups -- key = (g << 48) | the same interleave of 16-bit
 *   q = floor((x - lo_g) * (2^16 / E_g)) on the group's bounding cube
 *   (lower corner lo_g, side E_g = largest extent, 1 if 0).
 *   Sort: ascending by key, stable (equal keys keep caller order).
 * Outputs (device, capacity n each):
 *   keys_out[s]  sorted keys;   perm_out[s] = caller index of sorted slot s;
 *   cell_id_out[c], cell_start_out[c], cell_count_out[c] for the occupied
 *   cells at level L = params->cell_level (or the default rule): cell id =
 *   key >> 3(21 - L) (groups: 3(16 - L)), in ascending order;
 *   *n_cells_out (device int32) = number of occupied cells.
 * group_offsets: device int64[n_groups + 1], non-decreasing, offsets[0] = 0,
 * offsets[n_groups] = n; NULL iff n_groups == 0.  Requires n_groups < 65536.
 * The offsets stay on the device and are not checked synchronously: every
 * entry point first copies them into its workspace as offsets[0] = 0,
 * offsets[n_groups] = n and, in between, the running maximum of the given
 * values clamped to [0, n], which leaves well-formed offsets unchanged.
 * Malformed offsets therefore never make a kernel read outside the caller's
 * arrays; the results are those of the corrected groups (the Python binding
 * rejects malformed offsets on the host instead).
 * Any output pointer except keys_out and perm_out may be NULL; no output may
 * overlap the inputs, the workspace or another output. */
int sph_sort(const sph_params *params, int64_t n, int32_t n_groups,
             const int64_t *group_offsets,
             const void *x, const void *y, const void *z,
             uint64_t *keys_out, int32_t *perm_out,
             uint64_t *cell_id_out, int32_t *cell_start_out, int32_t *cell_count_out,
             int32_t *n_cells_out,
             void *ws, size_t ws_bytes, void *stream);

/* Density and smoothing-length solve (Eq. 1 with the recompute loop of
 * Sec. IV-A).  Per particle, starting from h = h_init (NULL: every particle
 * starts at 2 (V/n)^(1/3), V = box^3 periodic, or the group's bounding-box
 * volume with every extent taken at least 2^-16 of the largest extent),
 * repeat: evaluate at h the sums over neighbours j (r_ij^2 < h^2, minimum
 * image when periodic, same group when isolated)
 *     S0 = sum f(q), S1 = sum q f'(q), R = sum m_j f(q),   q = r_ij / h,
 * giving rho = sigma R/h^3, n = C S0, dn/dh = -C S1/h; stop per
 * `mode`; else set lo = h if n < N_t, else hi = h, and take the Newton step
 * h + (N_t - n)/(dn/dh) when dn/dh > 0 and the step lands strictly inside
 * (lo, hi) and within [h/2, 2h], otherwise 2h (no upper bracket yet), h/2 (no
 * lower bracket yet) or (lo + hi)/2.  Periodic h is capped at
 * box/2 (1 - 2^-20).
 * Outputs (device, caller order, io_dtype unless noted): rho_out, h_out,
 * nw_out (the weighted count n at the returned h), nngb_out (int32: number
 * of j with r_ij^2 < h^2, i included), status_out (int32, bits above).
 * Any output may be NULL except rho_out and h_out.
 * stats_out: NULL or device uint64[4], overwritten: [0] in-range pairs
 * evaluated over all trial h, [1] candidate pairs tested (particle against
 * candidate), [2] density passes made (sum over particles of updates + 1),
 * [3] candidates streamed from neighbour cells and tested once against the
 * region of the particles being solved together (the bounding box of their
 * positions widened by their largest h), before the pair tests. */
int sph_density_solve(const sph_params *params, int64_t n, int32_t n_groups,
                      const int64_t *group_offsets,
                      const void *x, const void *y, const void *z, const void *m,
                      const void *h_init,
                      void *rho_out, void *h_out, void *nw_out,
                      int32_t *nngb_out, int32_t *status_out, uint64_t *stats_out,
                      void *ws, size_t ws_bytes, void *stream);

/* Adjoint of sph_density_solve.  Given the forward's h (h_out) and
 * cotangents grad_rho (and optionally grad_h, NULL = 0), writes
 *   grad_x/y/z[k] = d/dx_k sum_i (grad_rho_i rho_i + grad_h_i h_i)
 *   grad_m[k]     = d/dm_k of the same,
 * with each h_i held on its implicit root n_i(h_i, x) = n_i(achieved):
 *   lambda_i = -(grad_rho_i drho_i/dh_i + grad_h_i) / (dn_i/dh_i)
 *   (0 when dn_i/dh_i = 0), and for each pair j in N(i), j != i, with
 *   q = r_ij/h_i and unit vector u = (x_i - x_j)/r_ij:
 *     c_ij = grad_rho_i m_j sigma f'(q)/h_i^4 + lambda_i C f'(q)/h_i,
 *     grad_x_i += c_ij u,  grad_x_j -= c_ij u,
 *     grad_m_j += grad_rho_i W(r_ij, h_i)   (self term included).
 * Computed in gather form (no floating-point atomics; bitwise reproducible).
 * Outputs are in caller order, io_dtype, and are overwritten. */
int sph_density_backward(const sph_params *params, int64_t n, int32_t n_groups,
                         const int64_t *group_offsets,
                         const void *x, const void *y, const void *z, const void *m,
                         const void *h, const void *grad_rho, const void *grad_h,
                         void *grad_x, void *grad_y, void *grad_z, void *grad_m,
                         void *ws, size_t ws_bytes, void *stream);

/* Pressure acceleration of the variational (grad-h) SPH equations (the
 * "other particle interaction computations" of the neighbour loop), at the
 * converged h of sph_density_solve (h_out) and its rho (rho_out), for
 * per-particle pressures P:
 *   a_k = -(1/m_k) dE/dx_k,  E = sum_i m_i u_i(rho_i),  du_i/drho_i = P_i/rho_i^2,
 * with every h_i held on its count constraint n_i(h_i, x) = n_i(achieved):
 * the sph_density_backward gradient for grad_rho_i = m_i P_i/rho_i^2 (and
 * grad_h = 0), divided by -m_k.  Pairwise antisymmetric: sum_k m_k a_k = 0
 * (and no torque for isolated groups) up to rounding.  rho and pressure are
 * inputs like x (in_stride); ax/ay/az outputs (out_stride), caller order,
 * io_dtype, overwritten.  SPH_KNN mode: SPH_E_UNSUPPORTED. */
int sph_pressure_force(const sph_params *params, int64_t n, int32_t n_groups,
                       const int64_t *group_offsets,
                       const void *x, const void *y, const void *z, const void *m,
                       const void *h, const void *rho, const void *pressure,
                       void *ax_out, void *ay_out, void *az_out,
                       void *ws, size_t ws_bytes, void *stream);

/* Scatter form of the density, Eq. (1) as printed (each neighbour j with its
 * own smoothing length h_j), at given h (e.g. sph_density_solve's h_out):
 *   rho_s_out[i]   = sum_{j: r_ij < h_j} m_j W(r_ij, h_j)     (i included)
 *   rho_sym_out[i] = (sum_{j: r_ij < h_i} m_j W(r_ij, h_i) + rho_s_out[i]) / 2
 *   nngb_s_out[i]  = number of j with r_ij < h_j (int32)
 * with the minimum image when periodic and the same group when isolated.
 * rho_sym_out and nngb_s_out may be NULL.  Particles with invalid inputs
 * (non-finite x/y/z/m/h, h <= 0, periodic coordinates outside [0, L)) get NaN
 * and 0 and are nobody's neighbour.  The mode and the h-iteration fields of
 * params are not used.  Computed in gather form over each particle's
 * reverse neighbours (no atomics; bitwise reproducible); outputs in caller
 * order, io_dtype, overwritten. */
int sph_density_scatter(const sph_params *params, int64_t n, int32_t n_groups,
                        const int64_t *group_offsets,
                        const void *x, const void *y, const void *z, const void *m,
                        const void *h, void *rho_s_out, void *rho_sym_out,
                        int32_t *nngb_s_out, void *ws, size_t ws_bytes, void *stream);

/* Launch-parameter autotuner of sph_density_solve (the batched persistent form
 * whose per-item work is uneven and unknown in advance: the dynamic scheduling
 * of Sec. IV-A).  Times sph_density_solve on the given input for every
 * combination of segment {8, 16, 32, 64}, waves_per_cu {8, 16, 32} and
 * tile_cell {-1, 0} (one warm-up call, then the median of three, timed with
 * HIP events on `stream`), and writes *params with the fastest combination to
 * *best_out (and its time in ms to *best_ms_out, if not NULL).  rho_out and
 * h_out (device, capacity n, io_dtype) are scratch outputs and are
 * overwritten; ws is a workspace as for sph_density_solve.
 * Results are cached in the process (mutex-guarded), keyed by the device
 * architecture, every parameter other than the three tuned ones, whether
 * h_init is given, floor(log2 n) and floor(log2(n_groups + 1)); a cached key
 * returns at once without touching the device.  If the environment variable
 * SPH_TUNE_CACHE names a file, entries are read from it on first use and new
 * ones appended.  The call synchronizes with `stream` (it must not be
 * captured into a graph).  Returns SPH_OK, or the first failing code of the
 * solves (SPH_E_INVALID / SPH_E_WORKSPACE / SPH_E_HIP). */
int sph_autotune(const sph_params *params, int64_t n, int32_t n_groups,
                 const int64_t *group_offsets,
                 const void *x, const void *y, const void *z, const void *m,
                 const void *h_init, void *rho_out, void *h_out,
                 void *ws, size_t ws_bytes, void *stream,
                 sph_params *best_out, float *best_ms_out);

/* sph_density_solve without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Arguments, outputs and results are those
 * of sph_density_solve; the workspace is a fixed scratch array of
 * SPH_NOALLOC_SCRATCH_BYTES held in the library's device memory (one per
 * device, kept until the process ends; its address is looked up once per
 * device, on the first call with that device current).  The call allocates
 * nothing.  A problem whose sph_workspace_size exceeds the scratch (about
 * 3e5 particles) returns SPH_E_WORKSPACE before anything is enqueued; use
 * sph_density_solve with a caller workspace for larger sets.  Every call on
 * one device shares that device's scratch, which keeps the last call's
 * contents (no call relies on them): calls that may overlap on one device
 * (different streams, or host threads without ordering) race and must not be
 * issued. */
#define SPH_NOALLOC_SCRATCH_BYTES (64u << 20)
int sph_density_solve_noalloc(const sph_params *params, int64_t n, int32_t n_groups,
                              const int64_t *group_offsets,
                              const void *x, const void *y, const void *z, const void *m,
                              const void *h_init,
                              void *rho_out, void *h_out, void *nw_out,
                              int32_t *nngb_out, int32_t *status_out, uint64_t *stats_out,
                              void *stream);

/* Static text for a return code. */
const char *sph_status_string(int code);

/* The HIP error code of the last SPH_E_HIP returned on the calling thread
 * (0 if none), and its text. */
int sph_last_hip_error(void);
const char *sph_last_hip_error_string(void);

/* Host only; synchronises with the current device.  The particle sort
 * (inside sph_sort and every call that sorts) scatters each radix pass in
 * tiles that take the output offsets of their digits from the tiles before
 * them as those publish their counts (a decoupled look-back over a chained
 * scan).  A tile waits only on tiles that started before it, so every wait
 * ends; each wait is still bounded, and one that reaches its bound lets the
 * tile go on with a wrong offset (that sort's outputs are then wrong).
 * *count receives how many waits reached the bound on the current device
 * since the last call (0 is the only expected value), and the count is
 * cleared.  Returns SPH_OK, SPH_E_INVALID (count NULL) or SPH_E_HIP. */
int sph_sort_wait_faults(uint32_t *count);

#ifdef __cplusplus
}
#endif

#endif /* SPH_H */
