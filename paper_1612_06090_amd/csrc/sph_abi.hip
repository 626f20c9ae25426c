// C ABI of libsph: argument validation, workspace planning and the launch
// sequence of each entry point.  Declarations and semantics: include/sph.h.
#include "sph_internal.h"

#include <math.h>
#include <string.h>

#include <mutex>

namespace sph {

static thread_local int g_last_hip = 0;

static int hip_fail(hipError_t e) {
    g_last_hip = (int)e;
    return SPH_E_HIP;
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

static int ceil_log2_i64(int64_t n) {
    int lg = 0;
    while (lg < 62 && ((int64_t)1 << lg) < n) ++lg;
    return lg;
}

int make_plan(const sph_params *p, int64_t n, int32_t G, void *ws, Plan *out) {
    Plan &pl = *out;
    pl = Plan();
    pl.prm = *p;
    pl.n = n;
    pl.G = G;
    pl.grouped = G > 0;
    pl.bits = pl.grouped ? 16 : 21;
    const int lg = ceil_log2_i64(n > 0 ? n : 1);
    if (p->cell_level >= 0) {
        pl.Lc = p->cell_level;
    } else {
        const int t = lg - 3;
        pl.Lc = t <= 0 ? 1 : (t + 2) / 3;
        if (pl.Lc < 1) pl.Lc = 1;
        if (pl.Lc > pl.bits) pl.Lc = pl.bits;
    }
    if (!pl.grouped) {
        int Ld = (lg + 2) / 3;
        if (Ld < 1) Ld = 1;
        if (Ld > 8) Ld = 8;
        pl.Ld = Ld;
        pl.table_n = ((int64_t)1 << (3 * Ld)) + 1;
    }
    pl.sort_rounds = n <= ((int64_t)1 << 21) ? 4 : 16;
    pl.sort_tile = (int64_t)256 * pl.sort_rounds;
    pl.nb_sort = ceil_div(n > 0 ? n : 1, pl.sort_tile);
    pl.nb_scan_n = ceil_div(n > 0 ? n : 1, kScanTile);
    pl.nb_scan_t = ceil_div(pl.table_n > 0 ? pl.table_n : 1, kScanTile);
    const int64_t seg = p->segment;
    pl.n_items = ceil_div(n > 0 ? n : 1, seg);
    const int64_t full = (int64_t)256 * p->waves_per_cu;
    pl.grid = (int)(pl.grouped ? full : (pl.n_items < full ? pl.n_items : full));
    if (pl.grid < 1) pl.grid = 1;
    const int64_t es = p->io_dtype == SPH_F32 ? 4 : 8;
    pl.in_stride = p->in_stride ? p->in_stride : es;
    pl.out_stride = p->out_stride ? p->out_stride : es;
    pl.out_stride_i = p->out_stride ? p->out_stride : 4;

    const bool f32c = p->precision == SPH_FP32C;
    const size_t N = (size_t)(n > 0 ? n : 1);
    size_t off = 0;
    char *base = static_cast<char *>(ws);
    auto take = [&](size_t bytes) -> void * {
        void *r = base ? base + off : nullptr;
        off = align256(off + bytes);
        return r;
    };
    pl.keysA = (uint64_t *)take(8 * N);
    pl.keysB = (uint64_t *)take(8 * N);
    pl.valsA = (int32_t *)take(4 * N);
    pl.valsB = (int32_t *)take(4 * N);
    pl.sweep_words = 2 * 256 * pl.nb_sort + 8 * 256 + 16;
    pl.sweep = (int32_t *)take(4 * (size_t)pl.sweep_words);
    if (pl.sweep) {
        pl.sweep_desc = reinterpret_cast<uint64_t *>(pl.sweep);
        pl.sweep_gh = reinterpret_cast<uint32_t *>(pl.sweep + 2 * 256 * pl.nb_sort);
        pl.sweep_ctr = pl.sweep + 2 * 256 * pl.nb_sort + 8 * 256;
    }
    pl.digit_tot = (uint32_t *)take(4 * 256);
    if (!f32c) {
        pl.sp = (double4 *)take(32 * N);
    } else {
        pl.qp = (int4 *)take(16 * N);
        pl.fp = (float4 *)take(16 * N);
    }
    pl.sh0 = (double *)take(8 * N);
    if (pl.table_n > 0) pl.table = (int32_t *)take(4 * (size_t)pl.table_n);
    int64_t nbs = pl.nb_scan_n;
    if (pl.nb_scan_t > nbs) nbs = pl.nb_scan_t;
    const int64_t nbg = ceil_div((int64_t)G + 1, kScanTile);
    if (nbg > nbs) nbs = nbg;
    pl.bsum = (int32_t *)take(4 * (size_t)(nbs + 1));
    if (pl.grouped) {
        pl.frame = (double *)take(8 * 8 * (size_t)G);
        pl.gitems = (int32_t *)take(4 * ((size_t)G + 1));
        pl.nb_gsort = ceil_div((int64_t)G, (int64_t)256 * 4);
        pl.gkeysA = (uint64_t *)take(8 * (size_t)G);
        pl.gkeysB = (uint64_t *)take(8 * (size_t)G);
        pl.gvalsA = (int32_t *)take(4 * (size_t)G);
        pl.gvalsB = (int32_t *)take(4 * (size_t)G);
        pl.ghist = (uint32_t *)take(4 * 256 * (size_t)pl.nb_gsort);
        pl.goff = (int64_t *)take(8 * ((size_t)G + 1));
    }
    pl.ctrl = (int32_t *)take(64);
    pl.stats = (uint64_t *)take(64);
    pl.adj = (double *)take(5 * 8 * N);
    pl.adj_rec = (float4 *)take(16 * N);
    pl.adj_g = (float *)take(4 * N);
    pl.rmq_levels = ceil_log2_i64((int64_t)N) + 1;
    pl.rmq = (float *)take(4 * N * (size_t)pl.rmq_levels);
    if (p->mode == SPH_KNN) {
        pl.knn_h = (double *)take(8 * N);
        pl.knn_st = (int32_t *)take(4 * N);
        // at most one entry per selection tile, also with groups (each
        // group's tiles start at its first particle)
        pl.knn_items = (int32_t *)take(4 * ((size_t)ceil_div((int64_t)N, (int64_t)kSelTile) +
                                            (size_t)G + 1));
    }
    pl.total = off;
    return SPH_OK;
}

static int check_params(const sph_params *p, int64_t n, int32_t G, const int64_t *goff) {
    if (!p) return SPH_E_INVALID;
    if (p->abi_version != SPH_ABI_VERSION) return SPH_E_INVALID;
    if (p->precision != SPH_FP64 && p->precision != SPH_FP32C) return SPH_E_INVALID;
    if (p->io_dtype != SPH_F64 && p->io_dtype != SPH_F32) return SPH_E_INVALID;
    if (p->mode != SPH_BAND && p->mode != SPH_ROOT && p->mode != SPH_KNN) return SPH_E_INVALID;
    if (p->periodic != 0 && p->periodic != 1) return SPH_E_INVALID;
    if (n < 0 || n >= ((int64_t)1 << 31) - 1) return SPH_E_INVALID;
    if (p->periodic) {
        if (G != 0 || goff) return SPH_E_INVALID;
        if (!(p->box > 0.0) || !isfinite(p->box)) return SPH_E_INVALID;
    } else {
        if (G < 1 || G >= 65536 || !goff) return SPH_E_INVALID;
    }
    if (!(p->n_target > 0.0) || !isfinite(p->n_target)) return SPH_E_INVALID;
    if (!(p->n_tol >= 0.0) || !isfinite(p->n_tol)) return SPH_E_INVALID;
    if (p->mode == SPH_ROOT && (!(p->root_tol > 0.0) || !isfinite(p->root_tol)))
        return SPH_E_INVALID;
    if (p->mode == SPH_KNN) {
        // K an integer in [2, 2^20] (K = 1 would give h = 0, the particle itself), the
        // count band slack an integer in [0, 48]
        if (p->n_target != floor(p->n_target) || p->n_target < 2.0 || p->n_target > 1048576.0)
            return SPH_E_INVALID;
        if (p->n_tol != floor(p->n_tol) || p->n_tol > 48.0) return SPH_E_INVALID;
    }
    if (p->max_iter < 0 || p->max_iter > 65535) return SPH_E_INVALID;
    const int bits = p->periodic ? 21 : 16;
    if (p->cell_level < -1 || p->cell_level > bits || p->cell_level == 0) return SPH_E_INVALID;
    if (p->tile_cell < -2 || p->tile_cell > 0) return SPH_E_INVALID;
    if (p->waves_per_cu < 1 || p->waves_per_cu > 32) return SPH_E_INVALID;
    if (p->segment != 8 && p->segment != 16 && p->segment != 32 && p->segment != 64)
        return SPH_E_INVALID;
    if (p->kernel != SPH_KERNEL_M4 && p->kernel != SPH_KERNEL_WENDLAND_C6) return SPH_E_INVALID;
    // strides: 0 (packed) or a positive multiple of the element size (and of 4 for
    // the int32 outputs), at most 64 KiB
    const int es = p->io_dtype == SPH_F32 ? 4 : 8;
    if (p->in_stride < 0 || p->in_stride > 65536 || p->in_stride % es != 0)
        return SPH_E_INVALID;
    if (p->out_stride < 0 || p->out_stride > 65536 || p->out_stride % es != 0)
        return SPH_E_INVALID;
    for (int k = 0; k < 5; ++k)
        if (p->reserved[k] != 0) return SPH_E_INVALID;
    return SPH_OK;
}

// Caller arrays must be aligned to their elements.
static bool aligned(const void *p, uintptr_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

static int check_ws(const sph_params *p, int64_t n, int32_t G, void *ws, size_t bytes, Plan *pl) {
    if (!ws) return SPH_E_INVALID;
    if (((uintptr_t)ws & 255u) != 0) return SPH_E_INVALID;
    Plan probe;
    make_plan(p, n, G, nullptr, &probe);
    if (bytes < probe.total) return SPH_E_WORKSPACE;
    return make_plan(p, n, G, ws, pl);
}

__global__ void k_store_i32(int32_t *p, int32_t v) { *p = v; }

// Group offsets as every kernel assumes them: out[0] = 0, out[G] = n and
// out[g] = the running maximum of the caller's offsets clamped to [0, n]
// in between.  Well-formed offsets are copied unchanged; malformed ones
// (decreasing, outside [0, n], wrong ends) are replaced by the nearest
// well-formed sequence, so that no kernel reads outside the particle arrays.
// One block of 1024 threads, each owning a contiguous run of entries.
constexpr int kCleanThreads = 1024;

__global__ __launch_bounds__(kCleanThreads) void k_clean_offsets(int32_t G, int64_t n,
                                                                 const int64_t *in,
                                                                 int64_t *out) {
    __shared__ int64_t run_max[kCleanThreads];
    const int t = threadIdx.x;
    const int64_t cnt = (int64_t)G + 1;
    const int64_t per = (cnt + kCleanThreads - 1) / kCleanThreads;
    const int64_t b = (int64_t)t * per;
    const int64_t e = b + per < cnt ? b + per : cnt;
    auto clampv = [&](int64_t g) -> int64_t {
        if (g == 0) return 0;
        if (g == G) return n;
        const int64_t v = in[g];
        return v < 0 ? 0 : (v > n ? n : v);
    };
    int64_t m = 0;
    for (int64_t g = b; g < e; ++g) m = clampv(g) > m ? clampv(g) : m;
    run_max[t] = m;
    __syncthreads();
    // inclusive max-scan over the threads' maxima (Hillis-Steele)
    for (int o = 1; o < kCleanThreads; o <<= 1) {
        const int64_t w = t >= o ? run_max[t - o] : 0;
        __syncthreads();
        if (w > run_max[t]) run_max[t] = w;
        __syncthreads();
    }
    int64_t acc = t > 0 ? run_max[t - 1] : 0;
    for (int64_t g = b; g < e; ++g) {
        const int64_t v = clampv(g);
        acc = v > acc ? v : acc;
        out[g] = acc;
    }
}

hipError_t run_clean_offsets(const Plan &pl, const int64_t *goff, hipStream_t st) {
    if (!pl.grouped) return hipSuccess;
    hipLaunchKernelGGL(k_clean_offsets, dim3(1), dim3(kCleanThreads), 0, st, pl.G, pl.n, goff,
                       pl.goff);
    return hipGetLastError();
}

// Scratch of sph_density_solve_noalloc: the workspace of a solve, held in the
// library's own device memory.  Each device that the library runs on keeps
// its copy until the process ends.  On the host `scratch` names a stand-in,
// never the device memory: host code uses only the address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t kNoAllocScratchBytes = (size_t)SPH_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// Device address of this device's scratch, looked up once per device with that
// device current.  Returns hipSuccess and sets *out, or the failing error.
static hipError_t scratch_ptr(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace sph

using namespace sph;

extern "C" {

void sph_default_params(sph_params *p) {
    if (!p) return;
    memset(p, 0, sizeof(*p));
    p->abi_version = SPH_ABI_VERSION;
    p->precision = SPH_FP64;
    p->io_dtype = SPH_F64;
    p->mode = SPH_BAND;
    p->periodic = 1;
    p->max_iter = 64;
    p->box = 1.0;
    p->n_target = 64.0;
    p->n_tol = 2.0;
    p->root_tol = 1e-12;
    p->cell_level = -1;
    p->tile_cell = -1;
    p->waves_per_cu = 16;
    p->segment = 16;
}

int sph_workspace_size(const sph_params *params, int64_t n, int32_t n_groups, size_t *bytes) {
    if (!bytes || !params) return SPH_E_INVALID;
    // group offsets are only inspected for presence; the size needs none
    const int64_t dummy = 0;
    const int rc = check_params(params, n, n_groups, params->periodic ? nullptr : &dummy);
    if (rc != SPH_OK) return rc;
    Plan pl;
    make_plan(params, n, n_groups, nullptr, &pl);
    *bytes = pl.total;
    return SPH_OK;
}

int sph_sort(const sph_params *params, int64_t n, int32_t n_groups, const int64_t *group_offsets,
             const void *x, const void *y, const void *z, uint64_t *keys_out, int32_t *perm_out,
             uint64_t *cell_id_out, int32_t *cell_start_out, int32_t *cell_count_out,
             int32_t *n_cells_out, void *ws, size_t ws_bytes, void *stream) {
    int rc = check_params(params, n, n_groups, group_offsets);
    if (rc != SPH_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (n == 0) {
        if (n_cells_out) {
            hipLaunchKernelGGL(k_store_i32, dim3(1), dim3(1), 0, st, n_cells_out, 0);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return hip_fail(e);
        }
        return SPH_OK;
    }
    if (!x || !y || !z || !keys_out || !perm_out) return SPH_E_INVALID;
    {
        const uintptr_t es = params->io_dtype == SPH_F32 ? 4 : 8;
        if (!aligned(x, es) || !aligned(y, es) || !aligned(z, es)) return SPH_E_INVALID;
    }
    Plan pl;
    rc = check_ws(params, n, n_groups, ws, ws_bytes, &pl);
    if (rc != SPH_OK) return rc;
    hipError_t e = run_clean_offsets(pl, group_offsets, st);
    const int64_t *goff = pl.goff;
    if (e == hipSuccess) e = run_keys_and_sort(pl, goff, x, y, z, st, keys_out, perm_out);
    if (e == hipSuccess && (cell_id_out || cell_start_out || cell_count_out || n_cells_out))
        e = run_contract_cells(pl, cell_id_out, cell_start_out, cell_count_out, n_cells_out, st);
    if (e != hipSuccess) return hip_fail(e);
    return SPH_OK;
}

int sph_density_solve(const sph_params *params, int64_t n, int32_t n_groups,
                      const int64_t *group_offsets, const void *x, const void *y, const void *z,
                      const void *m, const void *h_init, void *rho_out, void *h_out, void *nw_out,
                      int32_t *nngb_out, int32_t *status_out, uint64_t *stats_out, void *ws,
                      size_t ws_bytes, void *stream) {
    int rc = check_params(params, n, n_groups, group_offsets);
    if (rc != SPH_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (n == 0) {
        if (stats_out) {
            hipError_t e = run_zero_u64(stats_out, 4, st);
            if (e != hipSuccess) return hip_fail(e);
        }
        return SPH_OK;
    }
    if (!x || !y || !z || !m || !rho_out || !h_out) return SPH_E_INVALID;
    {
        const uintptr_t es = params->io_dtype == SPH_F32 ? 4 : 8;
        if (!aligned(x, es) || !aligned(y, es) || !aligned(z, es) || !aligned(m, es) ||
            !aligned(h_init, es) || !aligned(rho_out, es) || !aligned(h_out, es) ||
            !aligned(nw_out, es) || !aligned(nngb_out, 4) || !aligned(status_out, 4))
            return SPH_E_INVALID;
    }
    Plan pl;
    rc = check_ws(params, n, n_groups, ws, ws_bytes, &pl);
    if (rc != SPH_OK) return rc;
    const bool f32c = params->precision == SPH_FP32C;
    hipError_t e = run_clean_offsets(pl, group_offsets, st);
    const int64_t *goff = pl.goff;
    if (e == hipSuccess) e = run_keys_and_sort(pl, goff, x, y, z, st);
    if (e == hipSuccess) e = run_permute(pl, goff, x, y, z, m, h_init, f32c, st);
    if (e == hipSuccess) {
        if (!pl.grouped) e = run_dense_table(pl, st);
        else e = run_group_items(pl, goff, st);
    }
    if (e == hipSuccess)
        e = run_solve(pl, goff, rho_out, h_out, nw_out, nngb_out, status_out, stats_out, st);
    if (e != hipSuccess) return hip_fail(e);
    return SPH_OK;
}

int sph_density_backward(const sph_params *params, int64_t n, int32_t n_groups,
                         const int64_t *group_offsets, const void *x, const void *y,
                         const void *z, const void *m, const void *h, const void *grad_rho,
                         const void *grad_h, void *grad_x, void *grad_y, void *grad_z,
                         void *grad_m, void *ws, size_t ws_bytes, void *stream) {
    int rc = check_params(params, n, n_groups, group_offsets);
    if (rc != SPH_OK) return rc;
    if (params->mode == SPH_KNN) return SPH_E_UNSUPPORTED;
    if (n == 0) return SPH_OK;
    if (!x || !y || !z || !m || !h || !grad_rho || !grad_x || !grad_y || !grad_z || !grad_m)
        return SPH_E_INVALID;
    {
        const uintptr_t es = params->io_dtype == SPH_F32 ? 4 : 8;
        if (!aligned(x, es) || !aligned(y, es) || !aligned(z, es) || !aligned(m, es) ||
            !aligned(h, es) || !aligned(grad_rho, es) || !aligned(grad_h, es) ||
            !aligned(grad_x, es) || !aligned(grad_y, es) || !aligned(grad_z, es) ||
            !aligned(grad_m, es))
            return SPH_E_INVALID;
    }
    Plan pl;
    rc = check_ws(params, n, n_groups, ws, ws_bytes, &pl);
    if (rc != SPH_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    const bool f32c = params->precision == SPH_FP32C;
    // group work items of the adjoint are its tiles
    pl.prm.segment = kAdjTile;
    hipError_t e = run_clean_offsets(pl, group_offsets, st);
    const int64_t *goff = pl.goff;
    if (e == hipSuccess) e = run_keys_and_sort(pl, goff, x, y, z, st);
    if (e == hipSuccess) e = run_permute(pl, goff, x, y, z, m, h, f32c, st);
    if (e == hipSuccess) {
        if (!pl.grouped) e = run_dense_table(pl, st);
        else e = run_group_items(pl, goff, st);
    }
    if (e == hipSuccess)
        e = run_backward(pl, goff, h, grad_rho, grad_h, grad_x, grad_y, grad_z, grad_m, st);
    if (e != hipSuccess) return hip_fail(e);
    return SPH_OK;
}


int sph_pressure_force(const sph_params *params, int64_t n, int32_t n_groups,
                       const int64_t *group_offsets, const void *x, const void *y,
                       const void *z, const void *m, const void *h, const void *rho,
                       const void *pressure, void *ax_out, void *ay_out, void *az_out,
                       void *ws, size_t ws_bytes, void *stream) {
    int rc = check_params(params, n, n_groups, group_offsets);
    if (rc != SPH_OK) return rc;
    if (params->mode == SPH_KNN) return SPH_E_UNSUPPORTED;
    if (n == 0) return SPH_OK;
    if (!x || !y || !z || !m || !h || !rho || !pressure || !ax_out || !ay_out || !az_out)
        return SPH_E_INVALID;
    {
        const uintptr_t es = params->io_dtype == SPH_F32 ? 4 : 8;
        if (!aligned(x, es) || !aligned(y, es) || !aligned(z, es) || !aligned(m, es) ||
            !aligned(h, es) || !aligned(rho, es) || !aligned(pressure, es) ||
            !aligned(ax_out, es) || !aligned(ay_out, es) || !aligned(az_out, es))
            return SPH_E_INVALID;
    }
    Plan pl;
    rc = check_ws(params, n, n_groups, ws, ws_bytes, &pl);
    if (rc != SPH_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    const bool f32c = params->precision == SPH_FP32C;
    pl.prm.segment = kAdjTile;
    hipError_t e = run_clean_offsets(pl, group_offsets, st);
    const int64_t *goff = pl.goff;
    if (e == hipSuccess) e = run_keys_and_sort(pl, goff, x, y, z, st);
    if (e == hipSuccess) e = run_permute(pl, goff, x, y, z, m, h, f32c, st);
    if (e == hipSuccess) {
        if (!pl.grouped) e = run_dense_table(pl, st);
        else e = run_group_items(pl, goff, st);
    }
    if (e == hipSuccess)
        e = run_force(pl, goff, m, rho, pressure, ax_out, ay_out, az_out, st);
    if (e != hipSuccess) return hip_fail(e);
    return SPH_OK;
}

int sph_density_scatter(const sph_params *params, int64_t n, int32_t n_groups,
                        const int64_t *group_offsets, const void *x, const void *y,
                        const void *z, const void *m, const void *h, void *rho_s_out,
                        void *rho_sym_out, int32_t *nngb_s_out, void *ws, size_t ws_bytes,
                        void *stream) {
    int rc = check_params(params, n, n_groups, group_offsets);
    if (rc != SPH_OK) return rc;
    if (n == 0) return SPH_OK;
    if (!x || !y || !z || !m || !h || !rho_s_out) return SPH_E_INVALID;
    {
        const uintptr_t es = params->io_dtype == SPH_F32 ? 4 : 8;
        if (!aligned(x, es) || !aligned(y, es) || !aligned(z, es) || !aligned(m, es) ||
            !aligned(h, es) || !aligned(rho_s_out, es) || !aligned(rho_sym_out, es) ||
            !aligned(nngb_s_out, 4))
            return SPH_E_INVALID;
    }
    Plan pl;
    rc = check_ws(params, n, n_groups, ws, ws_bytes, &pl);
    if (rc != SPH_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    const bool f32c = params->precision == SPH_FP32C;
    // the walk's group work items are its tiles
    pl.prm.segment = kAdjTile;
    hipError_t e = run_clean_offsets(pl, group_offsets, st);
    const int64_t *goff = pl.goff;
    if (e == hipSuccess) e = run_keys_and_sort(pl, goff, x, y, z, st);
    if (e == hipSuccess) e = run_permute(pl, goff, x, y, z, m, h, f32c, st);
    if (e == hipSuccess) {
        if (!pl.grouped) e = run_dense_table(pl, st);
        else e = run_group_items(pl, goff, st);
    }
    if (e == hipSuccess) e = run_scatter(pl, goff, rho_s_out, rho_sym_out, nngb_s_out, st);
    if (e != hipSuccess) return hip_fail(e);
    return SPH_OK;
}

int sph_density_solve_noalloc(const sph_params *params, int64_t n, int32_t n_groups,
                              const int64_t *group_offsets, const void *x, const void *y,
                              const void *z, const void *m, const void *h_init, void *rho_out,
                              void *h_out, void *nw_out, int32_t *nngb_out, int32_t *status_out,
                              uint64_t *stats_out, void *stream) {
    int rc = check_params(params, n, n_groups, group_offsets);
    if (rc != SPH_OK) return rc;
    Plan probe;
    make_plan(params, n, n_groups, nullptr, &probe);
    if (probe.total > kNoAllocScratchBytes) return SPH_E_WORKSPACE;
    void *ws = nullptr;
    const hipError_t e = scratch_ptr(&ws);
    if (e != hipSuccess) return hip_fail(e);
    return sph_density_solve(params, n, n_groups, group_offsets, x, y, z, m, h_init, rho_out,
                             h_out, nw_out, nngb_out, status_out, stats_out, ws,
                             kNoAllocScratchBytes, stream);
}

const char *sph_status_string(int code) {
    switch (code) {
        case SPH_OK: return "SPH_OK: success";
        case SPH_E_INVALID: return "SPH_E_INVALID: invalid argument";
        case SPH_E_WORKSPACE: return "SPH_E_WORKSPACE: workspace too small";
        case SPH_E_HIP: return "SPH_E_HIP: a HIP call failed (see sph_last_hip_error)";
        case SPH_E_UNSUPPORTED: return "SPH_E_UNSUPPORTED: unsupported parameter combination";
        default: return "unknown status code";
    }
}

int sph_last_hip_error(void) { return g_last_hip; }

int sph_sort_wait_faults(uint32_t *count) {
    if (!count) return SPH_E_INVALID;
    const hipError_t e = read_sort_wait_faults(count);
    if (e != hipSuccess) return hip_fail(e);
    return SPH_OK;
}

const char *sph_last_hip_error_string(void) {
    return hipGetErrorString((hipError_t)g_last_hip);
}

}  // extern "C"
