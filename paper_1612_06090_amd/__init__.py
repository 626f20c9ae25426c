"""MI355X (gfx950) SPH density path: thin Python binding over libsph.so.

Argument marshalling only: every step of the path (Morton keys, radix sort,
cell tables, density and smoothing-length solve, adjoint) runs in the HIP
library.  PyTorch supplies device memory and the current stream.  There is no
fallback: if the library is missing, or a tensor is not on a GPU, the call
raises.

Functions mirror the C ABI of ``include/sph.h``:
``workspace_size``, ``sort``, ``density_solve``, ``density_backward``;
``density`` and :class:`SPHDensity` are conveniences on top.
"""
from __future__ import annotations

import ctypes as C
import os

__all__ = [
    "LIB_PATH", "Params", "SPHError", "load", "default_params", "workspace_size", "sort",
    "density_solve", "density_solve_noalloc", "density_backward", "density_scatter", "pressure_force", "autotune",
    "density", "SPHDensity",
    "status_string",
    "FP64", "FP32C", "F64", "F32", "BAND", "ROOT", "KNN", "KERNEL_M4", "KERNEL_WENDLAND_C6",
    "ST_NOCONV", "ST_HTOOLARGE", "ST_BADINPUT", "ST_UNREACHABLE",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsph.so")

FP64, FP32C = 0, 1
F64, F32 = 0, 1
BAND, ROOT, KNN = 0, 1, 2
ABI_VERSION = 1
OK, E_INVALID, E_WORKSPACE, E_HIP, E_UNSUPPORTED = 0, -1, -2, -3, -4
NOALLOC_SCRATCH_BYTES = 64 << 20
ST_NOCONV = 1 << 16
ST_HTOOLARGE = 1 << 17
ST_BADINPUT = 1 << 18
ST_UNREACHABLE = 1 << 19
KERNEL_M4, KERNEL_WENDLAND_C6 = 0, 1

EXPORTS = [
    "sph_default_params", "sph_workspace_size", "sph_sort", "sph_density_solve",
    "sph_density_backward", "sph_density_scatter", "sph_pressure_force", "sph_autotune",
    "sph_status_string",
    "sph_last_hip_error",
    "sph_last_hip_error_string",
    "sph_density_solve_noalloc",
    "sph_sort_wait_faults",
]


class Params(C.Structure):
    """Mirror of ``sph_params`` (include/sph.h)."""
    _fields_ = [
        ("abi_version", C.c_uint32),
        ("precision", C.c_int32),
        ("io_dtype", C.c_int32),
        ("mode", C.c_int32),
        ("periodic", C.c_int32),
        ("max_iter", C.c_int32),
        ("box", C.c_double),
        ("n_target", C.c_double),
        ("n_tol", C.c_double),
        ("root_tol", C.c_double),
        ("cell_level", C.c_int32),
        ("tile_cell", C.c_int32),
        ("waves_per_cu", C.c_int32),
        ("segment", C.c_int32),
        ("prof_events", C.c_void_p * 2),
        ("kernel", C.c_int32),
        ("in_stride", C.c_int32),
        ("out_stride", C.c_int32),
        ("reserved", C.c_int32 * 5),
    ]


class SPHError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = status_string(code)
        if code == E_HIP:
            lib = load()
            msg += f" (hip error {lib.sph_last_hip_error()}: " \
                   f"{lib.sph_last_hip_error_string().decode()})"
        super().__init__(f"{where}: {msg}")


_lib = None


def load():
    """Load libsph.so (built in-tree by ``__graft_entry__.build()``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "or python -m paper_1612_06090_amd.build")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    I64, I32, SZ = C.c_int64, C.c_int32, C.c_size_t
    PP = C.POINTER(Params)
    L.sph_default_params.argtypes = [PP]
    L.sph_default_params.restype = None
    L.sph_workspace_size.argtypes = [PP, I64, I32, C.POINTER(SZ)]
    L.sph_workspace_size.restype = C.c_int
    L.sph_sort.argtypes = [PP, I64, I32, P, P, P, P, P, P, P, P, P, P, P, SZ, P]
    L.sph_sort.restype = C.c_int
    L.sph_density_solve.argtypes = [PP, I64, I32, P, P, P, P, P, P, P, P, P, P, P, P, P, SZ, P]
    L.sph_density_solve.restype = C.c_int
    L.sph_density_solve_noalloc.argtypes = [PP, I64, I32, P, P, P, P, P, P, P, P, P, P, P, P, P]
    L.sph_density_solve_noalloc.restype = C.c_int
    L.sph_density_backward.argtypes = [PP, I64, I32, P, P, P, P, P, P, P, P, P, P, P, P, P, SZ, P]
    L.sph_density_backward.restype = C.c_int
    L.sph_density_scatter.argtypes = [PP, I64, I32, P, P, P, P, P, P, P, P, P, P, SZ, P]
    L.sph_density_scatter.restype = C.c_int
    L.sph_pressure_force.argtypes = [PP, I64, I32, P, P, P, P, P, P, P, P, P, P, P, P, SZ, P]
    L.sph_pressure_force.restype = C.c_int
    L.sph_autotune.argtypes = [PP, I64, I32, P, P, P, P, P, P, P, P, P, SZ, P, PP,
                               C.POINTER(C.c_float)]
    L.sph_autotune.restype = C.c_int
    L.sph_status_string.argtypes = [C.c_int]
    L.sph_status_string.restype = C.c_char_p
    L.sph_last_hip_error.argtypes = []
    L.sph_last_hip_error.restype = C.c_int
    L.sph_last_hip_error_string.argtypes = []
    L.sph_last_hip_error_string.restype = C.c_char_p
    L.sph_sort_wait_faults.argtypes = [C.POINTER(C.c_uint32)]
    L.sph_sort_wait_faults.restype = C.c_int
    _lib = L
    return L


def status_string(code: int) -> str:
    return load().sph_status_string(int(code)).decode()


def sort_wait_faults() -> int:
    """Look-back waits of the particle sort that reached their bound on the
    current device since the last call (synchronises; clears the count)."""
    v = C.c_uint32(0)
    rc = load().sph_sort_wait_faults(C.byref(v))
    if rc != OK:
        raise SPHError(rc, "sph_sort_wait_faults")
    return int(v.value)


def default_params(**kw) -> Params:
    """``sph_default_params`` then field overrides, e.g. ``precision=FP32C``."""
    p = Params()
    load().sph_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def workspace_size(params: Params, n: int, n_groups: int = 0) -> int:
    out = C.c_size_t(0)
    rc = load().sph_workspace_size(C.byref(params), int(n), int(n_groups), C.byref(out))
    if rc != OK:
        raise SPHError(rc, "sph_workspace_size")
    return int(out.value)


# ------------------------------------------------------------- marshalling

def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(device):
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


_ws_cache: dict = {}


def workspace(params: Params, n: int, n_groups: int, device):
    """A cached device workspace large enough for (params, n, n_groups)."""
    torch = _torch()
    need = workspace_size(params, n, n_groups)
    key = (str(device),)
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < need:
        buf = torch.empty(max(need, 256), dtype=torch.uint8, device=device)
        _ws_cache[key] = buf
    return buf


def _check_dev(*ts):
    dev = None
    for t in ts:
        if t is None:
            continue
        if not t.is_cuda:
            raise ValueError("libsph works on GPU tensors only")
        if t.dtype == _torch().int64 and not t.is_contiguous():
            raise ValueError("group offsets must be contiguous")
        if dev is None:
            dev = t.device
        elif t.device != dev:
            raise ValueError("all arrays must be on one device")
    return dev


def _check_offsets(goff, n):
    """Host check of group offsets: non-decreasing from 0 to n.

    The library itself replaces malformed offsets by the nearest well-formed
    ones on the device (so no kernel reads out of range); this check turns
    them into an error instead.  It reads the offsets back (a synchronising
    copy), so it is skipped while a HIP graph is being captured.
    """
    if goff is None:
        return
    torch = _torch()
    if goff.dtype != torch.int64 or goff.dim() != 1 or goff.shape[0] < 2:
        raise ValueError("group offsets must be a 1-D int64 tensor of n_groups + 1 entries")
    if torch.cuda.is_current_stream_capturing():
        return
    o = goff.cpu()
    if int(o[0]) != 0 or int(o[-1]) != n or bool((o[1:] < o[:-1]).any()):
        raise ValueError("group offsets must be non-decreasing with offsets[0] = 0 and "
                         "offsets[n_groups] = n")


def _stride_bytes(*ts):
    """Common byte stride of 1-D per-particle tensors (0: all packed).

    Packed arrays have stride 1; fields of an array of particle structs are
    strided views (e.g. ``P[:, 0]`` of an (n, k) tensor) that must share one
    byte stride, the struct size.
    """
    seen = set()
    for t in ts:
        if t is None:
            continue
        if t.dim() != 1:
            raise ValueError("per-particle arrays must be 1-D")
        if t.shape[0] > 1:
            seen.add(0 if t.stride(0) == 1 else t.stride(0) * t.element_size())
    if len(seen) > 1:
        raise ValueError("per-particle arrays must all be packed or share one byte stride")
    return seen.pop() if seen else 0


def _with_strides(params: Params, ins: int, outs: int) -> Params:
    q = Params.from_buffer_copy(params)
    q.in_stride = ins
    q.out_stride = outs
    return q


def _io(params: Params):
    torch = _torch()
    return torch.float32 if params.io_dtype == F32 else torch.float64


def sort(x, y, z, params: Params | None = None, group_offsets=None, cells=True):
    """Morton keys, stable radix sort and cell table (``sph_sort``).

    Returns dict(keys, perm, cell_id, cell_start, cell_count, n_cells) of
    device tensors, cells trimmed to n_cells.
    """
    torch = _torch()
    params = params or default_params()
    dev = _check_dev(x, y, z, group_offsets)
    n = x.shape[0]
    G = 0 if group_offsets is None else group_offsets.shape[0] - 1
    _check_offsets(group_offsets, n)
    ws = workspace(params, n, G, dev)
    keys = torch.empty(n, dtype=torch.int64, device=dev)
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    cid = torch.empty(max(n, 1), dtype=torch.int64, device=dev) if cells else None
    cst = torch.empty(max(n, 1), dtype=torch.int32, device=dev) if cells else None
    ccn = torch.empty(max(n, 1), dtype=torch.int32, device=dev) if cells else None
    nc = torch.zeros(1, dtype=torch.int32, device=dev) if cells else None
    params = _with_strides(params, _stride_bytes(x, y, z), 0)
    rc = load().sph_sort(C.byref(params), n, G, _ptr(group_offsets), _ptr(x), _ptr(y), _ptr(z),
                         _ptr(keys), _ptr(perm), _ptr(cid), _ptr(cst), _ptr(ccn), _ptr(nc),
                         _ptr(ws), ws.numel(), _stream(dev))
    if rc != OK:
        raise SPHError(rc, "sph_sort")
    out = dict(keys=keys, perm=perm)
    if cells:
        k = int(nc.item())
        out.update(cell_id=cid[:k], cell_start=cst[:k], cell_count=ccn[:k], n_cells=k)
    return out


def density_solve(x, y, z, m, h_init=None, params: Params | None = None, group_offsets=None,
                  stats=False, ws=None, out=None):
    """``sph_density_solve``: returns dict(rho, h, nw, nngb, status[, stats]).

    Inputs may be strided views into an array of particle structs (one common
    byte stride); ``out`` may hold preallocated outputs (rho and h required;
    nw, nngb, status optional), also strided views sharing one byte stride,
    which the library then writes in place.
    """
    torch = _torch()
    params = params or default_params()
    dev = _check_dev(x, y, z, m, h_init, group_offsets)
    n = x.shape[0]
    G = 0 if group_offsets is None else group_offsets.shape[0] - 1
    _check_offsets(group_offsets, n)
    if ws is None:
        ws = workspace(params, n, G, dev)
    dt = _io(params)
    if out is None:
        rho = torch.empty(n, dtype=dt, device=dev)
        h = torch.empty(n, dtype=dt, device=dev)
        nw = torch.empty(n, dtype=dt, device=dev)
        nngb = torch.empty(n, dtype=torch.int32, device=dev)
        status = torch.empty(n, dtype=torch.int32, device=dev)
    else:
        rho, h = out["rho"], out["h"]
        nw, nngb, status = out.get("nw"), out.get("nngb"), out.get("status")
        _check_dev(rho, h, nw, nngb, status)
    prm = _with_strides(params, _stride_bytes(x, y, z, m, h_init),
                        _stride_bytes(rho, h, nw, nngb, status))
    st = torch.zeros(4, dtype=torch.int64, device=dev) if stats else None
    rc = load().sph_density_solve(C.byref(prm), n, G, _ptr(group_offsets), _ptr(x), _ptr(y),
                                  _ptr(z), _ptr(m), _ptr(h_init), _ptr(rho), _ptr(h), _ptr(nw),
                                  _ptr(nngb), _ptr(status), _ptr(st), _ptr(ws), ws.numel(),
                                  _stream(dev))
    if rc != OK:
        raise SPHError(rc, "sph_density_solve")
    res = dict(rho=rho, h=h, nw=nw, nngb=nngb, status=status)
    if stats:
        res["stats"] = st
    return res


def density_solve_noalloc(x, y, z, m, h_init=None, params: Params | None = None,
                          group_offsets=None, stats=False, out=None):
    """``sph_density_solve_noalloc``: as ``density_solve``, with the library's
    fixed device scratch instead of a caller workspace (the C call allocates
    nothing; this wrapper allocates the outputs unless ``out`` gives them).
    Raises SPHError(E_WORKSPACE) when the set needs more than
    NOALLOC_SCRATCH_BYTES of workspace.
    """
    torch = _torch()
    params = params or default_params()
    dev = _check_dev(x, y, z, m, h_init, group_offsets)
    n = x.shape[0]
    G = 0 if group_offsets is None else group_offsets.shape[0] - 1
    _check_offsets(group_offsets, n)
    dt = _io(params)
    if out is None:
        out = dict(rho=torch.empty(n, dtype=dt, device=dev),
                   h=torch.empty(n, dtype=dt, device=dev),
                   nw=torch.empty(n, dtype=dt, device=dev),
                   nngb=torch.empty(n, dtype=torch.int32, device=dev),
                   status=torch.empty(n, dtype=torch.int32, device=dev))
    rho, h = out["rho"], out["h"]
    nw, nngb, status = out.get("nw"), out.get("nngb"), out.get("status")
    _check_dev(rho, h, nw, nngb, status)
    prm = _with_strides(params, _stride_bytes(x, y, z, m, h_init),
                        _stride_bytes(rho, h, nw, nngb, status))
    st = torch.zeros(4, dtype=torch.int64, device=dev) if stats else None
    rc = load().sph_density_solve_noalloc(C.byref(prm), n, G, _ptr(group_offsets), _ptr(x),
                                          _ptr(y), _ptr(z), _ptr(m), _ptr(h_init), _ptr(rho),
                                          _ptr(h), _ptr(nw), _ptr(nngb), _ptr(status),
                                          _ptr(st), _stream(dev))
    if rc != OK:
        raise SPHError(rc, "sph_density_solve_noalloc")
    res = dict(rho=rho, h=h, nw=nw, nngb=nngb, status=status)
    if stats:
        res["stats"] = st
    return res


def density_backward(x, y, z, m, h, grad_rho, grad_h=None, params: Params | None = None,
                     group_offsets=None, ws=None, out=None):
    """``sph_density_backward``: returns dict(gx, gy, gz, gm).

    Strided inputs and preallocated strided ``out`` (gx, gy, gz, gm) as in
    ``density_solve``.
    """
    torch = _torch()
    params = params or default_params()
    dev = _check_dev(x, y, z, m, h, grad_rho, grad_h, group_offsets)
    n = x.shape[0]
    G = 0 if group_offsets is None else group_offsets.shape[0] - 1
    _check_offsets(group_offsets, n)
    if ws is None:
        ws = workspace(params, n, G, dev)
    dt = _io(params)
    if out is None:
        gx, gy, gz, gm = (torch.empty(n, dtype=dt, device=dev) for _ in range(4))
    else:
        gx, gy, gz, gm = out["gx"], out["gy"], out["gz"], out["gm"]
        _check_dev(gx, gy, gz, gm)
    prm = _with_strides(params, _stride_bytes(x, y, z, m, h, grad_rho, grad_h),
                        _stride_bytes(gx, gy, gz, gm))
    rc = load().sph_density_backward(C.byref(prm), n, G, _ptr(group_offsets), _ptr(x), _ptr(y),
                                     _ptr(z), _ptr(m), _ptr(h), _ptr(grad_rho), _ptr(grad_h),
                                     _ptr(gx), _ptr(gy), _ptr(gz), _ptr(gm), _ptr(ws),
                                     ws.numel(), _stream(dev))
    if rc != OK:
        raise SPHError(rc, "sph_density_backward")
    return dict(gx=gx, gy=gy, gz=gz, gm=gm)


def density_scatter(x, y, z, m, h, params: Params | None = None, group_offsets=None, ws=None,
                    out=None):
    """``sph_density_scatter``: Eq. (1) with each neighbour's own h_j.

    Returns dict(rho_s, rho_sym, nngb_s); strided inputs and preallocated
    strided ``out`` (rho_s required, rho_sym and nngb_s optional) as in
    ``density_solve``.
    """
    torch = _torch()
    params = params or default_params()
    dev = _check_dev(x, y, z, m, h, group_offsets)
    n = x.shape[0]
    G = 0 if group_offsets is None else group_offsets.shape[0] - 1
    _check_offsets(group_offsets, n)
    if ws is None:
        ws = workspace(params, n, G, dev)
    dt = _io(params)
    if out is None:
        rs = torch.empty(n, dtype=dt, device=dev)
        rsym = torch.empty(n, dtype=dt, device=dev)
        cnt = torch.empty(n, dtype=torch.int32, device=dev)
    else:
        rs, rsym, cnt = out["rho_s"], out.get("rho_sym"), out.get("nngb_s")
        _check_dev(rs, rsym, cnt)
    prm = _with_strides(params, _stride_bytes(x, y, z, m, h), _stride_bytes(rs, rsym, cnt))
    rc = load().sph_density_scatter(C.byref(prm), n, G, _ptr(group_offsets), _ptr(x), _ptr(y),
                                    _ptr(z), _ptr(m), _ptr(h), _ptr(rs), _ptr(rsym), _ptr(cnt),
                                    _ptr(ws), ws.numel(), _stream(dev))
    if rc != OK:
        raise SPHError(rc, "sph_density_scatter")
    return dict(rho_s=rs, rho_sym=rsym, nngb_s=cnt)


def pressure_force(x, y, z, m, h, rho, pressure, params: Params | None = None,
                   group_offsets=None, ws=None, out=None):
    """``sph_pressure_force``: the grad-h SPH pressure acceleration,
    dict(ax, ay, az); strided inputs and preallocated strided ``out`` as in
    ``density_solve``."""
    torch = _torch()
    params = params or default_params()
    dev = _check_dev(x, y, z, m, h, rho, pressure, group_offsets)
    n = x.shape[0]
    G = 0 if group_offsets is None else group_offsets.shape[0] - 1
    _check_offsets(group_offsets, n)
    if ws is None:
        ws = workspace(params, n, G, dev)
    dt = _io(params)
    if out is None:
        ax, ay, az = (torch.empty(n, dtype=dt, device=dev) for _ in range(3))
    else:
        ax, ay, az = out["ax"], out["ay"], out["az"]
        _check_dev(ax, ay, az)
    prm = _with_strides(params, _stride_bytes(x, y, z, m, h, rho, pressure),
                        _stride_bytes(ax, ay, az))
    rc = load().sph_pressure_force(C.byref(prm), n, G, _ptr(group_offsets), _ptr(x), _ptr(y),
                                   _ptr(z), _ptr(m), _ptr(h), _ptr(rho), _ptr(pressure),
                                   _ptr(ax), _ptr(ay), _ptr(az), _ptr(ws), ws.numel(),
                                   _stream(dev))
    if rc != OK:
        raise SPHError(rc, "sph_pressure_force")
    return dict(ax=ax, ay=ay, az=az)


def autotune(x, y, z, m, h_init=None, params: Params | None = None, group_offsets=None, ws=None):
    """``sph_autotune``: returns (tuned Params, its time per solve in ms)."""
    torch = _torch()
    params = params or default_params()
    dev = _check_dev(x, y, z, m, h_init, group_offsets)
    n = x.shape[0]
    G = 0 if group_offsets is None else group_offsets.shape[0] - 1
    _check_offsets(group_offsets, n)
    if ws is None:
        ws = workspace(params, n, G, dev)
    dt = _io(params)
    rho = torch.empty(max(n, 1), dtype=dt, device=dev)
    h = torch.empty(max(n, 1), dtype=dt, device=dev)
    best = Params()
    ms = C.c_float(0.0)
    params = _with_strides(params, _stride_bytes(x, y, z, m, h_init), 0)
    rc = load().sph_autotune(C.byref(params), n, G, _ptr(group_offsets), _ptr(x), _ptr(y),
                             _ptr(z), _ptr(m), _ptr(h_init), _ptr(rho), _ptr(h), _ptr(ws),
                             ws.numel(), _stream(dev), C.byref(best), C.byref(ms))
    if rc != OK:
        raise SPHError(rc, "sph_autotune")
    return best, float(ms.value)


def density(pos, m, h_init=None, group_offsets=None, **params):
    """Solve for (rho, h, nw, nngb, status) from an (n, 3) position tensor."""
    prm = default_params(**params)
    if group_offsets is not None:
        prm.periodic = 0
    x, y, z = (pos[:, a].contiguous() for a in range(3))
    o = density_solve(x, y, z, m.contiguous(), None if h_init is None else h_init.contiguous(),
                      prm, group_offsets)
    return o["rho"], o["h"], o["nw"], o["nngb"], o["status"]


def _make_autograd():
    torch = _torch()

    class SPHDensity(torch.autograd.Function):
        """(rho, h) = SPHDensity.apply(pos, m, params[, group_offsets[, h_init]]).

        Backward runs the hand-written adjoint (``sph_density_backward``)
        with each h held on its implicit root, so gradients flow to
        positions (and masses) including the dependence through h.
        """

        @staticmethod
        def forward(ctx, pos, m, params, group_offsets=None, h_init=None):
            params = params or default_params()
            x, y, z = (pos[:, a].contiguous() for a in range(3))
            m = m.contiguous()
            h0 = None if h_init is None else h_init.detach().contiguous()
            o = density_solve(x, y, z, m, h0, params, group_offsets)
            ctx.save_for_backward(x, y, z, m, o["h"])
            ctx.params = params
            ctx.goff = group_offsets
            return o["rho"], o["h"]

        @staticmethod
        def backward(ctx, grad_rho, grad_h):
            x, y, z, m, h = ctx.saved_tensors
            gr = grad_rho.contiguous() if grad_rho is not None else torch.zeros_like(h)
            gh = grad_h.contiguous() if grad_h is not None else None
            g = density_backward(x, y, z, m, h, gr, gh, ctx.params, ctx.goff)
            gpos = torch.stack([g["gx"], g["gy"], g["gz"]], dim=1)
            # h_init only starts the iteration: the converged h does not depend on it
            return gpos, g["gm"], None, None, None

    return SPHDensity


class _Lazy:
    _cls = None

    def __get__(self, obj, owner):
        if _Lazy._cls is None:
            _Lazy._cls = _make_autograd()
        return _Lazy._cls


class _Namespace:
    SPHDensity = _Lazy()


def __getattr__(name):
    if name == "SPHDensity":
        return _Namespace.SPHDensity
    raise AttributeError(name)
