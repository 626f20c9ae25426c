"""CPU oracle for the SPH density path -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package.  The product (the HIP library and
its Python binding) never imports it, and it imports nothing from the
product: the two share only the seeded inputs drawn by ``sphgen``.

The arithmetic lives in ``sph_oracle.c`` (plain C, IEEE binary64, built with
``-ffp-contract=off``).  This module compiles it with gcc when the shared
object is missing or older than its source, and marshals NumPy arrays.

Paper: Baruffa et al., arXiv:1612.06090 -- Eq. (1) (density sum),
Listing 1 (neighbour loop with the in-support test), Sec. IV-A with
Listings 2/3 (recompute loop over particles whose neighbour criterion
fails, dynamic scheduling).  Readings where the paper is silent (kernel
function, whose h, update rule, tolerance band) are documented in the
C source header.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sph_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ST_NOCONV = 1 << 16
ST_HTOOLARGE = 1 << 17
ST_BADINPUT = 1 << 18
ST_UNREACHABLE = 1 << 19

BAND = 0
ROOT = 1


def build(force: bool = False) -> str:
    """Compile the oracle shared object with gcc (plain C11 + OpenMP)."""
    if (not force and os.path.exists(_LIB)
            and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC)):
        return _LIB
    tmp = _LIB + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


class _Cfg(C.Structure):
    _fields_ = [
        ("periodic", C.c_int32),
        ("box", C.c_double),
        ("ngroups", C.c_int32),
        ("offsets", C.c_void_p),
        ("n_target", C.c_double),
        ("n_tol", C.c_double),
        ("mode", C.c_int32),
        ("root_tol", C.c_double),
        ("max_iter", C.c_int32),
        ("search", C.c_int32),
        ("nthreads", C.c_int32),
        ("kernel", C.c_int32),
    ]


def lib():
    global _lib
    if _lib is None:
        # SPH_ORACLE_LIB names another build of the same source (the tests load
        # an AddressSanitizer / UBSan build this way)
        path = os.environ.get("SPH_ORACLE_LIB") or build()
        L = C.CDLL(path)
        P = C.c_void_p
        L.oracle_kernel_f.restype = C.c_double
        L.oracle_kernel_f.argtypes = [C.c_double]
        L.oracle_kernel_dfdq.restype = C.c_double
        L.oracle_kernel_dfdq.argtypes = [C.c_double]
        L.oracle_kernel_W.restype = C.c_double
        L.oracle_kernel_W.argtypes = [C.c_double, C.c_double]
        for name in ("oracle_wendland6_f", "oracle_wendland6_dfdq"):
            getattr(L, name).restype = C.c_double
            getattr(L, name).argtypes = [C.c_double]
        for name in ("oracle_f", "oracle_dfdq"):
            getattr(L, name).restype = C.c_double
            getattr(L, name).argtypes = [C.c_int32, C.c_double]
        for name in ("oracle_sigma", "oracle_count_const"):
            getattr(L, name).restype = C.c_double
            getattr(L, name).argtypes = [C.c_int32]
        L.oracle_morton_periodic.argtypes = [C.c_int64, P, P, P, C.c_double, P]
        L.oracle_morton_groups.argtypes = [C.c_int64, C.c_int32, P, P, P, P, P]
        L.oracle_group_frames.argtypes = [C.c_int32, P, P, P, P, P, P]
        L.oracle_stable_sort.argtypes = [C.c_int64, P, P, P]
        L.oracle_cell_level.restype = C.c_int32
        L.oracle_cell_level.argtypes = [C.c_int64, C.c_int32]
        L.oracle_cell_table.restype = C.c_int64
        L.oracle_cell_table.argtypes = [C.c_int64, P, C.c_int32, P, P, P]
        L.oracle_eval_at_h.argtypes = [C.POINTER(_Cfg), C.c_int64, P, P, P, P, P, P, P, P, P, P]
        L.oracle_solve.argtypes = [C.POINTER(_Cfg), C.c_int64, P, P, P, P, P, P, C.c_int64,
                                   P, P, P, P, P, P, P]
        L.oracle_backward.argtypes = [C.POINTER(_Cfg), C.c_int64, P, P, P, P, P, P, P,
                                      P, P, P, P]
        L.oracle_knn.argtypes = [C.POINTER(_Cfg), C.c_int64, P, P, P, P, P, C.c_int32,
                                 P, C.c_int64, P, P, P, P, P]
        L.oracle_scatter.argtypes = [C.POINTER(_Cfg), C.c_int64, P, P, P, P, P, P, P, P]
        L.oracle_max_threads.restype = C.c_int32
        L.oracle_max_threads.argtypes = []
        _lib = L
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def kernel_f(q: float) -> float:
    return lib().oracle_kernel_f(float(q))


def kernel_dfdq(q: float) -> float:
    return lib().oracle_kernel_dfdq(float(q))


def kernel_W(r: float, h: float) -> float:
    return lib().oracle_kernel_W(float(r), float(h))


M4, WENDLAND_C6 = 0, 1


def wendland6_f(q: float) -> float:
    return lib().oracle_wendland6_f(float(q))


def wendland6_dfdq(q: float) -> float:
    return lib().oracle_wendland6_dfdq(float(q))


def shape_f(kernel: int, q: float) -> float:
    """f(q) of the selected kernel (M4 or WENDLAND_C6)."""
    return lib().oracle_f(int(kernel), float(q))


def shape_dfdq(kernel: int, q: float) -> float:
    return lib().oracle_dfdq(int(kernel), float(q))


def sigma(kernel: int) -> float:
    """Normalisation: W(r, h) = sigma / h^3 f(r/h)."""
    return lib().oracle_sigma(int(kernel))


def count_const(kernel: int) -> float:
    """C in n = C sum_j f(r_ij / h)."""
    return lib().oracle_count_const(int(kernel))


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def morton_periodic(x, y, z, box: float) -> np.ndarray:
    x, y, z = _d(x), _d(y), _d(z)
    keys = np.empty(x.shape[0], dtype=np.uint64)
    lib().oracle_morton_periodic(x.shape[0], _p(x), _p(y), _p(z), float(box), _p(keys))
    return keys


def group_frames(offsets, x, y, z):
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    x, y, z = _d(x), _d(y), _d(z)
    g = offsets.shape[0] - 1
    org = np.empty(3 * g)
    sc = np.empty(g)
    lib().oracle_group_frames(g, _p(offsets), _p(x), _p(y), _p(z), _p(org), _p(sc))
    return org.reshape(g, 3), sc


def morton_groups(offsets, x, y, z) -> np.ndarray:
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    x, y, z = _d(x), _d(y), _d(z)
    keys = np.empty(x.shape[0], dtype=np.uint64)
    lib().oracle_morton_groups(x.shape[0], offsets.shape[0] - 1, _p(offsets), _p(x), _p(y),
                               _p(z), _p(keys))
    return keys


def stable_sort(keys):
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    n = keys.shape[0]
    srt = np.empty(n, dtype=np.uint64)
    perm = np.empty(n, dtype=np.int32)
    lib().oracle_stable_sort(n, _p(keys), _p(srt), _p(perm))
    return srt, perm


def cell_level(n: int, grouped: bool) -> int:
    return int(lib().oracle_cell_level(int(n), 16 if grouped else 21))


def cell_table(sorted_keys, level: int, grouped: bool):
    """Occupied cells at ``level``: (cell_id, start, count)."""
    sk = np.ascontiguousarray(sorted_keys, dtype=np.uint64)
    n = sk.shape[0]
    bits = 16 if grouped else 21
    shift = 3 * (bits - level)
    cid = np.empty(max(n, 1), dtype=np.uint64)
    st = np.empty(max(n, 1), dtype=np.int32)
    ct = np.empty(max(n, 1), dtype=np.int32)
    nc = lib().oracle_cell_table(n, _p(sk), shift, _p(cid), _p(st), _p(ct))
    return cid[:nc].copy(), st[:nc].copy(), ct[:nc].copy()


def sort(ps):
    """Keys, stable sort and contract cell table for a ParticleSet."""
    if ps.offsets is None:
        keys = morton_periodic(ps.x, ps.y, ps.z, ps.box)
    else:
        keys = morton_groups(ps.offsets, ps.x, ps.y, ps.z)
    srt, perm = stable_sort(keys)
    grouped = ps.offsets is not None
    lc = cell_level(ps.n, grouped)
    cid, st, ct = cell_table(srt, lc, grouped)
    return dict(keys=keys, sorted_keys=srt, perm=perm, level=lc, cell_id=cid,
                cell_start=st, cell_count=ct)


def _cfg(ps, mode=BAND, root_tol=1e-12, max_iter=64, search=1, nthreads=0, kernel=M4):
    off = None if ps.offsets is None else np.ascontiguousarray(ps.offsets, dtype=np.int64)
    c = _Cfg(
        periodic=1 if ps.periodic else 0, box=float(ps.box),
        ngroups=0 if off is None else off.shape[0] - 1,
        offsets=None if off is None else off.ctypes.data,
        n_target=float(ps.n_target), n_tol=float(ps.n_tol), mode=int(mode),
        root_tol=float(root_tol), max_iter=int(max_iter), search=int(search),
        nthreads=int(nthreads), kernel=int(kernel),
    )
    return c, off


def eval_at_h(ps, h, search=1, nthreads=0, kernel=M4):
    """rho, n, dn/dh, drho/dh and the integer neighbour count at given h."""
    c, _keep = _cfg(ps, search=search, nthreads=nthreads, kernel=kernel)
    x, y, z, m, h = _d(ps.x), _d(ps.y), _d(ps.z), _d(ps.m), _d(h)
    n = x.shape[0]
    rho, nw, dndh, drhodh = (np.empty(n) for _ in range(4))
    nngb = np.empty(n, dtype=np.int64)
    lib().oracle_eval_at_h(C.byref(c), n, _p(x), _p(y), _p(z), _p(m), _p(h), _p(rho), _p(nw),
                           _p(dndh), _p(drhodh), _p(nngb))
    return dict(rho=rho, nw=nw, dndh=dndh, drhodh=drhodh, nngb=nngb)


def solve(ps, h_init=None, subset=None, mode=BAND, root_tol=1e-12, max_iter=64, search=1,
          nthreads=0, kernel=M4):
    """Per-particle h iteration; returns rho, h, nw, dndh, nngb, status, pairs.

    With ``subset`` (array of particle indices) only those particles are
    solved, each against the full set, and outputs follow ``subset``'s order.
    """
    c, _keep = _cfg(ps, mode=mode, root_tol=root_tol, max_iter=max_iter, search=search,
                    nthreads=nthreads, kernel=kernel)
    x, y, z, m = _d(ps.x), _d(ps.y), _d(ps.z), _d(ps.m)
    h0 = _d(ps.h_init if h_init is None else h_init)
    n = x.shape[0]
    sub = None if subset is None else np.ascontiguousarray(subset, dtype=np.int64)
    cnt = n if sub is None else sub.shape[0]
    rho, h, nw, dndh = (np.empty(cnt) for _ in range(4))
    nngb = np.empty(cnt, dtype=np.int32)
    status = np.empty(cnt, dtype=np.int32)
    pairs = np.empty(cnt, dtype=np.int64)
    lib().oracle_solve(C.byref(c), n, _p(x), _p(y), _p(z), _p(m), _p(h0), _p(sub), cnt,
                       _p(rho), _p(h), _p(nw), _p(dndh), _p(nngb), _p(status), _p(pairs))
    return dict(rho=rho, h=h, nw=nw, dndh=dndh, nngb=nngb, status=status, pairs=pairs)


def knn(ps, K, h_init=None, subset=None, search=1, nthreads=0, kernel=M4):
    """Exact K-nearest criterion: h = distance of the K-th nearest particle
    (the particle itself first), rho etc. at that h; dict(rho, h, nw, nngb,
    status).  With ``subset`` only the listed particles are done (each against
    the full set) and outputs follow ``subset``'s order."""
    c, _keep = _cfg(ps, search=search, nthreads=nthreads, kernel=kernel)
    x, y, z, m = _d(ps.x), _d(ps.y), _d(ps.z), _d(ps.m)
    h0 = _d(ps.h_init if h_init is None else h_init)
    n = x.shape[0]
    sub = None if subset is None else np.ascontiguousarray(subset, dtype=np.int64)
    cnt = n if sub is None else sub.shape[0]
    rho, h, nw = (np.empty(cnt) for _ in range(3))
    nngb = np.empty(cnt, dtype=np.int32)
    status = np.empty(cnt, dtype=np.int32)
    lib().oracle_knn(C.byref(c), n, _p(x), _p(y), _p(z), _p(m), _p(h0), int(K),
                     None if sub is None else sub.ctypes.data_as(C.c_void_p), cnt, _p(rho),
                     _p(h), _p(nw), _p(nngb), _p(status))
    return dict(rho=rho, h=h, nw=nw, nngb=nngb, status=status)


def scatter(ps, h, search=1, nthreads=0, kernel=M4):
    """Eq. (1) with the neighbour's own h_j: dict(rho_s, rho_sym, nngb_s).

    rho_s_i = sum_j m_j W(r_ij, h_j) over r_ij < h_j (self included);
    rho_sym_i = (sum_j m_j W(r_ij, h_i) + rho_s_i) / 2; nngb_s_i = number of
    j whose sphere holds i.
    """
    c, _keep = _cfg(ps, search=search, nthreads=nthreads, kernel=kernel)
    x, y, z, m = _d(ps.x), _d(ps.y), _d(ps.z), _d(ps.m)
    h = _d(h)
    n = x.shape[0]
    rs, rsym = np.empty(n), np.empty(n)
    cnt = np.empty(n, dtype=np.int64)
    lib().oracle_scatter(C.byref(c), n, _p(x), _p(y), _p(z), _p(m), _p(h), _p(rs), _p(rsym),
                         cnt.ctypes.data_as(C.c_void_p))
    return dict(rho_s=rs, rho_sym=rsym, nngb_s=cnt)


def backward(ps, h, grad_rho, grad_h=None, search=1, nthreads=0, x=None, m=None, kernel=M4):
    """Analytic adjoint (gx, gy, gz, gm) of sum(grad_rho*rho + grad_h*h).

    ``x`` (an (n,3) array) and ``m`` override the set's positions / masses.
    """
    c, _keep = _cfg(ps, search=search, nthreads=nthreads, kernel=kernel)
    if x is None:
        px, py, pz = _d(ps.x), _d(ps.y), _d(ps.z)
    else:
        px, py, pz = _d(x[:, 0]), _d(x[:, 1]), _d(x[:, 2])
    mm = _d(ps.m if m is None else m)
    h = _d(h)
    gr = _d(grad_rho)
    gh = None if grad_h is None else _d(grad_h)
    n = px.shape[0]
    gx, gy, gz, gm = (np.empty(n) for _ in range(4))
    lib().oracle_backward(C.byref(c), n, _p(px), _p(py), _p(pz), _p(mm), _p(h), _p(gr), _p(gh),
                          _p(gx), _p(gy), _p(gz), _p(gm))
    return dict(gx=gx, gy=gy, gz=gz, gm=gm)


def pressure_force(ps, h, rho, P, search=1, nthreads=0, kernel=M4):
    """Pressure acceleration of the variational (grad-h) SPH equations with each
    h held on its count constraint: a_k = -(1/m_k) dE/dx_k for the thermal
    energy E = sum_i m_i u_i(rho_i) with du_i/drho_i = P_i/rho_i^2, which is
    the adjoint of the density with cotangent m_i P_i/rho_i^2 (implicit h
    included).  dict(ax, ay, az)."""
    m = _d(ps.m)
    gr = m * _d(P) / _d(rho) ** 2
    g = backward(ps, h, gr, None, search=search, nthreads=nthreads, kernel=kernel)
    return dict(ax=-g["gx"] / m, ay=-g["gy"] / m, az=-g["gz"] / m)
