"""Host-side checks of the C ABI (no GPU needed).

The library must load, export every function the header declares, agree with
a C compiler on the layout of ``sph_params``, and reject bad arguments on
the host before anything is enqueued.
"""
import ctypes as C
import os
import re
import subprocess

import pytest

import paper_1612_06090_amd as sph

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sph.h")


def _lib():
    if not os.path.exists(sph.LIB_PATH):
        from paper_1612_06090_amd import build
        build.build()
    return sph.load()


def test_exports_every_declared_function():
    text = open(HEADER).read()
    decl = set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(sph_\w+)\s*\(", text, re.M))
    assert {"sph_sort", "sph_density_solve", "sph_density_backward", "sph_workspace_size",
            "sph_status_string", "sph_default_params"} <= decl
    lib = _lib()
    for name in decl:
        assert hasattr(lib, name), name
    assert set(sph.EXPORTS) == decl
    out = subprocess.run(["nm", "-D", "--defined-only", sph.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    for name in decl:
        assert re.search(rf"\bT {name}\b", out), name


def test_params_layout_matches_c(tmp_path):
    src = tmp_path / "probe.c"
    fields = [f for f, _ in sph.Params._fields_]
    body = "\n".join(f'printf("{f} %zu\\n", offsetof(sph_params, {f}));' for f in fields)
    src.write_text(f'#include <stdio.h>\n#include <stddef.h>\n#include "{HEADER}"\n'
                   f'int main(void){{ printf("size %zu\\n", sizeof(sph_params));\n{body}\n'
                   f'return 0; }}\n')
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c11", "-o", str(exe), str(src)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                  check=True).stdout.splitlines())
    assert int(got["size"]) == C.sizeof(sph.Params)
    for f in fields:
        assert int(got[f]) == getattr(sph.Params, f).offset, f


def test_default_params():
    _lib()
    p = sph.default_params()
    assert p.abi_version == sph.ABI_VERSION
    assert (p.precision, p.io_dtype, p.mode, p.periodic) == (sph.FP64, sph.F64, sph.BAND, 1)
    assert (p.box, p.n_target, p.n_tol, p.root_tol) == (1.0, 64.0, 2.0, 1e-12)
    assert (p.max_iter, p.cell_level, p.segment, p.tile_cell) == (64, -1, 16, -1)
    assert p.waves_per_cu == 16 and p.kernel == sph.KERNEL_M4


def test_workspace_size_monotone_and_valid():
    _lib()
    p = sph.default_params()
    sizes = [sph.workspace_size(p, n) for n in (0, 1, 64, 4096, 1 << 20, 1 << 24)]
    assert all(b >= a for a, b in zip(sizes, sizes[1:]))
    assert sizes[-1] > 300 * (1 << 24) // 10
    q = sph.default_params(precision=sph.FP32C)
    assert sph.workspace_size(q, 1 << 20) > 0
    g = sph.default_params(periodic=0, n_target=32.0, n_tol=1.0)
    assert sph.workspace_size(g, 10000, 300) > 0


@pytest.mark.parametrize("field,value", [
    ("abi_version", 99), ("precision", 7), ("io_dtype", 3), ("mode", 3), ("periodic", 5),
    ("box", 0.0), ("box", float("nan")), ("n_target", 0.0), ("n_tol", -1.0),
    ("max_iter", -1), ("max_iter", 70000), ("cell_level", 22), ("cell_level", 0),
    ("tile_cell", 3), ("tile_cell", -3), ("kernel", 2), ("kernel", -1), ("waves_per_cu", 0), ("segment", 12), ("segment", 128),
    ("in_stride", 4), ("in_stride", -8), ("in_stride", 65544), ("in_stride", 12),
    ("out_stride", 20), ("out_stride", -224), ("out_stride", 1 << 20),
])
def test_invalid_params_rejected(field, value):
    _lib()
    p = sph.default_params()
    setattr(p, field, value)
    out = C.c_size_t(0)
    rc = sph.load().sph_workspace_size(C.byref(p), 100, 0, C.byref(out))
    assert rc == sph.E_INVALID


@pytest.mark.parametrize("k,dk,ok", [
    (64.0, 2.0, True), (2.0, 0.0, True), (1048576.0, 48.0, True),
    (1.0, 2.0, False), (0.0, 2.0, False), (32.5, 2.0, False), (1048577.0, 2.0, False),
    (64.0, 1.5, False), (64.0, 49.0, False), (64.0, -1.0, False),
])
def test_knn_params(k, dk, ok):
    # exact-K mode: K an integer in [2, 2^20], the count slack an integer in [0, 48]
    _lib()
    p = sph.default_params(mode=sph.KNN, n_target=k, n_tol=dk)
    out = C.c_size_t(0)
    rc = sph.load().sph_workspace_size(C.byref(p), 1000, 0, C.byref(out))
    assert rc == (sph.OK if ok else sph.E_INVALID)
    if ok:
        # the count stage keeps its h and status beside the band-mode workspace
        band = sph.workspace_size(sph.default_params(n_target=k, n_tol=dk), 1000)
        assert out.value >= band + 12 * 1000


def test_strides_accepted_and_alignment_checked():
    # strided (array-of-structs) I/O: multiples of the element size up to 64 KiB
    lib = _lib()
    out = C.c_size_t(0)
    for dt, es in ((sph.F64, 8), (sph.F32, 4)):
        for st in (0, es, 3 * es, 224, 65536):
            p = sph.default_params(io_dtype=dt, in_stride=st, out_stride=st)
            assert lib.sph_workspace_size(C.byref(p), 100, 0, C.byref(out)) == sph.OK
    # misaligned caller pointers are refused before anything is enqueued
    p = sph.default_params(in_stride=224, out_stride=224)
    ok, odd = C.c_void_p(0x1000), C.c_void_p(0x1004)
    ws = C.c_void_p(0x100000)
    for args in ((odd, ok, ok, ok, ok, ok), (ok, ok, ok, ok, odd, ok), (ok, ok, ok, ok, ok, odd)):
        x, y, z, m, rho, h = args
        assert lib.sph_density_solve(C.byref(p), 10, 0, None, x, y, z, m, None, rho, h, None,
                                     None, None, None, ws, 1 << 30, None) == sph.E_INVALID
    assert lib.sph_density_solve(C.byref(p), 10, 0, None, ok, ok, ok, ok, None, ok, ok, None,
                                 C.c_void_p(0x1002), None, None, ws, 1 << 30,
                                 None) == sph.E_INVALID
    assert lib.sph_sort(C.byref(p), 10, 0, None, odd, ok, ok, ok, ok, None, None, None, None,
                        ws, 1 << 30, None) == sph.E_INVALID


def test_force_and_scatter_host_checks():
    lib = _lib()
    fake, ws = C.c_void_p(0x1000), C.c_void_p(0x100000)
    p = sph.default_params()
    # missing pressure / outputs
    assert lib.sph_pressure_force(C.byref(p), 10, 0, None, fake, fake, fake, fake, fake, fake,
                                  None, fake, fake, fake, ws, 1 << 30, None) == sph.E_INVALID
    assert lib.sph_density_scatter(C.byref(p), 10, 0, None, fake, fake, fake, fake, fake, None,
                                   None, None, ws, 1 << 30, None) == sph.E_INVALID
    # exact-K h is not differentiable: no force from it
    k = sph.default_params(mode=sph.KNN, n_target=32.0, n_tol=2.0)
    assert lib.sph_pressure_force(C.byref(k), 10, 0, None, fake, fake, fake, fake, fake, fake,
                                  fake, fake, fake, fake, ws, 1 << 30, None) == sph.E_UNSUPPORTED
    # nothing to do
    assert lib.sph_pressure_force(C.byref(p), 0, 0, None, None, None, None, None, None, None,
                                  None, None, None, None, None, 0, None) == sph.OK
    assert lib.sph_density_scatter(C.byref(p), 0, 0, None, None, None, None, None, None, None,
                                   None, None, None, 0, None) == sph.OK


def test_knn_backward_unsupported():
    # h of the K-th neighbour is not differentiable in the positions: refused on the host
    lib = _lib()
    p = sph.default_params(mode=sph.KNN, n_target=32.0, n_tol=2.0)
    fake = C.c_void_p(0x1000)
    rc = lib.sph_density_backward(C.byref(p), 10, 0, None, fake, fake, fake, fake, fake, None,
                                  fake, fake, fake, fake, fake, C.c_void_p(0x100000), 1 << 30,
                                  None)
    assert rc == sph.E_UNSUPPORTED


def test_invalid_calls_rejected_before_any_launch():
    lib = _lib()
    p = sph.default_params()
    fake = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    # negative n, null inputs, groups on a periodic set, missing workspace
    assert lib.sph_density_solve(C.byref(p), -1, 0, None, fake, fake, fake, fake, None, fake,
                                 fake, None, None, None, None, fake, 1 << 30,
                                 None) == sph.E_INVALID
    assert lib.sph_density_solve(C.byref(p), 10, 0, None, None, fake, fake, fake, None, fake,
                                 fake, None, None, None, None, fake, 1 << 30,
                                 None) == sph.E_INVALID
    assert lib.sph_density_solve(C.byref(p), 10, 3, fake, fake, fake, fake, fake, None, fake,
                                 fake, None, None, None, None, fake, 1 << 30,
                                 None) == sph.E_INVALID
    assert lib.sph_density_solve(C.byref(p), 10, 0, None, fake, fake, fake, fake, None, fake,
                                 fake, None, None, None, None, None, 1 << 30,
                                 None) == sph.E_INVALID
    # workspace too small
    ws = C.c_void_p(0x100000)
    assert lib.sph_density_solve(C.byref(p), 1000, 0, None, fake, fake, fake, fake, None, fake,
                                 fake, None, None, None, None, ws, 16, None) == sph.E_WORKSPACE
    # misaligned workspace
    assert lib.sph_sort(C.byref(p), 1000, 0, None, fake, fake, fake, fake, fake, None, None,
                        None, None, C.c_void_p(0x100001), 1 << 30, None) == sph.E_INVALID
    # isolated groups need offsets and at most 65535 groups
    g = sph.default_params(periodic=0)
    assert lib.sph_sort(C.byref(g), 1000, 0, None, fake, fake, fake, fake, fake, None, None,
                        None, None, ws, 1 << 30, None) == sph.E_INVALID
    assert lib.sph_sort(C.byref(g), 1000, 70000, fake, fake, fake, fake, fake, fake, None, None,
                        None, None, ws, 1 << 30, None) == sph.E_INVALID
    # backward: null cotangent
    assert lib.sph_density_backward(C.byref(p), 10, 0, None, fake, fake, fake, fake, fake, None,
                                    None, fake, fake, fake, fake, ws, 1 << 30,
                                    None) == sph.E_INVALID


def test_status_strings():
    _lib()
    for code in (sph.OK, sph.E_INVALID, sph.E_WORKSPACE, sph.E_HIP, sph.E_UNSUPPORTED):
        s = sph.status_string(code)
        assert s.startswith("SPH_")
    assert "unknown" in sph.status_string(12345)


def test_product_does_not_touch_oracle():
    # the product path never imports the oracle (or any CPU fallback)
    pkg = os.path.join(ROOT, "paper_1612_06090_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "sph_oracle" not in text, f


def test_autotune_host_checks():
    lib = _lib()
    p = sph.default_params()
    best = sph.Params()
    ms = C.c_float(-1.0)
    # null result pointer, invalid parameters: rejected before any device call
    assert lib.sph_autotune(C.byref(p), 10, 0, None, None, None, None, None, None, None, None,
                            None, 0, None, None, None) == sph.E_INVALID
    bad = sph.default_params(segment=12)
    assert lib.sph_autotune(C.byref(bad), 10, 0, None, None, None, None, None, None, None, None,
                            None, 0, None, C.byref(best), None) == sph.E_INVALID
    # an empty input needs no device: the parameters come back unchanged
    assert lib.sph_autotune(C.byref(p), 0, 0, None, None, None, None, None, None, None, None,
                            None, 0, None, C.byref(best), C.byref(ms)) == sph.OK
    assert (best.segment, best.waves_per_cu, best.tile_cell) == (p.segment, p.waves_per_cu,
                                                                  p.tile_cell)
    assert ms.value == 0.0


def test_size_limits():
    # particle counts below 2^31 - 1 (32-bit sorted indices), group counts in
    # [1, 65535] for isolated groups and none for a periodic set
    lib = _lib()
    out = C.c_size_t(0)
    p = sph.default_params()
    for n, ok in ((0, True), ((1 << 31) - 2, True), ((1 << 31) - 1, False), (-1, False)):
        rc = lib.sph_workspace_size(C.byref(p), n, 0, C.byref(out))
        assert rc == (sph.OK if ok else sph.E_INVALID), n
    assert lib.sph_workspace_size(C.byref(p), 100, 3, C.byref(out)) == sph.E_INVALID
    g = sph.default_params(periodic=0, n_target=32.0, n_tol=1.0)
    for G, ok in ((1, True), (65535, True), (0, False), (65536, False)):
        rc = lib.sph_workspace_size(C.byref(g), 1000, G, C.byref(out))
        assert rc == (sph.OK if ok else sph.E_INVALID), G


def test_noalloc_host_checks():
    # the no-workspace solve validates like sph_density_solve and rejects a set
    # whose workspace would exceed its fixed scratch before touching a device
    lib = _lib()
    p = sph.default_params()
    dummy = C.c_void_p(256)
    args = [dummy] * 5 + [dummy, dummy, None, None, None, None, None]
    big = 1 << 20
    assert sph.workspace_size(p, big) > sph.NOALLOC_SCRATCH_BYTES
    assert lib.sph_density_solve_noalloc(C.byref(p), big, 0, None, *args) == sph.E_WORKSPACE
    bad = sph.default_params(n_target=-1.0)
    assert lib.sph_density_solve_noalloc(C.byref(bad), 1000, 0, None, *args) == sph.E_INVALID
    assert lib.sph_density_solve_noalloc(C.byref(p), -5, 0, None, *args) == sph.E_INVALID
