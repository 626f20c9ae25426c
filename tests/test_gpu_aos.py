"""Array-of-structs interop (Sec. IV-B): the caller keeps one particle struct
per particle (224 bytes in binary64, 112 in binary32) and passes pointers to
its fields with the struct size as the stride.  The library's own gather into
sorted arrays reads the structs, and its outputs are written through the sort
permutation straight into them.  Results must be bit-identical to the packed
path (which the other tests hold to the oracle), every other field of the
structs must be left as it was, and one case is checked against the oracle
directly.
"""
import numpy as np
import pytest

import oracle
import paper_1612_06090_amd as sph
import sphgen
from gpu_util import dev_arrays, params_for, rel, say

pytestmark = pytest.mark.gpu

WORDS = 28          # 28 words: 224 bytes in binary64
POS, MASS, HIN = 0, 6, 8
RHO, HOUT, NW, INTS = 9, 10, 11, 12   # INTS: nngb, status as two int32 (binary64 struct)
GX, GY, GZ, GM, GRHO = 13, 14, 15, 16, 17
SENTINEL = 7.25


def _structs(ps, dtype):
    import torch
    S = torch.full((ps.n, WORDS), SENTINEL, dtype=dtype, device="cuda")
    for c, k in ((POS, "x"), (POS + 1, "y"), (POS + 2, "z"), (MASS, "m"), (HIN, "h_init")):
        S[:, c] = torch.tensor(np.asarray(getattr(ps, k)), dtype=dtype, device="cuda")
    return S


def _int_cols(dtype):
    # nngb and status: the two int32 halves of word INTS (binary64 structs) or
    # words INTS and INTS + 1 (binary32 structs)
    import torch
    return (2 * INTS, 2 * INTS + 1) if dtype == torch.float64 else (INTS, INTS + 1)


def _aos_solve(ps, S, params, goff=None):
    import torch
    iv = S.view(torch.int32)
    ci = _int_cols(S.dtype)
    out = dict(rho=S[:, RHO], h=S[:, HOUT], nw=S[:, NW], nngb=iv[:, ci[0]], status=iv[:, ci[1]])
    sph.density_solve(S[:, POS], S[:, POS + 1], S[:, POS + 2], S[:, MASS], S[:, HIN], params,
                      goff, out=out)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy().copy() for k, v in out.items()}


def _untouched(S, used):
    import torch
    keep = [c for c in range(WORDS) if c not in used]
    if S.dtype == torch.float32:
        keep = [c for c in keep if c != INTS + 1]
    assert bool((S[:, keep] == SENTINEL).all()), "a struct field outside the outputs changed"


CASES = [
    ("uniform4096", sph.FP64, "float64", sph.BAND, sph.KERNEL_M4),
    ("clustered32k", sph.FP32C, "float64", sph.BAND, sph.KERNEL_M4),
    ("groups60", sph.FP64, "float32", sph.BAND, sph.KERNEL_M4),
    ("groups60", sph.FP32C, "float32", sph.BAND, sph.KERNEL_M4),
    ("clustered32k", sph.FP64, "float64", sph.KNN, sph.KERNEL_M4),
    ("clustered32k", sph.FP32C, "float64", sph.BAND, sph.KERNEL_WENDLAND_C6),
]


def _make(name):
    if name == "uniform4096":
        return sphgen.config("uniform4096")
    if name == "clustered32k":
        return sphgen.plummer_mixture(1 << 15, 20, seed=61)
    return sphgen.groups(60, seed=62, lo=40, hi=5000)


@pytest.mark.parametrize("name,prec,io,mode,kern", CASES)
def test_aos_solve_bit_identical(name, prec, io, mode, kern):
    import torch
    ps = _make(name)
    say(f"[aos] {name} n={ps.n} prec={prec} io={io} mode={mode} kernel={kern}")
    dt = getattr(torch, io)
    kw = dict(io_dtype=sph.F32 if io == "float32" else sph.F64, precision=prec, mode=mode,
              kernel=kern)
    if mode == sph.KNN:
        kw.update(n_target=64.0, n_tol=8.0)
    p = params_for(ps, **kw)
    d = dev_arrays(ps, io)
    packed = sph.density_solve(d["x"], d["y"], d["z"], d["m"], d["h_init"], p, d["goff"])
    torch.cuda.synchronize()
    S = _structs(ps, dt)
    a = _aos_solve(ps, S, p, d["goff"])
    for k in ("rho", "h", "nw", "nngb", "status"):
        assert np.array_equal(a[k], packed[k].cpu().numpy(), equal_nan=k in ("rho", "nw")), k
    _untouched(S, (POS, POS + 1, POS + 2, MASS, HIN, RHO, HOUT, NW, INTS))


def test_aos_against_oracle():
    ps = sphgen.config("uniform4096")
    import torch
    S = _structs(ps, torch.float64)
    a = _aos_solve(ps, S, params_for(ps))
    o = oracle.solve(ps)
    assert np.array_equal(a["nngb"], o["nngb"].astype(np.int32))
    assert rel(a["h"], o["h"]).max() < 1e-12 and rel(a["rho"], o["rho"]).max() < 1e-12
    assert np.array_equal(a["status"], o["status"])


@pytest.mark.parametrize("prec", [sph.FP64, sph.FP32C])
def test_aos_backward_bit_identical(prec):
    import torch
    ps = sphgen.plummer_mixture(1 << 14, 10, seed=63)
    p = params_for(ps, precision=prec, mode=sph.ROOT, root_tol=1e-10)
    d = dev_arrays(ps)
    f = sph.density_solve(d["x"], d["y"], d["z"], d["m"], d["h_init"], p)
    gr = torch.tensor(np.random.default_rng(64).standard_normal(ps.n), dtype=torch.float64,
                      device="cuda")
    packed = sph.density_backward(d["x"], d["y"], d["z"], d["m"], f["h"], gr, None, p)
    S = _structs(ps, torch.float64)
    S[:, HOUT] = f["h"]
    S[:, GRHO] = gr
    out = dict(gx=S[:, GX], gy=S[:, GY], gz=S[:, GZ], gm=S[:, GM])
    sph.density_backward(S[:, POS], S[:, POS + 1], S[:, POS + 2], S[:, MASS], S[:, HOUT],
                         S[:, GRHO], None, p, out=out)
    torch.cuda.synchronize()
    for k in ("gx", "gy", "gz", "gm"):
        assert torch.equal(out[k], packed[k]), k
    _untouched(S, (POS, POS + 1, POS + 2, MASS, HIN, HOUT, GX, GY, GZ, GM, GRHO))


def test_aos_sort_identical():
    import torch
    ps = sphgen.plummer_mixture(50000, 10, seed=65)
    d = dev_arrays(ps)
    a = sph.sort(d["x"], d["y"], d["z"])
    S = _structs(ps, torch.float64)
    b = sph.sort(S[:, POS], S[:, POS + 1], S[:, POS + 2])
    for k in ("keys", "perm", "cell_id", "cell_start", "cell_count"):
        assert torch.equal(a[k], b[k]), k


def test_aos_clustered2p20_fp32c():
    # the benchmarked set at full size, structs of 224 bytes
    import torch
    ps = sphgen.config("clustered2^20")
    say(f"[aos] clustered2^20 fp32c n={ps.n}")
    p = params_for(ps, precision=sph.FP32C)
    d = dev_arrays(ps)
    packed = sph.density_solve(d["x"], d["y"], d["z"], d["m"], d["h_init"], p)
    torch.cuda.synchronize()
    S = _structs(ps, torch.float64)
    a = _aos_solve(ps, S, p)
    for k in ("rho", "h", "nw", "nngb", "status"):
        assert np.array_equal(a[k], packed[k].cpu().numpy()), k
    _untouched(S, (POS, POS + 1, POS + 2, MASS, HIN, RHO, HOUT, NW, INTS))
