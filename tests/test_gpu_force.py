"""SPH pressure force of the variational (grad-h) equations on the GPU against
the oracle: a_k = -(1/m_k) dE/dx_k with each h on its count constraint, the
density adjoint for the cotangent m_i P_i/rho_i^2.

Both sides take the same h, rho (the GPU solve's, root mode) and P.  Bounds as
for the adjoint: FP64 within 1e-11 of the largest |a| component, FP32C within
2e-5 of it and 1e-5 in relative L2.  Invariants of the GPU output itself:
sum_k m_k a_k = 0 (pair antisymmetry) and no torque for isolated groups, to
the rounding of the sums.
"""
import numpy as np
import pytest

import oracle
import paper_1612_06090_amd as sph
import sphgen
from gpu_util import dev_arrays, params_for, say

pytestmark = pytest.mark.gpu


def _setup(name):
    rng = np.random.default_rng(50)
    kern = oracle.M4
    if name == "uniform4096":
        ps = sphgen.config("uniform4096")
    elif name == "clustered32k":
        ps = sphgen.plummer_mixture(1 << 15, 20, seed=51)
    elif name == "groups60":
        ps = sphgen.groups(60, seed=52, lo=40, hi=3000)
    elif name == "clustered32k_wc6":
        ps = sphgen.plummer_mixture(1 << 15, 20, seed=53, n_target=295.0)
        kern = oracle.WENDLAND_C6
    elif name == "coincident4396":
        # twins at r = 0: the pair's direction is undefined and its term
        # vanishes (f'(0) = 0) on both sides
        ps = sphgen.with_duplicates(sphgen.uniform(4096, seed=54), 300, seed=55)
    else:
        raise KeyError(name)
    ps.m = rng.uniform(0.5, 2.0, ps.n) / ps.n
    A = rng.uniform(0.5, 2.0, ps.n)
    return ps, A, kern


def _kern(k):
    return sph.KERNEL_WENDLAND_C6 if k == oracle.WENDLAND_C6 else sph.KERNEL_M4


def _gpu_force(ps, A, kern, precision, gamma=5.0 / 3.0):
    import torch
    rt = 1e-10 if precision == sph.FP64 else 1e-6   # binary32 sums settle near 1e-7
    p = params_for(ps, precision=precision, mode=sph.ROOT, root_tol=rt, kernel=_kern(kern))
    d = dev_arrays(ps)
    f = sph.density_solve(d["x"], d["y"], d["z"], d["m"], d["h_init"], p, d["goff"])
    P = torch.tensor(A, dtype=torch.float64, device="cuda") * f["rho"] ** gamma
    a = sph.pressure_force(d["x"], d["y"], d["z"], d["m"], f["h"], f["rho"], P, p, d["goff"])
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in a.items()}
    return out, f["h"].cpu().numpy(), f["rho"].cpu().numpy(), P.cpu().numpy(), \
        (f["status"].cpu().numpy() >> 16)


def _cmp(ps, g, o, tol_max, tol_l2=None):
    G = np.stack([g["ax"], g["ay"], g["az"]], 1)
    O = np.stack([o["ax"], o["ay"], o["az"]], 1)
    scale = np.abs(O).max()
    err = np.abs(G - O).max() / scale
    l2 = np.linalg.norm(G - O) / np.linalg.norm(O)
    say(f"  max err / max|a| {err:.2e}  rel L2 {l2:.2e}")
    assert err <= tol_max
    if tol_l2 is not None:
        assert l2 <= tol_l2
    return G


NAMES = ["uniform4096", "clustered32k", "groups60", "clustered32k_wc6", "coincident4396"]


@pytest.mark.parametrize("name", NAMES)
def test_force_fp64(name):
    ps, A, kern = _setup(name)
    say(f"[force fp64] {name} n={ps.n}")
    g, h, rho, P, flags = _gpu_force(ps, A, kern, sph.FP64)
    assert np.all(flags == 0)
    o = oracle.pressure_force(ps, h, rho, P, kernel=kern)
    G = _cmp(ps, g, o, 1e-11)
    F = G * ps.m[:, None]
    if ps.offsets is None:
        assert np.all(np.abs(F.sum(0)) < 1e-12 * np.abs(F).sum())
    else:
        for a, b in zip(ps.offsets[:-1], ps.offsets[1:]):
            if b - a < 2:
                continue
            s = np.abs(F[a:b]).sum()
            assert np.all(np.abs(F[a:b].sum(0)) < 1e-12 * s)
            r = ps.pos[a:b] - ps.pos[a:b].mean(0)
            assert np.all(np.abs(np.cross(r, F[a:b]).sum(0)) < 1e-12 * np.abs(r).max() * s)


@pytest.mark.parametrize("name", NAMES)
def test_force_fp32c(name):
    ps, A, kern = _setup(name)
    g, h, rho, P, flags = _gpu_force(ps, A, kern, sph.FP32C)
    o = oracle.pressure_force(ps, h, rho, P, kernel=kern)
    _cmp(ps, g, o, 2e-5, 1e-5)


def test_force_aos_bit_identical():
    import torch
    ps, A, kern = _setup("clustered32k")
    p = params_for(ps, mode=sph.ROOT, root_tol=1e-10)
    d = dev_arrays(ps)
    f = sph.density_solve(d["x"], d["y"], d["z"], d["m"], d["h_init"], p)
    P = torch.tensor(A, dtype=torch.float64, device="cuda") * f["rho"] ** (5.0 / 3.0)
    a = sph.pressure_force(d["x"], d["y"], d["z"], d["m"], f["h"], f["rho"], P, p)
    S = torch.full((ps.n, 28), 7.25, dtype=torch.float64, device="cuda")
    for c, v in ((0, d["x"]), (1, d["y"]), (2, d["z"]), (6, d["m"]), (10, f["h"]), (9, f["rho"]),
                 (21, P)):
        S[:, c] = v
    out = dict(ax=S[:, 3], ay=S[:, 4], az=S[:, 5])
    sph.pressure_force(S[:, 0], S[:, 1], S[:, 2], S[:, 6], S[:, 10], S[:, 9], S[:, 21], p,
                       out=out)
    torch.cuda.synchronize()
    for k in ("ax", "ay", "az"):
        assert torch.equal(out[k], a[k]), k
    keep = [c for c in range(28) if c not in (0, 1, 2, 3, 4, 5, 6, 9, 10, 21)]
    assert bool((S[:, keep] == 7.25).all())


def test_force_clustered2p20_fp32c():
    ps = sphgen.config("clustered2^20")
    A = np.random.default_rng(54).uniform(0.5, 2.0, ps.n)
    say(f"[force fp32c] clustered2^20 n={ps.n}")
    g, h, rho, P, flags = _gpu_force(ps, A, oracle.M4, sph.FP32C)
    assert np.all(flags == 0)
    o = oracle.pressure_force(ps, h, rho, P)
    _cmp(ps, g, o, 2e-5, 1e-5)
