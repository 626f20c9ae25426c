"""GPU parity of the hand-written adjoint against the CPU oracle's adjoint.

Both are evaluated at the same h (the GPU solve's), with standard-normal
cotangents on rho and, separately, on h.  FP64: every component within
1e-11 of the largest oracle component (the sums differ only in order).
FP32C: every component within 2e-5 of the largest, relative L2 <= 1e-5.
Invariants that need no oracle: translation invariance (position gradients of
each isolated set sum to zero), degree-1 homogeneity in the masses
(sum_k m_k dL/dm_k = sum_i grad_rho_i rho_i, h not depending on masses),
scaling of an isolated group (x -> s x takes h -> s h at fixed n and
rho -> s^-3 rho, so sum_k x_k . dL/dx_k = -3 sum gr rho + sum gh h), and the
symmetry of a cubic lattice (every position gradient vanishes).
"""
import numpy as np
import pytest

import oracle
import paper_1612_06090_amd as sph
import sphgen
from gpu_util import gpu_backward, gpu_solve, say

pytestmark = pytest.mark.gpu

COMP = ("gx", "gy", "gz", "gm")


def _straddle():
    # two tight clusters in opposite corners: Morton tiles straddle them
    rng = np.random.default_rng(16)
    pts = np.concatenate([0.2 + 0.01 * rng.standard_normal((100, 3)),
                          0.8 + 0.01 * rng.standard_normal((100, 3))]) % 1.0
    return sphgen.ParticleSet(x=pts[:, 0].copy(), y=pts[:, 1].copy(), z=pts[:, 2].copy(),
                              m=np.ones(200), h_init=np.full(200, 0.02), periodic=True,
                              box=1.0, n_target=32.0, n_tol=1.0)


def _clump_in_background():
    # density contrast 8000: a cube of 2000 particles (side 0.05) in 2000
    # uniform ones; background spheres near the clump reach into it, so the
    # clump's particles have reverse neighbours with ~20 times their radius
    bg = sphgen.uniform(2000, seed=62)
    cl = sphgen.uniform(2000, seed=63)
    x = np.concatenate([bg.x, 0.475 + 0.05 * cl.x])
    y = np.concatenate([bg.y, 0.475 + 0.05 * cl.y])
    z = np.concatenate([bg.z, 0.475 + 0.05 * cl.z])
    n = x.shape[0]
    return sphgen.ParticleSet(x=x, y=y, z=z, m=np.full(n, 1.0 / n),
                              h_init=np.full(n, sphgen.default_h_init(n, 1.0)), periodic=True,
                              box=1.0, n_target=64.0, n_tol=2.0)


CASES = {
    "uniform4096": lambda: sphgen.config("uniform4096"),
    "clump_in_background": _clump_in_background,
    "clustered32k": lambda: sphgen.plummer_mixture(1 << 15, 20, seed=45),
    "groups200": lambda: sphgen.groups(200, seed=47, lo=32, hi=5000),
    "ragged65": lambda: sphgen.uniform(65, seed=15, n_target=16.0, n_tol=1.0),
    "ragged4133": lambda: sphgen.uniform(4133, seed=58),
    "straddle": _straddle,
    # coincident pairs: r = 0 between distinct particles, where the pair's
    # direction is undefined and its term vanishes (f'(0) = 0)
    "coincident4396": lambda: sphgen.with_duplicates(sphgen.uniform(4096, seed=74), 300,
                                                     seed=75),
}


def _compare(g, o, tol_max, tol_l2=None, tag=""):
    for k in COMP:
        sc = max(np.abs(o[k]).max(), 1e-300)
        err = np.abs(g[k] - o[k]).max() / sc
        l2 = np.linalg.norm(g[k] - o[k]) / max(np.linalg.norm(o[k]), 1e-300)
        say(f"  {tag} {k}: max {err:.2e} l2 {l2:.2e}")
        assert err <= tol_max, k
        if tol_l2 is not None:
            assert l2 <= tol_l2, k


def _setup(name, precision=sph.FP64):
    ps = CASES[name]()
    s = gpu_solve(ps, precision=precision)
    gr = sphgen.cotangent(ps.n, 71)
    gh = sphgen.cotangent(ps.n, 72)
    return ps, s, gr, gh


@pytest.mark.parametrize("name", sorted(CASES))
def test_backward_fp64(name):
    ps, s, gr, gh = _setup(name)
    say(f"[backward fp64] {name} n={ps.n}")
    for ghv in (None, gh):
        g = gpu_backward(ps, s["h"], gr, ghv)
        o = oracle.backward(ps, s["h"], gr, ghv)
        _compare(g, o, 1e-11, tag=name)


@pytest.mark.parametrize("name", sorted(CASES))
def test_backward_fp32c(name):
    ps, s, gr, gh = _setup(name, precision=sph.FP32C)
    say(f"[backward fp32c] {name} n={ps.n}")
    g = gpu_backward(ps, s["h"], gr, gh, precision=sph.FP32C)
    o = oracle.backward(ps, s["h"], gr, gh)
    _compare(g, o, 2e-5, 1e-5, tag=name)


def test_backward_clustered2p20_full():
    # the full-size set, every particle compared
    ps = sphgen.config("clustered2^20")
    say(f"[backward] clustered2^20 n={ps.n}")
    s = gpu_solve(ps, precision=sph.FP32C)
    gr = sphgen.cotangent(ps.n, 73)
    o = oracle.backward(ps, s["h"], gr)
    g64 = gpu_backward(ps, s["h"], gr)
    _compare(g64, o, 1e-11, tag="fp64")
    g32 = gpu_backward(ps, s["h"], gr, precision=sph.FP32C)
    _compare(g32, o, 2e-5, 1e-5, tag="fp32c")


@pytest.mark.parametrize("name", ["clustered32k", "groups200"])
@pytest.mark.parametrize("precision", [sph.FP64, sph.FP32C])
def test_backward_invariants(name, precision):
    ps, s, gr, _ = _setup(name, precision)
    g = gpu_backward(ps, s["h"], gr, precision=precision)
    tol = 1e-12 if precision == sph.FP64 else 1e-6
    offs = [0, ps.n] if ps.offsets is None else list(ps.offsets)
    for a, b in zip(offs[:-1], offs[1:]):
        if b == a:
            continue
        for k in ("gx", "gy", "gz"):
            tot = abs(g[k][a:b].sum())
            assert tot <= tol * np.abs(g[k][a:b]).sum() + 1e-300, (k, a, b)
    lhs = float(np.dot(ps.m, g["gm"]))
    rhs = float(np.dot(gr, s["rho"]))
    say(f"  homogeneity: {lhs:.15e} vs {rhs:.15e}")
    assert abs(lhs - rhs) <= tol * np.dot(np.abs(gr), s["rho"])


@pytest.mark.parametrize("precision", [sph.FP64, sph.FP32C])
def test_backward_group_scaling(precision):
    ps, s, gr, gh = _setup("groups200", precision)
    g = gpu_backward(ps, s["h"], gr, gh, precision=precision)
    tol = 1e-11 if precision == sph.FP64 else 1e-5
    worst = 0.0
    for a, b in zip(ps.offsets[:-1], ps.offsets[1:]):
        if b == a:
            continue
        xg = ps.x[a:b] * g["gx"][a:b] + ps.y[a:b] * g["gy"][a:b] + ps.z[a:b] * g["gz"][a:b]
        lhs = xg.sum()
        rhs = -3.0 * np.dot(gr[a:b], s["rho"][a:b]) + np.dot(gh[a:b], s["h"][a:b])
        scale = (np.abs(xg).sum() + 3.0 * np.dot(np.abs(gr[a:b]), s["rho"][a:b])
                 + np.dot(np.abs(gh[a:b]), s["h"][a:b]))
        worst = max(worst, abs(lhs - rhs) / scale)
    say(f"  scaling identity: worst relative residual {worst:.2e}")
    assert worst <= tol


@pytest.mark.parametrize("precision", [sph.FP64, sph.FP32C])
def test_backward_lattice_symmetry(precision):
    # 16^3 lattice, h = 2.72 spacings for every particle: each site sees the
    # same symmetric neighbourhood, so d(sum rho)/dx = 0 and dL/dm = sum_j W
    ps = sphgen.lattice(16, h=0.17)
    h = np.full(ps.n, 0.17)
    ones = np.ones(ps.n)
    g = gpu_backward(ps, h, ones, ones, precision=precision)
    r = gpu_backward(ps, h, sphgen.cotangent(ps.n, 81), None, precision=precision)
    scale = np.abs(r["gx"]).max()
    tol = 1e-12 if precision == sph.FP64 else 1e-5
    for k in ("gx", "gy", "gz"):
        say(f"  lattice {k}: max {np.abs(g[k]).max() / scale:.2e} of the random-cotangent scale")
        assert np.abs(g[k]).max() <= tol * scale
    e = oracle.eval_at_h(ps, h, search=1)
    sumw = e["rho"] / ps.m
    assert np.abs(g["gm"] - sumw).max() <= (1e-13 if precision == sph.FP64 else 1e-6) * sumw.max()


def test_backward_clustered2p20_central_differences():
    # full-size set, FP64 root-mode solves: the directional derivative of
    # L = sum gr rho along 8 random unit directions over all (x, m), and 64
    # single-coordinate probes (x, y, z and m of 16 particles), against the
    # adjoint (FP64 and FP32C)
    import torch
    ps = sphgen.config("clustered2^20")
    n = ps.n
    prm = sph.default_params(mode=sph.ROOT, root_tol=1e-14, n_target=ps.n_target,
                             n_tol=ps.n_tol, max_iter=200)
    base = {k: torch.tensor(getattr(ps, k), dtype=torch.float64, device="cuda")
            for k in ("x", "y", "z", "m")}
    h0 = torch.tensor(ps.h_init, dtype=torch.float64, device="cuda")
    gr_np = sphgen.cotangent(n, 5)
    gr = torch.tensor(gr_np, device="cuda")

    def L(dx=None, dm=None, eps=0.0):
        x = {k: v.clone() for k, v in base.items()}
        if dx is not None:
            for a, k in enumerate("xyz"):
                x[k] = torch.remainder(x[k] + eps * dx[:, a], 1.0)
        if dm is not None:
            x["m"] = x["m"] + eps * dm
        o = sph.density_solve(x["x"], x["y"], x["z"], x["m"], h0, prm)
        return float((gr * o["rho"]).sum()), o

    L0, o0 = L()
    assert int(((o0["status"] >> 16) != 0).sum()) == 0
    h = o0["h"].cpu().numpy()
    g64 = gpu_backward(ps, h, gr_np)
    g32 = gpu_backward(ps, h, gr_np, precision=sph.FP32C)
    eps = 1e-6
    rng = np.random.default_rng(82)
    worst = {"fp64": 0.0, "fp32c": 0.0}
    for t in range(8):
        v = rng.standard_normal(4 * n)
        v /= np.linalg.norm(v)
        dx = torch.tensor(v[:3 * n].reshape(n, 3), device="cuda")
        dm = torch.tensor(v[3 * n:], device="cuda")
        fd = (L(dx, dm, eps)[0] - L(dx, dm, -eps)[0]) / (2 * eps)
        for tag, g in (("fp64", g64), ("fp32c", g32)):
            an = float(np.dot(v[:3 * n], np.stack([g["gx"], g["gy"], g["gz"]], 1).ravel())
                       + np.dot(v[3 * n:], g["gm"]))
            worst[tag] = max(worst[tag], abs(fd - an) / abs(fd))
        say(f"  direction {t}: fd {fd:.10e}")
    say(f"  worst relative error: {worst}")
    assert worst["fp64"] <= 1e-5 and worst["fp32c"] <= 1e-4
    # 64 single-coordinate probes: the three position coordinates and the mass
    # of 16 particles, 8 in the densest regions (largest rho) and 8 at random
    top = np.argsort(-o0["rho"].cpu().numpy())[:8]
    probes = list(top) + list(rng.choice(n, 8, replace=False))
    scale = np.abs(g64["gx"]).max()
    scale_m = np.abs(g64["gm"]).max()
    done = 0
    for k in probes:
        for a, key in enumerate(("gx", "gy", "gz")):
            dx = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
            dx[k, a] = 1.0
            step = 1e-6 * h[k]
            fd = (L(dx, None, step)[0] - L(dx, None, -step)[0]) / (2 * step)
            err = abs(fd - g64[key][k])
            assert err <= 1e-5 * max(abs(fd), 1e-3 * scale), (k, a, fd, g64[key][k])
            done += 1
        dm = torch.zeros(n, dtype=torch.float64, device="cuda")
        dm[k] = 1.0
        # rho is linear in each mass (h does not depend on masses), so a large
        # step keeps the difference far above the rounding of the full sum
        step = 0.5 * ps.m[k]
        fd = (L(None, dm, step)[0] - L(None, dm, -step)[0]) / (2 * step)
        err = abs(fd - g64["gm"][k])
        assert err <= 1e-5 * max(abs(fd), 1e-3 * scale_m), (k, "m", fd, g64["gm"][k])
        done += 1
    say(f"  {done} single-coordinate probes within 1e-5")
    assert done == 64


def test_backward_deterministic():
    ps, s, gr, gh = _setup("clustered32k")
    for prec in (sph.FP64, sph.FP32C):
        a = gpu_backward(ps, s["h"], gr, gh, precision=prec)
        b = gpu_backward(ps, s["h"], gr, gh, precision=prec)
        for k in COMP:
            assert np.array_equal(a[k], b[k]), k


def test_backward_bad_inputs():
    ps = sphgen.uniform(2000, seed=53)
    ps.x = ps.x.copy()
    ps.y = ps.y.copy()
    ps.m = ps.m.copy()
    ps.x[10] = np.nan
    ps.y[20] = 1.5
    ps.m[30] = np.inf
    s = gpu_solve(ps)
    gr = sphgen.cotangent(ps.n, 74)
    g = gpu_backward(ps, s["h"], gr)
    o = oracle.backward(ps, s["h"], gr)
    bad = [10, 20, 30]
    for k in COMP:
        assert np.all(g[k][bad] == 0.0), k
    _compare(g, o, 1e-11, tag="bad")


def test_backward_io_float32():
    ps = sphgen.uniform(3000, seed=75)
    for k in ("x", "y", "z", "m", "h_init"):
        setattr(ps, k, getattr(ps, k).astype(np.float32).astype(np.float64))
    s = gpu_solve(ps)
    h = s["h"].astype(np.float32).astype(np.float64)
    gr = sphgen.cotangent(ps.n, 76).astype(np.float32).astype(np.float64)
    g = gpu_backward(ps, h, gr, io="float32")
    o = oracle.backward(ps, h, gr)
    _compare(g, o, 1e-6, tag="io32")   # outputs rounded to binary32


def test_backward_empty():
    import torch
    z = torch.empty(0, dtype=torch.float64, device="cuda")
    o = sph.density_backward(z, z, z, z, z, z)
    torch.cuda.synchronize()
    assert all(v.numel() == 0 for v in o.values())


def test_autograd_function():
    # SPHDensity routes torch.autograd through the adjoint: its gradient equals
    # the direct call, and a central difference of the root-mode solve (where
    # each n_i sits on N_t, so h follows the implicit root exactly)
    import torch
    ps = sphgen.uniform(600, seed=77, n_target=32.0, n_tol=1.0)
    prm = sph.default_params(mode=sph.ROOT, root_tol=1e-14, n_target=32.0, n_tol=1.0,
                             max_iter=200)
    pos = torch.tensor(np.stack([ps.x, ps.y, ps.z], 1), dtype=torch.float64, device="cuda",
                       requires_grad=True)
    m = torch.tensor(ps.m, dtype=torch.float64, device="cuda", requires_grad=True)
    rho, h = sph.SPHDensity.apply(pos, m, prm)
    wr = torch.tensor(sphgen.cotangent(ps.n, 78), device="cuda")
    wh = torch.tensor(sphgen.cotangent(ps.n, 79), device="cuda")
    loss = (wr * rho).sum() + (wh * h).sum()
    loss.backward()
    gp = pos.grad.cpu().numpy()
    gm = m.grad.cpu().numpy()
    d = gpu_backward(ps, h.detach().cpu().numpy(), wr.cpu().numpy(), wh.cpu().numpy(),
                     mode=sph.ROOT, root_tol=1e-14, max_iter=200)
    assert np.array_equal(gp[:, 0], d["gx"]) and np.array_equal(gm, d["gm"])
    # directional central difference (positions kept inside the box)
    rng = np.random.default_rng(80)
    v = rng.standard_normal((ps.n, 3))
    vm = rng.standard_normal(ps.n)
    eps = 1e-6

    def L(t):
        with torch.no_grad():
            p2 = pos + t * torch.tensor(v, device="cuda")
            p2 = torch.remainder(p2, 1.0)
            m2 = m + t * torch.tensor(vm, device="cuda")
            r2, h2 = sph.SPHDensity.apply(p2, m2, prm)
            return float((wr * r2).sum() + (wh * h2).sum())

    fd = (L(eps) - L(-eps)) / (2 * eps)
    an = float((gp * v).sum() + (gm * vm).sum())
    say(f"  autograd: analytic {an:.10e} fd {fd:.10e}")
    assert abs(fd - an) <= 1e-6 * max(abs(an), np.abs(gp).sum() * 1e-3)
