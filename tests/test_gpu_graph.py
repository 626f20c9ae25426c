"""HIP-graph capture of the multi-launch entry points: exact K (count stage,
selection, evaluation), the scatter form, the pressure force, the adjoint,
and the solve of sets above 2^21 particles (whose sort clears its look-back
descriptors and tile counters with a fill kernel in every call) are captured
once and replayed between eager calls of the program's own; every replay
must equal an eager call bit for bit, also after the inputs are changed in
place."""
import numpy as np
import pytest

import paper_1612_06090_amd as sph
import sphgen
from gpu_util import dev_arrays, params_for

pytestmark = pytest.mark.gpu


def _check_graph(run, mutate):
    import torch

    def eager():
        o = run()
        torch.cuda.synchronize()
        return {k: v.clone() for k, v in o.items() if v is not None}

    ref = eager()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        out = run()
    for r in range(3):
        eager()
        graph.replay()
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(out[k], ref[k]), (r, k)
    mutate()
    ref2 = eager()
    graph.replay()
    torch.cuda.synchronize()
    for k in ref2:
        assert torch.equal(out[k], ref2[k]), k


@pytest.mark.parametrize("grouped", [False, True])
def test_graph_exact_k(grouped):
    ps = (sphgen.groups(40, seed=30, lo=80, hi=3000) if grouped
          else sphgen.plummer_mixture(1 << 14, 8, seed=31))
    p = params_for(ps, mode=sph.KNN, n_target=64.0, n_tol=8.0, precision=sph.FP32C)
    d = dev_arrays(ps)
    G = 0 if ps.offsets is None else len(ps.offsets) - 1
    ws = sph.workspace(p, ps.n, G, d["x"].device)
    _check_graph(lambda: sph.density_solve(d["x"], d["y"], d["z"], d["m"], d["h_init"], p,
                                           d["goff"], ws=ws),
                 lambda: d["y"].mul_(0.75))


def test_graph_scatter_force_adjoint():
    import torch
    ps = sphgen.plummer_mixture(1 << 14, 8, seed=32)
    p = params_for(ps, mode=sph.ROOT, root_tol=1e-10)
    d = dev_arrays(ps)
    f = sph.density_solve(d["x"], d["y"], d["z"], d["m"], d["h_init"], p)
    h, rho = f["h"].clone(), f["rho"].clone()
    P = rho ** (5.0 / 3.0)
    gr = torch.tensor(np.random.default_rng(33).standard_normal(ps.n), dtype=torch.float64,
                      device="cuda")
    ws = sph.workspace(p, ps.n, 0, d["x"].device)
    _check_graph(lambda: sph.density_scatter(d["x"], d["y"], d["z"], d["m"], h, p, ws=ws),
                 lambda: h.mul_(1.1))
    _check_graph(lambda: sph.pressure_force(d["x"], d["y"], d["z"], d["m"], h, rho, P, p,
                                            ws=ws),
                 lambda: P.mul_(2.0))
    _check_graph(lambda: sph.density_backward(d["x"], d["y"], d["z"], d["m"], h, gr, None, p,
                                              ws=ws),
                 lambda: gr.mul_(-1.0))


@pytest.mark.parametrize("grouped", [False, True])
def test_graph_solve_above_2p21(grouped):
    # periodic: keys with digit counts in one kernel; groups: a histogram
    # pass of its own; both then the single-sweep scatter passes
    ps = (sphgen.config("groups10k") if grouped
          else sphgen.uniform((1 << 21) + 4096, seed=34, n_target=32.0, n_tol=1.0))
    p = params_for(ps, precision=sph.FP32C)
    d = dev_arrays(ps)
    G = 0 if ps.offsets is None else len(ps.offsets) - 1
    ws = sph.workspace(p, ps.n, G, d["x"].device)
    _check_graph(lambda: sph.density_solve(d["x"], d["y"], d["z"], d["m"], d["h_init"], p,
                                           d["goff"], ws=ws),
                 lambda: d["x"].mul_(0.5))
