"""GPU test of sph_density_solve_noalloc, the solve that takes no workspace.

Called through the C ABI, twice in a row with the second set smaller than the
first (so that the second call finds the first call's contents in the
library's scratch), each against sph_density_solve with a caller workspace on
the same inputs: every output must be bit-identical (same kernels, same
inputs; the result never depends on what the workspace held).  The first
call is also checked against the oracle (FP64: counts exact, rho and h to
1e-12), so that a wrong scratch cannot pass by matching a wrong reference.
"""
import numpy as np
import pytest

import oracle
import paper_1612_06090_amd as sph
import sphgen
from gpu_util import dev_arrays, params_for, rel, say

pytestmark = pytest.mark.gpu


def _np(o):
    return {k: v.cpu().numpy() for k, v in o.items() if v is not None}


def _both(ps, **kw):
    import torch
    p = params_for(ps, **kw)
    d = dev_arrays(ps)
    a = sph.density_solve_noalloc(d["x"], d["y"], d["z"], d["m"], d["h_init"], p, d["goff"],
                                  stats=True)
    torch.cuda.synchronize()
    a = _np(a)
    b = sph.density_solve(d["x"], d["y"], d["z"], d["m"], d["h_init"], p, d["goff"], stats=True)
    torch.cuda.synchronize()
    b = _np(b)
    for k in ("rho", "h", "nw", "nngb", "status", "stats"):
        assert np.array_equal(a[k], b[k]), k
    return a


def test_noalloc_twice_smaller_second():
    ps1 = sphgen.plummer_mixture(20000, 12, seed=71)
    say(f"[noalloc] call 1: clustered n={ps1.n} FP64")
    a = _both(ps1)
    o = oracle.solve(ps1)
    e = oracle.eval_at_h(ps1, a["h"])
    assert np.array_equal(a["nngb"], e["nngb"].astype(np.int32))
    assert rel(a["h"], o["h"]).max() < 1e-12 and rel(a["rho"], o["rho"]).max() < 1e-12
    ps2 = sphgen.uniform(3001, seed=72)
    say(f"[noalloc] call 2: uniform n={ps2.n} FP32C")
    _both(ps2, precision=sph.FP32C)
    ps3 = sphgen.groups(40, seed=73, lo=32, hi=2048)
    say(f"[noalloc] call 3: {ps3.offsets.size - 1} groups n={ps3.n} FP32C")
    _both(ps3, precision=sph.FP32C)


def test_noalloc_rejects_sets_beyond_scratch():
    import torch
    p = sph.default_params()
    n = 1 << 20
    assert sph.workspace_size(p, n) > sph.NOALLOC_SCRATCH_BYTES
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(sph.SPHError) as ei:
        sph.density_solve_noalloc(x, x, x, x, None, p)
    assert ei.value.code == sph.E_WORKSPACE
