"""Helpers shared by the GPU tests: move a ParticleSet to the device and run
the library through its C ABI binding."""
import sys

import numpy as np

import paper_1612_06090_amd as sph


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev_arrays(ps, dtype="float64"):
    import torch
    dt = getattr(torch, dtype)
    d = {k: torch.tensor(np.asarray(getattr(ps, k)), dtype=dt, device="cuda")
         for k in ("x", "y", "z", "m", "h_init")}
    d["goff"] = None if ps.offsets is None else torch.tensor(ps.offsets, dtype=torch.int64,
                                                             device="cuda")
    return d


def params_for(ps, **kw):
    p = sph.default_params(periodic=1 if ps.periodic else 0, box=ps.box,
                           n_target=ps.n_target, n_tol=ps.n_tol)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def gpu_solve(ps, h_init="given", io="float64", stats=False, **kw):
    import torch
    p = params_for(ps, io_dtype=sph.F32 if io == "float32" else sph.F64, **kw)
    d = dev_arrays(ps, io)
    h0 = d["h_init"] if isinstance(h_init, str) else (
        None if h_init is None else torch.tensor(h_init, dtype=d["x"].dtype, device="cuda"))
    o = sph.density_solve(d["x"], d["y"], d["z"], d["m"], h0, p, d["goff"], stats=stats)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in o.items()}
    for k in ("rho", "h", "nw"):
        out[k] = out[k].astype(np.float64)
    return out


def gpu_sort(ps, io="float64", **kw):
    import torch
    p = params_for(ps, io_dtype=sph.F32 if io == "float32" else sph.F64, **kw)
    d = dev_arrays(ps, io)
    o = sph.sort(d["x"], d["y"], d["z"], p, d["goff"])
    torch.cuda.synchronize()
    out = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in o.items()}
    out["keys"] = out["keys"].view(np.uint64)
    if "cell_id" in out:
        out["cell_id"] = out["cell_id"].view(np.uint64)
    return out


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


def gpu_backward(ps, h, grad_rho, grad_h=None, io="float64", **kw):
    """sph_density_backward at the given h; returns numpy gx, gy, gz, gm."""
    import torch
    p = params_for(ps, io_dtype=sph.F32 if io == "float32" else sph.F64, **kw)
    d = dev_arrays(ps, io)
    dt = d["x"].dtype
    ht = torch.tensor(np.asarray(h), dtype=dt, device="cuda")
    gr = torch.tensor(np.asarray(grad_rho), dtype=dt, device="cuda")
    gh = None if grad_h is None else torch.tensor(np.asarray(grad_h), dtype=dt, device="cuda")
    o = sph.density_backward(d["x"], d["y"], d["z"], d["m"], ht, gr, gh, p, d["goff"])
    torch.cuda.synchronize()
    return {k: v.cpu().numpy().astype(np.float64) for k, v in o.items()}
