#!/usr/bin/env python3
"""Benchmark of the SPH density hot path on one MI355X.

A step is one full pass of the path over the 2^20-particle clustered set
(200 Plummer spheres + 30% uniform background, periodic unit cube, equal
masses, N_t = 64 +- 2, h_init = 2 N^(-1/3)): Morton keys, radix sort,
cell tables, and the FP32-compensated density + smoothing-length solve.
The same input is also timed with the plain FP64 solve, reported beside it.

Prints ONE JSON line.  ``value`` = in-range particle-neighbour pairs
evaluated per second over the whole step (every trial h counts);
``roofline`` is the density kernel's algorithmic FLOP rate (8 FLOP per
candidate pair tested, 31 per in-range pair in FP32C / 22 in FP64) over
its own duration, measured with HIP events on the launch stream, against
the MI355X FP32 vector peak.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-neighbour interactions/s and particles/s for density+h solve, FP32 vs FP64"
PEAK_FP32 = 157.3e12   # MI355X vector FP32 (packed) FLOP/s
PEAK_FP64 = 78.6e12    # MI355X vector FP64 FLOP/s
FLOP_CAND = 8.0        # 3 differences + r^2 (one multiply, two FMA; FMA = 2)
# A candidate streamed from a neighbour cell is first tested once against the
# tile's region (its distance from the particles' bounding box, the same 3
# differences and r^2) before the per-particle tests: 8 FLOP per region test.
FLOP_REGION = 8.0
# Algorithmic FLOP per in-range pair, the headline weights: the root, q, the
# spline's f and f', and the three sums S0, S1, R: 22 in FP64; the FP32C form
# adds a Kahan compensation to each of the three sums (3 x 3): 31.
FLOP_PAIR = {"fp32c": 31.0, "fp64": 22.0}
# Beside them, what this kernel's instructions do per in-range pair, the same in
# both forms: q^2 (or q = sqrt(r^2) / h) 2, the branch-free spline's f and q f'
# 11, three sums 4 (one FMA).  The binary32 form sums up to 64 terms per lane
# plainly and folds them into Kahan-compensated totals once per chunk round, so
# its compensation costs no FLOP per pair.
FLOP_PAIR_KERNEL = {"fp32c": 17.0, "fp64": 17.0}
# Wendland C6: q^2 and q 2 (FP32C) or 3 (FP64: sqrt, 1/h, q^2), the two
# polynomials and powers of (1 - q) 19, three sums 4
FLOP_PAIR_WC6 = {"fp32c": 25.0, "fp64": 26.0}


class HipEvents:
    """hipEvent_t pairs through the HIP runtime (timing only)."""

    def __init__(self):
        self.hip = C.CDLL("libamdhip64.so")
        self.hip.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        self.hip.hipEventSynchronize.argtypes = [C.c_void_p]
        self.hip.hipEventDestroy.argtypes = [C.c_void_p]

    def create(self):
        e = C.c_void_p()
        rc = self.hip.hipEventCreate(C.byref(e))
        if rc != 0:
            raise RuntimeError(f"hipEventCreate failed: {rc}")
        return e

    def elapsed_ms(self, a, b):
        self.hip.hipEventSynchronize(b)
        ms = C.c_float()
        rc = self.hip.hipEventElapsedTime(C.byref(ms), a, b)
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed: {rc}")
        return float(ms.value)


def run_form(sph, torch, d, ps, precision, steps, warmup, ev):
    p = sph.default_params(periodic=1, box=ps.box, n_target=ps.n_target, n_tol=ps.n_tol,
                           precision=precision)
    n = ps.n
    ws = sph.workspace(p, n, 0, d["x"].device)
    outs = None
    for _ in range(warmup):
        outs = sph.density_solve(d["x"], d["y"], d["z"], d["m"], d["h_init"], p, stats=True,
                                 ws=ws)
    torch.cuda.synchronize()
    pairs = [(ev.create(), ev.create()) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        p.prof_events[0] = pairs[k][0]
        p.prof_events[1] = pairs[k][1]
        outs = sph.density_solve(d["x"], d["y"], d["z"], d["m"], d["h_init"], p, stats=True,
                                 ws=ws)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [ev.elapsed_ms(a, b) for a, b in pairs]
    st = outs["stats"].cpu().numpy().astype(np.int64)
    status = outs["status"].cpu().numpy()
    nngb = outs["nngb"].cpu().numpy()
    for a, b in pairs:
        ev.hip.hipEventDestroy(a)
        ev.hip.hipEventDestroy(b)
    return dict(ms_per_step=1e3 * wall / steps, kernel_ms=float(np.mean(kern_ms)),
                kernel_ms_median=float(np.median(kern_ms)), pairs=int(st[0]), cands=int(st[1]), passes=int(st[2]), region=int(st[3]),
                final_pairs=int(nngb.astype(np.int64).sum()),
                flagged=int(((status >> 16) != 0).sum()),
                _rho=outs["rho"].cpu().numpy(), _h=outs["h"].cpu().numpy())


# adjoint: per in-range pair, 20 FLOP in the coefficient pass (sqrt, q, f, f',
# three sums) and 40 in the gradient pass (both sides of the pair: f' or f,
# c_ij, c/r and three products each)
FLOP_ADJ_PAIR = 60.0
SORT_BYTES_PER_PARTICLE = 300.0   # keys 36, 8 radix passes 192, digit histograms (one key read) 8, permute 64


def _executed(summary, flop, kms, form="fp32c"):
    """Counter-measured binary32 VALU work of a unit (all 64 lanes of every
    issued instruction) at this run's kernel time, beside the algorithmic
    count, and the VALU lane utilisation: the mean fraction of the 64 lanes
    active per issued VALU instruction (SQ_THREAD_CYCLES_VALU over
    64 x SQ_ACTIVE_INST_VALU), the GPU counterpart of the vector efficiency
    of Sec. IV-C (Eq. 2, speed-up over vector length).  None without a
    summary for the current source.  The FP64 form is counted in binary64
    FLOP against the binary64 peak (its binary32 work beside it)."""
    if summary is None:
        return None
    if form == "fp64":
        ex = summary["executed_f64_flop_per_launch"]
        peak = PEAK_FP64
    else:
        ex = summary["executed_f32_flop_per_launch"]
        peak = PEAK_FP32
    out = {"flop_per_launch": ex, "achieved": ex / (kms * 1e-3) / 1e12,
           "frac": ex / (kms * 1e-3) / peak, "algorithmic_over_executed": flop / ex}
    if form == "fp64":
        out["f32_flop_per_launch"] = summary["executed_f32_flop_per_launch"]
    c = summary.get("counters_per_launch", {})
    if c.get("SQ_ACTIVE_INST_VALU") and c.get("SQ_THREAD_CYCLES_VALU"):
        out["valu_lane_utilisation"] = c["SQ_THREAD_CYCLES_VALU"] / (
            64.0 * c["SQ_ACTIVE_INST_VALU"])
    if c.get("SQ_INSTS_VALU"):
        out["valu_wave_instructions"] = c["SQ_INSTS_VALU"]
    return out


def alu_roofline(cands, pairs, kms, form, kernel="k_solve", region=0):
    """Roofline of one density-kernel launch: algorithmic FLOP (8 per candidate
    test, FLOP_PAIR per in-range pair) over the launch's HIP-event time, and
    the same with this kernel's own per-pair count beside it."""
    peak = PEAK_FP32 if form == "fp32c" else PEAK_FP64
    flop = FLOP_REGION * region + FLOP_CAND * cands + FLOP_PAIR[form] * pairs
    flop_k = FLOP_REGION * region + FLOP_CAND * cands + FLOP_PAIR_KERNEL[form] * pairs
    sec = kms * 1e-3
    return {"bound": "alu", "achieved": flop / sec / 1e12, "peak": peak / 1e12,
            "unit": "TFLOP/s", "frac": flop / sec / peak, "kernel": kernel, "kernel_ms": kms,
            "flop_per_launch": flop,
            "flop_weights": {"region_test": FLOP_REGION, "candidate": FLOP_CAND,
                             "pair": FLOP_PAIR[form]},
            "region_tests": region,
            "kernel_counted": {"flop_per_launch": flop_k, "pair": FLOP_PAIR_KERNEL[form],
                               "achieved": flop_k / sec / 1e12, "frac": flop_k / sec / peak}}


def run_adjoint(sph, torch, d, ps, steps, warmup, ev):
    """FP32C root-mode solve, then the adjoint under a Gaussian cotangent on rho."""
    p = sph.default_params(periodic=1, box=ps.box, n_target=ps.n_target, n_tol=ps.n_tol,
                           precision=sph.FP32C, mode=sph.ROOT, root_tol=1e-6)
    n = ps.n
    ws = sph.workspace(p, n, 0, d["x"].device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fw = sph.density_solve(d["x"], d["y"], d["z"], d["m"], d["h_init"], p, ws=ws)
    torch.cuda.synchronize()
    fwd_ms = 1e3 * (time.perf_counter() - t0)
    h = fw["h"]
    import sphgen
    gr = torch.tensor(sphgen.cotangent(n, 5), dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        sph.density_backward(d["x"], d["y"], d["z"], d["m"], h, gr, None, p, ws=ws)
    torch.cuda.synchronize()
    pairs_ev = [(ev.create(), ev.create()) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        p.prof_events[0] = pairs_ev[k][0]
        p.prof_events[1] = pairs_ev[k][1]
        sph.density_backward(d["x"], d["y"], d["z"], d["m"], h, gr, None, p, ws=ws)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    kern = float(np.mean([ev.elapsed_ms(a, b) for a, b in pairs_ev]))
    for a, b in pairs_ev:
        ev.hip.hipEventDestroy(a)
        ev.hip.hipEventDestroy(b)
    pairs = int(fw["nngb"].to(torch.int64).sum().item())
    flop = FLOP_ADJ_PAIR * pairs
    ach = flop / (kern * 1e-3)
    flagged = int(((fw["status"] >> 16) != 0).sum().item())
    return {"workload": "clustered2^20, FP32C root-mode solve (root_tol 1e-6), then the adjoint "
                        "with grad_rho ~ N(0,1) (seed 5)",
            "forward_ms": fwd_ms, "ms_per_call": 1e3 * wall, "kernel_ms": kern,
            "pairs": pairs, "forward_flagged": flagged,
            "roofline": {"bound": "alu", "achieved": ach / 1e12, "peak": PEAK_FP32 / 1e12,
                         "unit": "TFLOP/s", "frac": ach / PEAK_FP32,
                         "kernel": "k_adjoint (both passes)", "flop_per_launch": flop,
                         "executed": _executed(measured_valu("k_adjoint"), flop, kern)}}


def run_sort(sph, torch, d, ps, steps):
    """Keys, radix sort, permutation and the cell table alone (sph_sort)."""
    p = sph.default_params(periodic=1, box=ps.box)
    sph.sort(d["x"], d["y"], d["z"], p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sph.sort(d["x"], d["y"], d["z"], p)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    gbs = SORT_BYTES_PER_PARTICLE * ps.n / (ms * 1e-3) / 1e9
    return {"ms_per_call": ms, "bytes_per_particle": SORT_BYTES_PER_PARTICLE,
            "achieved_GBps": gbs, "peak_GBps": 8000.0, "frac": gbs / 8000.0}


BATCHED = {
    "groups10k": "groups10k: 10000 isolated Plummer groups (sizes ~ n^-2 on [32, 131072], "
                 "scale radii log-uniform 0.005-0.05)",
    "groups10k_a1554": "groups10k_a1554: 10000 isolated Plummer groups (sizes ~ n^-1.554 on "
                       "[32, 131072], the slope whose expected total is ~1.6e7; scale radii "
                       "log-uniform 0.005-0.05)",
}


def run_batched(sph, torch, steps, warmup, ev, name="groups10k"):
    """Many isolated groups (sizes power-law on [32, 131072], N_t = 32 +- 1),
    FP32C, autotuned launch parameters, sort + solve replayed from a captured
    HIP graph; the solve kernel's own time from HIP events on eager calls."""
    import sphgen
    ps = sphgen.config(name)
    n, G = ps.n, len(ps.offsets) - 1
    d = {k: torch.tensor(getattr(ps, k), dtype=torch.float64, device="cuda")
         for k in ("x", "y", "z", "m", "h_init")}
    goff = torch.tensor(ps.offsets, dtype=torch.int64, device="cuda")
    p0 = sph.default_params(periodic=0, n_target=ps.n_target, n_tol=ps.n_tol,
                            precision=sph.FP32C)
    t0 = time.perf_counter()
    p, tuned_ms = sph.autotune(d["x"], d["y"], d["z"], d["m"], d["h_init"], p0, goff)
    tune_s = time.perf_counter() - t0
    ws = sph.workspace(p, n, G, d["x"].device)
    st = sph.density_solve(d["x"], d["y"], d["z"], d["m"], d["h_init"], p, goff, stats=True,
                           ws=ws)
    torch.cuda.synchronize()
    pairs = int(st["stats"][0].item())
    cands = int(st["stats"][1].item())
    region = int(st["stats"][3].item())
    final_pairs = int(st["nngb"].to(torch.int64).sum().item())
    flagged = int(((st["status"] >> 16) != 0).sum().item())
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(max(1, warmup)):
            sph.density_solve(d["x"], d["y"], d["z"], d["m"], d["h_init"], p, goff, ws=ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        sph.density_solve(d["x"], d["y"], d["z"], d["m"], d["h_init"], p, goff, ws=ws)
    graph.replay()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        graph.replay()
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    del graph
    kms = kernel_ms(ev, p, lambda: sph.density_solve(d["x"], d["y"], d["z"], d["m"],
                                                     d["h_init"], p, goff, ws=ws), steps)
    roof = alu_roofline(cands, pairs, kms, "fp32c", region=region)
    roof["replay_frac"] = roof["frac"] * kms / ms   # the same work over the whole replay
    return {"workload": f"{BATCHED[name]}, {n} particles, N_t = 32 +- 1, FP32C, autotuned, "
                        "sort + solve replayed from one HIP graph",
            "n": n, "groups": G, "ms_per_step": ms, "kernel_ms": kms,
            "interactions_per_s": pairs / (ms * 1e-3),
            "particles_per_s": n / (ms * 1e-3), "pairs_per_step": pairs,
            "candidates_per_step": cands, "final_pairs_per_s": final_pairs / (ms * 1e-3),
            "flagged": flagged, "roofline": roof,
            "tuned": {"segment": p.segment, "waves_per_cu": p.waves_per_cu,
                      "tile_cell": p.tile_cell, "ms": tuned_ms, "tuning_s": tune_s}}


def run_large(sph, torch, steps, ev):
    """clustered2^24: 2^24 particles, 2000 Plummer spheres (central contrast
    <= 1e5), N_t = 64 +- 1, FP32C, full sort in every call."""
    import sphgen
    ps = sphgen.config("clustered2^24")
    n = ps.n
    d = {k: torch.tensor(getattr(ps, k), dtype=torch.float64, device="cuda")
         for k in ("x", "y", "z", "m", "h_init")}
    p = sph.default_params(periodic=1, box=ps.box, n_target=ps.n_target, n_tol=ps.n_tol,
                           precision=sph.FP32C)
    ws = sph.workspace(p, n, 0, d["x"].device)
    o = sph.density_solve(d["x"], d["y"], d["z"], d["m"], d["h_init"], p, stats=True, ws=ws)
    torch.cuda.synchronize()
    pairs = int(o["stats"][0].item())
    flagged = int(((o["status"] >> 16) != 0).sum().item())
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        sph.density_solve(d["x"], d["y"], d["z"], d["m"], d["h_init"], p, ws=ws)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    cands = int(o["stats"][1].item())
    region = int(o["stats"][3].item())
    kms = kernel_ms(ev, p, lambda: sph.density_solve(d["x"], d["y"], d["z"], d["m"],
                                                     d["h_init"], p, ws=ws), steps)
    del o
    srt = run_sort(sph, torch, d, ps, steps)
    tr = measured_sort_traffic()
    srt["traffic"] = tr
    if tr is not None:
        # HBM bytes the counters saw per call, over the same call time
        srt["traffic_GBps"] = tr / (srt["ms_per_call"] * 1e-3) / 1e9
    return {"workload": "clustered2^24: 2^24 particles, 2000 Plummer spheres (contrast <= 1e5) "
                        "+ 30% background, N_t = 64 +- 1, FP32C, full sort every call",
            "n": n, "ms_per_step": ms, "interactions_per_s": pairs / (ms * 1e-3),
            "particles_per_s": n / (ms * 1e-3), "pairs_per_step": pairs,
            "candidates_per_step": cands, "flagged": flagged, "kernel_ms": kms,
            "roofline": alu_roofline(cands, pairs, kms, "fp32c", region=region), "sort": srt}


def run_wendland(sph, torch, d, ps, steps, ev):
    """The paper's kernel at the paper's scale: Wendland C6 with N_t = 295 +- 2
    on the clustered 2^20 set (FP32C and FP64), sort + solve per step; the
    roofline of its k_solve launch from the kernel's own counts."""
    out = {"workload": "clustered2^20, Wendland C6 kernel, N_t = 295 +- 2, h_init = 2 N^-1/3"}
    for prec, name in ((sph.FP32C, "fp32c"), (sph.FP64, "fp64")):
        p = sph.default_params(periodic=1, box=ps.box, n_target=295.0, n_tol=2.0,
                               precision=prec, kernel=sph.KERNEL_WENDLAND_C6)
        ws = sph.workspace(p, ps.n, 0, d["x"].device)
        o = sph.density_solve(d["x"], d["y"], d["z"], d["m"], d["h_init"], p, stats=True, ws=ws)
        torch.cuda.synchronize()
        pairs = int(o["stats"][0].item())
        flagged = int(((o["status"] >> 16) != 0).sum().item())
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            sph.density_solve(d["x"], d["y"], d["z"], d["m"], d["h_init"], p, ws=ws)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        cands = int(o["stats"][1].item())
        region = int(o["stats"][3].item())
        kms = kernel_ms(ev, p, lambda: sph.density_solve(d["x"], d["y"], d["z"], d["m"],
                                                         d["h_init"], p, ws=ws), steps)
        flop = FLOP_REGION * region + FLOP_CAND * cands + FLOP_PAIR_WC6[name] * pairs
        peak = PEAK_FP32 if name == "fp32c" else PEAK_FP64
        out[name] = {"ms_per_step": ms, "interactions_per_s": pairs / (ms * 1e-3),
                     "particles_per_s": ps.n / (ms * 1e-3), "pairs_per_step": pairs,
                     "candidates_per_step": cands, "flagged": flagged, "kernel_ms": kms,
                     "roofline": {"bound": "alu", "kernel": "k_solve",
                                  "achieved": flop / (kms * 1e-3) / 1e12,
                                  "peak": peak / 1e12, "unit": "TFLOP/s",
                                  "frac": flop / (kms * 1e-3) / peak, "flop_per_launch": flop}}
    out["fp32c_speedup_over_fp64"] = out["fp64"]["ms_per_step"] / out["fp32c"]["ms_per_step"]
    return out


def kernel_ms(ev, p, call, steps):
    """Mean time of the library's kernels over `steps` calls, from the hipEvent
    pair each call records on its stream (params.prof_events)."""
    pairs = [(ev.create(), ev.create()) for _ in range(steps)]
    for a, b in pairs:
        p.prof_events[0], p.prof_events[1] = a, b
        call()
    p.prof_events[0] = p.prof_events[1] = None
    ms = float(np.mean([ev.elapsed_ms(a, b) for a, b in pairs]))
    for a, b in pairs:
        ev.hip.hipEventDestroy(a)
        ev.hip.hipEventDestroy(b)
    return ms


def run_knn(sph, torch, d, ps, steps, dk=14.0):
    """The paper's own criterion at its scale: h = distance of the 295th
    nearest particle (itself first), Wendland C6, on the clustered 2^20 set
    (FP32C and FP64); sort + count stage + selection + evaluation per step."""
    out = {"workload": f"clustered2^20, Wendland C6 kernel, exact K = 295 (count band "
                       f"[K, K + {int(dk)}] then selection), h_init = 2 N^-1/3"}
    for prec, name in ((sph.FP32C, "fp32c"), (sph.FP64, "fp64")):
        p = sph.default_params(periodic=1, box=ps.box, n_target=295.0, n_tol=dk,
                               precision=prec, kernel=sph.KERNEL_WENDLAND_C6, mode=sph.KNN)
        ws = sph.workspace(p, ps.n, 0, d["x"].device)
        o = sph.density_solve(d["x"], d["y"], d["z"], d["m"], d["h_init"], p, ws=ws)
        torch.cuda.synchronize()
        flagged = int(((o["status"] >> 16) != 0).sum().item())
        iters = int((o["status"] & 0xFFFF).max().item())
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            sph.density_solve(d["x"], d["y"], d["z"], d["m"], d["h_init"], p, ws=ws)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        st = sph.density_solve(d["x"], d["y"], d["z"], d["m"], d["h_init"], p, ws=ws,
                               stats=True)
        torch.cuda.synchronize()
        cands = int(st["stats"][1].item())
        region = int(st["stats"][3].item())
        passes = int(st["stats"][2].item())
        final_pairs = int(st["nngb"].to(torch.int64).sum().item())
        kms = kernel_ms(HipEvents(), p, lambda: sph.density_solve(
            d["x"], d["y"], d["z"], d["m"], d["h_init"], p, ws=ws), steps)
        # algorithmic work, a lower bound: every candidate test of the three
        # stages, and the Wendland C6 pair terms of the evaluation stage only
        form = "fp32c" if prec == sph.FP32C else "fp64"
        flop = FLOP_REGION * region + FLOP_CAND * cands + FLOP_PAIR_WC6[form] * final_pairs
        peak = PEAK_FP32 if prec == sph.FP32C else PEAK_FP64
        out[name] = {"ms_per_step": ms, "particles_per_s": ps.n / (ms * 1e-3),
                     "flagged": flagged, "max_count_updates": iters, "kernel_ms": kms,
                     "candidates_per_step": cands, "final_pairs": final_pairs,
                     "passes_per_step": passes,
                     "roofline": {"bound": "alu", "kernel": "k_solve (exact-K stages)",
                                  "achieved": flop / (kms * 1e-3) / 1e12,
                                  "peak": peak / 1e12, "unit": "TFLOP/s",
                                  "frac": flop / (kms * 1e-3) / peak,
                                  "flop_per_launch": flop}}
    out["fp32c_speedup_over_fp64"] = out["fp64"]["ms_per_step"] / out["fp32c"]["ms_per_step"]
    return out


def run_aos(sph, torch, d, ps, steps):
    """Array-of-structs interop (Sec. IV-B) on the headline workload: the same
    FP32C sort + solve reading x, y, z, m, h_init from 224-byte particle structs
    and writing rho, h, nw, nngb, status back into them, against packed arrays.
    Alternating rounds; the best round of each."""
    n = ps.n
    p = sph.default_params(periodic=1, box=ps.box, n_target=ps.n_target, n_tol=ps.n_tol,
                           precision=sph.FP32C)
    ws = sph.workspace(p, n, 0, d["x"].device)
    S = torch.zeros((n, 28), dtype=torch.float64, device=d["x"].device)
    for c, k in ((0, "x"), (1, "y"), (2, "z"), (6, "m"), (8, "h_init")):
        S[:, c] = d[k]
    iv = S.view(torch.int32)
    out = dict(rho=S[:, 9], h=S[:, 10], nw=S[:, 11], nngb=iv[:, 24], status=iv[:, 25])

    def packed():
        sph.density_solve(d["x"], d["y"], d["z"], d["m"], d["h_init"], p, ws=ws)

    def aos():
        sph.density_solve(S[:, 0], S[:, 1], S[:, 2], S[:, 6], S[:, 8], p, ws=ws, out=out)

    best = {"packed": float("inf"), "aos": float("inf")}
    for _ in range(3):
        for name, fn in (("packed", packed), ("aos", aos)):
            fn()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(steps):
                fn()
            b.record()
            torch.cuda.synchronize()
            best[name] = min(best[name], a.elapsed_time(b) / steps)
    return {"workload": "clustered2^20 FP32C sort + solve; inputs and outputs in 224-byte "
                        "particle structs (stride 224) vs packed arrays",
            "packed_ms": best["packed"], "aos_ms": best["aos"],
            "overhead": best["aos"] / best["packed"] - 1.0}


# scatter form: per in-range pair (r < h_i or r < h_j) one square root, two
# kernel shapes (q, f: 9 each for M4) and three accumulations
FLOP_SCAT_PAIR = 24.0


def run_scatter(sph, torch, d, ps, steps):
    """Eq. (1) with each neighbour's own h_j (and the symmetric average) on the
    clustered 2^20 set at the h of the FP32C solve: sort + walk per call."""
    p = sph.default_params(periodic=1, box=ps.box, n_target=ps.n_target, n_tol=ps.n_tol,
                           precision=sph.FP32C)
    f = sph.density_solve(d["x"], d["y"], d["z"], d["m"], d["h_init"], p)
    h = f["h"]
    ws = sph.workspace(p, ps.n, 0, d["x"].device)
    o = sph.density_scatter(d["x"], d["y"], d["z"], d["m"], h, p, ws=ws)
    torch.cuda.synchronize()
    pairs_s = int(o["nngb_s"].to(torch.int64).sum().item())
    pairs_g = int(f["nngb"].to(torch.int64).sum().item())
    ev = HipEvents()
    kms = []
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        e0, e1 = ev.create(), ev.create()
        p.prof_events[0], p.prof_events[1] = e0, e1
        sph.density_scatter(d["x"], d["y"], d["z"], d["m"], h, p, ws=ws)
        kms.append((e0, e1))
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    kernel_ms = float(np.mean([ev.elapsed_ms(x, y) for x, y in kms]))
    for x, y in kms:
        ev.hip.hipEventDestroy(x)
        ev.hip.hipEventDestroy(y)
    # pairs with r < h_i or r < h_j: at most the sum of both counts
    flop = FLOP_SCAT_PAIR * max(pairs_s, pairs_g)
    return {"workload": "clustered2^20 at the FP32C solve's h: rho_s = sum_j m_j W(r_ij, h_j), "
                        "rho_sym, counts; FP32C; sort + walk per call",
            "ms_per_call": ms, "kernel_ms": kernel_ms,
            "interactions_per_s": pairs_s / (ms * 1e-3), "pairs_scatter": pairs_s,
            "pairs_gather": pairs_g,
            "roofline": {"bound": "alu", "achieved": flop / (kernel_ms * 1e-3) / 1e12,
                         "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                         "frac": flop / (kernel_ms * 1e-3) / PEAK_FP32,
                         "kernel": "k_adjoint (scatter phase)", "flop_per_launch": flop}}


def run_force(sph, torch, d, ps, steps):
    """The grad-h SPH pressure force (the adjoint for the cotangent m P/rho^2)
    on the clustered 2^20 set at the h and rho of an FP32C root-mode solve,
    P = A rho^(5/3) with A ~ U(0.5, 2) (seed 5)."""
    p = sph.default_params(periodic=1, box=ps.box, n_target=ps.n_target, n_tol=ps.n_tol,
                           precision=sph.FP32C, mode=sph.ROOT, root_tol=1e-6)
    f = sph.density_solve(d["x"], d["y"], d["z"], d["m"], d["h_init"], p)
    A = torch.tensor(np.random.default_rng(5).uniform(0.5, 2.0, ps.n), dtype=torch.float64,
                     device=d["x"].device)
    P = A * f["rho"] ** (5.0 / 3.0)
    ws = sph.workspace(p, ps.n, 0, d["x"].device)
    sph.pressure_force(d["x"], d["y"], d["z"], d["m"], f["h"], f["rho"], P, p, ws=ws)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        sph.pressure_force(d["x"], d["y"], d["z"], d["m"], f["h"], f["rho"], P, p, ws=ws)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    kms = kernel_ms(HipEvents(), p, lambda: sph.pressure_force(
        d["x"], d["y"], d["z"], d["m"], f["h"], f["rho"], P, p, ws=ws), steps)
    pairs = int(f["nngb"].to(torch.int64).sum().item())
    flop = FLOP_ADJ_PAIR * pairs
    return {"workload": "clustered2^20 FP32C, h and rho of a root-mode solve, P = A rho^(5/3); "
                        "sort + both walk passes + scaling per call",
            "ms_per_call": ms, "particles_per_s": ps.n / (ms * 1e-3), "kernel_ms": kms,
            "pairs": pairs,
            "roofline": {"bound": "alu", "kernel": "k_adjoint (both passes)",
                         "achieved": flop / (kms * 1e-3) / 1e12, "peak": PEAK_FP32 / 1e12,
                         "unit": "TFLOP/s", "frac": flop / (kms * 1e-3) / PEAK_FP32,
                         "flop_per_launch": flop}}


def _cpu_model():
    """The host CPU's model name (lscpu, else /proc/cpuinfo), with its family
    and model numbers where the name alone is generic."""
    import subprocess
    name, fam, mod = None, None, None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            k, _, v = ln.partition(":")
            if k.strip() == "Model name" and name is None:
                name = v.strip()
            elif k.strip() == "CPU family":
                fam = v.strip()
            elif k.strip() == "Model":
                mod = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    if name is None:
        try:
            for ln in open("/proc/cpuinfo"):
                if ln.startswith("model name"):
                    name = ln.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    if name is not None and fam is not None:
        name = f"{name} (family {fam}, model {mod})"
    return name


def cpu_baseline_child(budget_s):
    """Runs in its own process with the OpenMP placement fixed before the
    oracle's runtime starts: OMP_PROC_BIND=close, OMP_PLACES=cores."""
    import oracle
    import sphgen
    ps = sphgen.config("clustered2^20")
    rng = np.random.default_rng(12345)
    cores = oracle.max_threads()
    # two probes separate the fixed cost (tree build) from the per-particle cost
    t = []
    for k in (2000, 12000):
        t0 = time.perf_counter()
        oracle.solve(ps, subset=rng.choice(ps.n, k, replace=False))
        t.append(time.perf_counter() - t0)
    per = max((t[1] - t[0]) / 10000.0, 1e-7)
    fixed = max(t[0] - 2000 * per, 0.0)
    k = int(min(ps.n, max(2000, (budget_s - fixed) / per)))
    sub = rng.choice(ps.n, k, replace=False)
    runs = []
    pairs = 0
    for _ in range(3):
        t0 = time.perf_counter()
        r = oracle.solve(ps, subset=sub)
        runs.append(time.perf_counter() - t0)
        pairs = int(r["pairs"].sum())
    dt = float(np.median(runs))
    # the small configuration by brute force (O(N^2) neighbour search), the same
    # dynamic schedule: 4096 uniform particles, h_init = 0.125, N_t = 64 +- 2
    c1 = sphgen.config("uniform4096")
    bf = []
    for _ in range(3):
        t0 = time.perf_counter()
        rb = oracle.solve(c1, search=0)
        bf.append(time.perf_counter() - t0)
    bdt = float(np.median(bf))
    bpairs = int(rb["pairs"].sum())
    return {"value": pairs / dt, "unit": "interactions/s", "cores": cores, "kind": "oracle",
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
            "omp": {k: os.environ.get(k) for k in ("OMP_PROC_BIND", "OMP_PLACES",
                                                   "OMP_NUM_THREADS")},
            "sample": (f"all {k} particles of the clustered set" if k == ps.n else
                       f"{k} particles drawn uniformly from the {ps.n}-particle clustered set")
                      + f", each solved to convergence against the full set (FP64 k-d tree, "
                      f"OpenMP dynamic schedule; median of 3 runs {dt:.2f} s incl. tree "
                      f"build); particles/s = {k / dt:.4g}",
            "runs_s": runs, "particles_per_s": k / dt,
            "brute_force_uniform4096": {"ms": 1e3 * bdt, "runs_ms": [1e3 * v for v in bf],
                                        "interactions_per_s": bpairs / bdt,
                                        "particles_per_s": c1.n / bdt}}


def cpu_baseline(budget_s=6.0):
    """The oracle on the host's cores, in a child process (it uses no GPU) so
    that its OpenMP threads are pinned as asked before they start."""
    import subprocess
    env = dict(os.environ, OMP_PROC_BIND="close", OMP_PLACES="cores")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-child",
                        str(budget_s)], env=env, capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        raise RuntimeError("cpu baseline failed:\n" + r.stderr[-2000:])
    return json.loads(r.stdout.strip().splitlines()[-1])


SOLVE_SRC = os.path.join(ROOT, "paper_1612_06090_amd", "csrc", "solve.hip")
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "k_solve_clustered2p20_traffic.txt")
COPY_MIB = 256


def solve_source_sha():
    import hashlib
    return hashlib.sha256(open(SOLVE_SRC, "rb").read()).hexdigest()


def measured_traffic():
    """HBM bytes per k_solve launch from the committed counter summary, or None
    when the kernel source changed since the counters were taken."""
    try:
        d = json.load(open(TRAFFIC_JSON))
    except (OSError, ValueError):
        return None
    if d.get("solve_hip_sha256") != solve_source_sha():
        return None
    return d.get("bytes_per_launch")


def profile_run(steps, fp64=False):
    """FP32C (or FP64) solves plus one plain copy of COPY_MIB MiB (the counter
    calibration)."""
    import torch
    import paper_1612_06090_amd as sph
    import sphgen
    ps = sphgen.config("clustered2^20")
    d = {k: torch.tensor(getattr(ps, k), dtype=torch.float64, device="cuda")
         for k in ("x", "y", "z", "m", "h_init")}
    p = sph.default_params(n_target=ps.n_target, n_tol=ps.n_tol,
                           precision=sph.FP64 if fp64 else sph.FP32C)
    for _ in range(steps):
        sph.density_solve(d["x"], d["y"], d["z"], d["m"], d["h_init"], p)
    src = torch.ones(COPY_MIB << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(f"[bench] profile run: {steps} solves + one {COPY_MIB} MiB copy", flush=True)


def profile_adjoint_run(steps):
    """A root-mode FP32C solve of the clustered 2^20 set, then `steps` adjoint
    calls with the benchmark's cotangent (for rocprofv3 --pmc)."""
    import torch
    import paper_1612_06090_amd as sph
    import sphgen
    ps = sphgen.config("clustered2^20")
    d = {k: torch.tensor(getattr(ps, k), dtype=torch.float64, device="cuda")
         for k in ("x", "y", "z", "m", "h_init")}
    p = sph.default_params(periodic=1, box=ps.box, n_target=ps.n_target, n_tol=ps.n_tol,
                           precision=sph.FP32C, mode=sph.ROOT, root_tol=1e-6)
    fw = sph.density_solve(d["x"], d["y"], d["z"], d["m"], d["h_init"], p)
    gr = torch.tensor(sphgen.cotangent(ps.n, 5), dtype=torch.float64, device="cuda")
    for _ in range(steps):
        sph.density_backward(d["x"], d["y"], d["z"], d["m"], fw["h"], gr, None, p)
    torch.cuda.synchronize()
    print(f"[bench] adjoint profile run: one solve + {steps} adjoint calls", flush=True)


def summarize_traffic(fetch_csv, write_csv, cmd):
    """Per-launch k_solve HBM traffic from FETCH_SIZE / WRITE_SIZE (KiB per
    dispatch), each scaled by the same counter on the calibration copy."""
    import csv

    def per_kernel(path, counter):
        # the calibration copy is the largest non-solve dispatch of the run
        solve, other = [], []
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            v = float(r["Counter_Value"]) * 1024.0
            if "k_solve" in r["Kernel_Name"]:
                solve.append(v)
            else:
                other.append(v)
        return solve, [max(other)]

    fs, fc = per_kernel(fetch_csv, "FETCH_SIZE")
    ws, wc = per_kernel(write_csv, "WRITE_SIZE")
    nbytes = float(COPY_MIB << 20)
    kf = max(fc) / nbytes
    kw = max(wc) / nbytes
    fetch = float(np.mean(fs)) / kf
    write = float(np.mean(ws)) / kw
    out = {"kernel": "k_solve (FP32C, 16-particle tiles)", "workload": "clustered2^20",
           "solve_hip_sha256": solve_source_sha(),
           "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
           "bytes_per_launch": fetch + write,
           "copy_calibration": {"bytes": nbytes, "fetch_factor": kf, "write_factor": kw},
           "raw_bytes_per_dispatch": {"fetch_solve": fs, "write_solve": ws, "fetch_copy": fc,
                                      "write_copy": wc},
           "command": cmd}
    os.makedirs(os.path.dirname(TRAFFIC_JSON), exist_ok=True)
    json.dump(out, open(TRAFFIC_JSON, "w"), indent=1)
    print(json.dumps({k: out[k] for k in ("fetch_bytes_per_launch", "write_bytes_per_launch",
                                          "copy_calibration")}))


VALU_JSON = os.path.join(ROOT, "profiles", "k_solve_clustered2p20_valu.txt")
# wave-instruction counters -> operations on all 64 lanes (FMA = 2), masked lanes included
VALU_WEIGHTS = {"f32": {"SQ_INSTS_VALU_ADD_F32": 1, "SQ_INSTS_VALU_MUL_F32": 1,
                        "SQ_INSTS_VALU_FMA_F32": 2, "SQ_INSTS_VALU_TRANS_F32": 1},
                "f64": {"SQ_INSTS_VALU_ADD_F64": 1, "SQ_INSTS_VALU_MUL_F64": 1,
                        "SQ_INSTS_VALU_FMA_F64": 2, "SQ_INSTS_VALU_TRANS_F64": 1}}


VALU_TARGETS = {
    # kernel -> (summary file, source it is tied to, what one unit is)
    "k_solve": (VALU_JSON, SOLVE_SRC, "launch"),
    "k_solve_fp64": (os.path.join(ROOT, "profiles", "k_solve_fp64_clustered2p20_valu.txt"),
                     SOLVE_SRC, "launch"),
    "k_adjoint": (os.path.join(ROOT, "profiles", "k_adjoint_clustered2p20_valu.txt"),
                  os.path.join(ROOT, "paper_1612_06090_amd", "csrc", "backward.hip"),
                  "backward call (both passes)"),
}


def summarize_valu(cmd, *csvs, kernel="k_solve", calls=None):
    """Executed VALU work of one kernel from SQ instruction counters taken over
    several --pmc passes of the same profile run: per-dispatch sums over the
    counter's instances, then the mean per dispatch (or, given `calls`, the
    total over all dispatches divided by the number of calls)."""
    import csv
    import hashlib
    out_path, src, unit = VALU_TARGETS[kernel]
    if kernel == "k_solve":
        out_path = VALU_JSON
    match = "k_solve" if kernel.startswith("k_solve") else kernel
    per = {}
    for path in csvs:
        acc = {}
        for r in csv.DictReader(open(path)):
            if match not in r["Kernel_Name"]:
                continue
            key = (r["Counter_Name"], r["Dispatch_Id"])
            acc[key] = acc.get(key, 0.0) + float(r["Counter_Value"])
        for (name, _), v in acc.items():
            per.setdefault(name, []).append(v)
    if calls is None:
        mean = {k: float(np.mean(v)) for k, v in sorted(per.items())}
    else:
        mean = {k: float(np.sum(v)) / int(calls) for k, v in sorted(per.items())}
    flop = {t: 64.0 * sum(w * mean.get(c, 0.0) for c, w in ws.items())
            for t, ws in VALU_WEIGHTS.items()}
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    label = {"k_solve": "k_solve (FP32C, 16-particle tiles)",
             "k_solve_fp64": "k_solve (FP64, 16-particle tiles)"}.get(kernel, f"{kernel} (FP32C)")
    out = {"kernel": label,
           "workload": "clustered2^20", "unit": unit,
           ("solve_hip_sha256" if kernel.startswith("k_solve") else "source_sha256"): sha,
           "executed_f32_flop_per_launch": flop["f32"],
           "executed_f64_flop_per_launch": flop["f64"],
           "counters_per_launch": mean,
           "dispatches": {k: len(v) for k, v in sorted(per.items())},
           "note": "SQ_INSTS_VALU_* count wave instructions; FLOP = 64 lanes x (ADD + MUL + "
                   "TRANS + 2 FMA), lanes masked off included",
           "command": cmd}
    if mean.get("SQ_ACTIVE_INST_VALU"):
        out["thread_cycles_per_valu_cycle_raw"] = (mean.get("SQ_THREAD_CYCLES_VALU", 0.0) /
                                                   mean["SQ_ACTIVE_INST_VALU"])
    os.makedirs(os.path.dirname(out_path), exist_ok=True)
    json.dump(out, open(out_path, "w"), indent=1)
    print(json.dumps({k: out[k] for k in ("executed_f32_flop_per_launch",
                                          "executed_f64_flop_per_launch", "dispatches")}))


def measured_valu(kernel="k_solve"):
    """The committed counter summary of a kernel's executed VALU work (per
    k_solve launch, per backward call), or None when the kernel source changed
    since it was taken."""
    import hashlib
    path, src, _ = VALU_TARGETS[kernel]
    if kernel == "k_solve":
        path, key = VALU_JSON, "solve_hip_sha256"
    elif kernel.startswith("k_solve"):
        key = "solve_hip_sha256"
    else:
        key = "source_sha256"
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get(key) != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    return d


SORT_SRC = os.path.join(ROOT, "paper_1612_06090_amd", "csrc", "sort.hip")
SORT_TRAFFIC_JSON = os.path.join(ROOT, "profiles", "sph_sort_clustered2p24_traffic.txt")


def sort_source_sha():
    import hashlib
    return hashlib.sha256(open(SORT_SRC, "rb").read()).hexdigest()


def profile_sort_run(steps):
    """sph_sort calls on the clustered 2^24 set (as the large leg times them)
    plus one plain copy of COPY_MIB MiB (the counter calibration)."""
    import torch
    import paper_1612_06090_amd as sph
    import sphgen
    ps = sphgen.config("clustered2^24")
    d = {k: torch.tensor(getattr(ps, k), dtype=torch.float64, device="cuda")
         for k in ("x", "y", "z")}
    p = sph.default_params(periodic=1, box=ps.box)
    for _ in range(steps):
        sph.sort(d["x"], d["y"], d["z"], p)
    src = torch.ones(COPY_MIB << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(f"[bench] sort profile run: {steps} sorts of {ps.n} + one {COPY_MIB} MiB copy",
          flush=True)


def summarize_sort_traffic(fetch_csv, write_csv, cmd, steps="2"):
    """HBM bytes per sph_sort call at 2^24 from FETCH_SIZE / WRITE_SIZE (KiB
    per dispatch) over the library's dispatches, each counter scaled by its
    reading on the calibration copy; per kernel and in total."""
    import csv
    steps = int(steps)

    def read(path, counter):
        lib, other = {}, []
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            v = float(r["Counter_Value"]) * 1024.0
            name = r["Kernel_Name"]
            if "sph::" in name:
                short = name.split("sph::", 1)[1].split("(", 1)[0]
                lib[short] = lib.get(short, 0.0) + v
            else:
                other.append(v)
        return lib, max(other)

    lf, cf = read(fetch_csv, "FETCH_SIZE")
    lw, cw = read(write_csv, "WRITE_SIZE")
    nbytes = float(COPY_MIB << 20)
    kf, kw = cf / nbytes, cw / nbytes
    n = 1 << 24
    per_kernel = {k: {"fetch": lf.get(k, 0.0) / kf / steps, "write": lw.get(k, 0.0) / kw / steps}
                  for k in sorted(set(lf) | set(lw))}
    fetch = sum(v["fetch"] for v in per_kernel.values())
    write = sum(v["write"] for v in per_kernel.values())
    out = {"call": "sph_sort (keys, radix passes, permutation, cell table)",
           "workload": "clustered2^24", "n": n, "sort_hip_sha256": sort_source_sha(),
           "fetch_bytes_per_call": fetch, "write_bytes_per_call": write,
           "bytes_per_call": fetch + write, "bytes_per_particle": (fetch + write) / n,
           "algorithmic_bytes_per_particle": SORT_BYTES_PER_PARTICLE,
           "per_kernel_bytes_per_call": per_kernel,
           "copy_calibration": {"bytes": nbytes, "fetch_factor": kf, "write_factor": kw},
           "calls": steps, "command": cmd}
    os.makedirs(os.path.dirname(SORT_TRAFFIC_JSON), exist_ok=True)
    json.dump(out, open(SORT_TRAFFIC_JSON, "w"), indent=1)
    print(json.dumps({k: out[k] for k in ("bytes_per_call", "bytes_per_particle",
                                          "copy_calibration")}))


def measured_sort_traffic():
    """HBM bytes per sph_sort call at 2^24 from the committed counter summary,
    or None when the sort source changed since the counters were taken."""
    try:
        d = json.load(open(SORT_TRAFFIC_JSON))
    except (OSError, ValueError):
        return None
    if d.get("sort_hip_sha256") != sort_source_sha():
        return None
    return d.get("bytes_per_call")


TRACE_MD = os.path.join(ROOT, "profiles", "k_solve_clustered2p20_kernel_trace.md")
TRACE_KNN_MD = os.path.join(ROOT, "profiles", "k_solve_exactK295_clustered2p20_kernel_trace.md")
TRACE_BATCHED_MD = os.path.join(ROOT, "profiles", "k_solve_groups10k_kernel_trace.md")
TRACE_LARGE_MD = os.path.join(ROOT, "profiles", "k_solve_clustered2p24_kernel_trace.md")
TRACE_WC6_MD = os.path.join(ROOT, "profiles", "k_solve_wendland295_clustered2p20_kernel_trace.md")
TRACE_SORT_MD = os.path.join(ROOT, "profiles", "sph_sort_clustered2p24_kernel_trace.md")


def summarize_trace(stats_csv, cmd, which="headline"):
    """Kernel-time table from rocprofv3 --kernel-trace --stats (kernel_stats.csv)."""
    import csv
    rows = list(csv.DictReader(open(stats_csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    src = ("Solve", solve_source_sha())
    if which == "sort":
        path = TRACE_SORT_MD
        src = ("Sort", sort_source_sha())
        head = ["# sph_sort on clustered2^24 — rocprofv3 kernel trace", "",
                "Command (on the GPU host, from the repository root):", "", "    " + cmd, "",
                "Workload: Morton keys, radix sort, permutation and cell list of the "
                "2^24-particle clustered set (the large leg's sort), four calls, plus "
                "one plain copy (the counter calibration of the traffic runs; torch's "
                "kernels below). One call = a clear of the look-back descriptors, the "
                "digit histograms of all eight passes, eight single-sweep scatter "
                "passes (16-round tiles), then the cell list.", ""]
    elif which == "large":
        path = TRACE_LARGE_MD
        head = ["# Density solve on clustered2^24 — rocprofv3 kernel trace", "",
                "Command (on the GPU host, from the repository root):", "", "    " + cmd, "",
                "Workload: 2^24 particles, 2000 Plummer spheres (contrast <= 1e5) + 30% "
                "background, N_t = 64 +- 1, FP32C; one call = keys + digit histograms + "
                "single-sweep radix sort (16-round tiles) + permute + dense cell table + "
                "density/h solve.", ""]
    elif which == "wendland":
        path = TRACE_WC6_MD
        head = ["# Wendland C6 solve on clustered2^20 — rocprofv3 kernel trace", "",
                "Command (on the GPU host, from the repository root):", "", "    " + cmd, "",
                "Workload: the 2^20-particle clustered set, Wendland C6 kernel, band "
                "N_t = 295 +- 2, h_init = 2 N^-1/3; `k_solve<1, ..., 1, ...>` FP32C, "
                "`k_solve<0, ..., 1, ...>` FP64.", ""]
    elif which == "batched":
        path = TRACE_BATCHED_MD
        head = ["# Batched solve on groups10k — rocprofv3 kernel trace", "",
                "Command (on the GPU host, from the repository root):", "", "    " + cmd, "",
                "Workload: 10,000 isolated Plummer groups (sizes ~ n^-2 on [32, 131072]), "
                "2,246,696 particles, N_t = 32 +- 1, FP32C, the autotuned tile size; one "
                "replay of the HIP graph = group frames and keys, radix sort, permute, "
                "largest-first group order, group items, density/h solve. Calls include "
                "the autotuner's trial launches of other tile sizes.", ""]
    elif which == "knn":
        path = TRACE_KNN_MD
        head = ["# Exact-K stages on clustered2^20 (K = 295, Wendland C6) — rocprofv3 "
                "kernel trace", "",
                "Command (on the GPU host, from the repository root):", "", "    " + cmd, "",
                "Workload: the 2^20-particle clustered set, h = distance of the 295th "
                "nearest particle (itself first), Wendland C6, count band [K, K + 14]. "
                "One call = sort + four launches of the density kernel, told apart by "
                "its fifth template argument: 1 the count stage (h iterated on the "
                "integer count), 2 the selection of the K-th distance from per-lane lists "
                "of an outer shell (16-particle tiles, 4 lanes per particle), 4 the heap "
                "selection for the particles whose shell was too thin (only the tiles "
                "holding one), 3 the evaluation at that h. `k_solve<1, ...>` is FP32C, "
                "`k_solve<0, ...>` FP64.", ""]
    else:
        path = TRACE_MD
        head = ["# k_solve on clustered2^20 — rocprofv3 kernel trace", "",
                "Command (on the GPU host, from the repository root):", "", "    " + cmd, "",
                "Workload: the 2^20-particle clustered set (200 Plummer spheres + 30% "
                "background), N_t = 64 +- 2; one call = keys + radix sort + permute + dense "
                "cell table + density/h solve. `k_solve<1, ...>` is the FP32C solve, "
                "`k_solve<0, ...>` the FP64 one, both with 16-particle tiles.", ""]
    out = head + [f"{src[0]} source sha256: `{src[1]}`", "",
                  "| Kernel | Calls | Avg (us) | Share |", "|---|---|---|---|"]
    for r in rows[:14]:
        name = r["Name"].split("(")[0]
        out.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['Percentage']):.2f}% |")
    os.makedirs(os.path.dirname(path), exist_ok=True)
    open(path, "w").write("\n".join(out) + "\n")
    print("\n".join(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--no-wendland", action="store_true")
    ap.add_argument("--no-knn", action="store_true")
    ap.add_argument("--no-aos", action="store_true")
    ap.add_argument("--no-scatter", action="store_true")
    ap.add_argument("--no-force", action="store_true")
    ap.add_argument("--only-knn", action="store_true",
                    help="only the exact-K leg (for a kernel trace of its stages)")
    ap.add_argument("--profile-run", action="store_true",
                    help="only FP32C solves + a calibration copy (for rocprofv3 --pmc)")
    ap.add_argument("--profile-fp64", action="store_true",
                    help="with --profile-run: FP64 solves instead")
    ap.add_argument("--only-batched", action="store_true",
                    help="only the groups10k leg (for a kernel trace of its replays)")
    ap.add_argument("--only-large", action="store_true",
                    help="only the clustered 2^24 leg (for a kernel trace)")
    ap.add_argument("--only-wendland", action="store_true",
                    help="only the Wendland C6 N_t = 295 leg (for a kernel trace)")
    ap.add_argument("--profile-sort", action="store_true",
                    help="only sph_sort calls at 2^24 + a calibration copy (for rocprofv3 --pmc)")
    ap.add_argument("--summarize-sort-traffic", nargs="+", metavar="ARG",
                    help="FETCH_CSV WRITE_CSV CMD [CALLS]: write the sph_sort traffic summary")
    ap.add_argument("--summarize-trace", nargs="+", metavar="ARG",
                    help="STATS_CSV CMD [headline|knn|batched|large|wendland|sort]: write the "
                         "kernel-trace summary "
                         "from rocprofv3 --stats output")
    ap.add_argument("--summarize-traffic", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "CMD"),
                    help="write the k_solve traffic summary from two --pmc runs")
    ap.add_argument("--summarize-valu", nargs="+", metavar="ARG",
                    help="CMD CSV [CSV ...]: write the executed-VALU summary of --valu-kernel "
                         "from --pmc runs of SQ instruction counters")
    ap.add_argument("--valu-kernel", default="k_solve", choices=sorted(VALU_TARGETS))
    ap.add_argument("--valu-calls", type=int, default=None,
                    help="report totals per call over this many calls (default: per dispatch)")
    ap.add_argument("--profile-adjoint", action="store_true",
                    help="only one solve + adjoint calls (for rocprofv3 --pmc)")
    ap.add_argument("--cpu-baseline-child", type=float, default=None, metavar="BUDGET_S",
                    help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_baseline_child is not None:
        print(json.dumps(cpu_baseline_child(args.cpu_baseline_child)), flush=True)
        return
    if args.summarize_trace:
        if len(args.summarize_trace) not in (2, 3):
            ap.error("--summarize-trace takes STATS_CSV CMD "
                     "[headline|knn|batched|large|wendland|sort]")
        summarize_trace(*args.summarize_trace)
        return
    if args.summarize_traffic:
        summarize_traffic(*args.summarize_traffic)
        return
    if args.summarize_valu:
        if len(args.summarize_valu) < 2:
            ap.error("--summarize-valu takes CMD CSV [CSV ...]")
        summarize_valu(*args.summarize_valu, kernel=args.valu_kernel, calls=args.valu_calls)
        return
    if args.summarize_sort_traffic:
        if len(args.summarize_sort_traffic) not in (3, 4):
            ap.error("--summarize-sort-traffic takes FETCH_CSV WRITE_CSV CMD [CALLS]")
        summarize_sort_traffic(*args.summarize_sort_traffic)
        return
    if args.profile_run:
        profile_run(args.steps, fp64=args.profile_fp64)
        return
    if args.profile_sort:
        profile_sort_run(args.steps)
        return
    if args.profile_adjoint:
        profile_adjoint_run(args.steps)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the path is "
              "single-GPU: one process drives one MI355X.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1612_06090_amd as sph
    import sphgen

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    sph.load()
    ps = sphgen.config("clustered2^20")
    d = {k: torch.tensor(getattr(ps, k), dtype=torch.float64, device="cuda")
         for k in ("x", "y", "z", "m", "h_init")}
    ev = HipEvents()
    print(f"[bench] n={ps.n} steps={args.steps} warmup={args.warmup}", file=sys.stderr, flush=True)
    if args.only_knn:
        print(json.dumps({"exact_k": run_knn(sph, torch, d, ps, max(3, args.steps // 2))}),
              flush=True)
        return
    if args.only_batched:
        print(json.dumps({"batched": run_batched(sph, torch, max(3, args.steps), args.warmup,
                                                 ev)}), flush=True)
        return
    if args.only_large:
        print(json.dumps({"large": run_large(sph, torch, 3, ev)}), flush=True)
        return
    if args.only_wendland:
        print(json.dumps({"wendland_c6": run_wendland(sph, torch, d, ps,
                                                      max(3, args.steps // 2), ev)}), flush=True)
        return
    f32 = run_form(sph, torch, d, ps, sph.FP32C, args.steps, args.warmup, ev)
    print(f"[bench] fp32c { {k: v for k, v in f32.items() if k[0] != '_'} }", file=sys.stderr,
          flush=True)
    f64 = None
    if not args.no_fp64:
        f64 = run_form(sph, torch, d, ps, sph.FP64, max(3, args.steps // 2), 1, ev)
        print(f"[bench] fp64 { {k: v for k, v in f64.items() if k[0] != '_'} }",
              file=sys.stderr, flush=True)

    srt = run_sort(sph, torch, d, ps, max(3, args.steps))
    print(f"[bench] sort {srt}", file=sys.stderr, flush=True)
    adj = None
    if not args.no_adjoint:
        adj = run_adjoint(sph, torch, d, ps, max(3, args.steps // 2), 1, ev)
        print(f"[bench] adjoint {adj}", file=sys.stderr, flush=True)

    bat = bat2 = None
    if not args.no_batched:
        bat = run_batched(sph, torch, max(3, args.steps), args.warmup, ev)
        print(f"[bench] batched {bat}", file=sys.stderr, flush=True)
        bat2 = run_batched(sph, torch, 3, 1, ev, "groups10k_a1554")
        print(f"[bench] batched_a1554 {bat2}", file=sys.stderr, flush=True)

    wc6 = None
    if not args.no_wendland:
        wc6 = run_wendland(sph, torch, d, ps, max(3, args.steps // 2), ev)
        print(f"[bench] wendland {wc6}", file=sys.stderr, flush=True)
    scat = None
    if not args.no_scatter:
        scat = run_scatter(sph, torch, d, ps, max(3, args.steps // 2))
        print(f"[bench] scatter {scat}", file=sys.stderr, flush=True)
    frc = None
    if not args.no_force:
        frc = run_force(sph, torch, d, ps, max(3, args.steps // 2))
        print(f"[bench] force {frc}", file=sys.stderr, flush=True)
    aos = None
    if not args.no_aos:
        aos = run_aos(sph, torch, d, ps, max(3, args.steps // 2))
        print(f"[bench] aos {aos}", file=sys.stderr, flush=True)
    knn = None
    if not args.no_knn:
        knn = run_knn(sph, torch, d, ps, max(3, args.steps // 2))
        print(f"[bench] knn {knn}", file=sys.stderr, flush=True)
    big = None
    if not args.no_large:
        big = run_large(sph, torch, 3, ev)
        print(f"[bench] large {big}", file=sys.stderr, flush=True)

    def roof(r, form):
        out = alu_roofline(r["cands"], r["pairs"], r["kernel_ms"], form, region=r["region"])
        out["traffic"] = measured_traffic() if form == "fp32c" else None
        out["kernel_ms_median"] = r["kernel_ms_median"]
        # counter-measured VALU work of the same launch (all 64 lanes of every
        # issued instruction, masked lanes included), at this run's kernel time
        out["executed"] = _executed(measured_valu("k_solve" if form == "fp32c" else "k_solve_fp64"),
                                    out["flop_per_launch"], r["kernel_ms"], form)
        return out

    value = f32["pairs"] / (f32["ms_per_step"] * 1e-3)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "clustered2^20: 2^20 particles, 200 Plummer spheres (a log-uniform "
                               "0.005-0.05, mass slope -2) + 30% uniform background, periodic "
                               "unit cube, equal masses, M4 spline, N_t = 64 +- 2, "
                               "h_init = 2 N^-1/3, sort + FP32-compensated solve per step",
                   "n": ps.n, "precision": "fp32c", "parallelism": "single-gpu"},
        "particles_per_s": ps.n / (f32["ms_per_step"] * 1e-3),
        "final_pairs_per_s": f32["final_pairs"] / (f32["ms_per_step"] * 1e-3),
        "pairs_per_step": f32["pairs"],
        "candidates_per_step": f32["cands"],
        "passes_per_step": f32["passes"],
        "roofline": roof(f32, "fp32c"),
    }
    if f64 is not None:
        line["fp64"] = {
            "value": f64["pairs"] / (f64["ms_per_step"] * 1e-3), "unit": "interactions/s",
            "ms_per_step": f64["ms_per_step"],
            "particles_per_s": ps.n / (f64["ms_per_step"] * 1e-3),
            "roofline": roof(f64, "fp64"),
        }
        line["fp32c_speedup_over_fp64"] = f64["ms_per_step"] / f32["ms_per_step"]
        # per-particle error of the FP32C form; the FP64 path is the oracle's to 1e-12
        drho = np.abs(f32["_rho"] - f64["_rho"]) / f64["_rho"]
        dh = np.abs(f32["_h"] - f64["_h"]) / f64["_h"]
        line["fp32c_error_vs_fp64"] = {
            "rho_rel_max": float(drho.max()), "rho_rel_p99": float(np.quantile(drho, 0.99)),
            "h_rel_max": float(dh.max()), "h_rel_p99": float(np.quantile(dh, 0.99)),
            "frac_h_rel_le_1e-5": float((dh <= 1e-5).mean()),
            # particles whose iteration stopped at another h inside the band
            "band_flips": int((dh > 1e-5).sum())}
    line["sort"] = srt
    if bat is not None:
        line["batched"] = bat
    if bat2 is not None:
        line["batched_a1554"] = bat2
    if big is not None:
        line["large"] = big
    if wc6 is not None:
        line["wendland_c6"] = wc6
    if knn is not None:
        line["exact_k"] = knn
    if aos is not None:
        line["aos"] = aos
    if scat is not None:
        line["scatter"] = scat
    if frc is not None:
        line["pressure_force"] = frc
    if adj is not None:
        line["adjoint"] = adj
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
