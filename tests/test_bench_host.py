"""Host logic of the benchmark's counter summaries, on synthetic rocprofv3
counter-collection files: per-dispatch sums over counter instances, the
FLOP weights of the SQ instruction counters (64 lanes, FMA = 2), the copy
calibration of FETCH_SIZE / WRITE_SIZE, and that a summary taken on another
kernel source is ignored.
"""
import csv
import json

import pytest

import bench

HDR = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
       "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
       "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
       "Counter_Value", "Start_Timestamp", "End_Timestamp"]
SOLVE = "void sph::k_solve<1, false, 16, 0, 0, 64>(sph::SolveArgs)"


def _csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HDR)
        for disp, name, counter, value in rows:
            w.writerow([disp, disp, "Agent 1", 1, 1, 1, 64, 1, name, 64, 0, 0, 1, 0, 1, counter,
                        value, 0, 0])
    return str(path)


def test_valu_summary(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "VALU_JSON", str(tmp_path / "valu.txt"))
    other = "void sph::k_keys_periodic<double>(long)"
    rows_a, rows_b = [], []
    for disp, scale in ((3, 1.0), (7, 3.0)):       # two launches: the summary averages
        rows_a.append((disp - 1, other, "SQ_INSTS_VALU_FMA_F32", 1e9))   # not k_solve
        for c, v in (("SQ_INSTS_VALU_ADD_F32", 10), ("SQ_INSTS_VALU_MUL_F32", 20),
                     ("SQ_INSTS_VALU_FMA_F32", 30), ("SQ_INSTS_VALU_TRANS_F32", 5)):
            # two instances (e.g. shader engines) per dispatch: summed
            rows_a += [(disp, SOLVE, c, 0.25 * v * scale), (disp, SOLVE, c, 0.75 * v * scale)]
        for c, v in (("SQ_INSTS_VALU_FMA_F64", 7), ("SQ_THREAD_CYCLES_VALU", 3200),
                     ("SQ_ACTIVE_INST_VALU", 100)):
            rows_b.append((disp, SOLVE, c, v * scale))
    a = _csv(tmp_path / "a.csv", rows_a)
    b = _csv(tmp_path / "b.csv", rows_b)
    bench.summarize_valu("cmd", a, b)
    d = json.load(open(bench.VALU_JSON))
    assert d["executed_f32_flop_per_launch"] == pytest.approx(64 * (10 + 20 + 2 * 30 + 5) * 2.0)
    assert d["executed_f64_flop_per_launch"] == pytest.approx(64 * 2 * 7 * 2.0)
    assert d["thread_cycles_per_valu_cycle_raw"] == pytest.approx(32.0)
    assert d["dispatches"]["SQ_INSTS_VALU_FMA_F32"] == 2
    assert bench.measured_valu()["executed_f32_flop_per_launch"] == \
        d["executed_f32_flop_per_launch"]
    # lane utilisation: 3200 thread-cycles per 100 active VALU cycles = 32 of 64 lanes
    ex = bench._executed(bench.measured_valu(), 1.0, 1.0)
    assert ex["valu_lane_utilisation"] == pytest.approx(0.5)
    d["solve_hip_sha256"] = "0" * 64
    json.dump(d, open(bench.VALU_JSON, "w"))
    assert bench.measured_valu() is None


def test_sort_traffic_summary(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "SORT_TRAFFIC_JSON", str(tmp_path / "sort.txt"))
    copy = "__amd_rocclr_copyBuffer"
    nbytes = float(bench.COPY_MIB << 20)

    def rows(counter, factor, per_call):
        out, disp = [], 0
        for _ in range(2):                           # two calls: per-call figures halve
            for name, v in per_call:
                disp += 1
                out.append((disp, name, counter, v * factor / 1024.0))
        out.append((disp + 1, "void at::native::fill_kernel(int)", counter, 1.0))
        out.append((disp + 2, copy, counter, nbytes * factor / 1024.0))
        return out

    keys = "void sph::k_keys_periodic<double>(long, void const*)"
    up = "void sph::k_radix_up<16>(long, unsigned long const*)"
    n = 1 << 24
    f = _csv(tmp_path / "f.csv", rows("FETCH_SIZE", 0.5, [(keys, 24.0 * n), (up, 8.0 * n),
                                                         (up, 8.0 * n)]))
    w = _csv(tmp_path / "w.csv", rows("WRITE_SIZE", 1.0, [(keys, 12.0 * n), (up, 1.0 * n)]))
    bench.summarize_sort_traffic(f, w, "cmd", "2")
    d = json.load(open(bench.SORT_TRAFFIC_JSON))
    pk = d["per_kernel_bytes_per_call"]
    assert pk["k_keys_periodic<double>"]["fetch"] == pytest.approx(24.0 * n)
    assert pk["k_keys_periodic<double>"]["write"] == pytest.approx(12.0 * n)
    assert pk["k_radix_up<16>"]["fetch"] == pytest.approx(16.0 * n)
    assert d["bytes_per_particle"] == pytest.approx(24 + 12 + 16 + 1)
    assert d["copy_calibration"]["fetch_factor"] == pytest.approx(0.5)
    assert bench.measured_sort_traffic() == pytest.approx(d["bytes_per_call"])
    d["sort_hip_sha256"] = "0" * 64
    json.dump(d, open(bench.SORT_TRAFFIC_JSON, "w"))
    assert bench.measured_sort_traffic() is None


def test_solve_traffic_summary(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_JSON", str(tmp_path / "traffic.txt"))
    nbytes = float(bench.COPY_MIB << 20)
    f = _csv(tmp_path / "f.csv", [(1, SOLVE, "FETCH_SIZE", 1.15 * 4e8 / 1024),
                                  (2, SOLVE, "FETCH_SIZE", 1.15 * 6e8 / 1024),
                                  (3, "__amd_rocclr_copyBuffer", "FETCH_SIZE",
                                   1.15 * nbytes / 1024)])
    w = _csv(tmp_path / "w.csv", [(1, SOLVE, "WRITE_SIZE", 1e8 / 1024),
                                  (2, SOLVE, "WRITE_SIZE", 1e8 / 1024),
                                  (3, "__amd_rocclr_copyBuffer", "WRITE_SIZE", nbytes / 1024)])
    bench.summarize_traffic(f, w, "cmd")
    assert bench.measured_traffic() == pytest.approx(5e8 + 1e8)


def test_valu_summary_per_call(tmp_path, monkeypatch):
    # the adjoint: two dispatches per call, totals reported per call
    path = str(tmp_path / "adj.txt")
    _, src, unit = bench.VALU_TARGETS["k_adjoint"]
    monkeypatch.setitem(bench.VALU_TARGETS, "k_adjoint", (path, src, unit))
    adj = "void sph::k_adjoint<1, false, 0>(sph::AdjArgs)"
    rows = [(d, adj, "SQ_INSTS_VALU_FMA_F32", 10.0 * d) for d in (1, 2, 3, 4)]
    a = _csv(tmp_path / "a.csv", rows + [(5, SOLVE, "SQ_INSTS_VALU_FMA_F32", 1e6)])
    bench.summarize_valu("cmd", a, kernel="k_adjoint", calls=2)
    d = json.load(open(path))
    assert d["executed_f32_flop_per_launch"] == pytest.approx(64 * 2 * 100.0 / 2)
    assert bench.measured_valu("k_adjoint")["executed_f32_flop_per_launch"] == \
        d["executed_f32_flop_per_launch"]
    ex = bench._executed(d, 1600.0, 2.0)
    assert ex["algorithmic_over_executed"] == pytest.approx(0.25)
    assert "valu_lane_utilisation" not in ex    # no thread-cycle counters in this summary


def test_alu_roofline_weights():
    # headline: 8 FLOP per candidate test, 31 (FP32C) / 22 (FP64) per in-range
    # pair; the kernel's own count (17 per pair) beside it
    r = bench.alu_roofline(1e10, 4e9, 10.0, "fp32c")
    assert r["flop_per_launch"] == pytest.approx(8e10 + 31 * 4e9)
    assert r["frac"] == pytest.approx((8e10 + 31 * 4e9) / 1e-2 / 157.3e12)
    assert r["kernel_counted"]["flop_per_launch"] == pytest.approx(8e10 + 17 * 4e9)
    r = bench.alu_roofline(1e10, 4e9, 10.0, "fp64")
    assert r["flop_per_launch"] == pytest.approx(8e10 + 22 * 4e9)
    assert r["peak"] == pytest.approx(78.6)


def test_valu_summary_fp64(tmp_path, monkeypatch):
    # the FP64 solve: binary64 FLOP against the binary64 peak, binary32 beside it
    path = str(tmp_path / "fp64.txt")
    _, src, unit = bench.VALU_TARGETS["k_solve_fp64"]
    monkeypatch.setitem(bench.VALU_TARGETS, "k_solve_fp64", (path, src, unit))
    rows = [(1, SOLVE, "SQ_INSTS_VALU_FMA_F64", 100.0), (1, SOLVE, "SQ_INSTS_VALU_ADD_F64", 50.0),
            (1, SOLVE, "SQ_INSTS_VALU_ADD_F32", 20.0)]
    a = _csv(tmp_path / "a.csv", rows)
    bench.summarize_valu("cmd", a, kernel="k_solve_fp64")
    d = json.load(open(path))
    assert d["kernel"].startswith("k_solve (FP64")
    assert d["executed_f64_flop_per_launch"] == pytest.approx(64 * (2 * 100 + 50))
    ex = bench._executed(bench.measured_valu("k_solve_fp64"), 1.0, 1.0, "fp64")
    assert ex["flop_per_launch"] == pytest.approx(64 * 250)
    assert ex["frac"] == pytest.approx(64 * 250 / 1e-3 / bench.PEAK_FP64)
    assert ex["f32_flop_per_launch"] == pytest.approx(64 * 20)
