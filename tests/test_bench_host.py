"""Host-side logic of bench.py: the kernel-source hash that keys the committed counter
summaries ignores comments and whitespace, and a summary taken on other code is not used."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_code_only_drops_comments_and_whitespace_but_keeps_strings():
    a = 'int a = 1; // note\n/* block\n comment */ const char *s = "x // y /* z */";\n'
    b = 'int a=1;const char*s="x // y /* z */";'
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only("int a = 1;") != bench._code_only("int a = 2;")


def _write_profiles(tmp_path, monkeypatch, entries, h="h"):
    prof = tmp_path / "profiles"
    prof.mkdir(exist_ok=True)
    (prof / "traffic.json").write_text(json.dumps(entries))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # the hash itself reads the sources under the real root
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)


def test_counter_figures_only_for_the_current_code_and_launch(tmp_path, monkeypatch):
    ok = {"kernel_hash": "h", "launch": [256, 12, 1], "bytes_per_launch": 1.0e6}
    stale = {"kernel_hash": "0" * 16, "launch": [256, 12, 1], "bytes_per_launch": 2.0e6}
    _write_profiles(tmp_path, monkeypatch, {"c2:fp64": ok, "c2:mixed": stale})
    launch = (256, 12, 60, 1)   # tile, blocks per CU, graph steps, CFL sub-slots
    assert bench.counter_figures("c2", "fp64", 2 ** 20, 0.03, launch)["traffic"] == 1.0e6
    assert bench.counter_figures("c2", "mixed", 2 ** 20, 0.03, launch)["traffic"] is None
    assert bench.counter_figures("c3", "fp64", 2 ** 20, 0.03, launch)["traffic"] is None
    # taken at another launch: not used
    other = (256, 24, 60, 1)
    assert bench.counter_figures("c2", "fp64", 2 ** 20, 0.03, other)["traffic"] is None


def test_valu_issue_share_from_the_counter_summary(tmp_path, monkeypatch):
    ent = {"kernel_hash": "h", "valu_insts_per_edge": 640.0}
    _write_profiles(tmp_path, monkeypatch, {"c2:fp64": ent})
    # 640 instructions per edge, 2^20 edges: 2^14 waves x 640 x 4 cycles / 1024 SIMDs / 2.4 GHz
    busy = 2 ** 14 * 640 * 4 / 1024 / 2.4e9
    v = bench.counter_figures("c2", "fp64", 2 ** 20, busy * 2 * 1e3, None)["valu_issue"]
    assert v["insts_per_edge"] == 640.0 and abs(v["frac"] - 0.5) < 1e-12
    assert "active_frac" not in v
    assert bench.counter_figures("c3", "fp64", 2 ** 20, 1.0, None)["valu_issue"] is None
    # with the VALU-active counter: 704 four-cycle units per edge is 1.1 times the issue time
    ent["valu_active_per_edge"] = 704.0
    _write_profiles(tmp_path, monkeypatch, {"c2:fp64": ent})
    v = bench.counter_figures("c2", "fp64", 2 ** 20, busy * 2 * 1e3, None)["valu_issue"]
    assert abs(v["active_frac"] - 0.55) < 1e-12 and v["active_per_edge"] == 704.0


def test_counter_flop_rate_and_fraction(tmp_path, monkeypatch):
    ent = {"kernel_hash": "h", "flops_f64": 7.0e11, "flops_f32": 0.86e11}
    _write_profiles(tmp_path, monkeypatch, {"c5:fp64": ent, "c5:mixed": ent})
    cf = bench.counter_figures("c5", "fp64", 10 ** 8, 10.0, None)["counter_flops"]
    assert abs(cf["tflops"] - 78.6) < 1e-9 and abs(cf["frac"] - 1.0) < 1e-12
    assert abs(cf["per_edge_update"] - 7860.0) < 1e-9
    # the mixed form against the rate non-packed FP32 can issue (the FP64 rate)
    cm = bench.counter_figures("c5", "mixed", 10 ** 8, 20.0, None)["counter_flops"]
    assert cm["peak"] == 78.6 and abs(cm["frac"] - 0.5) < 1e-12


def test_valu_flops_counts_an_fma_twice():
    from paper_1912_04791_amd import profsum
    c = {"SQ_INSTS_VALU_ADD_F64": [1.0], "SQ_INSTS_VALU_MUL_F64": [2.0],
         "SQ_INSTS_VALU_FMA_F64": [3.0, 3.0, 5.0], "SQ_INSTS_VALU_TRANS_F64": [4.0],
         "SQ_INSTS_VALU_FMA_F32": [10.0]}
    f64, f32 = profsum.valu_flops(c)
    assert f64 == 64.0 * (1 + 2 + 2 * 3 + 4) and f32 == 64.0 * 20


def test_trace_runs_match_the_logged_runs(tmp_path):
    from paper_1912_04791_amd import profsum
    hdr = "Kind,Dispatch_Id,Kernel_Name,Start_Timestamp,End_Timestamp"
    rows, t, d = [], 0, 0

    def disp(name, dur):
        nonlocal t, d
        d += 1
        rows.append(f'KERNEL_DISPATCH,{d},"{name}",{t},{t + dur}')
        t += dur + 5

    s64, s32 = "dsve::k_step<3, 0, 0, false>(a)", "dsve::k_step<3, 1, 0, false>(a)"
    for name, n, dur in ((s64, 2, 100), (s64, 3, 90), (s32, 2, 70), (s32, 3, 60), (s64, 4, 95)):
        disp("dsve::k_fill_u64(x)", 1)
        disp("dsve::k_cfl<0, 0>(a)", 10)
        for _ in range(n):
            disp(name, dur)
    disp("dsve::k_cfl<0, 0>(a)", 10)   # a cfl_reduce call: no step kernels, no run
    (tmp_path / "run_kernel_trace.csv").write_text("\n".join([hdr] + rows) + "\n")
    log = tmp_path / "bench.err"
    log.write_text("\n".join([
        "[run] workload=c5 precision=fp64 solver=adot steps=2 kind=warmup",
        "[run] workload=c5 precision=fp64 solver=adot steps=3 kind=timed",
        "[bench] c5 fp64: ...",
        "[run] workload=c5 precision=mixed solver=adot steps=2 kind=warmup",
        "[run] workload=c5 precision=mixed solver=adot steps=3 kind=timed",
        "[run] workload=c5 precision=fp64 solver=adot steps=4 kind=full"]) + "\n")
    pairs = profsum.match_runs(profsum.read_runs(str(log)), profsum.trace_runs(str(tmp_path)))
    timed64 = [tr for lg, tr in pairs if lg["kind"] == "timed" and lg["precision"] == "fp64"]
    assert len(timed64) == 1 and timed64[0][1] == [90, 90, 90]
    st = profsum.dispatch_stats(timed64[0][1])
    assert st["n"] == 3 and abs(st["mean_us"] - 0.09) < 1e-12
    full = [tr for lg, tr in pairs if lg["kind"] == "full"]
    assert full[0][1] == [95] * 4
    # a missing log line is an error, not a silent mismatch
    import pytest
    with pytest.raises(ValueError):
        profsum.match_runs(profsum.read_runs(str(log))[1:], profsum.trace_runs(str(tmp_path)))


def test_host_cpu_threads_follow_the_cpu_share(monkeypatch):
    monkeypatch.setenv("OMP_NUM_THREADS", "3")
    c = bench.host_cpu()
    assert c["threads"] == min(3, c["affinity"]) and c["nproc"] >= c["affinity"] >= 1
    monkeypatch.delenv("OMP_NUM_THREADS")
    assert bench.host_cpu()["threads"] == bench.host_cpu()["affinity"]


def test_profile_calibration_is_the_first_copy(tmp_path):
    # a run whose later copies (the state copied back after an odd step count) are larger
    # than the calibration copy: the scale comes from the first copy dispatch
    from paper_1912_04791_amd import profsum
    hdr = ('"Correlation_Id","Dispatch_Id","Agent_Id","Queue_Id","Process_Id","Thread_Id",'
           '"Grid_Size","Kernel_Id","Kernel_Name","Workgroup_Size","LDS_Block_Size",'
           '"Scratch_Size","VGPR_Count","Accum_VGPR_Count","SGPR_Count","Counter_Name",'
           '"Counter_Value","Start_Timestamp","End_Timestamp"')
    def row(d, name, v):
        return f'{d},{d},"Agent 1",1,1,1,131072,1,"{name}",512,0,0,4,0,32,"FETCH_SIZE",{v},0,1'
    lines = [hdr, row(1, "fill_kernel", 17.0), row(2, "__amd_rocclr_copyBuffer", 131092.0),
             row(7, "dsve::k_step<3, 0, 0, false>", 500.0),
             row(9, "__amd_rocclr_copyBuffer", 590570.0),
             row(8, "dsve::k_step<3, 0, 0, false>", 520.0)]
    (tmp_path / "run_counter_collection.csv").write_text("\n".join(lines) + "\n")
    out, first = profsum.counters(str(tmp_path), "k_step<3, 0, 0, false>")
    assert first["FETCH_SIZE"] == 131092.0
    assert sorted(out["FETCH_SIZE"]) == [500.0, 520.0]


def test_effective_clock_from_busy_cycles_and_the_trace(tmp_path):
    # GRBM_GUI_ACTIVE counts busy cycles summed over the 8 XCDs: 8 x 2.0e9 x 1 ms of a 1 ms
    # dispatch is a 2.0 GHz clock; the trace's dispatch ids pair the two files
    from paper_1912_04791_amd import profsum
    hdr = ('"Correlation_Id","Dispatch_Id","Agent_Id","Queue_Id","Process_Id","Thread_Id",'
           '"Grid_Size","Kernel_Id","Kernel_Name","Workgroup_Size","LDS_Block_Size",'
           '"Scratch_Size","VGPR_Count","Accum_VGPR_Count","SGPR_Count","Counter_Name",'
           '"Counter_Value","Start_Timestamp","End_Timestamp"')
    k = "dsve::k_step<3, 0, 0, false>"
    rows = [hdr, f'5,5,"Agent 1",1,1,1,1,1,"{k}",256,0,0,4,0,32,"GRBM_GUI_ACTIVE",{8 * 2.0e9 * 1e-3},0,1',
            f'5,5,"Agent 1",1,1,1,1,1,"{k}",256,0,0,4,0,32,"SQ_ACTIVE_INST_VALU",{0.5 * 1024 * 2.0e6 / 4},0,1',
            f'6,6,"Agent 1",1,1,1,1,1,"{k}",256,0,0,4,0,32,"GRBM_GUI_ACTIVE",{8 * 1.9e9 * 2e-3},0,1']
    (tmp_path / "run_counter_collection.csv").write_text("\n".join(rows) + "\n")
    thdr = '"Kind","Agent_Id","Queue_Id","Kernel_Id","Kernel_Name","Correlation_Id","Dispatch_Id","Start_Timestamp","End_Timestamp"'
    trows = [thdr, f'"KERNEL_DISPATCH",1,1,1,"{k}",5,5,1000000,2000000',
             f'"KERNEL_DISPATCH",1,1,1,"{k}",6,6,3000000,5000000',
             f'"KERNEL_DISPATCH",1,1,1,"other",7,7,6000000,7000000']
    (tmp_path / "run_kernel_trace.csv").write_text("\n".join(trows) + "\n")
    got = profsum.clock_per_dispatch(str(tmp_path), "k_step<3, 0, 0, false>")
    assert [round(c / 1e9, 6) for _, c, _ in got] == [2.0, 1.9]
    d, f, c = got[0]
    assert abs(c["SQ_ACTIVE_INST_VALU"] * 4 / (1024 * d * f) - 0.5) < 1e-12


def test_more_than_one_gpu_is_refused_with_a_message():
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stderr and out.stdout == ""


def test_alu_roofline_peaks():
    fp64 = bench.alu_roofline("fp64", 20.0)
    assert fp64["peak"] == 78.6 and abs(fp64["frac"] - 20.0 / 78.6) < 1e-12
    mixed = bench.alu_roofline("mixed", 30.0)
    assert mixed["peak"] == 157.3 and abs(mixed["frac"] - 30.0 / 157.3) < 1e-12
    assert mixed["peak_nonpacked"] == 78.6 and abs(mixed["frac_nonpacked"] - 30.0 / 78.6) < 1e-12


def test_profile_timing_note_wording():
    from paper_1912_04791_amd import profsum
    assert "below it" in profsum.timing_note(3500.0, 3400.0)
    assert "above it" in profsum.timing_note(27.0, 29.0)


def test_relative_l1_floor_in_the_units_of_each_variable():
    # bench.py and the tests measure parity the same way: per variable, relative to the
    # reference's L1 norm or, where that is smaller, to a thousandth of the variable's natural
    # size in its own units (the depth for h and z, the critical discharge h sqrt(g h) for q)
    import numpy as np
    sys.path.insert(0, os.path.dirname(__file__))
    from common import max_rel_l1
    rng = np.random.default_rng(3)
    h = rng.uniform(0.5, 3.0, 500)
    ref = (h, 1e-7 * rng.standard_normal(500), rng.uniform(-0.2, 0.2, 500))
    got = tuple(r + 1e-9 * rng.standard_normal(500) for r in ref)
    assert bench.rel_l1_max(got, ref) == max_rel_l1(got, ref)
    # q is near zero everywhere: its floor is 1e-3 * sum(h sqrt(g h)), not its own norm
    eq = np.abs(got[1] - ref[1]).sum() / (1e-3 * (h * np.sqrt(9.81 * h)).sum())
    eh = np.abs(got[0] - ref[0]).sum() / np.abs(ref[0]).sum()
    ez = np.abs(got[2] - ref[2]).sum() / max(np.abs(ref[2]).sum(), 1e-3 * h.sum())
    assert bench.rel_l1_max(got, ref) == max(eh, eq, ez)
