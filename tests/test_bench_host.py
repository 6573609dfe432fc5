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


def test_traffic_is_used_only_for_the_current_code(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    ok = {"kernel_hash": bench.kernel_source_hash(), "bytes_per_launch": 1.0e6}
    stale = {"kernel_hash": "0" * 16, "bytes_per_launch": 2.0e6}
    (prof / "traffic.json").write_text(json.dumps({"c2:fp64": ok, "c2:mixed": stale}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # the hash itself reads the sources under the real root
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: ok["kernel_hash"])
    assert bench.measured_traffic("c2", "fp64") == 1.0e6
    assert bench.measured_traffic("c2", "mixed") is None
    assert bench.measured_traffic("c3", "fp64") is None


def test_valu_issue_share_from_the_counter_summary(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    ent = {"kernel_hash": "h", "valu_insts_per_edge": 640.0}
    (prof / "traffic.json").write_text(json.dumps({"c2:fp64": ent}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "h")
    # 640 instructions per edge, 2^20 edges: 2^14 waves x 640 x 4 cycles / 1024 SIMDs / 2.4 GHz
    busy = 2 ** 14 * 640 * 4 / 1024 / 2.4e9
    v = bench.valu_issue("c2", "fp64", 2 ** 20, busy * 2 * 1e3)
    assert v["insts_per_edge"] == 640.0 and abs(v["frac"] - 0.5) < 1e-12
    assert "active_frac" not in v
    assert bench.valu_issue("c3", "fp64", 2 ** 20, 1.0) is None
    # with the VALU-active counter: 704 four-cycle units per edge is 1.1 times the issue time
    ent["valu_active_per_edge"] = 704.0
    (prof / "traffic.json").write_text(json.dumps({"c2:fp64": ent}))
    v = bench.valu_issue("c2", "fp64", 2 ** 20, busy * 2 * 1e3)
    assert abs(v["active_frac"] - 0.55) < 1e-12 and v["active_per_edge"] == 704.0


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
    assert "is higher" in profsum.timing_note("26.5-28.5", 33.4)
    assert "agrees with it within 2%" in profsum.timing_note("398", 399.5)
    assert "agrees with it within 2%" in profsum.timing_note("415", 412.4)
