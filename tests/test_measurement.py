"""Host-side checks of the measurement plumbing (no GPU): bench.py's contract
on the GPU count and its counter-traffic lookup, and the arithmetic of the
rocprofv3 counter summary (FETCH_SIZE / WRITE_SIZE scaled by what the same
counters read for a copy kernel of known size)."""
import argparse
import hashlib
import importlib.util
import json
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SRC = os.path.join(ROOT, "paper_2312_03019_amd", "csrc", "qaoa_kernels.hip")


def _load(name, path):
    spec = importlib.util.spec_from_file_location(name, path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_counter_traffic_is_used_only_for_the_current_kernel(tmp_path):
    bench = _load("bench_under_test", os.path.join(ROOT, "bench.py"))
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    k = "k_fwd<float, 5, 13, 2, 2, 2, 0, 0, 1>"
    good = tmp_path / "good.md"
    good.write_text(f"text\n- traffic {k}: 1.5e+10\n- kernel_source_sha256: {sha}\n")
    t, src = bench.pmc_traffic(str(good), k)
    assert t == 1.5e10 and src.endswith("good.md")
    t, src = bench.pmc_traffic(str(good), "k_fwd<float, 5, 13, 3, 1, 0, 0, 0, 1>")
    assert t is None and "no counters" in src
    stale = tmp_path / "stale.md"
    stale.write_text(f"- traffic {k}: 1.5e+10\n- kernel_source_sha256: " + "0" * 64 + "\n")
    t, src = bench.pmc_traffic(str(stale), k)
    assert t is None and "changed" in src
    t, src = bench.pmc_traffic(str(tmp_path / "missing.md"), k)
    assert t is None


def _pmc_csv(path, counter, rows):
    with open(path, "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for d, name, v in rows:
            f.write(f'{d},"{name}",{counter},{v}\n')


def test_counter_summary_scales_by_the_copy_kernel(tmp_path, capsys):
    ps = _load("profile_summary_under_test", os.path.join(ROOT, "paper_2312_03019_amd", "profile_summary.py"))
    copy = "void qaoa::k_copy<4>(HIP_vector_type<float, 4u> const*, HIP_vector_type<float, 4u>*, long)"
    fwd = "void qaoa::k_fwd<float, 5, 13, 3, 1, 0, 0, 0, 1>(qaoa::PassDesc const*, int)"
    mrg = "void qaoa::k_fwd<float, 5, 13, 2, 2, 2, 0, 0, 1>(qaoa::PassDesc const*, int)"
    # the copy moves 1 MiB each way; FETCH_SIZE reports half the bytes read (split over two
    # rows of one dispatch), WRITE_SIZE all of the bytes written
    _pmc_csv(tmp_path / "f.csv", "FETCH_SIZE", [(1, copy, 300.0), (1, copy, 212.0), (2, fwd, 1000.0), (3, fwd, 1200.0),
                                                (4, mrg, 900.0)])
    _pmc_csv(tmp_path / "w.csv", "WRITE_SIZE", [(1, copy, 1024.0), (2, fwd, 1500.0), (3, fwd, 1700.0), (4, mrg, 2000.0)])
    a = argparse.Namespace(fetch=str(tmp_path / "f.csv"), write=str(tmp_path / "w.csv"), copy_bytes=float(1 << 20),
                           cmd="synthetic")
    ps.counters(a)
    out = capsys.readouterr().out
    fields = dict(re.findall(r"^- ([\w ,<>-]+): (\S+)$", out, re.M))
    assert float(fields["fetch_scale"]) == pytest.approx(2.0)
    assert float(fields["write_scale"]) == pytest.approx(1.0)
    # per kernel: mean over its dispatches, FETCH_SIZE x2 + WRITE_SIZE x1
    assert float(fields["traffic k_fwd<float, 5, 13, 3, 1, 0, 0, 0, 1>"]) == pytest.approx((1100.0 * 2 + 1600.0) * 1024)
    assert float(fields["traffic k_fwd<float, 5, 13, 2, 2, 2, 0, 0, 1>"]) == pytest.approx((900.0 * 2 + 2000.0) * 1024)
    assert fields["kernel_source_sha256"] == hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    # with launch sizes in the CSV, whole-pass and chunk launches of one kernel are kept apart
    with open(tmp_path / "f2.csv", "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Grid_Size,Workgroup_Size,Counter_Name,Counter_Value\n")
        f.write(f'1,"{copy}",262144,256,FETCH_SIZE,512.0\n2,"{mrg}",33554432,256,FETCH_SIZE,900.0\n'
                f'3,"{mrg}",524288,256,FETCH_SIZE,14.0\n')
    with open(tmp_path / "w2.csv", "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Grid_Size,Workgroup_Size,Counter_Name,Counter_Value\n")
        f.write(f'1,"{copy}",262144,256,WRITE_SIZE,1024.0\n2,"{mrg}",33554432,256,WRITE_SIZE,2000.0\n'
                f'3,"{mrg}",524288,256,WRITE_SIZE,31.0\n')
    ps.counters(argparse.Namespace(fetch=str(tmp_path / "f2.csv"), write=str(tmp_path / "w2.csv"),
                                   copy_bytes=float(1 << 20), cmd="synthetic"))
    out2 = capsys.readouterr().out
    f2 = dict(re.findall(r"^- ([\w ,<>-]+): (\S+)$", out2, re.M))
    assert float(f2["traffic k_fwd<float, 5, 13, 2, 2, 2, 0, 0, 1> x131072"]) == pytest.approx((900.0 * 2 + 2000.0) * 1024)
    assert float(f2["traffic k_fwd<float, 5, 13, 2, 2, 2, 0, 0, 1> x2048"]) == pytest.approx((14.0 * 2 + 31.0) * 1024)
    assert f2["traffic k_fwd<float, 5, 13, 2, 2, 2, 0, 0, 1>"] == f2["traffic k_fwd<float, 5, 13, 2, 2, 2, 0, 0, 1> x131072"]
    # bench reads the dominant kernel's figure from such a summary
    bench = _load("bench_under_test2", os.path.join(ROOT, "bench.py"))
    (tmp_path / "c.md").write_text(out)
    t, src = bench.pmc_traffic(str(tmp_path / "c.md"), "k_fwd<float, 5, 13, 2, 2, 2, 0, 0, 1>")
    assert t == pytest.approx((900.0 * 2 + 2000.0) * 1024, rel=1e-6)


def test_stats_summary_splits_launch_sizes(tmp_path, capsys):
    """Whole-pass and chunk launches of one kernel get separate averages, so the
    per-launch figure the benchmark reports can be found in the summary."""
    import paper_2312_03019_amd.profile_summary as ps
    mrg = "void qaoa::k_fwd<float, 5, 13, 2, 2, 2, 0, 0, 1>(qaoa::PassDesc const*, int, qaoa::LaunchMap)"
    with open(tmp_path / "b_kernel_stats.csv", "w") as f:
        f.write('"Name","Calls","TotalDurationNs","AverageNs","Percentage","MinNs","MaxNs"\n')
        f.write(f'"{mrg}",4,8300000,2075000,90.0,100000,4000000\n')
    with open(tmp_path / "b_kernel_trace.csv", "w") as f:
        f.write('"Kernel_Name","Grid_Size_X","Workgroup_Size_X","Start_Timestamp","End_Timestamp"\n')
        for start, dur, wgs in ((0, 4000000, 131072), (5000000, 4000000, 131072), (10000000, 100000, 2048),
                                (11000000, 200000, 2048)):
            f.write(f'"{mrg}",{wgs * 256},256,{start},{start + dur}\n')
    ps.stats(argparse.Namespace(dir=str(tmp_path), prefix="b", cmd="synthetic"))
    out = capsys.readouterr().out
    fields = dict(re.findall(r"^- (avg_ms [^:]+): (\S+)$", out, re.M))
    assert float(fields["avg_ms k_fwd<float, 5, 13, 2, 2, 2, 0, 0, 1> x131072"]) == pytest.approx(4.0)
    assert float(fields["avg_ms k_fwd<float, 5, 13, 2, 2, 2, 0, 0, 1> x2048"]) == pytest.approx(0.15)
    assert float(fields["avg_ms k_fwd<float, 5, 13, 2, 2, 2, 0, 0, 1>"]) == pytest.approx(2.075)
