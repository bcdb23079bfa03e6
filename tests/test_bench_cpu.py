"""The benchmark's contract on the CPU: one GPU only, the traffic figure read
from the committed profile only while the kernel sources match it, and the
same kernel identity for the tuning cache and the profile."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_traffic_is_read_only_for_matching_kernel_sources(tmp_path, monkeypatch):
    b = load_bench()
    h = b.kernel_source_hash()
    prof = tmp_path / "profiles"
    prof.mkdir()
    body = ("# summary\n\n- shoot kernel sources sha256: `{}`\n- binning mode: 1\n"
            "- fetch bytes per launch: 1.5e+06\n- write bytes per launch: 2.5e+09\n"
            "- executed FP32 flops per evaluation: 8.8\n")
    (prof / "traffic_shoot_fp32c_w.md").write_text(body.format(h))
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    monkeypatch.setattr(b, "kernel_source_hash", lambda: h)
    t = b.measured_traffic("w")
    assert t["bytes"] == 1.5e6 + 2.5e9 and t["executed_flops_per_eval"] == 8.8
    (prof / "traffic_shoot_fp32c_w.md").write_text(body.format("0" * 64))
    assert b.measured_traffic("w") is None
    assert b.measured_traffic("absent") is None


def test_profile_and_tuning_cache_name_the_same_kernel_build():
    b = load_bench()
    spec = importlib.util.spec_from_file_location("rl_build", os.path.join(ROOT, "paper_1406_0559_amd",
                                                                           "build.py"))
    bld = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bld)
    assert b.kernel_source_hash().startswith(bld.kernel_id())
