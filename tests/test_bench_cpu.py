"""Host-side logic of bench.py: the one-GPU guard and the rule that committed
HBM counter figures are used only for the kernel source they were taken on."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_before_any_device_work():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""


@pytest.fixture
def bench_module(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic_%s_%s_%s.json"))
    return bench, tmp_path


def _write(tmp_path, sha, nodes, bpd):
    with open(tmp_path / "traffic_fused_fp32_config2.json", "w") as fh:
        json.dump({"kernel_source_sha256": sha, "nodes": nodes, "bytes_per_dispatch": bpd}, fh)


def test_traffic_is_used_for_the_current_kernel_source(bench_module):
    bench, tmp = bench_module
    sha = hashlib.sha256(open(bench.KERNEL_SRC, "rb").read()).hexdigest()
    _write(tmp, sha, 2621440, 1.9e8)
    assert bench.traffic_from_profile(2621440, "fused", "config2") == pytest.approx(1.9e8)


@pytest.mark.parametrize("sha_ok,nodes", [(False, 2621440), (True, 2621441)])
def test_traffic_is_null_for_another_source_or_size(bench_module, sha_ok, nodes):
    bench, tmp = bench_module
    sha = hashlib.sha256(open(bench.KERNEL_SRC, "rb").read()).hexdigest()
    _write(tmp, sha if sha_ok else "0" * 64, 2621440, 1.9e8)
    assert bench.traffic_from_profile(nodes, "fused", "config2") is None


def test_traffic_is_null_without_counter_runs(bench_module):
    bench, tmp = bench_module
    assert bench.traffic_from_profile(2621440, "fused", "config5") is None
    # counters of the FP32 kernel say nothing about another storage precision
    sha = hashlib.sha256(open(bench.KERNEL_SRC, "rb").read()).hexdigest()
    _write(tmp, sha, 2621440, 1.9e8)
    assert bench.traffic_from_profile(2621440, "fused", "config2", "bf16") is None


def test_committed_counter_summaries_name_a_kernel_source():
    for name in os.listdir(os.path.join(ROOT, "profiles")):
        if name.startswith("traffic_") and name.endswith(".json"):
            with open(os.path.join(ROOT, "profiles", name)) as fh:
                t = json.load(fh)
            assert len(t["kernel_source_sha256"]) == 64
            assert t["nodes"] > 0 and t["bytes_per_dispatch"] > 0


def test_launch_duration_of_each_schedule(bench_module):
    bench, _ = bench_module
    # fused: one launch per step, so the timed region over its launches
    assert bench.launch_ms(2, 0.5, 10000, 0.047) == pytest.approx(0.05)
    # two kernels per step: the per-dispatch events of the collide kernel
    assert bench.launch_ms(0, 0.5, 10000, 0.031) == 0.031


def test_run_log_has_one_flat_record_per_measured_leg(bench_module):
    bench, _ = bench_module
    out = {"steps": 20, "value": 7.5e4, "config": {"workload": "sweep", "precision": "fp32", "nodes_per_step": 10},
           "roofline": {"achieved": 5.4e3, "frac": 0.68, "cache_resident": True,
                        "hbm_resident": [{"workload": "grid", "mlups": 6.3e4, "frac": 0.57}]},
           "bf16_batched": {"value": 6.6e4, "steps": 20}, "fp64_plain": {"value": 1.1e4, "config": "one run"},
           "d3q19": {"workload": "drop", "fp32": {"mlups": 2.5e4}, "fp64": {"mlups": 1.3e4}},
           "mc": {"workload": "mix", "fp32": {"mlups": 3.0e4}},
           "accuracy": {"pass": True}, "cpu_baseline": {"value": 46.0, "cores": 16}}
    recs = bench.jsonl_records(out, "config2")
    legs = [(r["leg"], r.get("precision")) for r in recs]
    assert legs == [("headline", "fp32"), ("hbm_resident", "fp32"), ("bf16_batched", "bf16"),
                    ("fp64_plain", "fp64"), ("d3q19", "fp32"), ("d3q19", "fp64"), ("mc", "fp32"),
                    ("accuracy", None), ("cpu_baseline", "fp64")]
    assert [r.get("mlups") for r in recs[:7]] == [7.5e4, 6.3e4, 6.6e4, 1.1e4, 2.5e4, 1.3e4, 3.0e4]
    assert recs[0]["frac"] == 0.68 and recs[-1]["cores"] == 16
    assert all(r["workload_id"] == "config2" for r in recs)
    for r in recs:
        json.loads(json.dumps(r))


def test_extension_traffic_follows_its_own_kernel_source(bench_module):
    bench, tmp = bench_module
    src3 = os.path.join(ROOT, "paper_1306_6445_amd", "csrc", "lbm3d_kernels.hip")
    sha3 = hashlib.sha256(open(src3, "rb").read()).hexdigest()
    with open(tmp / "traffic_fused3_fp32_d3q19.json", "w") as fh:
        json.dump({"kernel_source_sha256": sha3, "nodes": 16777216, "bytes_per_dispatch": 2.7e9}, fh)
    assert bench.traffic_from_profile(16777216, "fused3", "d3q19", "fp32", src3) == pytest.approx(2.7e9)
    # the 2D kernel source (the default) does not match the 3D counters
    assert bench.traffic_from_profile(16777216, "fused3", "d3q19", "fp32") is None
