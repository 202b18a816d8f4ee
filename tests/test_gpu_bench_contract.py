"""bench.py's output contract on a short run (needs an MI355X): one JSON line
with the required keys, the roofline and CPU-baseline objects, and values of
the right kinds.  Runs bench.py as a child process."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_prints_one_json_line_with_the_required_fields(tmp_path):
    log = str(tmp_path / "run.jsonl")
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "400", "--warmup", "40",
                        "--accuracy-steps", "0", "--cpu-seconds", "2", "--timing-steps", "20", "--jsonl", log],
                       capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert p.returncode == 0, p.stderr[-2000:]
    lines = [l for l in p.stdout.splitlines() if l.strip()]
    assert len(lines) == 1, p.stdout[-2000:]
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 400 and d["warmup"] == 40
    assert d["unit"] == "MLUPS" and d["value"] > 0 and d["higher_is_better"] is True
    assert d["dtype"] == "f32" and d["data"] == "synthetic" and "workload" in d["config"]
    r = d["roofline"]
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["achieved"] > 0 and r["frac"] == pytest.approx(r["achieved"] / r["peak"])
    assert r["traffic"] is None or r["traffic"] > 0
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and c["value"] > 0 and c["cores"] >= 1 and c["sample"]
    assert d["ms_per_step"] == pytest.approx(1e3 * d["config"]["nodes_per_step"] / (d["value"] * 1e6), rel=1e-6)
    # the default workload is cache-resident: the HBM-resident legs stand beside it
    assert r["cache_resident"] is True and r["working_set_bytes"] > 0
    legs = r["hbm_resident"]
    assert len(legs) == 2 and all(0 < l["frac"] < 1 and l["cache_resident"] is False for l in legs)
    # extension legs, FP32 and FP64
    for ext in ("d3q19", "mc"):
        for prec in ("fp32", "fp64"):
            leg = d[ext][prec]
            assert leg["mlups"] > 0 and 0 < leg["frac"] < 1, (ext, prec)
    # the run log: one record per measured leg, the headline first
    recs = [json.loads(l) for l in open(log)]
    assert recs[0]["leg"] == "headline" and recs[0]["mlups"] == pytest.approx(d["value"])
    assert {"hbm_resident", "d3q19", "mc", "cpu_baseline"} <= {x["leg"] for x in recs}
