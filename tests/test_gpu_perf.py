"""Throughput regression guard on the benchmark's default workload (needs an
MI355X): the 40 x 256^2 FP32 droplet batch in its launch shape.  The bounds
sit well below the measured figures (about 79k MLUPS fused, 52k with two
kernels per step), so only a real regression trips them."""
import sys
import time

import pytest
import torch

from paper_1306_6445_amd import lbm, workloads as WL

pytestmark = pytest.mark.gpu


def _mlups(L, nodes, k):
    L.step(64)
    L.synchronize()
    torch.cuda.synchronize()
    best = 0.0
    for _ in range(3):
        t0 = time.perf_counter()
        L.step(k)
        L.synchronize()
        torch.cuda.synchronize()
        best = max(best, nodes * k / (time.perf_counter() - t0) / 1e6)
    return best


def test_fp32_batch_throughput_and_fused_gain():
    runs = WL.config2()
    nodes = sum(r.nodes for r in runs)
    with lbm.Lattice(runs, precision="fp32", tile=(64, 4), fused=2) as L:
        L.init_all()
        fused = _mlups(L, nodes, 2000)
        L.set_fused(0)
        two = _mlups(L, nodes, 2000)
        assert not L.status().any()
    print("  fused %.0f MLUPS, two kernels %.0f MLUPS" % (fused, two), file=sys.stderr, flush=True)
    assert fused > 55000
    assert fused > 1.25 * two
