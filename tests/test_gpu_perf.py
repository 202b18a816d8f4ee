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


def test_extension_kernels_throughput():
    """The extensions in their default launch shapes: the 256^3 D3Q19 drop
    (measured about 26k MLUPS FP32 fused, 21k two-pass) and the 2048^2
    two-component mixture (about 31k FP32, 16k FP64)."""
    run3 = WL.config3d(256)
    with lbm.Lattice3(run3, precision="fp32") as L:
        L.init_all()
        fused = _mlups(L, run3.nodes, 40)
        L.set_schedule(0, 64, 8, 64)
        two = _mlups(L, run3.nodes, 40)
    runm = WL.mc_spinodal_run(2048)
    mc = {}
    for prec in ("fp32", "fp64"):
        with lbm.LatticeMC(runm, precision=prec) as L:
            L.init_all()
            mc[prec] = _mlups(L, runm.nodes, 200)
    print("  d3q19 fused %.0f, two-pass %.0f; mc fp32 %.0f, fp64 %.0f MLUPS" % (fused, two, mc["fp32"], mc["fp64"]),
          file=sys.stderr, flush=True)
    assert fused > 19000 and two > 16000 and fused > two
    assert mc["fp32"] > 23000 and mc["fp64"] > 12000
