"""The FP32 and bf16-storage step kernels run no binary64 arithmetic (CPU only).

The step's arithmetic is FP32 in those precisions: the density is a
compensated FP32 sum, the EOS, force, source term and collision are FP32, and
FP64 is reserved for the diagnostics reductions and the host.  This test
compiles the kernel sources for gfx950 to assembly with the library's own
flags and checks that no vector instruction of any FP32 or bf16 step kernel
(fused, psi and collide, 2D and 3D, every template instance) operates on f64,
while the FP64 instances do (so the check itself sees such instructions).
"""
import os
import re
import subprocess

import pytest

from paper_1306_6445_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1306_6445_amd", "csrc")


def kernels_asm(src, out):
    flags = [f for f in B.FLAGS if f not in ("-shared", "-fPIC")]
    subprocess.run([B.HIPCC] + flags + ["-I", CSRC, "--cuda-device-only", "-S", "-o", out, src],
                   check=True, capture_output=True, text=True, timeout=900)
    lines = open(out).read().splitlines()
    bodies = {}
    name = None
    for line in lines:
        m = re.match(r"^(_Z\S+):", line)
        if m:
            name, bodies[m.group(1)] = m.group(1), []
        elif name is not None:
            if "s_endpgm" in line:
                name = None
            elif line.startswith("\t") and line.strip().startswith("v_"):
                bodies[name].append(line.strip().split()[0])
    return bodies


STEP = re.compile(r"(fused3?_kernel|collide3?_kernel|psi3?_kernel)I(f|NS_6bf16_tE|d)")


@pytest.mark.skipif(not os.path.exists(B.HIPCC), reason="hipcc not installed")
@pytest.mark.parametrize("src", ["lbm_kernels.hip", "lbm3d_kernels.hip"])
def test_fp32_and_bf16_step_kernels_have_no_fp64_instructions(src, tmp_path):
    bodies = kernels_asm(os.path.join(CSRC, src), str(tmp_path / "k.s"))
    seen = {"f": 0, "NS_6bf16_tE": 0, "d": 0}
    f64_in_fp64 = 0
    for name, ops in bodies.items():
        m = STEP.search(name)
        if not m:
            continue
        seen[m.group(2)] += 1
        f64 = [op for op in ops if "_f64" in op]
        if m.group(2) == "d":
            f64_in_fp64 += len(f64)
        else:
            assert not f64, (name, sorted(set(f64)))
    assert seen["f"] >= 3 and seen["d"] >= 3, seen
    if src == "lbm_kernels.hip":
        assert seen["NS_6bf16_tE"] >= 3, seen
    assert f64_in_fp64 > 0
