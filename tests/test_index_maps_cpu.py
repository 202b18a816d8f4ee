"""The GPU kernels' AA streaming index maps, checked on the host (CPU only).

tests/index_maps_check.hip includes the same header functions the kernels
call (neighbours, the even and odd slot rules, the fixed-offset interior
form, the upwind node, psi_coord) and checks, for every node and direction of
80 grids (tiny, ragged, periodic and wall axes, padded rows), that every slot
is in bounds, that each step's loads and stores are bijections onto the grid,
that each node writes only the slots it reads (in-place AA without races),
and that what one step writes is what the next reads (Eq. 4 with halfway
bounce-back).  For the D3Q19 collide pass it checks on 88 grids that the
tiles cover every node once, that the per-axis neighbour offsets give the
psi_coord neighbours, and that the 19 streamed reads of all nodes (slot a of
x - e_a, or the node's own opposite slot across a wall) read every slot of
the source exactly once; for
the fused 3D step, that each LDS psi plane (tile and ring) is written exactly
once, that every psi a node reads is its psi_coord neighbour, and that the
work items and z chunks collide every node exactly once (1320 layouts: five
tile shapes, three z chunks); and for the two-component fused step, that every
tile shape covers the grid once, writes each cell of its density plane (tile
and ring) once and reads the psi_coord neighbours, and that the streamed
reads take every source slot once (1296 layouts).  It
is compiled for the host only; no GPU is involved.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_aa_index_maps_are_in_bounds_bijective_and_race_free(tmp_path):
    exe = str(tmp_path / "index_maps_check")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "--cuda-host-only", "-O1", "-std=c++17",
                    "-I", os.path.join(ROOT, "include"), "-o", exe,
                    os.path.join(ROOT, "tests", "index_maps_check.hip")],
                   check=True, capture_output=True, text=True, timeout=600)
    p = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert p.returncode == 0, p.stdout + p.stderr
    assert p.stdout.startswith("ok: 80 grids, 88 3d grids, 1320 fused 3d layouts, 1296 two-component layouts")
