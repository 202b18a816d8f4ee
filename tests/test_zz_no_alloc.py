"""The allocation-free step (lbm_step_noalloc) against lbm_step (needs an MI355X).

lbm_step_noalloc advances one FP64 run in place on the caller's device array,
with its psi array, run record and tile list in the library's static device
scratch; it runs the same kernels as the two-kernel schedule of a context, so
its populations must equal lbm_step's bit for bit.  Two calls in a row, the
second on a smaller grid (the scratch keeps the first call's contents), each
split at an odd step so that the in-place layout of both parities crosses
the call boundary."""
import sys

import numpy as np
import pytest

from paper_1306_6445_amd import lbm, workloads as WL
from tests.helpers import small_run

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_allocation_free_step_matches_lbm_step():
    import torch

    cases = [(small_run(96, 80, "cs", kappa=0.6, bc_y=WL.BC_WALL, seed=41), (3, 5)),
             (small_run(40, 24, "pw", kappa=0.3, seed=42), (5, 3))]
    for run, chunks in cases:
        say("  noalloc", run.label, run.nx, run.ny, chunks)
        with lbm.Lattice([run], precision="fp64") as L:
            L.init_all()
            f0 = L.populations(0)
            L.step(sum(chunks))
            ref = L.populations(0)
            assert L.status()[0] == 0
        f = torch.tensor(f0, dtype=torch.float64, device="cuda").contiguous()
        status = torch.full((1,), 7, dtype=torch.int32, device="cuda")
        stream = torch.cuda.current_stream()
        t = 0
        for n in chunks:
            lbm.step_noalloc(run, f.data_ptr(), t, n, status.data_ptr(), stream.cuda_stream)
            t += n
        torch.cuda.synchronize()
        got = f.cpu().numpy()
        np.testing.assert_array_equal(got, ref)
        assert int(status.item()) == 0
