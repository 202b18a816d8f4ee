"""The C ABI library loads on a machine without a GPU, exports every entry
point include/lbm.h declares, and validates parameters on the host (CPU only)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1306_6445_amd import lbm, workloads as WL
from tests.helpers import small_run

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", n) for n in sorted(os.listdir(os.path.join(ROOT, "include")))
           if n.endswith(".h")]


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lbm.LIB_PATH):
        from paper_1306_6445_amd import build
        build.build(verbose=False)
    return lbm.load_library()


def declared_functions():
    text = "\n".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm(?:3d)?_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_paper_entry_points():
    names = declared_functions()
    for required in ("lbm_create", "lbm_init_density", "lbm_step", "lbm_moments", "lbm3d_create",
                     "lbm3d_init_density", "lbm3d_step", "lbm3d_moments"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
    # and the binding knows the signature of each
    assert set(names) == set(lbm.SIGNATURES)
    out = subprocess.run(["nm", "-D", "--defined-only", lbm.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (lbm(?:3d)?_[a-z0-9_]+)", out))
    assert set(names) <= exported


def test_validation_accepts_workload_runs(lib):
    for run in (WL.config1(), small_run(8, 8, "pw"), small_run(8, 8, "exp"), WL.config3(256, 512, 256)):
        assert lbm.validate(run) == lbm.LBM_OK, lbm.last_error()


@pytest.mark.parametrize("field,value", [
    ("nx", 0), ("ny", -3), ("kappa", 1.0), ("kappa", -0.1), ("epsilon", -1.0),
    ("epsilon", float("nan")), ("G", 0.5), ("bc_x", 7), ("eos_kind", 9),
])
def test_validation_rejects_bad_parameters(lib, field, value):
    run = small_run(8, 8, "cs")
    setattr(run, field, value)
    assert lbm.validate(run) == lbm.LBM_EINVAL
    assert lbm.last_error()


@pytest.mark.parametrize("rates", [(1, 0.8, 0.8, 1, 1.1, 2.0), (1, 0.0, 0.0, 1, 1.1, 1.0),
                                   (1, 0.8, 0.9, 1, 1.1, 1.0)])
def test_validation_rejects_bad_rates(lib, rates):
    # rates must lie in (0, 2); epsilon != 0 needs s_zeta == s_e (Eq. 8)
    run = small_run(8, 8, "cs")
    run.rates = rates
    assert lbm.validate(run) == lbm.LBM_EINVAL


def test_validation_of_eos_parameters(lib):
    run = small_run(8, 8, "pw")
    run.eos = (0.1, -0.02, 1 / 3, 95.0, 1.49, 0.0)  # rho1 > rho2
    assert lbm.validate(run) == lbm.LBM_EINVAL
    run = small_run(8, 8, "exp")
    run.eos = (0.0, 200.0, 0, 0, 0, 0)
    assert lbm.validate(run) == lbm.LBM_EINVAL
    run = small_run(8, 8, "exp")
    run.G = 0.0  # the exponential potential allows G = 0 (no interaction) when epsilon = 0
    assert lbm.validate(run) == lbm.LBM_OK


def test_workspace_sizes(lib):
    a = small_run(100, 100)
    b = small_run(256, 256)
    s64 = lbm.workspace_bytes([a], "fp64")
    s32 = lbm.workspace_bytes([a], "fp32")
    s16 = lbm.workspace_bytes([a], "bf16")
    assert s64 > s32 > s16 > 9 * 2 * 100 * 100
    assert lbm.workspace_bytes([a, b], "fp32") > lbm.workspace_bytes([b], "fp32")
    g = lbm.Grid(0, 5, 0, 0)
    assert lib.lbm_workspace_bytes(ctypes.byref(g), 1) == 0


def test_empty_batches_and_grid_limits_are_rejected_on_the_host(lib):
    """No runs, an unknown precision or a run beyond 2^31 nodes (flat node
    indices within a run are 32-bit) fail before any device call."""
    assert lib.lbm_batch_workspace_bytes(0, None, 1) == 0
    a = (lbm.RunDesc * 1)(lbm.run_desc(small_run(8, 8)))
    assert lib.lbm_batch_workspace_bytes(1, a, 7) == 0
    ctx = ctypes.c_void_p()
    assert lib.lbm_batch_create(0, None, 1, None, 0, None, ctypes.byref(ctx)) == lbm.LBM_EINVAL
    assert not ctx.value and "run" in lbm.last_error()
    assert lib.lbm_batch_create(1, a, 7, None, 0, None, ctypes.byref(ctx)) == lbm.LBM_EINVAL
    assert not ctx.value and "precision" in lbm.last_error()
    run = small_run(8, 8)
    run.nx, run.ny = 65536, 32768  # exactly 2^31 nodes
    assert lbm.validate(run) == lbm.LBM_OK, lbm.last_error()
    run.ny = 32769
    assert lbm.validate(run) == lbm.LBM_EINVAL and "too large" in lbm.last_error()


def test_rows_are_dense(lib):
    """Device rows are stored unpadded: the population and node arrays grow
    with every node of width (row padding was measured and not adopted).
    Each direction's array is rounded up to 256 bytes and followed by a skew of
    17 x 256 bytes (so the nine arrays of a power-of-two grid do not share
    their offset modulo the HBM interleave), which the sizes include."""
    def ws(nx, prec, ny=20):
        return lbm.workspace_bytes([small_run(nx, ny)], prec)
    for prec, b in (("fp64", 8), ("fp32", 4), ("bf16", 2)):
        # two population buffers + psi (+ two writer-density arrays for bf16)
        # + the FP64 staging area, for 20 more nodes
        per_node = 2 * 9 * b + (8 if prec == "fp64" else 4) + (8 if prec == "bf16" else 0) + 9 * 8
        d = ws(97, prec) - ws(96, prec)
        slack = 2 * 9 * 256 + 1024
        assert 20 * per_node - slack <= d <= 20 * per_node + slack, (prec, d)
        n = 4096 * 2048
        assert ws(4096, prec, 2048) >= 2 * 9 * (n * b + 17 * 256), prec


def test_surrogate_entry_points_validate_on_the_host(lib):
    """lbm_mlp_*: sizes and argument checks that need no device."""
    assert lib.lbm_mlp_workspace_bytes(0) == 0
    assert lib.lbm_mlp_workspace_bytes(1 << 21) == 0
    small, big = lib.lbm_mlp_workspace_bytes(32), lib.lbm_mlp_workspace_bytes(4096)
    assert 0 < small < big
    # the per-chunk gradient slots dominate: one 4611-float slot per 32 samples
    assert big >= 4611 * 4 * (4096 // 32)
    h = ctypes.c_void_p()
    p = (ctypes.c_float * lbm.MLP_PARAMS)()
    assert lib.lbm_mlp_create(32, None, None, 0, None, ctypes.byref(h)) == lbm.LBM_EINVAL
    assert lib.lbm_mlp_create(32, p, None, small, None, ctypes.byref(h)) == lbm.LBM_EINVAL
    assert "workspace" in lbm.last_error()
    assert lib.lbm_mlp_create(0, p, ctypes.c_void_p(256), small, None, ctypes.byref(h)) == lbm.LBM_EINVAL
    p[7] = float("nan")
    assert lib.lbm_mlp_create(32, p, ctypes.c_void_p(256), small, None, ctypes.byref(h)) == lbm.LBM_EINVAL
    assert "finite" in lbm.last_error()
    assert lib.lbm_mlp_steps_taken(None) == -1
    assert lib.lbm_mlp_forward(None, None, 1, None) == lbm.LBM_EINVAL


def test_allocation_free_step_validates_on_the_host(lib):
    """lbm_step_noalloc rejects bad arguments and grids beyond its scratch
    (4,194,304 nodes, 65,536 tiles of 64 x 4) before any device call, and
    returns at once for zero steps."""
    run = small_run(64, 64)
    d = lbm.run_desc(run)

    def call(desc, f=ctypes.c_void_p(256), t0=0, n=1):
        return lib.lbm_step_noalloc(ctypes.byref(desc.grid), ctypes.byref(desc.eos), desc.G,
                                    ctypes.byref(desc.rates), desc.kappa, desc.epsilon, f, t0, n, None, None)

    assert call(d, f=None) == lbm.LBM_EINVAL and "population" in lbm.last_error()
    assert call(d, n=-1) == lbm.LBM_EINVAL and call(d, t0=-2) == lbm.LBM_EINVAL
    assert call(d, n=0) == lbm.LBM_OK
    big = lbm.run_desc(run)
    big.grid.nx, big.grid.ny = 4096, 1025
    assert call(big) == lbm.LBM_EINVAL and "4194304" in lbm.last_error()
    tall = lbm.run_desc(run)
    tall.grid.nx, tall.grid.ny = 1, 262148  # 65,537 tiles of one column
    assert call(tall) == lbm.LBM_EINVAL and "tiles" in lbm.last_error()
    bad = lbm.run_desc(run)
    bad.kappa = 1.0
    assert call(bad) == lbm.LBM_EINVAL and "kappa" in lbm.last_error()


def test_3d_entry_points_validate_on_the_host(lib):
    """lbm3d_validate / lbm3d_workspace_bytes / lbm3d_create reject bad
    arguments before any device call."""
    from tests.helpers import small_run3

    run = small_run3(8, 6, 5)
    g, e, G, r, kappa, eps = lbm.run3_args(run)
    assert lib.lbm3d_validate(ctypes.byref(g), ctypes.byref(e), G, ctypes.byref(r), kappa, eps) == lbm.LBM_OK
    bad = lbm.Rates3(*[float(v) for v in run.rates])
    bad.s_pi = 2.0
    assert lib.lbm3d_validate(ctypes.byref(g), ctypes.byref(e), G, ctypes.byref(bad), kappa, eps) == lbm.LBM_EINVAL
    assert "rates" in lbm.last_error()
    assert lib.lbm3d_validate(ctypes.byref(g), ctypes.byref(e), G, ctypes.byref(r), 1.0, eps) == lbm.LBM_EINVAL
    assert lib.lbm3d_validate(ctypes.byref(g), ctypes.byref(e), 0.5, ctypes.byref(r), kappa, eps) == lbm.LBM_EINVAL
    g0 = lbm.Grid3(8, 0, 5, 0, 0, 0)
    assert lib.lbm3d_validate(ctypes.byref(g0), ctypes.byref(e), G, ctypes.byref(r), kappa, eps) == lbm.LBM_EINVAL
    assert lib.lbm3d_workspace_bytes(ctypes.byref(g0), lbm.FP32) == 0
    # 2^31 - 1 nodes in one x column: the collide pass's 64 x 4 tiles would need
    # 2^31 workgroups of 256 threads; a 2^31-node grid of full tiles is fine
    thin = lbm.Grid3(1, 1, (1 << 31) - 1, 0, 0, 0)
    assert lib.lbm3d_validate(ctypes.byref(thin), ctypes.byref(e), G, ctypes.byref(r), kappa, eps) == lbm.LBM_EINVAL
    assert "2^32" in lbm.last_error()
    full = lbm.Grid3(1024, 1024, 2048, 0, 0, 0)
    assert lib.lbm3d_validate(ctypes.byref(full), ctypes.byref(e), G, ctypes.byref(r), kappa, eps) == lbm.LBM_OK
    # bf16 storage is 2D only; FP64 needs twice the FP32 population bytes
    assert lib.lbm3d_workspace_bytes(ctypes.byref(g), lbm.FP32_BF16STORE) == 0
    b32, b64 = lib.lbm3d_workspace_bytes(ctypes.byref(g), lbm.FP32), lib.lbm3d_workspace_bytes(ctypes.byref(g), lbm.FP64)
    assert b64 > b32 >= 2 * 19 * 4 * 240
    ctx = ctypes.c_void_p()
    assert lib.lbm3d_create(ctypes.byref(g), ctypes.byref(e), G, ctypes.byref(r), kappa, eps, lbm.FP32_BF16STORE,
                            None, 0, None, ctypes.byref(ctx)) == lbm.LBM_EINVAL
    assert not ctx.value and "FP64" in lbm.last_error()


def test_two_component_entry_points_validate_on_the_host(lib):
    """lbm_mc_validate / lbm_mc_workspace_bytes / lbm_mc_create reject bad
    arguments before any device call."""
    from tests.helpers import small_mc_run

    run = small_mc_run(12, 9)
    g, p = lbm.mc_args(run)
    assert lib.lbm_mc_validate(ctypes.byref(g), ctypes.byref(p)) == lbm.LBM_OK
    for field, value in (("G", 0.0), ("G", -1.0), ("G", float("inf")), ("kappa", 1.0), ("kappa", -0.2)):
        q = lbm.McParams(p.G, p.kappa, p.rates)
        setattr(q, field, value)
        assert lib.lbm_mc_validate(ctypes.byref(g), ctypes.byref(q)) == lbm.LBM_EINVAL, (field, value)
    q = lbm.McParams(p.G, p.kappa, p.rates)
    q.rates.s_j = 2.0
    assert lib.lbm_mc_validate(ctypes.byref(g), ctypes.byref(q)) == lbm.LBM_EINVAL
    assert "rates" in lbm.last_error()
    for bad in (lbm.Grid(0, 5, 0, 0), lbm.Grid(5, 5, 3, 0), lbm.Grid(1 << 16, 1 << 15, 0, 0)):
        assert lib.lbm_mc_validate(ctypes.byref(bad), ctypes.byref(p)) == lbm.LBM_EINVAL
    assert lib.lbm_mc_workspace_bytes(ctypes.byref(lbm.Grid(0, 5, 0, 0)), lbm.FP32) == 0
    assert lib.lbm_mc_workspace_bytes(ctypes.byref(g), lbm.FP32_BF16STORE) == 0
    b32, b64 = lib.lbm_mc_workspace_bytes(ctypes.byref(g), lbm.FP32), lib.lbm_mc_workspace_bytes(ctypes.byref(g), lbm.FP64)
    assert b64 > b32 >= 2 * 18 * 4 * 12 * 9
    ctx = ctypes.c_void_p()
    assert lib.lbm_mc_create(ctypes.byref(g), ctypes.byref(p), lbm.FP32_BF16STORE, None, 0, None,
                             ctypes.byref(ctx)) == lbm.LBM_EINVAL
    assert not ctx.value and "FP64" in lbm.last_error()
