"""The two-component extension on the GPU against its FP64 oracle (needs an MI355X).

Parity through the C ABI of include/lbm_mc.h; error = max over components,
directions and nodes of |f_gpu - f_oracle| / (rho_A + rho_B)(x).  FP64: 1e-13
per step on tiny and ragged grids with every boundary combination and every
tile shape class, 1e-11 after a few hundred steps, read-outs to 1e-9; FP32:
2e-6 per step from a common state (round-off of ~40 operations at 6e-8),
sampled at full size in the benchmark's launch shape; FP64 sampled past
4 GiB buffers (the 64-bit addressing).  Tile shapes give the same bits.  Physics: a settled slab keeps its compositions when kappa changes,
the Laplace tension scales as 1 - kappa, FP32 against FP64.
"""
import sys

import numpy as np
import pytest

from oracle import binary as B
from paper_1306_6445_amd import lbm, workloads as WL
from tests.helpers import oracle_mc_params, rel_err_mc, small_mc_run

pytestmark = pytest.mark.gpu
P, W = WL.BC_PERIODIC, WL.BC_WALL


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def lattice(run, precision, tile=None):
    say("  lattice_mc", precision, run.label, (run.nx, run.ny), (run.bc_x, run.bc_y), tile)
    L = lbm.LatticeMC(run, precision=precision)
    if tile:
        L.set_tile(*tile)
    L.init_all()
    return L


TINY = [((3, 3), (P, P)), ((1, 24), (P, W)), ((2, 5), (P, P)), ((7, 6), (W, P)), ((12, 9), (P, W)),
        ((17, 3), (W, W)), ((33, 20), (P, P)), ((70, 13), (W, W))]
TILES = [None, (32, 2, 1), (64, 8, 4), (256, 2, 2)]


@pytest.mark.parametrize("case", TINY, ids=lambda c: "%dx%d_bc%d%d" % (c[0] + c[1]))
def test_fp64_matches_oracle_step_by_step(case):
    (nx, ny), bc = case
    run = small_mc_run(nx, ny, bc=bc, seed=nx * 31 + ny)
    Pa = oracle_mc_params(run)
    f = B.init(Pa, run.rhoA, run.rhoB)
    for tile in TILES:
        g = f
        with lattice(run, "fp64", tile) as L:
            np.testing.assert_allclose(L.populations(), f, rtol=1e-15, atol=0)
            for k in range(1, 4):
                L.step(1)
                g = B.step(Pa, g)
                err = rel_err_mc(L.populations(), g)
                assert err < 1e-13, (tile, k, err)
        say("  ", tile, "3 steps ok")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tile_shapes_give_identical_bits(prec):
    runs = [small_mc_run(70, 13, bc=(W, W), seed=3), small_mc_run(65, 47, bc=(P, P), seed=4),
            small_mc_run(1, 40, bc=(P, W), seed=5)]
    for run in runs:
        ref = None
        for tile in [(64, 4, 2), (32, 2, 1), (64, 8, 4), (256, 2, 2), (128, 1, 4), (32, 8, 4)]:
            with lattice(run, prec, tile) as L:
                L.step(5)
                f = L.populations()
            if ref is None:
                ref = f
            else:
                assert np.array_equal(f, ref), (run.label, tile)


def test_fp64_drop_300_steps_and_read_outs():
    run = small_mc_run(40, 36, bc=(P, W), seed=8, R=9.0)
    Pa = oracle_mc_params(run)
    fo = B.run(Pa, B.init(Pa, run.rhoA, run.rhoB), 300)
    with lattice(run, "fp64") as L:
        L.step(300)
        fg = L.populations()
        mg = L.moments()
        dg = L.diagnostics(run.cx, run.cy, 2.0, 14.0)
    err = rel_err_mc(fg, fo)
    say("  300 steps err", err)
    assert err < 1e-11
    mo = B.moments(Pa, fo)
    np.testing.assert_allclose(mg[0], mo[0], rtol=1e-11)
    np.testing.assert_allclose(mg[1], mo[1], rtol=1e-11)
    vmax = max(np.abs(mo[2]).max(), np.abs(mo[3]).max())
    for a, b in zip(mg[2:], mo[2:]):
        assert np.abs(a - b).max() < 1e-9 * vmax + 1e-15
    do = B.diagnostics(Pa, fo, run.cx, run.cy, 2.0, 14.0)
    for k in B.DIAG_KEYS:
        assert dg[k] == pytest.approx(do[k], rel=1e-9, abs=1e-13), k
    assert dg["status"] == 0


def test_fp32_single_step_from_common_state():
    run = small_mc_run(48, 40, bc=(P, W), seed=6, R=10.0)
    Pa = oracle_mc_params(run)
    f0 = B.run(Pa, B.init(Pa, run.rhoA, run.rhoB), 30)
    with lattice(run, "fp32") as L:
        L.set_populations(f0)
        g0 = L.populations()
        L.step(1)
        got = L.populations()
    err = rel_err_mc(got, B.step(Pa, g0))
    say("  fp32 step err", err)
    assert err < 2e-6


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rest_state_and_conservation(prec):
    import dataclasses

    run = small_mc_run(20, 14, bc=(W, P), seed=2)
    rest = dataclasses.replace(run, rhoA=np.full(run.rhoA.shape, 0.3), rhoB=np.full(run.rhoB.shape, 0.6))
    with lattice(rest, prec) as L:
        f0 = L.populations()
        L.step(100)
        f1 = L.populations()
    np.testing.assert_allclose(f1, f0, rtol=1e-13 if prec == "fp64" else 1e-6, atol=0)
    with lattice(run, prec) as L:
        m0 = L.populations().sum(axis=(1, 2, 3))
        L.step(300)
        m1 = L.populations().sum(axis=(1, 2, 3))
    np.testing.assert_allclose(m1, m0, rtol=1e-12 if prec == "fp64" else 2e-6)


def test_divergence_is_flagged():
    run = small_mc_run(16, 16, seed=7)
    with lattice(run, "fp64") as L:
        f = L.populations()
        f[:, :, 5, 5] = -1.0  # a node with negative total density
        L.set_populations(f)
        L.step(2)
        with pytest.raises(lbm.LbmError):
            L.moments()
        assert L.diagnostics(8, 8, 2, 6)["status"] == 1


def _slab(kappa, prec, ny=128, steps=20000):
    import dataclasses

    run = WL.mc_drop_run(0, 1.0, kappa, shape=(4, ny))
    y = np.arange(ny)[:, None] * np.ones((1, 4))
    prof = 0.5 * (np.tanh((y - ny / 4) / 2) - np.tanh((y - 3 * ny / 4) / 2))
    run = dataclasses.replace(run, rhoA=0.05 + 0.95 * prof, rhoB=0.05 + 0.95 * (1 - prof))
    with lattice(run, prec) as L:
        L.step(steps)
        a, b, _, uy = L.moments()
    return a[ny // 2, 0], a[0, 0], np.abs(uy).max()


def test_flat_interface_compositions_do_not_move_with_kappa():
    res = {k: _slab(k, "fp64") for k in (0.0, 0.5, 0.9)}
    say("  slab", res)
    for k in (0.5, 0.9):
        assert res[k][0] == pytest.approx(res[0.0][0], rel=5e-4)
        assert res[k][1] == pytest.approx(res[0.0][1], rel=5e-3)
    # FP32 storage after 20,000 steps: within its accumulated rounding (5e-5 observed)
    f32 = _slab(0.9, "fp32")
    assert f32[0] == pytest.approx(res[0.9][0], rel=2e-4)
    assert f32[1] == pytest.approx(res[0.9][1], rel=2e-3)


def test_laplace_tension_scales_with_one_minus_kappa_fp32_vs_fp64():
    """Drops of A (R = 32 in 128^2, G = 1): sigma = dp R_eq at kappa = 0, 0.5,
    0.9 follows 1 - kappa; FP32 gives the FP64 tension within 0.5%."""
    sig = {}
    for prec in ("fp64", "fp32"):
        for kappa in (0.0, 0.5, 0.9):
            run = WL.mc_drop_run(128, 32.0, kappa, seed=WL.BASE_SEED + 12)
            with lattice(run, prec) as L:
                L.step(12000)
                d = L.diagnostics(run.cx, run.cy, *run.diag_radii())
            assert d["status"] == 0
            sig[(prec, kappa)] = d["dp"] * d["r_eq"]
    say("  sigma", sig)
    s0 = sig[("fp64", 0.0)]
    assert s0 > 0.03
    for kappa in (0.5, 0.9):
        assert sig[("fp64", kappa)] / s0 == pytest.approx(1 - kappa, abs=0.01 * (1 - kappa) + 2e-3)
    for kappa in (0.0, 0.5, 0.9):
        assert abs(sig[("fp32", kappa)] - sig[("fp64", kappa)]) < 5e-3 * s0


def test_full_size_fp32_sampled_in_the_benchmark_shape():
    """The 2048^2 spinodal-decomposition workload (FP32, default tile): sampled
    nodes of two consecutive steps against the oracle's sampled step."""
    run = WL.mc_spinodal_run(2048)
    Pa = oracle_mc_params(run)
    rng = np.random.default_rng(13)
    with lattice(run, "fp32") as L:
        L.step(20)
        for _ in range(2):
            f_t = L.populations()
            L.step(1)
            f_n = L.populations()
            idx = rng.choice(run.nodes, 2000, replace=False)
            ref = B.step_sampled(Pa, f_t, idx)
            got = f_n.reshape(2, 9, -1)[:, :, idx].transpose(2, 0, 1)
            err = float((np.abs(got - ref) / ref.sum(axis=(1, 2))[:, None, None]).max())
            say("  2048^2 fp32 sampled err", err)
            assert err < 2e-6


def test_population_round_trip_and_tile_validation():
    """FP64: reading the populations back and setting them again (a
    checkpoint) continues bit for bit; invalid tiles are rejected and leave
    the context usable."""
    run = small_mc_run(37, 29, bc=(W, P), seed=21)
    with lattice(run, "fp64") as L:
        L.step(7)
        blob = L.populations()
        L.step(9)
        ref = L.populations()
    with lattice(run, "fp64") as L:
        L.set_populations(blob)
        L.step(9)
        assert np.array_equal(L.populations(), ref)
        for bad in ((48, 4, 1), (64, 16, 1), (32, 1, 1), (256, 4, 1), (64, 4, 3)):
            with pytest.raises(lbm.LbmError):
                L.set_tile(*bad)
        L.step(1)
        assert L.steps_taken == 10


@pytest.mark.parametrize("prec,n,tol", [("fp64", 5504, 1e-13), ("fp32", 7744, 2e-6)])
def test_buffers_past_4_gib_match_the_oracle(prec, n, tol):
    """A mixture with walls in y whose population buffers hold more than
    4 GiB (FP64 5504^2: 4.4 GB; FP32 7744^2: 4.3 GB), past the 32-bit byte
    offsets the fused kernel uses on smaller grids, so it takes its 64-bit
    addressing.  Sampled nodes (both walls and the periodic seam among them)
    of two consecutive steps match the oracle's step from the same state."""
    import dataclasses

    run = dataclasses.replace(WL.mc_spinodal_run(n, seed=WL.BASE_SEED + 31), bc_y=W, label="mc_past_4GiB")
    assert 18 * (8 if prec == "fp64" else 4) * run.nodes > 2 ** 32
    Pa = oracle_mc_params(run)
    rng = np.random.default_rng(29)
    nx = run.nx
    with lattice(run, prec) as L:
        L.step(2)
        for _ in range(2):
            f_t = L.populations()
            L.step(1)
            f_n = L.populations()
            idx = np.concatenate([rng.choice(run.nodes, 600, replace=False), rng.integers(0, nx, 100),
                                  run.nodes - nx + rng.integers(0, nx, 100), rng.integers(0, run.ny, 100) * nx,
                                  rng.integers(0, run.ny, 100) * nx + nx - 1])
            ref = B.step_sampled(Pa, f_t, idx)
            got = f_n.reshape(2, 9, -1)[:, :, idx].transpose(2, 0, 1)
            err = float((np.abs(got - ref) / ref.sum(axis=(1, 2))[:, None, None]).max())
            say("  past 4 GiB %s sampled err" % prec, err)
            assert err < tol
            del f_t, f_n


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_checkpoint_continues_bit_for_bit(prec):
    """lbm_mc_save_state / lbm_mc_load_state: a restore into a fresh context
    (initialised from another field, so its FP32 base densities differ)
    continues bit for bit, in FP32 too; a checkpoint of another grid is
    refused and leaves the context usable."""
    run = small_mc_run(37, 29, bc=(W, P), seed=51)
    with lattice(run, prec) as L:
        L.step(7)
        blob = L.save_state()
        L.step(9)
        ref = L.populations()
    with lattice(small_mc_run(37, 29, bc=(W, P), seed=52), prec) as L:
        L.load_state(blob)
        assert L.steps_taken == 7
        L.step(9)
        assert np.array_equal(L.populations(), ref)
    with lattice(small_mc_run(36, 29, bc=(W, P), seed=53), prec) as L:
        with pytest.raises(lbm.LbmError):
            L.load_state(blob)
        L.step(1)
        assert L.steps_taken == 1


def test_autotune_picks_a_candidate_and_keeps_the_bits():
    """lbm_mc_autotune sets one of its candidate tiles; stepping with it gives
    the default tile's bits."""
    run = small_mc_run(70, 45, bc=(P, W), seed=62)
    with lattice(run, "fp32") as L:
        L.step(3)
        ref = L.populations()
    with lattice(run, "fp32") as L:
        choice = L.autotune(2)
        say("  autotune choice", choice)
        assert choice in {(128, 4, 1), (64, 8, 1), (128, 4, 2), (256, 2, 1), (64, 4, 2), (128, 2, 2), (256, 2, 2),
                          (64, 8, 2), (32, 8, 2), (64, 4, 1)}
        L.init_all()
        L.step(3)
        assert np.array_equal(L.populations(), ref)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_graph_replays_give_the_eager_bits(prec):
    """lbm_mc_step replays captured graphs of 2k steps: several replays with
    single launches, tile changes and read-backs between them give, after
    every phase, the bits of a context that launches every step."""
    run = small_mc_run(70, 45, bc=(W, P), seed=72)
    phases = [(4, None), (1, None), (8, None), (3, (32, 8, 4)), (4, None), (5, (256, 2, 2)), (9, None)]
    with lattice(run, prec) as G, lattice(run, prec) as E:
        G.set_graph_steps(2)
        E.set_graph_steps(0)
        for n, tile in phases:
            if tile:
                G.set_tile(*tile)
                E.set_tile(*tile)
            G.step(n)
            E.step(n)
            assert np.array_equal(G.populations(), E.populations()), (n, tile)
        assert G.steps_taken == E.steps_taken == sum(n for n, _ in phases)
        with pytest.raises(lbm.LbmError):
            G.set_graph_steps(5000)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32", 2e-5)])
def test_mixture_velocity_read_out_against_the_closed_form(prec, tol):
    """Eq. (6) for the mixture on the GPU, checked against a value computed
    here and not by the oracle: on resting sinusoidal densities the mixture
    velocity is (F_A + F_B) / (2 rho) with each F_s of Eq. (7) in closed form
    from the partner's density, and the diagnostics' largest speed is its
    largest norm."""
    import dataclasses

    G, nx, ny = 1.0, 24, 18
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    ka = 2 * np.pi * np.array([2 / nx, -1 / ny])
    kb = 2 * np.pi * np.array([1 / nx, 2 / ny])
    pha, phb = 1.1 + ka[0] * x + ka[1] * y, 0.4 + kb[0] * x + kb[1] * y
    rhoA, rhoB = 0.5 + 0.2 * np.cos(pha), 0.6 + 0.25 * np.cos(phb)
    run = dataclasses.replace(small_mc_run(nx, ny, seed=3, G=G), rhoA=rhoA, rhoB=rhoB, label="sinusoidal_mixture")

    def g(k):
        return [(2 / 3) * np.sin(k[0]) + (1 / 3) * np.sin(k[0]) * np.cos(k[1]),
                (2 / 3) * np.sin(k[1]) + (1 / 3) * np.sin(k[1]) * np.cos(k[0])]

    assert run.G == G
    rho = rhoA + rhoB
    FA = [-G * rhoA * (-0.25 * np.sin(phb)) * gi for gi in g(kb)]
    FB = [-G * rhoB * (-0.2 * np.sin(pha)) * gi for gi in g(ka)]
    want = [(a + b) / (2 * rho) for a, b in zip(FA, FB)]
    vmax = max(np.abs(w).max() for w in want)
    with lattice(run, prec) as L:
        a, b, ux, uy = L.moments()
        d = L.diagnostics(nx / 2, ny / 2, 2.0, 6.0)
    np.testing.assert_allclose(a, rhoA, rtol=1e-13 if prec == "fp64" else 1e-6)
    np.testing.assert_allclose(b, rhoB, rtol=1e-13 if prec == "fp64" else 1e-6)
    for got, w in zip((ux, uy), want):
        assert np.abs(got - w).max() < tol * vmax
    assert d["max_speed"] == pytest.approx(float(np.hypot(*want).max()), rel=tol)
