"""Parity of the HIP path with the FP64 oracle (needs an MI355X).

Every test drives the library through its C ABI (ctypes binding) and compares
with the oracle on the same seeded inputs.  Error measure: max over nodes and
directions of |f_gpu - f_oracle| / rho_oracle(x).
Tolerances: FP64 1e-13 per few steps (round-off of a few dozen operations;
FMA contraction and summation order differ from the oracle), 1e-10 after the
5,000 steps of the 100x100 droplet; FP32 2e-6 per step from a common state
(FP32 unit round-off 6e-8 times the ~30 operations on the longest path),
measured against max(rho(x), rho_ref) where the storage holds deviations from
the rest state at a base density rho_ref.
"""
import dataclasses
import sys

import numpy as np
import pytest

import oracle as O
from paper_1306_6445_amd import lbm, workloads as WL
from tests.helpers import oracle_params, rel_err, rel_err_scaled, small_run

pytestmark = pytest.mark.gpu

P, W = WL.BC_PERIODIC, WL.BC_WALL


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def lattice(runs, precision, **kw):
    say("  lattice", precision, [(r.label, r.nx, r.ny) for r in runs][:6], kw)
    L = lbm.Lattice(runs, precision=precision, **kw)
    L.init_all()
    return L


TINY = [
    dict(nx=3, ny=3, kind="cs", bc_x=P, bc_y=P),
    dict(nx=1, ny=40, kind="cs", bc_x=P, bc_y=W),
    dict(nx=2, ny=5, kind="pw", bc_x=P, bc_y=P),
    dict(nx=8, ny=8, kind="pw", bc_x=P, bc_y=W),
    dict(nx=17, ny=12, kind="exp", bc_x=W, bc_y=P),
    dict(nx=64, ny=4, kind="pw", bc_x=W, bc_y=W),
    dict(nx=130, ny=70, kind="cs", bc_x=P, bc_y=W),
    dict(nx=257, ny=9, kind="exp", bc_x=P, bc_y=P),
]


@pytest.mark.parametrize("fused", [1, 4, 0], ids=["fused1", "fused4", "twokernel"])
@pytest.mark.parametrize("case", TINY, ids=lambda c: "%s_%dx%d_bc%d%d" % (c["kind"], c["nx"], c["ny"], c["bc_x"], c["bc_y"]))
def test_fp64_matches_oracle_step_by_step(case, fused):
    run = small_run(case["nx"], case["ny"], case["kind"], kappa=0.6, bc_x=case["bc_x"], bc_y=case["bc_y"],
                    seed=case["nx"] * 31 + case["ny"])
    Pa = oracle_params(run)
    f = O.init(Pa, run.rho)
    with lattice([run], "fp64", graph_steps=0, fused=fused) as L:
        np.testing.assert_allclose(L.populations(0), f, rtol=1e-15, atol=0)
        for k in range(1, 5):
            L.step(1)
            f = O.step(Pa, f)
            err = rel_err(L.populations(0), f)
            say("  step", k, "err", err)
            assert err < 1e-13, (k, err)


def test_fp64_config1_5000_steps_within_1e10():
    run = WL.config1()
    Pa = oracle_params(run)
    f0 = O.init(Pa, run.rho)
    say("  oracle 5000 steps of 100x100 ...")
    fo = O.run(Pa, f0, 5000)
    with lattice([run], "fp64") as L:
        L.step(5000)
        fg = L.populations(0)
        rho_g, ux_g, uy_g = L.moments(0)
        dg = L.diagnostics([(run.cx, run.cy, *run.diag_radii())])[0]
    err = rel_err(fg, fo)
    say("  config1 per-node relative error after 5000 steps:", err)
    assert err < 1e-10
    rho_o, ux_o, uy_o = O.moments(Pa, fo)
    assert np.abs(rho_g - rho_o).max() < 1e-10 * rho_o.max()
    assert np.abs(ux_g - ux_o).max() < 1e-10 * max(np.abs(ux_o).max(), 1e-300) + 1e-15
    do = O.diagnostics(Pa, fo, run.cx, run.cy, *run.diag_radii())
    for k in ("mass", "rho_in", "rho_out", "p_in", "p_out", "r_eq", "max_speed"):
        assert dg[k] == pytest.approx(do[k], rel=1e-9), k
    assert dg["dp"] == pytest.approx(do["dp"], rel=1e-6)
    assert dg["status"] == 0


def eq7_force(psi, G, wall_y):
    """F = -G psi(x) sum_a w_a psi(x + e_a) e_a (Eq. 7) on a 2D field psi[y, x]
    that is periodic in x and periodic or walled in y (beyond a wall psi takes
    the value of the adjacent row), with w = 1/3 on the axes, 1/12 diagonally."""
    p = np.pad(psi, ((1, 1), (0, 0)), mode="edge" if wall_y else "wrap")
    p = np.pad(p, ((0, 0), (1, 1)), mode="wrap")
    c = lambda dx, dy: p[1 + dy:p.shape[0] - 1 + dy, 1 + dx:p.shape[1] - 1 + dx]
    sx = (c(1, 0) - c(-1, 0)) / 3 + (c(1, 1) - c(-1, -1) + c(1, -1) - c(-1, 1)) / 12
    sy = (c(0, 1) - c(0, -1)) / 3 + (c(1, 1) - c(-1, -1) + c(-1, 1) - c(1, -1)) / 12
    return -G * psi * sx, -G * psi * sy


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-6)])
def test_eq6_velocity_of_a_resting_sinusoidal_psi_field(precision, tol):
    """lbm_moments and lbm_diagnostics return the Eq. (6) velocity: on a rest
    equilibrium whose exponential pseudopotential is exactly
    A + B cos(theta + k x + l y), it is F / (2 rho) with F of Eq. (7) in closed
    form (no oracle involved)."""
    nx, ny, A, B, theta = 48, 40, 2.0, 0.35, 0.7
    k, l = 2 * np.pi * 3 / nx, 2 * np.pi * -2 / ny
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    phase = theta + k * x + l * y
    psi = A + B * np.cos(phase)
    kind, eos = WL.exp_eos()
    assert tuple(eos[:2]) == (4.0, 200.0)
    rho = -200.0 / np.log(psi / 4.0)
    run = WL.Run(nx=nx, ny=ny, eos_kind=kind, eos=eos, G=-40.0, rates=WL.rates(0.1), kappa=0.5,
                 epsilon=0.0, rho=rho, cx=nx / 2, cy=ny / 2, R0=8.0, label="sinusoidal_psi")
    sx = 2 * (np.sin(k) / 3 + np.sin(k + l) / 12 - np.sin(l - k) / 12)
    sy = 2 * (np.sin(l) / 3 + np.sin(k + l) / 12 + np.sin(l - k) / 12)
    Fx = 40.0 * psi * (-B * np.sin(phase)) * sx
    Fy = 40.0 * psi * (-B * np.sin(phase)) * sy
    with lattice([run], precision) as L:
        r, ux, uy = L.moments(0)
        d = L.diagnostics([(run.cx, run.cy, 4.0, 12.0)])[0]
    vmax = np.abs(Fx / (2 * rho)).max()
    say("  ", precision, "max |u| closed form", vmax, "GPU", d["max_speed"])
    # FP32: rho ~ 300 stored to 6e-8 relative moves psi (exp(-200/rho)) by
    # about 4e-8 relative, and F, a difference of psi values, by more
    scale = 1.0 if precision == "fp64" else 50.0
    assert np.abs(ux - Fx / (2 * rho)).max() < scale * tol * vmax
    assert np.abs(uy - Fy / (2 * rho)).max() < scale * tol * vmax
    assert d["max_speed"] == pytest.approx(float(np.max(np.hypot(Fx, Fy) / (2 * rho))), rel=scale * tol)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
def test_pressure_read_out_is_the_eos_of_the_density(precision):
    """lbm_run_pressure returns p_EOS(rho) per node (the bulk pressure of the
    Laplace law), for the three EOS forms, on a run in a batch; it equals the
    oracle's EOS (pinned separately) at the density lbm_run_moments returns."""
    runs = [small_run(40, 30, "cs", bc_y=W, seed=61), small_run(33, 20, "pw", seed=62),
            small_run(24, 24, "exp", seed=63)]
    with lattice(runs, precision) as L:
        L.step(7)
        for i, r in enumerate(runs):
            rho = L.moments(i)[0]
            p = L.pressure(i)
            ref = O.eos(oracle_params(r), rho)[0]
            # p_EOS is a difference of terms up to ~100 times larger than p
            scale = np.abs(ref).max()
            say("  ", precision, r.label, "max |dp| / max |p|", np.abs(p - ref).max() / scale)
            assert np.abs(p - ref).max() <= 1e-11 * scale


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 2e-6)])
def test_batch_diagnostics_of_top_hat_disks(precision, tol):
    """lbm_batch_diagnostics on two runs of different sizes in one batch (one
    periodic, one with walls in y), each a disk of rho_l in rho_v at rest:
    region means, the EOS pressure jump, the mass by node count and
    R_eq = sqrt(nodes of the disk / pi) are known without stepping."""
    rl, rv = 0.36, 0.009
    runs, expect = [], []
    for nx, ny, bcy, cx, cy, R in ((96, 80, P, 40.0, 37.0, 13.5), (70, 110, W, 30.0, 60.0, 17.5)):
        base = small_run(nx, ny, "cs", bc_y=bcy, noise=0.0)
        y, x = np.mgrid[0:ny, 0:nx]
        dx = np.abs(x - cx)
        dx = np.minimum(dx, nx - dx)
        dy = np.abs(y - cy) if bcy == W else np.minimum(np.abs(y - cy), ny - np.abs(y - cy))
        inside = np.hypot(dx, dy) <= R
        run = dataclasses.replace(base, rho=np.where(inside, rl, rv), cx=cx, cy=cy, R0=R)
        n_in = int(inside.sum())
        Pa = oracle_params(run)
        p = O.eos(Pa, np.array([rl, rv]))[0]
        # at rest sum_a e_a f_a = 0, so the Eq. 6 velocity is F / (2 rho), with F
        # of Eq. (7) on the disk's psi (periodic wrap, wall ghost = adjacent row)
        psi = O.eos(Pa, run.rho)[1]
        Fx, Fy = eq7_force(psi, Pa.G, bcy == W)
        vmax = float(np.max(np.hypot(Fx, Fy) / (2 * run.rho)))
        expect.append({"mass": n_in * rl + (nx * ny - n_in) * rv, "rho_in": rl, "rho_out": rv,
                       "p_in": p[0], "p_out": p[1], "r_eq": np.sqrt(n_in / np.pi), "max_speed": vmax})
        runs.append(run)
    with lattice(runs, precision) as L:
        got = L.diagnostics([(r.cx, r.cy, r.R0 / 2, r.R0 + 4) for r in runs])
    for g, e in zip(got, expect):
        say("  ", precision, {k: g[k] for k in e})
        for k in ("mass", "rho_in", "rho_out", "r_eq"):
            assert g[k] == pytest.approx(e[k], rel=tol), k
        # p_EOS here is a difference of terms about 100 times larger than p
        # (and psi, hence F in the speed, a root of one), so the density's
        # rounding reaches them amplified by that much
        for k in ("p_in", "p_out", "max_speed"):
            assert g[k] == pytest.approx(e[k], rel=100 * tol), k
        assert g["dp"] == pytest.approx(e["p_in"] - e["p_out"], rel=300 * tol)
        assert g["status"] == 0


@pytest.mark.parametrize("fused", [1, 0], ids=["fused", "twokernel"])
@pytest.mark.parametrize("kind", ["cs", "pw", "exp"])
def test_fp32_single_step_from_common_state(kind, fused):
    run = small_run(70, 33, kind, kappa=0.8, bc_y=W, seed=5)
    Pa = oracle_params(run)
    with lattice([run], "fp32", graph_steps=0, fused=fused) as L:
        L.step(37)
        for k in range(2):  # both parities
            f_t = L.populations(0)
            L.step(1)
            err = rel_err_scaled(L.populations(0), O.step(Pa, f_t), 0.0)
            say("  fp32", kind, "parity", (37 + k) % 2, "err", err)
            assert err < 2e-6


@pytest.mark.parametrize("tile,fused", [((64, 4), 1), ((32, 8), 1), ((32, 2), 1), ((256, 1), 1), ((64, 4), 2),
                                        ((32, 2), 4), ((128, 2), 4), ((64, 4), 0), ((256, 1), 0), ((32, 2), 0)])
def test_batch_of_uneven_runs_matches_oracle(tile, fused):
    runs = [small_run(33, 20, "cs", kappa=0.1, seed=1), small_run(5, 70, "pw", kappa=0.9, bc_y=W, seed=2),
            small_run(64, 64, "exp", kappa=0.5, seed=3), small_run(1, 16, "cs", kappa=0.0, bc_y=W, seed=4),
            small_run(100, 3, "pw", kappa=0.3, bc_x=W, seed=5)]
    with lattice(runs, "fp64", tile=tile, fused=fused) as L:
        L.step(7)
        for i, r in enumerate(runs):
            fo = O.run(oracle_params(r), O.init(oracle_params(r), r.rho), 7)
            err = rel_err(L.populations(i), fo)
            say("  run", i, r.label, "err", err)
            assert err < 1e-13


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_schedules_tiles_and_graphs_agree_bitwise(prec):
    """The arithmetic per node depends neither on the tile shape nor on the
    schedule (the fused kernel computes the halo densities and psi exactly as
    the psi pass does), nor on graph replay: bitwise equal throughout, also
    with odd step counts (the fused state then sits in the second buffer)."""
    runs = [small_run(96, 40, "cs", seed=8), small_run(37, 61, "pw", bc_y=W, seed=9),
            small_run(70, 9, "exp", bc_x=W, bc_y=W, seed=10)]

    def go(tile, gk, fused, chunks=(41,)):
        with lattice(runs, prec, tile=tile, graph_steps=gk, fused=fused) as L:
            for n in chunks:
                L.step(n)
            assert L.steps_taken == sum(chunks)
            return [L.populations(i) for i in range(len(runs))]

    ref = go((64, 4), 16, 0)
    for tile, gk, fused, chunks in [((64, 4), 0, 0, (41,)), ((64, 4), 4, 1, (41,)), ((64, 4), 0, 1, (41,)),
                                    ((128, 2), 3, 0, (41,)), ((32, 8), 3, 1, (41,)), ((256, 1), 2, 1, (5, 9, 27)),
                                    ((32, 2), 3, 0, (41,)), ((32, 4), 2, 1, (1, 1, 39)), ((64, 4), 2, 2, (41,)),
                                    ((32, 4), 3, 4, (5, 36)), ((64, 2), 0, 4, (41,)), ((128, 2), 4, 2, (3, 38))]:
        for u, v in zip(ref, go(tile, gk, fused, chunks)):
            np.testing.assert_array_equal(u, v)


@pytest.mark.parametrize("prec", ["fp32", "fp64", "bf16"])
def test_interior_and_edge_tiles_agree_bitwise(prec):
    """Tiles whose halo and upwind neighbours lie inside the grid take the
    fused kernel's interior path (fixed slot offsets); other tiles of a run
    periodic on both axes (the 257 x 130 run, the multi-range run) take the
    path with the wall tests folded away (FP64, FP32), and tiles at a wall
    the general one.  Grids large enough to hold all three, with walls,
    ragged sizes and a multi-range run: every fused shape agrees bit for bit
    with the two-kernel schedule."""
    mr = WL.paper_multirange_run("B", n=160, R=40.0)
    mr.rho = mr.rho * (1 + WL.noise(mr.rho.shape, 1e-3, 9))
    runs = [small_run(300, 200, "cs", kappa=0.6, bc_y=W, seed=31), small_run(257, 130, "pw", kappa=0.3, seed=32),
            small_run(200, 190, "exp", kappa=0.0, bc_x=W, bc_y=W, seed=33)]

    def go(rs, tile, fu):
        with lattice(rs, prec, tile=tile, graph_steps=2, fused=fu) as L:
            L.step(9)
            return [L.populations(i) for i in range(len(rs))]

    for rs in (runs, runs[:1] + [mr]):
        ref = go(rs, (64, 4), 0)
        for tile, fu in (((64, 4), 2), ((32, 8), 1), ((128, 2), 4), ((256, 1), 4), ((256, 2), 4), ((128, 4), 2),
                         ((64, 8), 1), ((64, 8), 0)):
            for u, v in zip(ref, go(rs, tile, fu)):
                np.testing.assert_array_equal(u, v)


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
def test_diagnostics_agree_across_tile_shapes(prec):
    """The FP64 diagnostics reduce per tile of the step's work list (tiles of
    64 to 512 threads) and then per run in a fixed order: the same state gives
    the same figures to round-off under every tile shape."""
    runs = [small_run(150, 70, "cs", kappa=0.5, bc_y=W, seed=41), small_run(33, 47, "pw", seed=42)]
    regions = [(r.cx, r.cy, *r.diag_radii()) for r in runs]
    out = []
    for tile in ((64, 4), (128, 4), (256, 2), (32, 2)):
        with lattice(runs, prec, tile=tile, graph_steps=2, fused=0) as L:
            L.step(12)
            out.append(L.diagnostics(regions))
    for d in out[1:]:
        for a, b in zip(out[0], d):
            for k in ("mass", "rho_in", "rho_out", "p_in", "p_out", "r_eq", "max_speed"):
                assert a[k] == pytest.approx(b[k], rel=1e-12, abs=1e-300), k


def test_switching_schedule_mid_run_is_bitwise():
    """The fused schedule's state may sit in either population buffer; every
    read-back, checkpoint and the two-kernel schedule take it from there."""
    runs = [small_run(66, 34, "pw", bc_y=W, seed=21), small_run(40, 40, "cs", seed=22)]
    with lattice(runs, "fp32", graph_steps=2) as L:
        L.step(23)
        ref = [L.populations(i) for i in range(2)]
    with lattice(runs, "fp32", graph_steps=2, fused=1) as L:
        L.step(7)  # odd: the state is in the second buffer
        rho_a = L.moments(0)[0]
        L.set_fused(0)
        L.step(6)
        L.set_fused(1)
        L.step(5)
        L.set_tile(32, 8)
        L.step(3)
        L.set_fused(4)
        L.step(2)
        for i in range(2):
            np.testing.assert_array_equal(L.populations(i), ref[i])
    with lattice(runs, "fp32", graph_steps=2) as L:
        L.step(7)
        np.testing.assert_array_equal(L.moments(0)[0], rho_a)


@pytest.mark.parametrize("kind", ["cs", "pw"])
def test_fp32_deviation_storage_step(kind):
    """FP32 populations stored as deviations from the rest state at a chosen
    base density: one step from a common state, error bounded relative to
    max(rho(x), rho_ref)."""
    run = small_run(48, 40, kind, kappa=0.7, bc_y=W, seed=15)
    Pa = oracle_params(run)
    with lattice([run], "fp32", graph_steps=0) as L:
        L.step(9)
        f_plain = L.populations(0)
        ref = float(run.rho.max())
        L.set_reference_density(0, ref)
        assert rel_err_scaled(L.populations(0), f_plain, ref) < 1e-7  # re-encoding
        for k in range(2):
            f_t = L.populations(0)
            L.step(1)
            err = rel_err_scaled(L.populations(0), O.step(Pa, f_t), ref)
            say("  fp32 deviation", kind, "err", err)
            assert err < 2e-6


def test_autotune_keeps_the_physics():
    """The autotuner times real steps under several schedules; the state must
    still be the oracle's after that many steps."""
    runs = [small_run(70, 40, "cs", seed=31), small_run(33, 65, "pw", bc_y=W, seed=32)]
    with lattice(runs, "fp64", graph_steps=2) as L:
        choice = L.autotune(4)
        n = L.steps_taken
        say("  autotune chose", choice, "after", n, "steps")
        assert n > 0 and choice["tile"][0] in (32, 64, 128, 256)
        for i, r in enumerate(runs):
            fo = O.run(oracle_params(r), O.init(oracle_params(r), r.rho), n)
            assert rel_err(L.populations(i), fo) < 1e-12


@pytest.mark.parametrize("fused", [0, 1])
def test_checkpoint_restart_is_bitwise(fused):
    runs = [small_run(50, 30, "pw", bc_y=W, seed=12)]
    with lattice(runs, "fp32", fused=fused) as L:
        L.step(11)
        blob = L.save_state()
        L.step(10)
        a = L.populations(0)
        L.load_state(blob)
        assert L.steps_taken == 11
        L.step(10)
        np.testing.assert_array_equal(a, L.populations(0))
    # a checkpoint does not depend on the schedule that wrote it
    with lattice(runs, "fp32", fused=1 - fused, tile=(32, 8)) as L:
        L.load_state(blob)
        L.step(10)
        np.testing.assert_array_equal(a, L.populations(0))


def test_set_and_get_populations_roundtrip_at_both_parities():
    run = small_run(20, 11, "exp", bc_x=W, seed=3)
    Pa = oracle_params(run)
    f = O.run(Pa, O.init(Pa, run.rho), 3)
    with lattice([run], "fp64") as L:
        for parity in (0, 1):
            if L.steps_taken % 2 != parity:
                L.step(1)
            assert L.steps_taken % 2 == parity
            L.set_populations(0, f)
            np.testing.assert_array_equal(L.populations(0), f)
            L.step(1)
            assert rel_err(L.populations(0), O.step(Pa, f)) < 1e-13


def test_init_with_velocity_matches_oracle():
    run = small_run(16, 16, "cs", seed=4)
    rng = np.random.default_rng(0)
    run.ux = rng.uniform(-0.02, 0.02, run.rho.shape)
    run.uy = rng.uniform(-0.02, 0.02, run.rho.shape)
    Pa = oracle_params(run)
    with lattice([run], "fp64") as L:
        np.testing.assert_allclose(L.populations(0), O.init(Pa, run.rho, run.ux, run.uy), rtol=1e-14)


@pytest.mark.parametrize("prec,fused", [("fp64", 2), ("fp64", 0), ("fp32", 2), ("fp32", 0), ("bf16", 2), ("bf16", 0)])
def test_uniform_fluid_at_rest_stays_at_rest(prec, fused):
    """A uniform density at rest is a fixed point of the step: uniform psi
    gives F = 0 (Eq. 7) and Q = 0 (Eq. 19), and the collision leaves the rest
    equilibrium (Eq. 3) in place.  Populations stay put to round-off in every
    precision and schedule, for each EOS, across periodic seams and walls (and
    bf16 stores only the rounding residue of f - w rho); the velocity stays
    exactly zero by symmetry; zero steps change nothing."""
    runs = []
    for kind, rho0, bcx, bcy in (("cs", 0.35, P, P), ("pw", 100.0, P, W), ("exp", 300.0, W, W)):
        r = small_run(70, 36, kind, kappa=0.7, bc_x=bcx, bc_y=bcy, seed=3)
        r.rho = np.full((36, 70), rho0)
        runs.append(r)
    tol = {"fp64": 1e-14, "fp32": 1e-6, "bf16": 1e-6}[prec]
    with lattice(runs, prec, fused=fused, graph_steps=2) as L:
        f0 = [L.populations(i) for i in range(len(runs))]
        L.step(0)
        assert L.steps_taken == 0
        for i in range(len(runs)):
            np.testing.assert_array_equal(L.populations(i), f0[i])
        L.step(11)
        assert not L.status().any()
        for i in range(len(runs)):
            err = np.abs(L.populations(i) - f0[i]).max() / f0[i].max()
            rho, ux, uy = L.moments(i)
            say("  rest", prec, fused, runs[i].label or i, "err", err, "max|u|", np.abs(ux).max(), np.abs(uy).max())
            assert err <= tol
            assert np.abs(ux).max() == 0.0 and np.abs(uy).max() == 0.0
            assert np.abs(rho / rho.mean() - 1).max() <= tol


def test_divergence_is_flagged_not_faulted():
    good = small_run(16, 16, "cs", seed=1)
    bad = small_run(16, 16, "cs", seed=2)
    bad.rho = np.full((16, 16), 0.999)  # eta close to 1: psi is not real there
    with lattice([good, bad], "fp32") as L:
        L.step(4)
        st = L.status()
        assert list(st) == [0, 1]
        with pytest.raises(lbm.LbmError) as e:
            L.moments(1)
        assert e.value.code == lbm.LBM_EDIVERGED
        L.moments(0)  # the healthy run is unaffected


def test_mass_conserved_on_gpu_fp64_with_walls():
    run = small_run(120, 80, "pw", kappa=0.95, bc_y=W, seed=21)
    with lattice([run], "fp64") as L:
        m0 = L.populations(0).sum()
        L.step(500)
        assert abs(L.populations(0).sum() - m0) < 1e-12 * m0


# ------------------------------------------------------------- full sizes

def _sample(nx, ny, rng, n=400):
    idx = rng.choice(nx * ny, size=n, replace=False)
    edges = [0, nx - 1, (ny - 1) * nx, ny * nx - 1, (ny // 2) * nx, nx // 2, (ny - 1) * nx + nx // 2]
    return np.unique(np.concatenate([idx, edges]))


def test_config2_full_size_batched_fp32_sampled():
    """40 runs of 256x256 in one batch, the benchmark's launch configuration."""
    runs = WL.config2()
    rng = np.random.default_rng(99)
    with lattice(runs, "fp32") as L:
        L.step(64)
        for i in (0, 13, 39):
            for _ in range(2):
                f_t = L.populations(i)
                L.step(1)
                f_n = L.populations(i)
                idx = _sample(256, 256, rng)
                ref = O.step_sampled(oracle_params(runs[i]), f_t, idx)
                got = f_n.reshape(9, -1)[:, idx].T
                err = float((np.abs(got - ref) / ref.sum(axis=1, keepdims=True)).max())
                say("  config2 run", i, "err", err)
                assert err < 2e-6


@pytest.mark.parametrize("precision,tol", [("fp32", 2e-6), ("fp64", 1e-13)])
def test_config3_full_size_capillary_sampled(precision, tol):
    """4096 x 2048 with bounce-back walls in y; samples include wall rows.  The
    benchmark's launch configuration: 256 x 2 threads, four nodes each."""
    run = WL.config3(256)
    Pa = oracle_params(run)
    rng = np.random.default_rng(7)
    with lattice([run], precision, tile=(256, 2), fused=4) as L:
        L.step(3)
        for _ in range(2):
            f_t = L.populations(0)
            L.step(1)
            f_n = L.populations(0)
            idx = _sample(run.nx, run.ny, rng, 2000)
            ref = O.step_sampled(Pa, f_t, idx)
            got = f_n.reshape(9, -1)[:, idx].T
            err = float((np.abs(got - ref) / ref.sum(axis=1, keepdims=True)).max())
            say("  config3", precision, "err", err)
            assert err < tol


def test_config5_full_size_splash_sampled():
    """2048 x 1024 droplet splash (wall below and above, step-function
    viscosity of Section V.C) in FP32, the benchmark's launch configuration;
    samples include both walls and the film surface."""
    run = WL.config5(0.584, 0.6245, 1.7)
    Pa = oracle_params(run)
    assert Pa.rho_nu > 0
    rng = np.random.default_rng(11)
    with lattice([run], "fp32", tile=(64, 4), fused=2) as L:
        L.step(5)
        for _ in range(2):
            f_t = L.populations(0)
            L.step(1)
            f_n = L.populations(0)
            film = [int(y) * run.nx + int(x) for y in (100, 101, 102) for x in rng.integers(0, run.nx, 20)]
            idx = np.unique(np.concatenate([_sample(run.nx, run.ny, rng, 2000), film]))
            ref = O.step_sampled(Pa, f_t, idx)
            got = f_n.reshape(9, -1)[:, idx].T
            err = float((np.abs(got - ref) / ref.sum(axis=1, keepdims=True)).max())
            say("  config5 err", err)
            assert err < 2e-6


def _window(run, x0, y0, w, h):
    """The run cut to columns x0 .. x0 + w - 1 (taken periodically) and rows
    y0 .. y0 + h - 1, with the same physics and boundary kinds."""
    xs = np.arange(x0, x0 + w) % run.nx

    def cut(a):
        return None if a is None else np.ascontiguousarray(a[y0:y0 + h][:, xs])

    return dataclasses.replace(run, nx=w, ny=h, rho=cut(run.rho), ux=cut(run.ux), uy=cut(run.uy))


@pytest.mark.parametrize("case", ["config3_wall", "config3_interface", "config5_impact"])
def test_fp64_prefix_at_full_size_against_oracle_window(case):
    """FP64 on the full 4096 x 2048 capillary grid and the 2048 x 1024 splash,
    200 steps from the seeded initial state in the benchmark's launch shape,
    against the oracle run on a window of the same initial field.  A node's
    state after n steps depends only on nodes within 2 n of it (it streams
    from x - e_a, whose collision reads psi at that node's neighbours), so on
    a window reaching 2 n + 2 beyond the compared block the window's own edges
    cannot reach the block, and the oracle computes it exactly; rows at a
    wall of the grid are kept with the wall inside the window."""
    n, b = 200, 200
    m = 2 * n + 2
    if case.startswith("config3"):
        run = WL.config3(256)
        tile, fused = (256, 2), 4
        # 1024 columns (four wavelengths): the window's periodic cut joins
        # equal phases of the wave
        bx0, bw, mx = 1000, b, 412
        by0, bh = (0, b) if case.endswith("wall") else (run.ny // 2 - b // 2, b)
    else:
        run = WL.config5(0.584, 0.6245, 1.7)
        tile, fused = (64, 4), 2
        bx0, bw, by0, bh, mx = run.nx // 2 - b // 2, b, 0, run.ny, m
    assert mx >= m
    wy0, wy1 = max(0, by0 - m), min(run.ny, by0 + bh + m)
    win = _window(run, bx0 - mx, wy0, bw + 2 * mx, wy1 - wy0)
    say("  ", case, "block", (bx0, by0, bw, bh), "window", (win.nx, win.ny))
    with lattice([run], "fp64", tile=tile, fused=fused) as L:
        L.step(n)
        got = L.populations(0)[:, by0:by0 + bh, bx0:bx0 + bw]
    Pw = oracle_params(win)
    ref = O.run(Pw, O.init(Pw, win.rho, win.ux, win.uy), n)[:, by0 - wy0:by0 - wy0 + bh, mx:mx + bw]
    err = rel_err(got, ref)
    say("  ", case, "err", err)
    # round-off of 200 FP64 steps (observed up to 1.3e-14)
    assert err < 1e-12


@pytest.mark.parametrize("case", ["config2", "config4"])
def test_fp64_batched_prefix_against_oracle(case):
    """FP64 batches of the droplet sweep (all 40 runs) and the ensemble (all
    512), stepped in the benchmark's launch shapes, against the oracle on whole
    runs: six of the sweep (R = 20, 40 at kappa = 0, 0.5, 0.95) after 1,000
    steps, and the smallest, the median and the largest ensemble run after 200."""
    if case == "config2":
        runs, tile, fused, n = WL.config2(), (64, 4), 2, 1000
        pick = [i for i, r in enumerate(runs) if r.R0 in (20, 40) and r.kappa in (0.0, 0.5, 0.95)]
    else:
        runs, tile, fused, n = WL.config4(), (128, 2), 4, 200
        order = sorted(range(len(runs)), key=lambda i: runs[i].nodes)
        pick = [order[0], order[len(order) // 2], order[-1]]
    with lattice(runs, "fp64", tile=tile, fused=fused) as L:
        L.step(n)
        got = {i: L.populations(i) for i in pick}
    for i in pick:
        r = runs[i]
        Pa = oracle_params(r)
        ref = O.run(Pa, O.init(Pa, r.rho, r.ux, r.uy), n)
        err = rel_err(got[i], ref)
        say("  ", case, "run", i, (r.nx, r.ny), "err", err)
        # round-off only (observed up to 2.1e-14 after 1,000 steps)
        assert err < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_window_read_back_matches_the_full_read_back(precision):
    """lbm_run_get_window returns the populations of a sub-rectangle, wrapped on
    periodic axes, at either step parity (and writer-referenced bf16)."""
    runs = [small_run(37, 23, "cs", bc_y=W, seed=71), small_run(20, 30, "pw", bc_x=W, seed=72)]
    with lattice(runs, precision) as L:
        for steps in (0, 3, 2):
            L.step(steps)
            for i, r in enumerate(runs):
                full = L.populations(i)
                for x0, y0, w, h in ((0, 0, 5, 4), (r.nx - 3, 2, 7, 5), (4, r.ny - 6, 6, 6), (1, 1, r.nx - 2, 3)):
                    if r.bc_x == W and (x0 + w > r.nx):
                        x0 = r.nx - w
                    if r.bc_y == W and (y0 + h > r.ny):
                        y0 = r.ny - h
                    xs, ys = (np.arange(x0, x0 + w) % r.nx), (np.arange(y0, y0 + h) % r.ny)
                    np.testing.assert_array_equal(L.window(i, x0, y0, w, h), full[:, ys][:, :, xs])
        with pytest.raises(lbm.LbmError):
            L.window(0, 0, runs[0].ny - 2, 4, 4)  # crosses the wall in y


def oracle_window_step(run, win, x0, y0, x, y):
    """f(t+1) at node (x, y) from the window win = f(t) on [x0, x0 + w) x
    [y0, y0 + h) (wrapped on periodic axes, inside the grid on wall axes),
    which reaches at least three nodes beyond (x, y) or to a wall: the oracle
    steps the window as a grid of its own (a node's next state depends on nodes
    within two), walls where the window ends at a real one."""
    h, w = win.shape[1:]
    bcx = W if run.bc_x == W and (x0 == 0 or x0 + w == run.nx) else P
    bcy = W if run.bc_y == W and (y0 == 0 or y0 + h == run.ny) else P
    Pw = oracle_params(run).replace(nx=w, ny=h, bc_x=bcx, bc_y=bcy)
    return O.step(Pw, win)[:, (y - y0) % run.ny, (x - x0) % run.nx]


def test_largest_single_run_beyond_32_bit_offsets():
    """One FP32 run of 16384 x 32768 nodes (537 M): its population block has
    9 N = 4.8e9 elements, past both 2^31 and 2^32, so every direction above
    the first lives at offsets that 32-bit index arithmetic would wrap.  Two
    steps (both parities) on the default schedule; sampled nodes, including
    both walls and the last rows, are checked against the oracle stepping a
    7 x 7 window read back around each (no full-grid copy on the host)."""
    import torch

    nx, ny = 16384, 32768
    free, _ = torch.cuda.mem_get_info()
    if free < 100e9:
        pytest.skip("needs about 80 GB of device memory")
    run = WL.config3(256, nx=nx, ny=ny, kappa=0.5)
    rng = np.random.default_rng(17)
    m = 3
    with lattice([run], "fp32", graph_steps=0) as L:
        L.step(1)
        for _ in range(2):
            idx = _sample(nx, ny, rng, 300)
            idx = np.unique(np.concatenate([idx, (ny - 1) * nx + rng.integers(0, nx, 20),
                                            (ny - 2) * nx + rng.integers(0, nx, 20), rng.integers(0, nx, 20)]))
            wins = []
            for k in idx:
                y, x = divmod(int(k), nx)
                y0, y1 = max(0, y - m), min(ny, y + m + 1)  # walls in y
                wins.append((x, y, x - m, y0, L.window(0, x - m, y0, 2 * m + 1, y1 - y0)))
            L.step(1)
            err = 0.0
            for x, y, x0, y0, win in wins:
                ref = oracle_window_step(run, win, x0, y0, x, y)
                got = L.window(0, x, y, 1, 1)[:, 0, 0]
                err = max(err, float(np.abs(got - ref).max() / ref.sum()))
            say("  16384x32768 err", err, "over", len(wins), "nodes")
            assert err < 2e-6


def test_config4_ensemble_sampled():
    """512 uneven periodic droplets in one batch, the benchmark's launch
    configuration (128 x 2 threads, four nodes each)."""
    runs = WL.config4()
    rng = np.random.default_rng(5)
    with lattice(runs, "fp32", tile=(128, 2), fused=4) as L:
        L.step(20)
        st = L.status()
        say("  config4 diverged after 20 steps:", int(st.sum()))
        for i in rng.choice(len(runs), 6, replace=False):
            if st[i]:
                continue
            f_t = L.populations(int(i))
            L.step(1)
            idx = _sample(runs[i].nx, runs[i].ny, rng, 300)
            ref = O.step_sampled(oracle_params(runs[i]), f_t, idx)
            got = L.populations(int(i)).reshape(9, -1)[:, idx].T
            err = float((np.abs(got - ref) / ref.sum(axis=1, keepdims=True)).max())
            say("  config4 run", int(i), runs[i].nx, "err", err)
            assert err < 2e-6


# ------------------------------------------------------------ bf16 storage

WT = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
EX = [0, 1, 0, -1, 0, 1, -1, -1, 1]
EY = [0, 0, 1, 0, -1, 1, 1, -1, -1]


def writer_density(rho, a, bc_x, bc_y):
    """rho(x - e_a), or rho(x) where x - e_a lies beyond a wall."""
    r = np.roll(rho, (EY[a], EX[a]), axis=(0, 1))
    if bc_y == W:
        if EY[a] > 0:
            r[0, :] = rho[0, :]
        if EY[a] < 0:
            r[-1, :] = rho[-1, :]
    if bc_x == W:
        if EX[a] > 0:
            r[:, 0] = rho[:, 0]
        if EX[a] < 0:
            r[:, -1] = rho[:, -1]
    return r


@pytest.mark.parametrize("kind", ["cs", "pw"])
def test_bf16_step_from_common_state(kind):
    """bf16 storage keeps f_a - w_a rho_w, rho_w the density of the node that
    wrote the population (its upwind node at the previous step).  One step
    from a common state: the stored deviations carry 8 significant bits, so
    the error is bounded by a few bf16 ulps of the largest deviation d_a
    (measured on the oracle's own states) plus FP32 round-off."""
    run = small_run(48, 40, kind, kappa=0.7, bc_y=W, seed=15)
    Pa = oracle_params(run)
    f_t = O.run(Pa, O.init(Pa, run.rho), 9)
    f_n = O.step(Pa, f_t)
    rho_t = f_t.sum(axis=0)
    d = np.stack([f_n[a] - WT[a] * writer_density(rho_t, a, run.bc_x, run.bc_y) for a in range(9)])
    bound = 4 * 2.0 ** -8 * np.abs(d).max() + 2e-6 * rho_t.max()
    with lattice([run], "bf16", graph_steps=0) as L:
        for parity in (0, 1):
            if L.steps_taken % 2 != parity:
                L.step(1)
            L.set_populations(0, f_t)
            back = L.populations(0)
            L.step(1)
            got = L.populations(0)
            err = np.abs(got - f_n).max()
            say("  bf16", kind, "parity", parity, "err", err, "bound", bound, "max|d|", np.abs(d).max(),
                "re-encode err", np.abs(back - f_t).max())
            assert err < bound


def test_bf16_graph_eager_and_checkpoint_are_bitwise():
    """Stochastic rounding draws its bits from a counter hash of (step, node,
    direction): graph replay and eager launches give the same bits, and a
    restart from a checkpoint continues bit for bit."""
    runs = [small_run(50, 30, "pw", bc_y=W, seed=12), small_run(37, 20, "cs", seed=13)]
    out = []
    for k in (0, 3):
        with lattice(runs, "bf16", graph_steps=k) as L:
            L.step(21)
            out.append([L.populations(i) for i in range(len(runs))])
    for u, v in zip(*out):
        np.testing.assert_array_equal(u, v)
    with lattice(runs, "bf16", graph_steps=2) as L:
        L.step(11)
        blob = L.save_state()
        L.step(10)
        a = [L.populations(i) for i in range(len(runs))]
        L.load_state(blob)
        L.step(10)
        for i in range(len(runs)):
            np.testing.assert_array_equal(a[i], L.populations(i))
        np.testing.assert_array_equal(a[0], out[0][0])


def test_bf16_rejects_constant_base():
    run = small_run(20, 12, "cs", seed=5)
    with lattice([run], "bf16") as L:
        with pytest.raises(lbm.LbmError):
            L.set_reference_density(0, 0.1)
        with pytest.raises(lbm.LbmError):
            L.set_fused(3)


@pytest.mark.parametrize("fused", [1, 2, 4])
def test_bf16_fused_matches_two_kernel_bitwise(fused):
    """The fused kernel decodes halo populations with writer densities staged
    with an H + 1 halo (across a wall centred on the clamped boundary node),
    derives each step's rounding seed as the psi pass does and writes its
    nodes' densities for the next step: the same bits as psi pass + collide,
    over walls on both axes, periodic wraps, grids smaller than a tile, a
    multi-range run (two-node halo), graph replay and mid-run switches."""
    mr = WL.paper_multirange_run("C", n=40, R=12.0)
    mr.rho = mr.rho * (1 + WL.noise(mr.rho.shape, 1e-3, 7))
    mr.bc_x, mr.bc_y = W, P
    runs = [small_run(50, 30, "pw", bc_x=W, bc_y=W, seed=12), small_run(37, 20, "cs", seed=13),
            small_run(5, 70, "pw", bc_y=W, seed=2), small_run(70, 9, "exp", bc_x=W, bc_y=W, seed=10)]

    def go(rs, tile, fu, gk, chunks):
        with lattice(rs, "bf16", tile=tile, graph_steps=gk, fused=fu) as L:
            for n in chunks:
                L.step(n)
            return [L.populations(i) for i in range(len(rs))]

    for rs in (runs, runs[:2] + [mr]):
        ref = go(rs, (64, 4), 0, 0, (23,))
        for tile, gk, chunks in [((64, 4), 3, (23,)), ((32, 2), 0, (1, 22)), ((128, 2), 2, (7, 16)),
                                 ((128, 4), 2, (7, 16))]:
            for u, v in zip(ref, go(rs, tile, fused, gk, chunks)):
                np.testing.assert_array_equal(u, v)
    # switching schedules mid-run and a checkpoint taken under the fused one
    with lattice(runs, "bf16", graph_steps=2, fused=fused) as L:
        L.step(9)
        blob = L.save_state()
        L.set_fused(0)
        L.step(5)
        L.set_fused(fused)
        L.step(9)
        a = [L.populations(i) for i in range(len(runs))]
    for u, v in zip(go(runs, (64, 4), 0, 2, (23,)), a):
        np.testing.assert_array_equal(u, v)
    with lattice(runs, "bf16", fused=0) as L:
        L.load_state(blob)
        L.step(14)
        for i in range(len(runs)):
            np.testing.assert_array_equal(L.populations(i), a[i])


def test_bf16_mass_and_phase_survive_long_runs():
    """A droplet with walls in bf16 for 4,000 steps: mass within 1e-4 and bulk
    densities within 0.5% of FP64 (stochastic rounding has zero mean)."""
    run = small_run(96, 80, "cs", kappa=0.5, bc_y=W, seed=8, noise=1e-6, R=24)
    res = {}
    for prec in ("fp64", "bf16"):
        with lattice([run], prec) as L:
            L.step(4000)
            res[prec] = L.diagnostics([(run.cx, run.cy, *run.diag_radii())])[0]
    a, b = res["fp64"], res["bf16"]
    say("  bf16 vs fp64: mass", b["mass"] / a["mass"] - 1, "rho_in", b["rho_in"] / a["rho_in"] - 1,
        "rho_out", b["rho_out"] / a["rho_out"] - 1)
    assert abs(b["mass"] / a["mass"] - 1) < 1e-4
    assert abs(b["rho_in"] / a["rho_in"] - 1) < 5e-3
    assert abs(b["rho_out"] / a["rho_out"] - 1) < 5e-3


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
def test_density_column_matches_moments(precision):
    """lbm_run_density_column decodes the storage like lbm_run_moments."""
    runs = [small_run(40, 24, "cs", bc_y=W, seed=9), small_run(30, 50, "pw", seed=10)]
    with lattice(runs, precision) as L:
        for n in (3, 4):  # both parities
            L.step(n)
            for i, r in enumerate(runs):
                rho = L.moments(i)[0]
                for x in (0, r.nx // 2, r.nx - 1):
                    np.testing.assert_allclose(L.density_column(i, x), rho[:, x], rtol=1e-12)


@pytest.mark.parametrize("fused", [0, 1])
def test_step_viscosity_matches_oracle(fused):
    """Section V.C step-function viscosity (nu_V below the threshold): FP64
    against the oracle step by step, both schedules."""
    run = small_run(40, 30, "pw", kappa=0.3, bc_y=W, seed=17)
    run.rho_nu, run.s_nu_low = 10.0, WL.s_nu(0.2)
    Pa = oracle_params(run)
    assert Pa.rho_nu == 10.0
    f = O.init(Pa, run.rho)
    with lattice([run], "fp64", fused=fused, graph_steps=0) as L:
        for k in range(4):
            L.step(1)
            f = O.step(Pa, f)
            assert rel_err(L.populations(0), f) < 1e-13, k


@pytest.mark.parametrize("fused", [0, 1], ids=["twokernel", "fused"])
@pytest.mark.parametrize("bc", [(P, P), (P, W), (W, W)], ids=["periodic", "walls_y", "walls_xy"])
def test_multirange_force_matches_oracle(bc, fused):
    """Eq. (9) multi-range force (two-node psi halo in the collide tile; psi
    beyond a wall clamped to the boundary node): FP64 against the oracle step by
    step, also with an ordinary run in the same batch, under both schedules."""
    mr = WL.paper_multirange_run("C", n=40, R=12.0)
    mr.rho = mr.rho * (1 + WL.noise(mr.rho.shape, 1e-3, 7))
    mr.bc_x, mr.bc_y = bc
    plain = small_run(33, 21, "exp", kappa=0.0, bc_y=bc[1], seed=8)
    runs = [mr, plain]
    Ps = [oracle_params(r) for r in runs]
    assert Ps[0].G2 != 0.0
    fs = [O.init(Pa, r.rho) for Pa, r in zip(Ps, runs)]
    with lattice(runs, "fp64", graph_steps=0, fused=fused) as L:
        for k in range(4):
            L.step(1)
            for i in range(2):
                fs[i] = O.step(Ps[i], fs[i])
                assert rel_err(L.populations(i), fs[i]) < 1e-13, (k, i)
        rho, ux, uy = L.moments(0)
        ro, uxo, uyo = O.moments(Ps[0], fs[0])
        assert np.abs(ux - uxo).max() < 1e-12 * max(np.abs(uxo).max(), 1e-30) + 1e-16
