"""Invariants the equations fix, checked on the oracle (CPU only).

* a uniform fluid at rest stays at rest (uniform psi => F = Q = 0, Eqs. 7, 19);
* mass is conserved (S0 = C0 = 0 in Eqs. 5, 18) with periodic and wall boundaries;
* total momentum is conserved on a periodic grid (pairwise antisymmetry of Eq. 7,
  and j* = j + F by Eqs. 2, 5, 6);
* the rates of the conserved moments do not matter (Eqs. 2, 6);
* a centred droplet keeps the D4 symmetry of the lattice (Eqs. 7, 19);
* the sampled single-node step agrees with the full step;
* information travels at most two nodes per step (streaming from x - e_a, whose
  collision reads psi at its own neighbours), so a window of the initial field
  with a margin of 2 n + 2 gives the same state after n steps;
* the step-function viscosity of Section V.C relaxes the stress moments at the
  rate of the density's side of the threshold (shear-wave decay at nu k^2);
* the diagnostics return the known values of a top-hat disk and a uniform flow.
"""
import numpy as np
import pytest

import oracle as O
from oracle import theory

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)

RHO_C, T_C = theory.critical_point(0.25, 4.0, 1.0)


def cs(nx, ny, kappa=0.0, eps=1.93, tr=0.7, **kw):
    return O.Params(nx=nx, ny=ny, eos_kind=O.EOS_CS, eos=(0.25, 4.0, 1.0, tr * T_C), G=-1.0,
                    kappa=kappa, sigma=O.sigma_from_epsilon(eps, -1.0), **kw)


def piecewise(nx, ny, kappa=0.0, **kw):
    return O.Params(nx=nx, ny=ny, eos_kind=O.EOS_PIECEWISE,
                    eos=(0.49 / 3, -0.06 / 3, 1 / 3, 1.49, 94.65), G=-1.0, sigma=0.087,
                    kappa=kappa, **kw)


def expo(nx, ny, kappa=0.0, **kw):
    return O.Params(nx=nx, ny=ny, eos_kind=O.EOS_EXP, eos=(4.0, 200.0), G=-40.0, kappa=kappa, **kw)


def droplet_rho(P, rl, rv, R, seed=None, amp=0.0, W=5.0):
    y, x = np.mgrid[0:P.ny, 0:P.nx]
    r = np.hypot(x - P.nx / 2, y - P.ny / 2)
    rho = (rl + rv) / 2 - (rl - rv) / 2 * np.tanh(2 * (r - R) / W)
    if seed is not None:
        rho = rho + np.random.default_rng(seed).uniform(-amp, amp, rho.shape)
    return rho


@pytest.mark.parametrize("make,rho0", [(cs, 0.2), (piecewise, 30.0), (expo, 300.0)])
@pytest.mark.parametrize("walls", [False, True])
def test_uniform_rest_state_stays_at_rest(make, rho0, walls):
    P = make(9, 7, kappa=0.6, bc_y=O.BC_WALL if walls else O.BC_PERIODIC)
    f = O.init(P, np.full((7, 9), rho0))
    f2 = O.run(P, f, 2000)
    rho, ux, uy = O.moments(P, f2)
    assert np.abs(rho - rho0).max() <= 1e-13 * rho0
    assert max(np.abs(ux).max(), np.abs(uy).max()) <= 1e-15


@pytest.mark.parametrize("walls", [False, True])
def test_mass_conservation(walls):
    P = cs(40, 36, kappa=0.5, bc_y=O.BC_WALL if walls else O.BC_PERIODIC)
    f = O.init(P, droplet_rho(P, 0.358, 0.0093, 10, seed=11, amp=1e-3))
    m0 = f.sum()
    f = O.run(P, f, 300)
    assert abs(f.sum() - m0) <= 1e-13 * m0


def test_momentum_conservation_periodic():
    P = piecewise(33, 30, kappa=0.3)
    rng = np.random.default_rng(7)
    rho = droplet_rho(P, 100.0, 1.0, 9) + rng.uniform(-0.05, 0.05, (30, 33))
    ux = rng.uniform(-0.01, 0.01, rho.shape)
    f = O.init(P, rho, ux, None)
    j0 = np.array([np.tensordot(EX, f, 1).sum(), np.tensordot(EY, f, 1).sum()])
    for _ in range(5):
        f = O.run(P, f, 40)
        j = np.array([np.tensordot(EX, f, 1).sum(), np.tensordot(EY, f, 1).sum()])
        assert np.abs(j - j0).max() <= 1e-12 * f.sum()


def test_conserved_moment_rates_do_not_matter():
    base = cs(24, 20, kappa=0.4)
    P1 = base.replace(s=O.rates(s_rho=1.0, s_j=1.0))
    P2 = base.replace(s=O.rates(s_rho=0.37, s_j=1.61))
    f = O.init(P1, droplet_rho(P1, 0.358, 0.0093, 6, seed=3, amp=1e-3))
    a = O.run(P1, f, 200)
    b = O.run(P2, f, 200)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=0)


def test_centred_droplet_keeps_lattice_symmetry():
    P = piecewise(32, 32, kappa=0.5)
    f = O.run(P, O.init(P, droplet_rho(P, 100.0, 1.0, 8)), 300)
    rho, _, _ = O.moments(P, f)
    # the centre is node (16, 16): mirror x -> 32 - x (mod 32), and transpose
    mirror = np.roll(rho[:, ::-1], 1, axis=1)
    np.testing.assert_allclose(mirror, rho, rtol=1e-11)
    np.testing.assert_allclose(rho.T, rho, rtol=1e-11)


@pytest.mark.parametrize("walls", [False, True])
def test_state_after_n_steps_depends_on_a_2n_neighbourhood(walls):
    n, b = 12, 10
    m = 2 * n + 2
    bcy = O.BC_WALL if walls else O.BC_PERIODIC
    P = cs(90, 80, kappa=0.5, tr=0.6, bc_y=bcy, rho_nu=0.2, s_nu_low=1.2)
    rho = droplet_rho(P, 0.41, 0.003, 14, seed=3, amp=1e-3)
    uy = -0.05 * (rho > 0.2)
    full = O.run(P, O.init(P, rho, None, uy), n)
    # a block in the interior and, with walls, one at the bottom wall (its
    # window from row 0); the window's own cut edges are walls
    blocks = [(30, 35, 35 - m)] + ([(40, 0, 0)] if walls else [])
    for bx0, by0, wy0 in blocks:
        W = cs(b + 2 * m, b + m + (by0 - wy0), kappa=0.5, tr=0.6, bc_y=O.BC_WALL, rho_nu=0.2, s_nu_low=1.2)
        xs = np.arange(bx0 - m, bx0 + b + m) % P.nx
        cut = lambda a: np.ascontiguousarray(a[wy0:wy0 + W.ny][:, xs])
        win = O.run(W, O.init(W, cut(rho), None, cut(uy)), n)
        got = win[:, by0 - wy0:by0 - wy0 + b, m:m + b]
        np.testing.assert_array_equal(got, full[:, by0:by0 + b, bx0:bx0 + b])
    # a margin two nodes short of the reach differs
    W = cs(b + 2 * (m - 4), P.ny, kappa=0.5, tr=0.6, bc_y=bcy, rho_nu=0.2, s_nu_low=1.2)
    xs = np.arange(40 - (m - 4), 40 + b + m - 4) % P.nx
    short = O.run(W, O.init(W, np.ascontiguousarray(rho[:, xs]), None, np.ascontiguousarray(uy[:, xs])), n)
    assert np.abs(short[:, :, m - 4:m - 4 + b] - full[:, :, 40:40 + b]).max() > 0


@pytest.mark.parametrize("walls", [False, True])
def test_sampled_step_matches_full_step(walls):
    P = piecewise(17, 12, kappa=0.7, bc_y=O.BC_WALL if walls else O.BC_PERIODIC)
    f = O.run(P, O.init(P, droplet_rho(P, 100.0, 1.0, 4, seed=5, amp=0.01)), 20)
    g = O.step(P, f)
    idx = np.array([0, 16, 17 * 11, 17 * 12 - 1, 5 * 17 + 8, 17 + 3])
    out = O.step_sampled(P, f, idx)
    ref = g.reshape(9, -1)[:, idx].T
    np.testing.assert_array_equal(out, ref)


def test_oracle_rejects_undefined_psi():
    # T above the range where p_EOS < rho cs^2 for this density: psi is not real
    P = cs(4, 4, tr=0.7)
    f = O.init(P, np.full((4, 4), 0.9999))
    with pytest.raises(O.OracleError):
        O.step(P, f)


# ------------------------------------- step-function viscosity (Section V.C)

def _shear_wave_decay(rho0, rho_nu, s_nu, s_nu_low, t1=200, t2=2000, ny=64):
    """Decay rate of u_x = U sin(k y) in a uniform fluid (no interaction force:
    psi is uniform, so F = Q = 0), between t1 and t2 so that the start-up
    transient of the equilibrium initial state drops out."""
    P = piecewise(4, ny, s=O.rates(s_nu=s_nu), rho_nu=rho_nu, s_nu_low=s_nu_low)
    y = np.arange(ny)[:, None] * np.ones((1, 4))
    U = 1e-3
    f = O.init(P, np.full((ny, 4), rho0), U * np.sin(2 * np.pi * y / ny), np.zeros((ny, 4)))
    sk = np.sin(2 * np.pi * np.arange(ny) / ny)
    f = O.run(P, f, t1)
    a1 = np.sum(O.moments(P, f)[1][:, 0] * sk)
    f = O.run(P, f, t2 - t1)
    a2 = np.sum(O.moments(P, f)[1][:, 0] * sk)
    return np.log(a1 / a2) / (t2 - t1), (2 * np.pi / ny) ** 2


def test_step_viscosity_picks_the_rate_by_density():
    """A shear wave decays at nu k^2 with nu = (1/s_nu - 1/2)/3: the low-density
    rate below the threshold, the other at or above it, the plain rate when the
    step is off.  Densities on the stable branches of Eq. (23) (vapour 1,
    liquid 100)."""
    s_l, s_v = 1.0 / (3 * 0.01 + 0.5), 1.0 / (3 * 0.2 + 0.5)
    nu = {s: (1.0 / s - 0.5) / 3.0 for s in (s_l, s_v)}
    for rho0, rho_nu, expect in ((1.0, 1.49, s_v), (100.0, 1.49, s_l), (1.0, 0.5, s_l), (100.0, 200.0, s_v),
                                 (1.0, 0.0, s_l)):
        rate, k2 = _shear_wave_decay(rho0, rho_nu, s_l, s_v)
        assert rate == pytest.approx(nu[expect] * k2, rel=5e-3), (rho0, rho_nu)


def test_step_viscosity_off_is_the_plain_step():
    P = piecewise(24, 20, kappa=0.4)
    y, x = np.mgrid[0:20, 0:24].astype(float)
    rho = 50.5 - 49.5 * np.tanh(2 * (np.hypot(x - 12, y - 10) - 6) / 5.0)
    f = O.init(P, rho)
    a = O.step(P, f)
    b = O.step(P.replace(rho_nu=0.0, s_nu_low=1.7), f)
    np.testing.assert_array_equal(a, b)
    # with the step on, only nodes below the threshold change
    c = O.step(P.replace(rho_nu=10.0, s_nu_low=1.7), f)
    low = f.sum(axis=0) < 10.0
    assert np.abs(c - a).max() > 0
    # a node's collision changes only if it is below the threshold; its
    # populations then stream to the neighbours (Eq. 4)
    changed = (np.abs(c - a) > 0).any(axis=0)
    near = low | np.roll(low, 1, 0) | np.roll(low, -1, 0) | np.roll(low, 1, 1) | np.roll(low, -1, 1) \
        | np.roll(np.roll(low, 1, 0), 1, 1) | np.roll(np.roll(low, 1, 0), -1, 1) \
        | np.roll(np.roll(low, -1, 0), 1, 1) | np.roll(np.roll(low, -1, 0), -1, 1)
    assert not (changed & ~near).any()


@pytest.mark.parametrize("walls", [False, True])
def test_diagnostics_of_a_top_hat_disk_and_a_uniform_flow(walls):
    """The FP64 diagnostics (Section V.A's Laplace-law inputs) on fields whose
    values are known: a disk of density rho_l in rho_v gives the two densities
    as region means, p_in - p_out from the EOS of each, the mass by counting
    nodes, and R_eq = sqrt(nodes of the disk / pi); a uniform flow at rest
    density gives |u| as the largest speed (uniform psi, so F = 0 in Eq. 6)."""
    bcy = O.BC_WALL if walls else O.BC_PERIODIC
    P = cs(64, 48, bc_y=bcy)
    rl, rv, R, cx, cy = 0.36, 0.009, 11.5, 30.0, 25.0
    y, x = np.mgrid[0:P.ny, 0:P.nx]
    dx = np.abs(x - cx)
    dx = np.minimum(dx, P.nx - dx)
    dy = np.abs(y - cy) if walls else np.minimum(np.abs(y - cy), P.ny - np.abs(y - cy))
    inside = np.hypot(dx, dy) <= R
    rho = np.where(inside, rl, rv)
    d = O.diagnostics(P, O.init(P, rho), cx, cy, R / 2, R + 4)
    n_in = int(inside.sum())
    pl, _ = O.eos(P, np.array([rl]))
    pv, _ = O.eos(P, np.array([rv]))
    assert d["mass"] == pytest.approx(n_in * rl + (P.nx * P.ny - n_in) * rv, rel=1e-12)
    assert d["rho_in"] == pytest.approx(rl, rel=1e-12) and d["rho_out"] == pytest.approx(rv, rel=1e-12)
    assert d["dp"] == pytest.approx(pl[0] - pv[0], rel=1e-12)
    assert d["r_eq"] == pytest.approx(np.sqrt(n_in / np.pi), rel=1e-12)
    u = (0.031, -0.017)
    f = O.init(P, np.full((P.ny, P.nx), 0.2), np.full((P.ny, P.nx), u[0]), np.full((P.ny, P.nx), u[1]))
    d = O.diagnostics(P, f, cx, cy, 4, 20)
    assert d["max_speed"] == pytest.approx(np.hypot(*u), rel=1e-12)
