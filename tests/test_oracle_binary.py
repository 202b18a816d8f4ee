"""Pins of the two-component oracle (CPU only).

Each test checks the oracle against something other than itself: textbook
velocity-space forms (the second-order equilibrium, BGK with Guo forcing, the
Hermite form of a momentum-flux shift), closed forms of the lattice sums for a
sinusoidal psi, conservation laws, the A <-> B symmetry of the model, the
spinodal that the model's bulk pressure p = rho/3 + G rho_A rho_B fixes
(G^2 rho_A rho_B = 1/9, i.e. G rho = 2/3 for a 50/50 mixture), and the two
properties the two-component form of the source term is derived to have:
flat-interface compositions that do not move with kappa, and a Laplace
tension proportional to 1 - kappa (the two-component Eq. 22).
"""
import numpy as np
import pytest

from oracle import binary as B

EX, EY = B.EX.astype(float), B.EY.astype(float)
W_EQ = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
W_INT = np.array([0.0] + [1 / 3] * 4 + [1 / 12] * 4)


def textbook_feq(rho, u):
    eu = EX * u[0] + EY * u[1]
    return W_EQ * rho * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * (u[0] ** 2 + u[1] ** 2))


def textbook_guo(u, F):
    eu = EX * u[0] + EY * u[1]
    eF = EX * F[0] + EY * F[1]
    return W_EQ * (3 * ((EX - u[0]) * F[0] + (EY - u[1]) * F[1]) + 9 * eu * eF)


def hermite_shift(dxx, dyy, dxy):
    # second-order equilibrium change for a momentum-flux shift: w (9/2) dPi : (e e - I/3)
    return W_EQ * 4.5 * (dxx * (EX * EX - 1 / 3) + dyy * (EY * EY - 1 / 3) + 2 * dxy * EX * EY)


def params(**kw):
    base = dict(nx=8, ny=6, G=1.0, s=B.rates(), kappa=0.0)
    base.update(kw)
    return B.ParamsMC(**base)


def test_matrix_inverse():
    M, Mi = B.matrices()
    np.testing.assert_allclose(M @ Mi, np.eye(9), atol=1e-14)


def test_unit_rates_relax_to_the_textbook_equilibrium():
    """All rates 1, no force, no source: f* = f_eq(rho_s, u), so Eq. (3) and M
    are the textbook D2Q9 equilibrium."""
    P = params(s=(1.0,) * 9)
    rng = np.random.default_rng(3)
    f = 0.1 + rng.random(9) * 0.05
    u = np.array([0.03, -0.05])
    got = B.collide_node(P, f, u, np.zeros(2), np.zeros(3))
    np.testing.assert_allclose(got, textbook_feq(f.sum(), u), atol=1e-15)


@pytest.mark.parametrize("s", [0.7, 1.3])
def test_equal_rates_give_bgk_with_guo_forcing(s):
    """Equal rates: f* = f - s (f - f_eq(rho_s, u)) + (1 - s/2) F_Guo(u, F_s),
    the mixture velocity u in both (Eq. 5 and the (I - Lambda/2) factor)."""
    P = params(s=(s,) * 9)
    rng = np.random.default_rng(4)
    f = 0.1 + rng.random(9) * 0.05
    u, F = np.array([0.02, 0.04]), np.array([-0.003, 0.007])
    got = B.collide_node(P, f, u, F, np.zeros(3))
    want = f - s * (f - textbook_feq(f.sum(), u)) + (1 - s / 2) * textbook_guo(u, F)
    np.testing.assert_allclose(got, want, atol=1e-15)


@pytest.mark.parametrize("q", [(1e-3, -2e-3, 5e-4), (0.0, 0.0, -7e-4), (3e-3, 3e-3, 0.0)])
def test_source_term_is_the_flux_shift_three_quarters_trace_minus_q(q):
    """With equal rates s the source of Eq. (18) adds s times the Hermite
    equilibrium change for the flux shift dPi = (3/4) tr(Q) I - Q."""
    s = 1.1
    P = params(s=(s,) * 9)
    rng = np.random.default_rng(5)
    f = 0.1 + rng.random(9) * 0.05
    u, F = np.array([0.01, -0.02]), np.array([0.002, 0.001])
    Q = np.array(q)
    d = B.collide_node(P, f, u, F, Q) - B.collide_node(P, f, u, F, np.zeros(3))
    tr = Q[0] + Q[1]
    want = s * hermite_shift(0.75 * tr - Q[0], 0.75 * tr - Q[1], -Q[2])
    np.testing.assert_allclose(d, want, atol=1e-16)


@pytest.mark.parametrize("kx,ky,theta", [(0.3, 0.0, 0.2), (0.5, -0.7, 1.1), (2.0, 1.3, -0.4)])
def test_force_and_source_exact_for_a_sinusoidal_partner(kx, ky, theta):
    """psi_o = A + B cos(k.x + theta) around the node: the lattice sums have
    closed forms (sum w sin(k.e) e_x = (2/3) sin kx + (1/3) sin kx cos ky,
    sum w (cos(k.e) - 1) e_x e_x = (2/3)(cos kx - 1) + (1/3)(cos kx cos ky - 1),
    sum w (cos(k.e) - 1) e_x e_y = -(1/3) sin kx sin ky)."""
    G, kappa, Av, Bv, psi_s = 1.3, 0.6, 0.5, 0.2, 0.8
    P = params(G=G, kappa=kappa)
    psi_o = Av + Bv * np.cos(kx * EX + ky * EY + theta)
    F, Q = B.force_and_q(P, psi_s, psi_o)
    gx = (2 / 3) * np.sin(kx) + (1 / 3) * np.sin(kx) * np.cos(ky)
    gy = (2 / 3) * np.sin(ky) + (1 / 3) * np.sin(ky) * np.cos(kx)
    # sum w psi_o(x + e) e = -B sin(theta) (gx, gy)
    np.testing.assert_allclose(F, -G * psi_s * (-Bv * np.sin(theta)) * np.array([gx, gy]), atol=1e-15)
    qxx = (2 / 3) * (np.cos(kx) - 1) + (1 / 3) * (np.cos(kx) * np.cos(ky) - 1)
    qyy = (2 / 3) * (np.cos(ky) - 1) + (1 / 3) * (np.cos(kx) * np.cos(ky) - 1)
    qxy = -(1 / 3) * np.sin(kx) * np.sin(ky)
    k = kappa * G / 2 * psi_s * Bv * np.cos(theta)
    np.testing.assert_allclose(Q, k * np.array([qxx, qyy, qxy]), atol=1e-15)


@pytest.mark.parametrize("ma,mb,tha,thb", [((1, 0), (0, 1), 0.3, -0.8), ((2, -1), (1, 2), 1.1, 0.4),
                                             ((3, 1), (-2, 1), -2.0, 2.5)])
def test_eq6_mixture_velocity_of_resting_sinusoidal_densities(ma, mb, tha, thb):
    """Eq. (6) for the mixture: (rho_A + rho_B) u = sum_s (sum_a e_a f^s_a +
    F_s / 2).  On rest equilibria the sums vanish, so u = (F_A + F_B) / (2 rho)
    with each F_s of Eq. (7) in closed form from the partner's sinusoidal
    density (psi_s = rho_s).  Dropping either force, halving them or flipping
    their sign fails here; the diagnostics' largest speed is the largest
    |u|."""
    G, nx, ny = 1.3, 24, 18
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    ka = 2 * np.pi * np.array([ma[0] / nx, ma[1] / ny])
    kb = 2 * np.pi * np.array([mb[0] / nx, mb[1] / ny])
    pha, phb = tha + ka[0] * x + ka[1] * y, thb + kb[0] * x + kb[1] * y
    rhoA, rhoB = 0.5 + 0.2 * np.cos(pha), 0.6 + 0.25 * np.cos(phb)
    P = params(nx=nx, ny=ny, G=G, kappa=0.6)
    f = B.init(P, rhoA, rhoB)
    a, b, ux, uy = B.moments(P, f)
    np.testing.assert_allclose(a, rhoA, rtol=1e-14)
    np.testing.assert_allclose(b, rhoB, rtol=1e-14)

    def g(k):  # sum_a w_a sin(k.e_a) e_a
        return np.array([(2 / 3) * np.sin(k[0]) + (1 / 3) * np.sin(k[0]) * np.cos(k[1]),
                         (2 / 3) * np.sin(k[1]) + (1 / 3) * np.sin(k[1]) * np.cos(k[0])])

    FA = [-G * rhoA * (-0.25 * np.sin(phb)) * gi for gi in g(kb)]  # A feels B's psi
    FB = [-G * rhoB * (-0.2 * np.sin(pha)) * gi for gi in g(ka)]
    assert np.abs(np.array(FA)).max() > 0.05 and np.abs(np.array(FB)).max() > 0.05  # both forces matter
    rho = rhoA + rhoB
    np.testing.assert_allclose(ux, (FA[0] + FB[0]) / (2 * rho), rtol=1e-11, atol=1e-16)
    np.testing.assert_allclose(uy, (FA[1] + FB[1]) / (2 * rho), rtol=1e-11, atol=1e-16)
    d = B.diagnostics(P, f, nx / 2, ny / 2, 2.0, 6.0)
    speed = np.hypot(FA[0] + FB[0], FA[1] + FB[1]) / (2 * rho)
    assert d["max_speed"] == pytest.approx(float(speed.max()), rel=1e-11)


def _mixture(P, seed, noise=1e-2):
    rng = np.random.default_rng(seed)
    rA = 0.5 + noise * rng.standard_normal(P.shape)
    rB = 0.55 + noise * rng.standard_normal(P.shape)
    return rA, rB


@pytest.mark.parametrize("bc", [(0, 0), (1, 0), (1, 1)])
def test_masses_conserved_and_periodic_momentum_exact(bc):
    """Each component's mass is conserved with any boundaries; on a periodic
    box the cross forces cancel in sum (Newton's third law of Eq. 7's pair
    interaction), so the total momentum of the Eq. (6) velocity stays zero."""
    P = params(nx=12, ny=10, G=1.1, kappa=0.7, bc_x=bc[0], bc_y=bc[1])
    rA, rB = _mixture(P, 7)
    f0 = B.init(P, rA, rB)
    f = B.run(P, f0, 120)
    np.testing.assert_allclose(f.sum(axis=(1, 2, 3)), f0.sum(axis=(1, 2, 3)), rtol=1e-13)
    if bc == (0, 0):
        a, b, ux, uy = B.moments(P, f)
        rho = a + b
        assert abs((rho * ux).sum()) < 1e-12 and abs((rho * uy).sum()) < 1e-12


@pytest.mark.parametrize("bc", [(0, 0), (1, 1)])
def test_uniform_mixture_stays_at_rest(bc):
    P = params(nx=7, ny=5, G=0.5, kappa=0.9, bc_x=bc[0], bc_y=bc[1])
    rA, rB = np.full(P.shape, 0.3), np.full(P.shape, 0.6)
    f0 = B.init(P, rA, rB)
    np.testing.assert_allclose(B.run(P, f0, 100), f0, rtol=1e-13, atol=0)


def test_swapping_the_components_swaps_the_result():
    """The model is symmetric under A <-> B (same rates, cross interaction only)."""
    P = params(nx=10, ny=9, G=1.2, kappa=0.4, bc_y=1)
    rA, rB = _mixture(P, 9, noise=0.05)
    fa = B.run(P, B.init(P, rA, rB), 40)
    fb = B.run(P, B.init(P, rB, rA), 40)
    np.testing.assert_allclose(fa[::-1], fb, rtol=1e-12, atol=1e-15)


def _composition_amplitude(G, L=32, steps=4000, d=1e-3):
    P = params(nx=L, ny=1, G=G)
    x = np.arange(L)
    w = d * np.cos(2 * np.pi * x / L)
    f = B.run(P, B.init(P, (0.5 + w)[None, :], (0.5 - w)[None, :]), steps)
    a, b, _, _ = B.moments(P, f)
    return np.abs(np.fft.rfft(a[0] - b[0])[1]) / L / d


@pytest.mark.parametrize("G,grows", [(0.5, False), (0.64, False), (0.7, True), (0.8, True)])
def test_spinodal_of_the_equal_mixture(G, grows):
    """p = rho/3 + G rho_A rho_B makes a uniform mixture unstable to
    composition waves when G^2 rho_A rho_B > 1/9: at rho_A = rho_B = 1/2,
    G > 2/3 (a wave of length 32 raises that by a factor k / sin k < 1.01)."""
    amp = _composition_amplitude(G)
    assert (amp > 1.5) if grows else (amp < 0.5), amp


def _slab(kappa, G=1.0, ny=64, steps=8000):
    P = params(nx=1, ny=ny, G=G, kappa=kappa)
    y = np.arange(ny)
    prof = 0.5 * (np.tanh((y - ny / 4) / 2) - np.tanh((y - 3 * ny / 4) / 2))
    f = B.run(P, B.init(P, (0.05 + 0.95 * prof)[:, None], (0.05 + 0.95 * (1 - prof))[:, None]), steps)
    a, _, _, uy = B.moments(P, f)
    return a[ny // 2, 0], a[0, 0], np.abs(uy).max()


def test_flat_interface_compositions_do_not_move_with_kappa():
    """The flux shift has no normal-normal part on a flat interface, so the
    bulk compositions of a settled slab stay as at kappa = 0 (to the
    neglected higher-order terms) while the tension changes."""
    base = _slab(0.0)
    for kappa in (0.5, 0.9):
        maj, mino, u = _slab(kappa)
        assert maj == pytest.approx(base[0], rel=5e-4)
        assert mino == pytest.approx(base[1], rel=5e-3)
        assert u < 1e-6
    # phase separation happened: a rich and a lean phase
    assert base[0] > 1.0 and base[1] < 0.06


def _drop_sigma(kappa, n=64, R=16, G=1.0, steps=5000):
    P = params(nx=n, ny=n, G=G, kappa=kappa)
    y, x = np.mgrid[0:n, 0:n]
    prof = 0.5 * (1 - np.tanh((np.hypot(x - n / 2, y - n / 2) - R) / 2))
    f = B.run(P, B.init(P, 0.05 + 0.95 * prof, 0.05 + 0.95 * (1 - prof)), steps)
    d = B.diagnostics(P, f, n / 2, n / 2, R / 4, R + 8)
    return d["dp"] * d["r_eq"], d


def test_laplace_tension_scales_with_one_minus_kappa():
    """A drop of A in B: sigma = dp R_eq scales as 1 - kappa (the two-component
    form of Eq. 22), and the drop's composition barely moves."""
    s0, d0 = _drop_sigma(0.0)
    for kappa in (0.5, 0.9):
        s, d = _drop_sigma(kappa)
        assert s / s0 == pytest.approx(1 - kappa, abs=0.01 * (1 - kappa) + 2e-3)
        assert d["rhoA_in"] == pytest.approx(d0["rhoA_in"], rel=1e-2)
    assert s0 > 0.03 and d0["rhoA_in"] > 1.0 and d0["rhoA_out"] < 0.06


def test_step_sampled_matches_the_full_step():
    P = params(nx=9, ny=7, G=1.1, kappa=0.5, bc_x=1)
    rA, rB = _mixture(P, 11, noise=0.05)
    f = B.run(P, B.init(P, rA, rB), 3)
    full = B.step(P, f)
    idx = np.array([0, 5, 8, 9, 30, 62])
    got = B.step_sampled(P, f, idx)
    want = full.reshape(2, 9, -1)[:, :, idx].transpose(2, 0, 1)
    np.testing.assert_array_equal(got, want)
