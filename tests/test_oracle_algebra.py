"""Pins of the oracle's node arithmetic against closed forms that do not come
from the oracle itself (CPU only).

* The moment matrix M is a reading (Section II prints no M).  It is pinned by
  requiring that the textbook D2Q9 equilibrium maps onto the printed m_eq of
  Eq. (3), and that M^-1 is an inverse.
* The forcing moments of Eq. (5) are pinned against the velocity-space forcing
  of Guo et al. (reference [34] of the paper): S = M F_Guo.
* With all relaxation rates equal, Eq. (2) must collapse to BGK with Guo forcing.
* The force of Eq. (7) and the source tensor of Eq. (19) are pinned by exact
  trigonometric closed forms for a sinusoidal psi field.
* Streaming (Eq. 4) and halfway bounce-back are pinned by pure advection.
"""
import numpy as np
import pytest

import oracle as O
from oracle import theory

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)
# textbook D2Q9 lattice weights (rest 4/9, axis 1/9, diagonal 1/36)
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def feq_textbook(rho, ux, uy):
    eu = EX * ux + EY * uy
    return W * rho * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * (ux * ux + uy * uy))


def guo_forcing(ux, uy, Fx, Fy):
    eu = EX * ux + EY * uy
    eF = EX * Fx + EY * Fy
    return W * (3 * ((EX - ux) * Fx + (EY - uy) * Fy) + 9 * eu * eF)


def eq3(rho, vx, vy):
    v2 = vx * vx + vy * vy
    return rho * np.array([1, -2 + 3 * v2, 1 - 3 * v2, vx, -vx, vy, -vy, vx * vx - vy * vy, vx * vy])


def params(**kw):
    base = dict(nx=8, ny=8, eos_kind=O.EOS_EXP, eos=(4.0, 200.0), G=-40.0)
    base.update(kw)
    return O.Params(**base)


def test_matrix_maps_textbook_equilibrium_to_eq3():
    M, _ = O.matrices()
    rng = np.random.default_rng(1)
    for _ in range(20):
        rho = rng.uniform(0.01, 500)
        ux, uy = rng.uniform(-0.2, 0.2, 2)
        np.testing.assert_allclose(M @ feq_textbook(rho, ux, uy), eq3(rho, ux, uy),
                                   rtol=1e-13, atol=1e-13 * rho)


def test_matrix_inverse_and_orthogonal_rows():
    M, Mi = O.matrices()
    np.testing.assert_allclose(M @ Mi, np.eye(9), atol=1e-15)
    np.testing.assert_allclose(Mi @ M, np.eye(9), atol=1e-15)
    G = M @ M.T
    np.testing.assert_allclose(G, np.diag([9, 36, 36, 6, 12, 6, 12, 4, 4]), atol=1e-13)
    # conserved rows: density and momentum are the plain sums sum f, sum e f
    np.testing.assert_array_equal(M[0], np.ones(9))
    np.testing.assert_array_equal(M[3], EX)
    np.testing.assert_array_equal(M[5], EY)


def test_rest_and_moving_equilibrium_initialisation():
    P = params(nx=3, ny=2)
    rho = np.array([[0.3, 1.0, 7.0], [100.0, 0.01, 2.5]])
    f = O.init(P, rho)
    for a in range(9):
        np.testing.assert_allclose(f[a], W[a] * rho, rtol=1e-14)
    ux = np.full_like(rho, 0.05)
    uy = np.full_like(rho, -0.03)
    f = O.init(P, rho, ux, uy)
    for j in range(2):
        for i in range(3):
            np.testing.assert_allclose(f[:, j, i], feq_textbook(rho[j, i], 0.05, -0.03), rtol=1e-13)


def test_forcing_moments_equal_guo_forcing():
    M, _ = O.matrices()
    P = params(sigma=0.0)
    rng = np.random.default_rng(2)
    for _ in range(20):
        v = rng.uniform(-0.1, 0.1, 2)
        F = rng.uniform(-1, 1, 2)
        S = O.forcing_moments(P, v, F, psi=1.3)
        np.testing.assert_allclose(S, M @ guo_forcing(v[0], v[1], F[0], F[1]), atol=1e-14)


def test_equal_rates_reduce_to_bgk_with_guo_forcing():
    tau = 0.83
    P = params(s=[1 / tau] * 9, sigma=0.0)
    rng = np.random.default_rng(3)
    for _ in range(20):
        rho = rng.uniform(0.5, 3.0)
        f = feq_textbook(rho, *rng.uniform(-0.05, 0.05, 2)) * rng.uniform(0.9, 1.1, 9)
        F = rng.uniform(-0.02, 0.02, 2)
        fs = O.collide_node(P, f, F, np.zeros(3), psi=1.0)
        r = f.sum()
        vx = (EX @ f + F[0] / 2) / r
        vy = (EY @ f + F[1] / 2) / r
        ref = f - (f - feq_textbook(r, vx, vy)) / tau + (1 - 1 / (2 * tau)) * guo_forcing(vx, vy, *F)
        np.testing.assert_allclose(fs, ref, rtol=1e-12, atol=1e-15)


def _wave(A, B, k, l, theta):
    """psi at the nine lattice offsets for psi = A + B cos(theta + k x + l y)."""
    return A + B * np.cos(theta + k * EX + l * EY)


@pytest.mark.parametrize("k,l,theta", [(0.3, 0.0, 0.4), (0.21, -0.55, 1.9), (1.1, 0.7, -2.2)])
def test_force_exact_for_sinusoidal_psi(k, l, theta):
    G = -1.7
    A, B = 2.0, 0.35
    P = params(G=G)
    psi9 = _wave(A, B, k, l, theta)
    F, _ = O.force_and_q(P, psi9)
    # sum w psi(x+e) e = -B sin(theta) * 2 * sum over half the stencil of w e sin(k.e)
    sx = 2 * (np.sin(k) / 3 + np.sin(k + l) / 12 - np.sin(l - k) / 12)
    sy = 2 * (np.sin(l) / 3 + np.sin(k + l) / 12 + np.sin(l - k) / 12)
    ref = -G * psi9[0] * (-B * np.sin(theta)) * np.array([sx, sy])
    np.testing.assert_allclose(F, ref, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("k,l,theta", [(0.3, 0.0, 0.4), (0.21, -0.55, 1.9), (1.1, 0.7, -2.2)])
def test_source_tensor_exact_for_sinusoidal_psi(k, l, theta):
    G, kappa = -1.3, 0.7
    A, B = 1.5, 0.2
    P = params(G=G, kappa=kappa)
    psi9 = _wave(A, B, k, l, theta)
    _, Q = O.force_and_q(P, psi9)
    ck, cl, cp, cm = np.cos(k) - 1, np.cos(l) - 1, np.cos(k + l) - 1, np.cos(l - k) - 1
    T = 2 * (ck / 3 * np.array([[1, 0], [0, 0]]) + cl / 3 * np.array([[0, 0], [0, 1]])
             + cp / 12 * np.array([[1, 1], [1, 1]]) + cm / 12 * np.array([[1, -1], [-1, 1]]))
    ref = kappa * G / 2 * psi9[0] * B * np.cos(theta) * T
    np.testing.assert_allclose(Q, [ref[0, 0], ref[1, 1], ref[0, 1]], rtol=1e-12, atol=1e-16)


def test_uniform_psi_gives_no_force_and_no_source():
    P = params(G=-1.0, kappa=0.9)
    F, Q = O.force_and_q(P, np.full(9, 3.7))
    assert np.all(F == 0.0) and np.all(np.abs(Q) == 0.0)


def _advect_params(L, walls):
    return O.Params(nx=L, ny=L, eos_kind=O.EOS_EXP, eos=(1.0, 1.0), G=0.0, s=[0.0] * 9,
                    bc_y=O.BC_WALL if walls else O.BC_PERIODIC)


def test_pure_streaming_periodic_returns_after_one_lap():
    L = 7
    P = _advect_params(L, walls=False)
    rng = np.random.default_rng(4)
    f0 = rng.uniform(0.5, 1.5, (9, L, L)) * W[:, None, None]
    f1 = O.step(P, f0)
    for a in range(9):  # one step moves each population by e_a
        np.testing.assert_allclose(f1[a], np.roll(f0[a], (int(EY[a]), int(EX[a])), axis=(0, 1)),
                                   rtol=1e-13)
    np.testing.assert_allclose(O.run(P, f0, L), f0, rtol=1e-12)


def test_pure_streaming_with_walls_bounces_back():
    L = 6
    P = _advect_params(L, walls=True)
    f0 = np.zeros((9, L, L))
    f0 += 1e-3 * W[:, None, None]  # positive background keeps rho > 0
    f0[2, L - 1, 3] += 1.0          # moving up (e2) in the top row
    f1 = O.step(P, f0)
    # it reaches the wall half-way and returns to the same node moving down (e4)
    assert f1[4, L - 1, 3] == pytest.approx(1.0 + 1e-3 * W[2], rel=1e-12)
    f2 = O.step(P, f1)
    assert f2[4, L - 2, 3] == pytest.approx(1.0 + 1e-3 * W[2], rel=1e-12)
    rng = np.random.default_rng(5)
    g0 = rng.uniform(0.5, 1.5, (9, L, L)) * W[:, None, None]
    # every population is back after travelling to both walls and back
    np.testing.assert_allclose(O.run(P, g0, 2 * L), g0, rtol=1e-12)


def test_carnahan_starling_critical_point():
    # a = 0.25, b = 4, R = 1: published CS values T_c = 0.3773 a / (b R), eta_c = 0.1304
    rho_c, T_c = theory.critical_point(0.25, 4.0, 1.0)
    assert T_c * 4.0 / 0.25 == pytest.approx(0.3773, abs=2e-4)
    assert 4.0 * rho_c / 4.0 == pytest.approx(0.1304, abs=1e-4)


def test_piecewise_eos_transcription(golden):
    g = golden["piecewise_setup"]
    cs2 = 1 / 3
    P = O.Params(nx=1, ny=1, eos_kind=O.EOS_PIECEWISE, G=g["G"],
                 eos=(g["thetaV_over_cs2"] * cs2, g["thetaM_over_cs2"] * cs2,
                      g["thetaL_over_cs2"] * cs2, g["rho1"], g["rho2"]))
    p, psi = O.eos(P, np.array([g["rho_V"], g["rho_L"], g["rho2"], 97.0, 120.0]))
    # the prescribed phases rho_V = 1 and rho_L = 100 sit at (nearly) equal pressure
    assert p[0] == pytest.approx(p[1], rel=2e-3)
    # thetaL = cs^2 makes psi constant on the liquid branch, so F = 0 in bulk liquid
    assert np.ptp(psi[2:]) < 1e-12 * psi[2]


@pytest.mark.parametrize("k,l,theta", [(0.3, 0.0, 0.4), (0.21, -0.55, 1.9), (1.1, 0.7, -2.2)])
def test_multirange_force_exact_for_sinusoidal_psi(k, l, theta):
    """Eq. (9): the second range adds -G2 psi(x) sum w psi(x + 2e) e, whose
    discrete sum for psi = A + B cos(theta + k.x) is the first-range sum at the
    doubled wave vector."""
    G1, G2 = -1.7, 0.4
    A, B = 2.0, 0.35
    P = params(G=G1).replace(G2=G2)
    psi9 = _wave(A, B, k, l, theta)
    psi2 = _wave(A, B, 2 * k, 2 * l, theta)
    F, _ = O.force_multirange(P, psi9, psi2)

    def s(k, l):
        return np.array([2 * (np.sin(k) / 3 + np.sin(k + l) / 12 - np.sin(l - k) / 12),
                         2 * (np.sin(l) / 3 + np.sin(k + l) / 12 + np.sin(l - k) / 12)])
    ref = -psi9[0] * (-B * np.sin(theta)) * (G1 * s(k, l) + G2 * s(2 * k, 2 * l))
    np.testing.assert_allclose(F, ref, rtol=1e-13, atol=1e-15)
    # G2 = 0 is the Eq. (7) force
    F1, _ = O.force_and_q(P.replace(G2=0.0), psi9)
    F2, _ = O.force_multirange(P.replace(G2=0.0), psi9, psi2)
    np.testing.assert_array_equal(F1, F2)


def test_multirange_eos_uses_g1_plus_2g2():
    """Section III.A: p0 = rho cs^2 + (G1 + 2 G2) psi^2 / 2 (exp psi), and the
    sqrt psi forms invert with G1 + 2 G2."""
    P = O.Params(nx=1, ny=1, eos_kind=O.EOS_EXP, eos=(4.0, 200.0), G=-1.3 * 40.0, G2=0.15 * 40.0)
    p, psi = O.eos(P, np.array([200.0]))
    assert p[0] == pytest.approx(200 / 3 - 20 * (4 / np.e) ** 2, rel=1e-14)
    Pc = O.Params(nx=1, ny=1, eos_kind=O.EOS_PIECEWISE, eos=(0.49 / 3, -0.06 / 3, 1 / 3, 1.49, 94.65),
                  G=-1.3, G2=0.15)
    Pr = Pc.replace(G=-1.0, G2=0.0)
    np.testing.assert_allclose(O.eos(Pc, np.array([0.7, 50.0, 120.0])), O.eos(Pr, np.array([0.7, 50.0, 120.0])),
                               rtol=1e-15)


def test_exponential_potential_eos():
    P = O.Params(nx=1, ny=1, eos_kind=O.EOS_EXP, eos=(4.0, 200.0), G=-40.0)
    p, psi = O.eos(P, np.array([200.0]))
    assert psi[0] == pytest.approx(4.0 / np.e, rel=1e-15)
    assert p[0] == pytest.approx(200 / 3 - 20 * (4 / np.e) ** 2, rel=1e-14)


def _sinusoidal_exp_field(nx, ny, m, n, theta, A=2.0, B=0.35, psi0=4.0, rho0=200.0):
    """Density whose exponential pseudopotential psi0 exp(-rho0 / rho) is exactly
    A + B cos(theta + k x + l y) on a periodic nx x ny grid (k = 2 pi m / nx,
    l = 2 pi n / ny): rho = -rho0 / ln(psi / psi0)."""
    k, l = 2 * np.pi * m / nx, 2 * np.pi * n / ny
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    phase = theta + k * x + l * y
    psi = A + B * np.cos(phase)
    return -rho0 / np.log(psi / psi0), psi, phase, k, l


@pytest.mark.parametrize("m,n,theta", [(1, 0, 0.4), (2, -1, 1.9), (3, 2, -2.2)])
def test_eq6_velocity_of_a_resting_sinusoidal_psi_field(m, n, theta):
    """Eq. (6): rho v = sum_a e_a f_a + F / 2.  On a rest equilibrium the first
    sum vanishes (f_a = w_a rho), so the read-out velocity is exactly
    F / (2 rho), with F of Eq. (7) known in closed form for a sinusoidal psi.
    Dropping the F / 2 term, flipping its sign or halving it fails here; the
    diagnostics' largest speed is the largest |F| / (2 rho) of the field."""
    G = -40.0
    nx, ny = 24, 18
    rho, psi, phase, k, l = _sinusoidal_exp_field(nx, ny, m, n, theta)
    P = params(nx=nx, ny=ny, G=G, kappa=0.6)
    f = O.init(P, rho)
    r, ux, uy = O.moments(P, f)
    np.testing.assert_allclose(r, rho, rtol=1e-14)
    sx = 2 * (np.sin(k) / 3 + np.sin(k + l) / 12 - np.sin(l - k) / 12)
    sy = 2 * (np.sin(l) / 3 + np.sin(k + l) / 12 + np.sin(l - k) / 12)
    Fx = -G * psi * (-0.35 * np.sin(phase)) * sx
    Fy = -G * psi * (-0.35 * np.sin(phase)) * sy
    assert np.abs(Fx).max() + np.abs(Fy).max() > 1.0  # the force term is not negligible
    np.testing.assert_allclose(ux, Fx / (2 * rho), rtol=1e-11, atol=1e-15)
    np.testing.assert_allclose(uy, Fy / (2 * rho), rtol=1e-11, atol=1e-15)
    d = O.diagnostics(P, f, nx / 2, ny / 2, 3.0, 8.0)
    assert d["max_speed"] == pytest.approx(float(np.max(np.hypot(Fx, Fy) / (2 * rho))), rel=1e-11)
