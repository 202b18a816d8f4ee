"""Pins of the D3Q19 oracle (the 3D extension that Section VI leaves as future
work) against what does not come from the oracle itself (CPU only).

* M: the orthogonal D3Q19 basis of d'Humieres et al.; pinned by its inverse,
  its row norms and by mapping the textbook equilibrium and Guo forcing onto
  their closed-form moments.
* The source-term rule (Lambda M df for a momentum-flux shift dPi): df moves
  exactly the flux; in 2D the same rule with dPi = 3/4 tr Q I - Q is Eq. (18)
  and with dPi = 2 sigma |F|^2 / psi^2 I the Eq. (8) term, checked against the
  (pinned) 2D oracle.
* F (Eq. 7) and Q (Eq. 19) with the 3D weights: trigonometric closed forms for a
  sinusoidal psi.
* Invariants: rest state, mass and momentum, the conserved moments' rates.
* Physics: flat-interface coexistence against the Eq. 16 quadrature and its
  kappa invariance (Section IV); the Laplace law on cylinders gives a tension
  that scales as 1 - kappa.
"""
import numpy as np
import pytest

import oracle as O
from oracle import d3q19 as D
from oracle import theory
from paper_1306_6445_amd import workloads as WL

RHO_C, T_C = theory.critical_point(0.25, 4.0, 1.0)

# the D3Q19 velocities and textbook BGK weights, written out here independently
E = np.array([(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
              (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1),
              (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)], dtype=float)
C2 = (E ** 2).sum(axis=1)
W = np.where(C2 == 0, 1 / 3, np.where(C2 == 1, 1 / 18, 1 / 36))


def feq_textbook(rho, v):
    eu = E @ v
    return W * rho * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * (v @ v))


def eq_moments(rho, v):
    """Closed-form equilibrium moments of the d'Humieres basis for the BGK
    equilibrium (w_eps = 3, w_epsj = -11/2, w_xx = -1/2)."""
    vx, vy, vz = v
    v2 = v @ v
    pxx, pww = rho * (3 * vx * vx - v2), rho * (vy * vy - vz * vz)
    return np.array([rho, rho * (-11 + 19 * v2), rho * (3 - 5.5 * v2), rho * vx, -2 / 3 * rho * vx,
                     rho * vy, -2 / 3 * rho * vy, rho * vz, -2 / 3 * rho * vz, pxx, -pxx / 2, pww, -pww / 2,
                     rho * vx * vy, rho * vy * vz, rho * vx * vz, 0, 0, 0])


def params(**kw):
    base = dict(nx=6, ny=5, nz=4, eos_kind=O.EOS_EXP, eos=(4.0, 200.0), G=-40.0)
    base.update(kw)
    return D.Params3(**base)


def cs_params(n=(8, 6, 5), T=0.7, **kw):
    kind, eos = WL.cs_eos(T)
    return D.Params3(nx=n[0], ny=n[1], nz=n[2], eos_kind=kind, eos=eos, G=-1.0,
                     sigma=O.sigma_from_epsilon(1.93, -1.0), **kw)


# ------------------------------------------------------------------ algebra

def test_matrix_inverse_norms_and_conserved_rows():
    M, Mi = D.matrices()
    np.testing.assert_allclose(M @ Mi, np.eye(19), atol=1e-14)
    np.testing.assert_allclose(M @ M.T, np.diag([19, 2394, 252, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24, 4, 4, 4,
                                                 8, 8, 8]), atol=1e-12)
    np.testing.assert_array_equal(M[0], np.ones(19))
    for r, axis in ((3, 0), (5, 1), (7, 2)):
        np.testing.assert_array_equal(M[r], E[:, axis])


def test_equilibrium_maps_to_closed_form_moments():
    M, _ = D.matrices()
    rng = np.random.default_rng(1)
    for _ in range(20):
        rho = rng.uniform(0.01, 300)
        v = rng.uniform(-0.15, 0.15, 3)
        np.testing.assert_allclose(D.feq(rho, v), feq_textbook(rho, v), rtol=1e-13, atol=1e-15 * rho)
        np.testing.assert_allclose(M @ feq_textbook(rho, v), eq_moments(rho, v), rtol=1e-12, atol=1e-12 * rho)


def test_guo_forcing_moments_are_the_force_derivative_of_the_equilibrium():
    """Guo's forcing moves each equilibrium moment as d m_eq/dt under
    d(rho v)/dt = F: j by F, e by 38 v.F, eps by -11 v.F, 3pxx by
    2 (3 vx Fx - v.F), pxy by vx Fy + vy Fx, q by -2F/3, m by 0."""
    M, _ = D.matrices()
    rng = np.random.default_rng(2)
    for _ in range(20):
        v, F = rng.uniform(-0.1, 0.1, 3), rng.uniform(-1, 1, 3)
        vF = v @ F
        pxx, pww = 2 * (3 * v[0] * F[0] - vF), 2 * (v[1] * F[1] - v[2] * F[2])
        ref = np.array([0, 38 * vF, -11 * vF, F[0], -2 / 3 * F[0], F[1], -2 / 3 * F[1], F[2], -2 / 3 * F[2],
                        pxx, -pxx / 2, pww, -pww / 2, v[0] * F[1] + v[1] * F[0], v[1] * F[2] + v[2] * F[1],
                        v[0] * F[2] + v[2] * F[0], 0, 0, 0])
        np.testing.assert_allclose(M @ D.guo(v, F), ref, atol=1e-13)


def test_equal_rates_reduce_to_bgk_with_guo_forcing():
    tau = 0.83
    P = params(s=[1 / tau] * 19)
    rng = np.random.default_rng(3)
    for _ in range(10):
        rho = rng.uniform(0.5, 3.0)
        f = feq_textbook(rho, rng.uniform(-0.05, 0.05, 3)) * rng.uniform(0.9, 1.1, 19)
        F = rng.uniform(-0.02, 0.02, 3)
        fs = D.collide_node(P, f, F, np.zeros(6), psi=1.0)
        r = f.sum()
        v = (E.T @ f + F / 2) / r
        eu, eF = E @ v, E @ F
        guo = W * (3 * ((E - v) @ F) + 9 * eu * eF)
        ref = f - (f - feq_textbook(r, v)) / tau + (1 - 1 / (2 * tau)) * guo
        np.testing.assert_allclose(fs, ref, rtol=1e-12, atol=1e-15)


def _sym(d):
    xx, yy, zz, xy, yz, xz = d
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])


def test_flux_shift_moves_only_the_momentum_flux():
    rng = np.random.default_rng(4)
    for _ in range(10):
        dPi = rng.normal(size=6)
        df = D.flux_shift(dPi)
        assert abs(df.sum()) < 1e-14
        np.testing.assert_allclose(E.T @ df, 0, atol=1e-14)
        np.testing.assert_allclose(np.einsum("a,ai,aj->ij", df, E, E), _sym(dPi), atol=1e-13)


def test_the_flux_shift_rule_in_2d_is_eq18_and_the_eq8_term():
    """The 3D source term is the rule C = Lambda M df(dPi) with
    dPi = 3/(d+2) tr Q I - Q; in D2Q9 (d = 2) the same rule must give the
    paper's Eq. (18) exactly, and the flux shift 2 sigma |F|^2/psi^2 I the
    Eq. (8) term (with tau_zeta = tau_e), as the 2D oracle computes them."""
    M2, _ = O.matrices()
    ex = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1.0])
    ey = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1.0])
    w2 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)

    def df2(d):
        xx, yy, xy = d
        return w2 * 4.5 * (xx * (ex * ex - 1 / 3) + yy * (ey * ey - 1 / 3) + 2 * xy * ex * ey)

    s = O.rates(s_e=0.8, s_zeta=0.8, s_q=1.1, s_nu=1.3)
    P = O.Params(nx=4, ny=4, eos_kind=O.EOS_EXP, eos=(4.0, 200.0), G=-40.0, s=s, kappa=0.7, sigma=0.11)
    rng = np.random.default_rng(5)
    for _ in range(10):
        Q = rng.normal(size=3)  # (xx, yy, xy)
        tr = Q[0] + Q[1]
        rule = np.array(s) * (M2 @ df2((0.75 * tr - Q[0], 0.75 * tr - Q[1], -Q[2])))
        np.testing.assert_allclose(rule, O.source_moments(P, Q), atol=1e-13)
        v, F, psi = rng.uniform(-0.1, 0.1, 2), rng.uniform(-1, 1, 2), rng.uniform(0.5, 3)
        eq8 = (1 - 0.5 * np.array(s)) * (O.forcing_moments(P, v, F, psi) - O.forcing_moments(
            P.replace(sigma=0.0), v, F, psi))
        a = 2 * P.sigma * (F @ F) / psi ** 2
        np.testing.assert_allclose(np.array(s) * (M2 @ df2((a, a, 0.0))), eq8, atol=1e-13)


def _wave3(A, B, k, theta):
    return A + B * np.cos(theta + E @ k)


@pytest.mark.parametrize("k,theta", [((0.3, 0.0, 0.0), 0.4), ((0.21, -0.55, 0.9), 1.9), ((1.1, 0.7, -0.35), -2.2)])
def test_force_and_source_exact_for_sinusoidal_psi(k, theta):
    k = np.array(k)
    G, kappa, A, B = -1.3, 0.7, 1.8, 0.3
    P = params(G=G, kappa=kappa)
    psi19 = _wave3(A, B, k, theta)
    F, Q = D.force_and_q(P, psi19)
    kx, ky, kz = k
    c, s_ = np.cos, np.sin
    # sum_a w_a psi(x + e_a) e_a = -B sin(theta) sum_a w_a sin(k.e_a) e_a, in closed form
    sx = s_(kx) / 3 * (1 + c(ky) + c(kz))
    sy = s_(ky) / 3 * (1 + c(kx) + c(kz))
    sz = s_(kz) / 3 * (1 + c(kx) + c(ky))
    np.testing.assert_allclose(F, -G * psi19[0] * (-B * s_(theta)) * np.array([sx, sy, sz]), rtol=1e-12,
                               atol=1e-15)
    # sum_a w_a (psi(x + e_a) - psi(x)) e_a e_a = B cos(theta) sum_a w_a (cos(k.e_a) - 1) e_a e_a
    txx = (c(kx) - 1) / 3 + (c(kx) * (c(ky) + c(kz)) - 2) / 3
    tyy = (c(ky) - 1) / 3 + (c(ky) * (c(kx) + c(kz)) - 2) / 3
    tzz = (c(kz) - 1) / 3 + (c(kz) * (c(kx) + c(ky)) - 2) / 3
    txy, tyz, txz = -s_(kx) * s_(ky) / 3, -s_(ky) * s_(kz) / 3, -s_(kx) * s_(kz) / 3
    ref = kappa * G / 2 * psi19[0] * B * c(theta) * np.array([txx, tyy, tzz, txy, tyz, txz])
    np.testing.assert_allclose(Q, ref, rtol=1e-11, atol=1e-15)


@pytest.mark.parametrize("m,theta", [((1, 0, 0), 0.4), ((2, -1, 1), 1.9), ((1, 2, -1), -2.2)])
def test_eq6_velocity_of_a_resting_sinusoidal_psi_field(m, theta):
    """Eq. (6) in 3D: rho v = sum_a e_a f_a + F / 2.  On a rest equilibrium
    the first sum vanishes, so the read-out velocity is exactly F / (2 rho),
    with F of Eq. (7) in closed form for psi = A + B cos(theta + k.x) (the
    exponential potential inverted for rho).  Dropping, halving or flipping
    the F / 2 term fails here; the diagnostics' largest speed is the largest
    |F| / (2 rho)."""
    G, Aw, Bw = -40.0, 2.0, 0.35
    nx, ny, nz = 12, 10, 8
    k = 2 * np.pi * np.array(m) / np.array([nx, ny, nz])
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx].astype(float)
    phase = theta + k[0] * x + k[1] * y + k[2] * z
    psi = Aw + Bw * np.cos(phase)
    rho = -200.0 / np.log(psi / 4.0)
    P = params(nx=nx, ny=ny, nz=nz, G=G, kappa=0.6)
    f = D.init(P, rho)
    r, ux, uy, uz = D.moments(P, f)
    np.testing.assert_allclose(r, rho, rtol=1e-14)
    c, s_ = np.cos, np.sin
    kx, ky, kz = k
    g = [s_(kx) / 3 * (1 + c(ky) + c(kz)), s_(ky) / 3 * (1 + c(kx) + c(kz)), s_(kz) / 3 * (1 + c(kx) + c(ky))]
    F = [-G * psi * (-Bw * s_(phase)) * gi for gi in g]
    assert max(np.abs(Fi).max() for Fi in F) > 1.0  # the force term is not negligible
    for u, Fi in zip((ux, uy, uz), F):
        np.testing.assert_allclose(u, Fi / (2 * rho), rtol=1e-11, atol=1e-15)
    d = D.diagnostics(P, f, 3, nx / 2, ny / 2, nz / 2, 2.0, 4.0)
    speed = np.sqrt(F[0] ** 2 + F[1] ** 2 + F[2] ** 2) / (2 * rho)
    assert d["max_speed"] == pytest.approx(float(speed.max()), rel=1e-11)


# --------------------------------------------------------------- invariants

@pytest.mark.parametrize("make", ["cs", "exp", "pw"])
@pytest.mark.parametrize("walls", [False, True])
def test_uniform_rest_state_stays_at_rest(make, walls):
    bc = O.BC_WALL if walls else O.BC_PERIODIC
    if make == "cs":
        P, rho0 = cs_params(kappa=0.5, bc_z=bc), 0.2
    elif make == "exp":
        P, rho0 = params(kappa=0.5, bc_y=bc), 300.0
    else:
        kind, eos = WL.piecewise_eos()
        P, rho0 = D.Params3(7, 5, 6, kind, eos, -1.0, kappa=0.9, sigma=0.087, bc_x=bc), 50.0
    f0 = D.init(P, np.full(P.shape, rho0))
    f = D.run(P, f0, 200)
    # uniform psi gives F = Q = 0 exactly; what remains is the round-off of the
    # dense 19 x 19 products (entries up to 24, moments up to 11 rho)
    np.testing.assert_allclose(f, f0, rtol=1e-12, atol=0)
    _, ux, uy, uz = D.moments(P, f)
    assert max(np.abs(ux).max(), np.abs(uy).max(), np.abs(uz).max()) < 1e-13


def _blob(P, rl, rv, R, seed=0):
    z, y, x = np.mgrid[0:P.nz, 0:P.ny, 0:P.nx].astype(float)
    r = np.sqrt((x - P.nx / 2) ** 2 + (y - P.ny / 2) ** 2 + (z - P.nz / 2) ** 2)
    rho = (rl + rv) / 2 - (rl - rv) / 2 * np.tanh(2 * (r - R) / 5)
    return rho * (1 + WL.noise(rho.shape, 1e-3, seed))


@pytest.mark.parametrize("walls", [False, True])
def test_mass_conservation(walls):
    P = cs_params(n=(12, 10, 9), kappa=0.6, bc_y=O.BC_WALL if walls else O.BC_PERIODIC)
    rl, rv = WL.coexistence_seed(0.7, 1.93)
    f0 = D.init(P, _blob(P, rl, rv, 3.0))
    f = D.run(P, f0, 60)
    assert f.sum() == pytest.approx(f0.sum(), rel=1e-13)


def test_momentum_conservation_periodic():
    """Eq. (7) is pair-antisymmetric, the flux shifts and the forcing carry no
    net momentum: total momentum is constant (up to round-off)."""
    P = cs_params(n=(12, 10, 9), kappa=0.6)
    rl, rv = WL.coexistence_seed(0.7, 1.93)
    z, y, x = np.mgrid[0:P.nz, 0:P.ny, 0:P.nx].astype(float)
    f0 = D.init(P, _blob(P, rl, rv, 3.0), 0.02 * np.sin(2 * np.pi * y / P.ny), None, 0.01 * np.cos(2 * np.pi * x / P.nx))
    p0 = np.einsum("a,ai->i", f0.reshape(19, -1).sum(axis=1), E)
    f = D.run(P, f0, 40)
    p1 = np.einsum("a,ai->i", f.reshape(19, -1).sum(axis=1), E)
    np.testing.assert_allclose(p1, p0, atol=1e-12 * f0.sum())


def test_conserved_moment_rates_do_not_matter():
    P = cs_params(n=(8, 7, 6), kappa=0.4)
    rl, rv = WL.coexistence_seed(0.7, 1.93)
    f0 = D.init(P, _blob(P, rl, rv, 2.0))
    a = D.run(P, f0, 10)
    s = list(P.s)
    for i in (0, 3, 5, 7):
        s[i] = 0.37
    b = D.run(P.replace(s=s), f0, 10)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-15)


def test_sampled_step_matches_full_step():
    P = cs_params(n=(9, 7, 6), kappa=0.5, bc_z=O.BC_WALL)
    rl, rv = WL.coexistence_seed(0.7, 1.93)
    f0 = D.init(P, _blob(P, rl, rv, 2.0))
    f1 = D.step(P, f0)
    idx = np.arange(0, P.nx * P.ny * P.nz, 7)
    np.testing.assert_allclose(D.step_sampled(P, f0, idx), f1.reshape(19, -1)[:, idx].T, rtol=1e-14, atol=0)


# ------------------------------------------------------------------ physics

def _slab3(P, rl, rv, steps):
    """A liquid slab of half the height across z (the 2D slab profile along z)."""
    rho = WL.slab(1, P.nz, rl, rv, P.nz / 2)[:, 0][:, None, None] * np.ones(P.shape)
    f = D.run(P, D.init(P, rho), steps)
    r = D.moments(P, f)[0]
    return r[P.nz // 2, 0, 0], r[0, 0, 0]


def test_flat_interface_coexistence_matches_eq16_in_3d():
    """With the 3D weights the flat-interface balance is the 2D one (Eq. 16 with
    epsilon = -16 G sigma), so a slab's densities match the same quadrature."""
    eps = 1.93
    kind, eos = WL.cs_eos(0.7)
    P2 = O.Params(nx=1, ny=1, eos_kind=kind, eos=eos, G=-1.0, sigma=O.sigma_from_epsilon(eps, -1.0))
    rl_t, rv_t, _ = theory.coexistence(P2, eps)
    P = D.Params3(1, 1, 256, kind, eos, -1.0, sigma=O.sigma_from_epsilon(eps, -1.0))
    rl, rv = _slab3(P, rl_t, rv_t, 20000)
    assert rl == pytest.approx(rl_t, rel=5e-3)
    assert rv == pytest.approx(rv_t, rel=3e-2)


def test_kappa_leaves_3d_coexistence_unchanged(golden):
    g = golden["piecewise_setup"]
    cs2 = 1 / 3
    eos = (g["thetaV_over_cs2"] * cs2, g["thetaM_over_cs2"] * cs2, g["thetaL_over_cs2"] * cs2, g["rho1"], g["rho2"])
    res = []
    for kappa in (0.0, 0.9):
        P = D.Params3(1, 1, 256, O.EOS_PIECEWISE, eos, g["G"], kappa=kappa, sigma=g["sigma"])
        res.append(_slab3(P, 100.0, 1.0, 12000))
    assert res[1][1] == pytest.approx(res[0][1], rel=1e-2)
    assert res[1][0] == pytest.approx(res[0][0], rel=1e-4)


def test_cylinder_tension_scales_with_one_minus_kappa(golden):
    """Laplace law for a cylinder along z (dp = sigma / R): sigma = dp R_eq at
    kappa = 0 and 0.5 (Eq. 22: the tension coefficient becomes 1 - kappa); the
    kappa = 0 value is near the flat-interface theory of the same EOS."""
    g = golden["piecewise_setup"]
    cs2 = 1 / 3
    eos = (g["thetaV_over_cs2"] * cs2, g["thetaM_over_cs2"] * cs2, g["thetaL_over_cs2"] * cs2, g["rho1"], g["rho2"])
    sig = []
    for kappa in (0.0, 0.5):
        P = D.Params3(48, 48, 1, O.EOS_PIECEWISE, eos, g["G"], kappa=kappa, sigma=g["sigma"],
                      s=D.rates(s_nu=1.0))
        y, x = np.mgrid[0:48, 0:48].astype(float)
        r = np.hypot(x - 24, y - 24)
        rho = (100.0 + 1.0) / 2 - (100.0 - 1.0) / 2 * np.tanh(2 * (r - 14) / 5)
        f = D.run(P, D.init(P, rho[None]), 5000)
        d = D.diagnostics(P, f, 2, 24, 24, 0, 3.5, 22)
        sig.append(d["dp"] * d["r_eq"])
    assert sig[1] / sig[0] == pytest.approx(0.5, rel=0.04)
    P2 = O.Params(nx=1, ny=1, eos_kind=O.EOS_PIECEWISE, eos=eos, G=g["G"], sigma=g["sigma"])
    assert sig[0] == pytest.approx(theory.flat_surface_tension(P2, -16 * g["G"] * g["sigma"]), rel=0.12)
