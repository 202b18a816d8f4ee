"""Physics pins of the oracle against what the paper prints (CPU only).

Each test names the passage it checks.  Tolerances are stated with the reason.
The droplet runs use the paper's own set-ups (Section III.B / V.A) but stop
earlier than a production run: the densities converge within a few thousand
steps; pressure-jump tests use tau_v = 1 so that the breathing mode of the
drop decays within the run.
"""
import numpy as np
import pytest

import oracle as O
from oracle import theory
from paper_1306_6445_amd import workloads as WL

RHO_C, T_C = theory.critical_point(0.25, 4.0, 1.0)


def piecewise_params(g, n, kappa=0.0, s=None, **kw):
    cs2 = 1 / 3
    return O.Params(nx=n, ny=kw.pop("ny", n), eos_kind=O.EOS_PIECEWISE, G=g["G"], sigma=g["sigma"],
                    eos=(g["thetaV_over_cs2"] * cs2, g["thetaM_over_cs2"] * cs2,
                         g["thetaL_over_cs2"] * cs2, g["rho1"], g["rho2"]),
                    kappa=kappa, s=s or O.rates(), **kw)


def exp_params(g, kappa=0.0):
    return O.Params(nx=g["nx"], ny=g["ny"], eos_kind=O.EOS_EXP, eos=(g["psi0"], g["rho0"]),
                    G=g["G"], kappa=kappa, s=O.rates(s_nu=O.s_nu_from_viscosity(g["nu"])))


def run_droplet(P, rl, rv, R, steps, r_out_pad=15.0):
    rho = WL.droplet(P.nx, P.ny, R, rl, rv)
    f = O.run(P, O.init(P, rho), steps)
    return O.diagnostics(P, f, P.nx / 2, P.ny / 2, R / 4, R + r_out_pad)


def run_slab(P, rl, rv, steps):
    f = O.run(P, O.init(P, WL.slab(P.nx, P.ny, rl, rv, P.ny / 2)), steps)
    rho, _, _ = O.moments(P, f)
    return rho[P.ny // 2, 0], rho[0, 0]


# --------------------------------------------------------------- theory tool

def test_maxwell_construction_matches_paper(golden):
    g = golden["exp_maxwell"]
    s = golden["exp_potential_setup"]
    P = O.Params(nx=1, ny=1, eos_kind=O.EOS_EXP, eos=(s["psi0"], s["rho0"]), G=s["G"])
    rl, rv, _ = theory.maxwell(P)
    # the paper quotes "approximately 514 and 79.5"
    assert rl == pytest.approx(g["rho_L"], rel=2e-3)
    assert rv == pytest.approx(g["rho_V"], rel=5e-3)
    # for this potential Eq. (16) with epsilon = 0 is the Maxwell rule
    rl2, rv2, _ = theory.coexistence(P, 0.0)
    assert rl2 == pytest.approx(rl, rel=1e-8) and rv2 == pytest.approx(rv, rel=1e-7)


def test_flat_tension_theory_close_to_paper(golden):
    # leading-order flat-interface tension vs the droplet values of Tables 2 and 3
    s = golden["exp_potential_setup"]
    Pe = O.Params(nx=1, ny=1, eos_kind=O.EOS_EXP, eos=(s["psi0"], s["rho0"]), G=s["G"])
    assert theory.flat_surface_tension(Pe, 0.0) == pytest.approx(golden["table2"]["tension"][0], rel=0.04)
    g = golden["piecewise_setup"]
    Pp = piecewise_params(g, 1)
    eps = -16 * g["G"] * g["sigma"]
    assert theory.flat_surface_tension(Pp, eps) == pytest.approx(golden["table3"]["tension"][0], rel=0.04)


# -------------------------------------------------- mechanical stability (Eq. 16)

def test_flat_interface_cs_satisfies_mechanical_stability():
    eps = 1.93
    P = O.Params(nx=1, ny=256, eos_kind=O.EOS_CS, eos=(0.25, 4.0, 1.0, 0.7 * T_C), G=-1.0,
                 sigma=O.sigma_from_epsilon(eps, -1.0), s=O.rates())
    rl_t, rv_t, _ = theory.coexistence(P, eps)
    rl, rv = run_slab(P, rl_t, rv_t, 20000)
    # leading-order theory neglects higher-order gradient terms: the paper's own gap
    # between Table 3 and this theory is ~5% in the vapour density
    assert rl == pytest.approx(rl_t, rel=5e-3)
    assert rv == pytest.approx(rv_t, rel=3e-2)


def test_flat_interface_piecewise_and_kappa_invariance(golden):
    g = golden["piecewise_setup"]
    eps = -16 * g["G"] * g["sigma"]
    res = []
    for kappa in (0.0, 0.9):
        P = piecewise_params(g, 1, kappa=kappa, ny=256)
        res.append(run_slab(P, 100.0, 1.0, 12000))
    rl_t, rv_t, _ = theory.coexistence(piecewise_params(g, 1), eps)
    for rl, rv in res:
        assert rl == pytest.approx(rl_t, rel=1e-3)
        assert rv == pytest.approx(rv_t, rel=3e-2)
    # Section IV: kappa changes the surface tension but not the coexistence densities
    assert res[1][1] == pytest.approx(res[0][1], rel=1e-2)
    assert res[1][0] == pytest.approx(res[0][0], rel=1e-4)


# -------------------------------------------------- Tables 2 and 3 (droplets)

def test_table3_droplet_densities(golden):
    g, t3 = golden["piecewise_setup"], golden["table3"]
    P = piecewise_params(g, 120, kappa=0.0, s=O.rates(s_nu=O.s_nu_from_viscosity(0.1)))
    d = run_droplet(P, g["rho_L"], g["rho_V"], 40, 6000)
    assert d["rho_in"] == pytest.approx(t3["rho_L"][0], rel=1e-3)
    assert d["rho_out"] == pytest.approx(t3["rho_V"][0], rel=1.5e-2)


def test_exponential_potential_droplet_densities(golden):
    s, e = golden["exp_potential_setup"], golden["exp_droplet_densities"]
    d = run_droplet(exp_params(s), 514.6, 79.7, s["R"], 6000)
    assert d["rho_in"] == pytest.approx(e["rho_L"][0], rel=2e-3)
    assert d["rho_out"] == pytest.approx(e["rho_V"][0], rel=5e-3)
    assert d["rho_in"] / d["rho_out"] == pytest.approx(e["ratio"][0], rel=5e-3)


def test_surface_tension_scales_with_one_minus_kappa(golden):
    """Section IV / Table 3: the tension coefficient becomes (1 - kappa) while the
    densities barely move."""
    g, t3 = golden["piecewise_setup"], golden["table3"]
    out = {}
    for kappa in (0.0, 0.5, 0.95):
        P = piecewise_params(g, 72, kappa=kappa, s=O.rates(s_nu=1.0))
        d = run_droplet(P, g["rho_L"], g["rho_V"], 20, 3000, r_out_pad=10.0)
        out[kappa] = (d["dp"] * d["r_eq"], d["rho_in"], d["rho_out"])
    s0 = out[0.0][0]
    # Laplace tension at R = 20 vs Table 3 (R = 40): curvature corrections ~2%
    assert s0 == pytest.approx(t3["tension"][0], rel=0.05)
    assert out[0.5][0] / s0 == pytest.approx(t3["tension"][1] / t3["tension"][0], abs=0.03)
    assert out[0.95][0] / s0 == pytest.approx(t3["tension"][2] / t3["tension"][0], abs=0.015)
    ratios = [v[1] / v[2] for v in out.values()]
    assert max(ratios) / min(ratios) - 1 < 0.03


def test_laplace_law_is_linear_in_inverse_radius(golden):
    g, t3 = golden["piecewise_setup"], golden["table3"]
    P = piecewise_params(g, 72, kappa=0.0, s=O.rates(s_nu=1.0))
    xs, ys = [], []
    for R in (12, 16, 20):
        d = run_droplet(P, g["rho_L"], g["rho_V"], R, 3000, r_out_pad=10.0)
        xs.append(1 / d["r_eq"])
        ys.append(d["dp"])
    slope, icpt = np.polyfit(xs, ys, 1)
    fit = slope * np.array(xs) + icpt
    assert np.abs(fit - ys).max() < 2e-3 * max(ys)
    # small drops carry a curvature correction: slope ~10% under the R = 40 value
    assert slope == pytest.approx(t3["tension"][0], rel=0.12)
    assert abs(icpt) < 0.1 * min(ys)


# -------------------------------------------------- capillary waves (Eq. 24)

def _interface(col, m):
    i = np.where((col[:-1] >= m) & (col[1:] < m))[0][0]
    return i + (col[i] - m) / (col[i] - col[i + 1])


def capillary_period(g, L, kappa, steps):
    H = int(3.5 * L)
    P = piecewise_params(g, L, kappa=kappa, ny=H, s=O.rates(s_nu=O.s_nu_from_viscosity(0.01)),
                         bc_y=O.BC_WALL)
    rl, rv = 100.13, 1.012
    f = O.init(P, WL.wave(L, H, rl, rv, L, 0.125 * L))
    m = (rl + rv) / 2
    amp, ts = [], []
    for t in range(0, steps, 10):
        rho, _, _ = O.moments(P, f)
        amp.append(0.5 * (_interface(rho[:, 0], m) - _interface(rho[:, L // 2], m)))
        ts.append(t)
        f = O.run(P, f, 10)
    amp = np.array(amp)
    z = [ts[i] + 10 * amp[i] / (amp[i] - amp[i + 1]) for i in range(len(amp) - 1)
         if amp[i] * amp[i + 1] < 0]
    return 2 * np.mean(np.diff(z))


def test_capillary_wave_follows_dispersion(golden):
    """Eq. (24) read as omega^2 = sigma k^3 / (rho_L + rho_V); scaled-down Table 4 set-up."""
    g, t3 = golden["piecewise_setup"], golden["table3"]
    L = 64
    k = 2 * np.pi / L
    periods = {}
    for kappa, steps in ((0.0, 2600), (0.5, 3800)):
        periods[kappa] = capillary_period(g, L, kappa, steps)
        omega = np.sqrt(t3["tension"][0] * (1 - kappa) * k ** 3 / (g["rho_L"] + g["rho_V"]))
        # the paper's own numerical periods differ from Eq. (24) by up to 3.5% (Table 4)
        assert periods[kappa] == pytest.approx(2 * np.pi / omega, rel=0.06)
    # omega^2 proportional to the tension: T(kappa = 0.5) / T(0) = sqrt(2)
    assert periods[0.5] / periods[0.0] == pytest.approx(np.sqrt(2), rel=0.05)
