"""Physics of the HIP path at the paper's own set-ups (needs an MI355X).

These are not parity tests (those compare with the oracle node by node); they
check that the GPU path, in FP64 and in FP32, reproduces what the paper
reports: Table 2 (exponential psi) and Table 3 (Eq. 23) droplet tensions and
densities, Table 4 capillary periods, and, for the Carnahan-Starling fluid of
the capillary workload, the dispersion relation Eq. (24) with the tension from
a Laplace fit.  FP32 is also held to FP64 within 0.5% on the same runs.
"""
import sys

import numpy as np
import pytest

from paper_1306_6445_amd import analysis as A, lbm, workloads as WL

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def droplet_table(precision, steps):
    runs = ([WL.paper_droplet_run("exp", k) for k in (0.0, 0.5, 0.95, 0.99)]
            + [WL.paper_droplet_run("pw", k) for k in (0.0, 0.5, 0.95, 0.99)])
    say("  droplets", precision, steps, [r.label for r in runs])
    with lbm.Lattice(runs, precision=precision) as L:
        L.init_all()
        L.step(steps)
        d = L.diagnostics([(r.cx, r.cy, *r.diag_radii()) for r in runs])
    return runs, d


def test_tables_2_and_3_droplet_tension_on_gpu(golden):
    """Table 2 (exp psi) and Table 3 (Eq. 23) at R = 40: sigma = dp R matches
    the paper for kappa <= 0.5 and scales as (1 - kappa) (Section IV); the
    densities match Table 3 and barely move with kappa; FP32 against FP64."""
    t2, t3 = golden["table2"], golden["table3"]
    res = {p: droplet_table(p, 20000) for p in ("fp64", "fp32")}
    runs, d64 = res["fp64"]
    _, d32 = res["fp32"]
    sig64 = [d["dp"] * d["r_eq"] for d in d64]
    sig32 = [d["dp"] * d["r_eq"] for d in d32]
    for r, a, b, x, y in zip(runs, sig64, sig32, d64, d32):
        say("  %-16s sigma fp64 %.5g fp32 %.5g  rho %.6g/%.6g ratio %.6g  fp32 ratio %.6g  mass fp32/fp64-1 %.2e"
            % (r.label, a, b, x["rho_in"], x["rho_out"], x["rho_in"] / x["rho_out"], y["rho_in"] / y["rho_out"],
               y["mass"] / x["mass"] - 1))
        assert x["status"] == 0 and y["status"] == 0
    say("  paper Table 2", t2["tension"], "Table 3", t3["tension"])
    for blk, table in ((0, t2["tension"]), (4, t3["tension"])):
        s0 = sig64[blk]
        # kappa = 0 and 0.5 against the printed tensions; 5% covers the
        # curvature correction at R = 40 and the tanh seed
        assert s0 == pytest.approx(table[0], rel=0.05)
        assert sig64[blk + 1] == pytest.approx(table[1], rel=0.05)
        # sigma(kappa) / sigma(0) = 1 - kappa, to 1.5% of sigma(0)
        for i in range(4):
            assert sig64[blk + i] / s0 == pytest.approx(1.0 - runs[blk + i].kappa, abs=0.015)
        # kappa moves the density ratio by at most 2% (Table 3 itself: 1.4%)
        ratios = [x["rho_in"] / x["rho_out"] for x in d64[blk:blk + 4]]
        assert max(ratios) / min(ratios) - 1 < 0.02
        # FP32: tension error below 0.5% of sigma(0) (relative error at
        # kappa = 0 below 0.5%); density ratio within 0.5%
        for i in range(4):
            assert abs(sig32[blk + i] - sig64[blk + i]) < 5e-3 * s0, runs[blk + i].label
    for i in range(4):
        assert d64[4 + i]["rho_in"] == pytest.approx(t3["rho_L"][i], rel=1e-3)
        assert d64[4 + i]["rho_out"] == pytest.approx(t3["rho_V"][i], rel=2e-2)
    for x, y in zip(d64, d32):
        assert abs((y["rho_in"] / y["rho_out"]) / (x["rho_in"] / x["rho_out"]) - 1) < 5e-3


def test_table4_capillary_periods_on_gpu(golden):
    """Table 4: capillary periods for 1 - kappa = 1, 0.5, 0.25 against Eq. (24)
    and against the paper's own numerical periods, FP64 and FP32."""
    t4 = golden["table4"]
    kappas = [1.0 - v for v in t4["one_minus_kappa"]]
    runs = [WL.paper_wave_run(k) for k in kappas]
    L = runs[0].nx
    periods = {}
    for prec in ("fp64", "fp32"):
        say("  waves", prec, [r.label for r in runs])
        with lbm.Lattice(runs, precision=prec) as lat:
            lat.init_all()
            tr = A.track_standing_wave(lat, list(range(len(runs))), L, 27000, 20, 0.5 * (100.13 + 1.012))
            assert not lat.status().any()
        periods[prec] = [A.crossing_period(tr["t"], a) for a in tr["a"]]
        say("  periods", prec, periods[prec], "paper numerical", t4["numerical"], "analytic", t4["analytic"])
    for T, an, num in zip(periods["fp64"], t4["analytic"], t4["numerical"]):
        # the paper's numerical periods are within 3.5% of Eq. (24)
        assert T == pytest.approx(an, rel=0.06)
        assert T == pytest.approx(num, rel=0.05)
    assert periods["fp64"][1] / periods["fp64"][0] == pytest.approx(np.sqrt(2), rel=0.05)
    assert periods["fp64"][2] / periods["fp64"][0] == pytest.approx(2.0, rel=0.06)
    for a, b in zip(periods["fp64"], periods["fp32"]):
        assert abs(b / a - 1) < 5e-3


def test_capillary_dispersion_cs_fluid_on_gpu():
    """The capillary workload's fluid (CS EOS, T/Tc = 0.6, nu = 0.01): omega of
    a lambda = 256 standing wave against Eq. (24) with the flat-interface tension
    from FP64 droplets; FP32 keeps omega and rho_l / rho_v within 0.5% of FP64,
    bf16 storage omega within 1% and the ratio within 0.5%."""
    lap = A.laplace_sigma(lbm, 0.6, 1.93)
    say("  laplace", {k: lap[k] for k in ("sigma", "sigma_flat", "tolman_length", "rho_l", "rho_v")})
    lam = 256
    run = WL.config3(wavelength=lam, nx=lam, ny=2 * lam)
    ex = A.capillary_experiment(lbm, run, ("fp64", "fp32", "bf16"), lam, 30000, 100)
    ref = ex["fp64"]
    w_th = A.capillary_omega(lap["sigma_flat"], lam, ref["rho_l"], ref["rho_v"])
    for p, e in ex.items():
        say("  %s omega %.6g (theory %.6g) gamma %.3g rho %.6g/%.6g" % (p, e["fit"]["omega"], w_th,
                                                                       e["fit"]["gamma"], e["rho_l"], e["rho_v"]))
    assert ref["fit"]["omega"] == pytest.approx(w_th, rel=0.06)
    f32 = ex["fp32"]
    assert abs(f32["fit"]["omega"] / ref["fit"]["omega"] - 1) < 5e-3
    assert abs((f32["rho_l"] / f32["rho_v"]) / (ref["rho_l"] / ref["rho_v"]) - 1) < 5e-3
    # bf16 storage (8 significant bits per stored deviation, stochastic
    # rounding): omega within 1%, the density ratio within 0.5%
    b16 = ex["bf16"]
    assert b16["status"] == 0
    assert abs(b16["fit"]["omega"] / ref["fit"]["omega"] - 1) < 1e-2
    assert abs((b16["rho_l"] / b16["rho_v"]) / (ref["rho_l"] / ref["rho_v"]) - 1) < 5e-3


@pytest.mark.parametrize("lam,steps,precs", [(512, 50000, ("fp64", "fp32", "bf16")),
                                              (1024, 130000, ("fp64", "fp32", "bf16"))],
                         ids=["lambda512", "lambda1024"])
def test_capillary_long_waves_on_the_full_grid(lam, steps, precs):
    """The capillary workload's long waves on its full 4096 x 2048 grid
    (periodic in x, walls in y, liquid depth 1024: deep for both): lambda =
    512 over its 50,000 steps (1.2 periods) and lambda = 1024 over 130,000
    steps (1.1 periods; 50,000 steps hold only 0.42 of its period).  FP64 omega
    within 6% of Eq. (24) with the flat-interface Laplace tension (observed
    +2.3% / +2.5%), the omega(512) / omega(1024) ratio within 3% of the
    k^(3/2) law's 2^(3/2); FP32 omega and rho_l / rho_v within 0.5% of FP64,
    bf16 storage omega within 1% and the ratio within 0.5%."""
    lap = A.laplace_sigma(lbm, 0.6, 1.93)
    run = WL.config3(wavelength=lam)
    say("  lambda", lam, "steps", steps, (run.nx, run.ny))
    ex = A.capillary_experiment(lbm, run, precs, lam, steps, 250)
    ref = ex["fp64"]
    w_th = A.capillary_omega(lap["sigma_flat"], lam, ref["rho_l"], ref["rho_v"])
    for p, e in ex.items():
        say("  %s omega %.6g (theory %.6g, period %.0f steps) crossings %d rho %.6g/%.6g"
            % (p, e["fit"]["omega"], w_th, 2 * np.pi / w_th, e["fit"]["crossings"], e["rho_l"], e["rho_v"]))
        assert e["status"] == 0
    assert ref["fit"]["crossings"] >= 2
    assert ref["fit"]["omega"] == pytest.approx(w_th, rel=0.06)
    # the crossing period agrees with the fitted one (a clean, lightly damped wave)
    assert A.crossing_period(ref["t"], ref["a"]) == pytest.approx(2 * np.pi / ref["fit"]["omega"], rel=0.03)
    _LONG_WAVE_OMEGA[lam] = ref["fit"]["omega"]
    if len(_LONG_WAVE_OMEGA) == 2:
        assert _LONG_WAVE_OMEGA[512] / _LONG_WAVE_OMEGA[1024] == pytest.approx(2 ** 1.5, rel=0.03)
    ratio = ref["rho_l"] / ref["rho_v"]
    for p, tol in (("fp32", 5e-3), ("bf16", 1e-2)):
        e = ex[p]
        assert abs(e["fit"]["omega"] / ref["fit"]["omega"] - 1) < tol, p
        assert abs((e["rho_l"] / e["rho_v"]) / ratio - 1) < 5e-3, p


_LONG_WAVE_OMEGA = {}


def test_table5_splash_spread_radius_on_gpu(golden):
    """Section V.C set-up (Eq. 23, rho_L/rho_V = 100, R = 50, U = 0.125, Re =
    1000, nu_V/nu_L = 20 switched at rho1, film 25), kappa = 0: the spreading
    radius one row above the film grows as in Table 5.  The paper's top and
    sides are open boundaries (unspecified); here a top wall and periodic
    sides, so the comparison is coarse: within 20% of the printed radii and of
    1.3 sqrt(t*).  FP32 gives the FP64 radii to the node."""
    t5 = golden["table5"]
    D, U = 100.0, 0.125
    times = [int(round(ts * D / U)) for ts in t5["t_star"]]
    run = WL.paper_splash_run(0.0)
    res = {}
    for prec in ("fp64", "fp32"):
        with lbm.Lattice([run], precision=prec) as L:
            L.init_all()
            res[prec] = A.splash_history(L, 0, times, 28, 50.5, run.nx / 2)
            assert L.status()[0] == 0
    r64 = np.array(res["fp64"]["r"]) / D
    say("  r/D fp64", np.round(r64, 4), "paper", t5["kappa0"], "1.3 sqrt(t*)", t5["power_law"])
    assert np.all(np.diff(r64) > 0)
    for r, p, law, ts in zip(r64, t5["kappa0"], t5["power_law"], t5["t_star"]):
        if ts >= 0.25:
            assert r == pytest.approx(p, rel=0.2)
            assert r == pytest.approx(law, rel=0.2)
    np.testing.assert_allclose(np.array(res["fp32"]["r"]), np.array(res["fp64"]["r"]), atol=1.0)
    m = res["fp64"]["mass"]
    assert abs(m[-1] / m[0] - 1) < 1e-12


def test_table1_multirange_potential_on_gpu(golden):
    """Section III.B / Table 1: with the multi-range force of Eq. (9) the
    tension falls from case A to D but stays of the same order (the continuum
    pressure tensor Eq. 10 would scale it by (G1 + 8 G2)/G = 0.01 at D), and the
    coexistence densities move with (G1, G2) (the text: vapour density and
    ratio off by about 10% and 9% at D).  Tensions dp R at R = 40 after 30,000
    steps: A and B within 5% of Table 1, C and D within 15%; FP32 within 0.5%
    of FP64."""
    t1 = golden["table1"]
    runs = [WL.paper_multirange_run(c) for c in t1["case"]]
    res = {}
    for prec in ("fp64", "fp32"):
        with lbm.Lattice(runs, precision=prec) as L:
            L.init_all()
            L.step(30000)
            res[prec] = L.diagnostics([(r.cx, r.cy, *r.diag_radii()) for r in runs])
    d64 = res["fp64"]
    sig = [d["dp"] * d["r_eq"] for d in d64]
    rv = [d["rho_out"] for d in d64]
    ratio = [d["rho_in"] / d["rho_out"] for d in d64]
    say("  tension", np.round(sig, 4), "Table 1", t1["tension"])
    say("  rho_v", np.round(rv, 3), "ratio", np.round(ratio, 4))
    for i, (s_, t) in enumerate(zip(sig, t1["tension"])):
        assert s_ == pytest.approx(t, rel=0.05 if i < 2 else 0.15), t1["case"][i]
    # Section III.B's reading of Eq. (14): sigma = a sigma_1 + b sigma_2 with
    # a = (G1 + 8 G2)/G and b = -2 G2/G, sigma_1 and sigma_2 the same in every
    # case.  Solving B and C for them must predict D (the paper's own numbers
    # do so to 4%); the gap to the printed C and D lies in sigma_2 alone.
    coef = [((g1 + 8 * g2), -2 * g2) for g1, g2 in (WL.MULTIRANGE_CASES[c] for c in t1["case"])]
    s1, s2 = np.linalg.solve(np.array([coef[1], coef[2]]), np.array([sig[1], sig[2]]))
    d_est = coef[3][0] * s1 + coef[3][1] * s2
    say("  Eq. 14 split: sigma_1 %.4f sigma_2 %.4f -> case D %.4f (measured %.4f)" % (s1, s2, d_est, sig[3]))
    assert d_est == pytest.approx(sig[3], rel=0.02)
    assert s1 == pytest.approx(sig[0], rel=0.08)
    assert all(a > b for a, b in zip(sig, sig[1:]))
    assert sig[3] > 0.25 * sig[0]
    assert all(a > b for a, b in zip(rv, rv[1:])) and all(a < b for a, b in zip(ratio, ratio[1:]))
    assert -0.12 < rv[3] / rv[0] - 1 < -0.06
    assert 0.03 < ratio[3] / ratio[0] - 1 < 0.12
    for a, b in zip(d64, res["fp32"]):
        assert abs(b["dp"] * b["r_eq"] / (a["dp"] * a["r_eq"]) - 1) < 5e-3
        assert abs((b["rho_in"] / b["rho_out"]) / (a["rho_in"] / a["rho_out"]) - 1) < 5e-3
