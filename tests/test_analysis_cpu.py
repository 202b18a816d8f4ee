"""Host-side post-processing (paper_1306_6445_amd/analysis.py) on synthetic
inputs, no GPU: the time-averaged Laplace estimator, the Laplace fit, the
damped-cosine fit and interface tracking."""
import math

import numpy as np
import pytest

from paper_1306_6445_amd import analysis as A


class FakeLattice:
    """Stands in for lbm.Lattice: a step counter and diagnostics that ring
    around a fixed pressure jump, dp(t) = dp0 (1 + a cos(w t))."""

    def __init__(self, dp0, amp, omega):
        self.t = 0
        self.dp0, self.amp, self.omega = dp0, amp, omega
        self.calls = []

    def step(self, n):
        assert n >= 0
        self.t += n

    def diagnostics(self, regions):
        self.calls.append(self.t)
        out = []
        for i, _ in enumerate(regions):
            dp = self.dp0[i] * (1 + self.amp * math.cos(self.omega * self.t))
            out.append({"dp": dp, "r_eq": 10.0 + i, "rho_in": 1.0, "rho_out": 0.1, "p_in": dp, "p_out": 0.0,
                        "mass": 1.0, "max_speed": 0.0, "status": 1 if self.t == 150 and i == 1 else 0})
        return out


def test_averaged_diagnostics_samples_the_window_and_averages():
    L = FakeLattice([1e-3, 2e-3], amp=5.0, omega=2 * math.pi / 200.0)
    snap, mean = A.averaged_diagnostics(L, [(0, 0, 1, 2), (0, 0, 1, 2)], steps=1000, window=400, every=50)
    assert L.t == 1000
    assert L.calls == list(range(600, 1001, 50))  # both ends of the window included
    # nine samples over two periods of four: the cosines cancel except for the
    # closing sample (cos = 1), so the mean is dp0 (1 + amp / 9)
    for i, d in enumerate(mean):
        assert d["dp"] == pytest.approx(L.dp0[i] * (1 + 5.0 / 9), rel=1e-12)
        assert d["r_eq"] == 10.0 + i
    assert snap[0]["dp"] == pytest.approx(1e-3 * 6.0)  # cos(0) at t = 1000: the snapshot is off by the swing
    assert mean[1]["status"] == 0 and max(c for c in L.calls) == 1000
    # a status raised at any sample is kept
    L2 = FakeLattice([1e-3, 2e-3], amp=0.0, omega=0.0)
    _, mean2 = A.averaged_diagnostics(L2, [(0, 0, 1, 2)] * 2, steps=200, window=100, every=50)
    assert mean2[1]["status"] == 1 and mean2[0]["status"] == 0


def test_averaged_diagnostics_window_longer_than_run_and_ragged_every():
    L = FakeLattice([1.0], amp=0.0, omega=0.0)
    snap, mean = A.averaged_diagnostics(L, [(0, 0, 1, 2)], steps=120, window=500, every=50)
    assert L.calls == [0, 50, 100, 120]
    assert mean[0]["dp"] == pytest.approx(1.0) and snap[0]["dp"] == pytest.approx(1.0)


def test_laplace_fit_recovers_slope_and_skips_diverged():
    class R:
        def __init__(self, k):
            self.kappa = k
    sigma = {0.0: 0.02, 0.5: 0.01}
    runs, diags = [], []
    for k, s in sigma.items():
        for Req in (20.0, 30.0, 40.0):
            runs.append(R(k))
            diags.append({"r_eq": Req, "dp": s / Req + 1e-5, "status": 0})
    runs.append(R(0.5))
    diags.append({"r_eq": 25.0, "dp": 1.0, "status": 1})  # diverged: ignored
    fit = A.laplace_fit(diags, runs)
    for k, s in sigma.items():
        assert fit[k][0] == pytest.approx(s, rel=1e-12)
        assert fit[k][1] == pytest.approx(1e-5, abs=1e-12)


def test_damped_cosine_fit_and_crossing_period():
    t = np.arange(0, 3000, 10.0)
    w, g = 2 * math.pi / 700.0, 4e-4
    a = 2.0 * np.exp(-g * t) * np.cos(w * t + 0.3) + 0.1
    fit = A.damped_cosine_fit(t, a)
    assert fit["omega"] == pytest.approx(w, rel=1e-6)
    assert fit["gamma"] == pytest.approx(g, rel=1e-4)
    assert A.crossing_period(t, np.cos(w * t)) == pytest.approx(700.0, rel=1e-3)


def test_cosine_fit_given_decay_over_less_than_a_period():
    """0.4 of a period: with the decay and offset given, omega comes back
    exactly, also from starting values 3% off."""
    t = np.arange(0, 50000, 250.0)
    w, g, c = 2 * math.pi / 125000.0, 2e-6, -0.4
    a = 10.0 * np.exp(-g * t) * np.cos(w * t - 0.05) + c
    assert A.cosine_fit_given_decay(t, a, g, c, 9.0, 1.03 * w, 0.0) == pytest.approx(w, rel=1e-8)


def test_interface_height_interpolates_the_crossing():
    y = np.arange(64, dtype=float)
    col = 0.5 - 0.4 * np.tanh((y - 30.25) / 3.0)  # liquid below, vapour above, midpoint 0.5 at y = 30.25
    assert A.interface_height(col, 0.5) == pytest.approx(30.25, abs=2e-2)
    assert math.isnan(A.interface_height(np.ones(8), 0.5))
