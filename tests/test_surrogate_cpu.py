"""Host logic of the surrogate-guided parameter selection (CPU only): when the
network-guided picks miss the target within their budget, the full LB search
(here a stand-in verifier with a closed-form response) takes over as the
fallback, and every solve is counted."""
import math

import numpy as np

from paper_1306_6445_amd import surrogate as S


class StandInVerifier:
    """Counts solves like surrogate.Verifier; its response follows the trends
    of Section IV: the density ratio falls with T/T_c and does not depend on
    kappa, the tension scales as 1 - kappa."""

    def __init__(self):
        self.solves = 0

    def __call__(self, T, k, eps):
        self.solves += 1
        ratio = math.exp(12.0 * (0.85 - T)) * (1.0 + 0.1 * (eps - 1.5))
        sigma = 0.004 * (0.9 - T) * (1.0 - k)
        return S.Verified(T, k, eps, ratio, sigma, True)


class WrongNetwork:
    """A network whose predictions are far off (never near the target)."""

    def predict(self, P):
        P = np.atleast_2d(P)
        return np.stack([np.full(len(P), 2.0), np.full(len(P), 1.0), np.full(len(P), 1e-6)], axis=1)


def test_missed_network_budget_hands_over_to_the_lb_search():
    truth = StandInVerifier()(0.7, 0.4, 1.5)
    v = StandInVerifier()
    r = S.surrogate_select(WrongNetwork(), v, truth.ratio, truth.sigma, 1.5, max_solves=3)
    assert r["network_solves"] == 3 and r["fallback"]
    assert r["hit"], r
    assert r["solves"] == r["network_solves"] + r["fallback_solves"] == v.solves
    assert abs(r["final"].ratio / truth.ratio - 1) < 0.01 and abs(r["final"].sigma / truth.sigma - 1) < 0.01


def test_no_fallback_when_disabled_or_not_needed():
    truth = StandInVerifier()(0.7, 0.4, 1.5)
    v = StandInVerifier()
    r = S.surrogate_select(WrongNetwork(), v, truth.ratio, truth.sigma, 1.5, max_solves=2, fallback_solves=0)
    assert not r["fallback"] and not r["hit"] and r["solves"] == 2 == v.solves
    # the physics-aware search alone, from its default start, also hits
    v2 = StandInVerifier()
    p = S.physics_select(v2, truth.ratio, truth.sigma, 1.5)
    assert p["hit"] and p["solves"] == v2.solves
