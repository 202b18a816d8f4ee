"""Host-side analysis of GPU runs: Laplace fits and capillary-wave tracking.

Only post-processing of what the HIP library returns (diagnostics, density
columns); no lattice-Boltzmann arithmetic.

* Laplace law (Section IV): the pressure jump across a droplet is
  dp = sigma / R in two dimensions, so sigma is the slope of dp against 1/R.
* Capillary waves: a small standing wave a(t) cos(k x) on a flat interface
  between two deep layers oscillates as a(t) ~ cos(omega t) exp(-gamma t) with
  omega^2 = sigma k^3 / (rho_l + rho_v) (linear inviscid theory, depth >> 1/k).
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence

import numpy as np


def laplace_fit(diags: Sequence[dict], runs: Sequence, key=lambda r: r.kappa) -> Dict:
    """Per group (default: kappa): (slope, intercept) of dp against 1/R_eq over
    the runs of the group that did not diverge."""
    out = {}
    for g in sorted(set(key(r) for r in runs)):
        xs = [1.0 / d["r_eq"] for d, r in zip(diags, runs) if key(r) == g and d["status"] == 0]
        ys = [d["dp"] for d, r in zip(diags, runs) if key(r) == g and d["status"] == 0]
        if len(xs) >= 2:
            s, b = np.polyfit(xs, ys, 1)
            out[g] = (float(s), float(b))
    return out


def averaged_diagnostics(lattice, regions, steps: int, window: int, every: int):
    """Advance `lattice` by `steps` steps and return (snapshot, mean): the
    per-run diagnostics at the end, and the same with dp, r_eq, rho_in,
    rho_out, p_in and p_out averaged over the last `window` steps (sampled
    every `every` steps, both ends included).  A droplet relaxing from its
    initial profile rings acoustically for many thousand steps (small,
    weakly damped drops at large kappa swing by several times their mean
    pressure jump); the Laplace pressure jump is the time average."""
    window = min(window, steps)
    lattice.step(steps - window)
    samples = [lattice.diagnostics(regions)]
    t = 0
    while t < window:
        n = min(every, window - t)
        lattice.step(n)
        t += n
        samples.append(lattice.diagnostics(regions))
    mean = []
    for i in range(len(regions)):
        d = dict(samples[-1][i])
        for key in ("dp", "r_eq", "rho_in", "rho_out", "p_in", "p_out"):
            d[key] = float(np.mean([s[i][key] for s in samples]))
        d["status"] = max(s[i]["status"] for s in samples)
        mean.append(d)
    return samples[-1], mean


def interface_height(column: np.ndarray, rho_mid: float) -> float:
    """Height of the liquid-below / vapour-above interface in a density column:
    the downward crossing of rho_mid nearest to mid-height, linearly
    interpolated between nodes.  NaN if the column has no such crossing."""
    s = np.asarray(column, dtype=float) - rho_mid
    idx = np.nonzero((s[:-1] > 0) & (s[1:] <= 0))[0]
    if idx.size == 0:
        return float("nan")
    i = int(idx[np.argmin(np.abs(idx - 0.5 * (s.size - 1)))])
    return i + s[i] / (s[i] - s[i + 1])


def bulk_densities(column: np.ndarray, margin: int = 16) -> tuple:
    """(rho_l, rho_v) of a column with liquid below and vapour above, from the
    quarter-heights (away from the interface and from the walls)."""
    n = len(column)
    lo = column[max(margin, n // 4 - margin): n // 4 + margin]
    hi = column[3 * n // 4 - margin: min(n - margin, 3 * n // 4 + margin)]
    return float(np.mean(lo)), float(np.mean(hi))


def damped_cosine_fit(t: np.ndarray, a: np.ndarray) -> dict:
    """Least-squares fit a(t) = A exp(-gamma t) cos(omega t + phi) + c.

    The starting omega comes from the mean spacing of the zero crossings of
    a - mean(a); the fit then polishes (A, gamma, omega, phi, c)."""
    from scipy.optimize import curve_fit

    t = np.asarray(t, dtype=float)
    a = np.asarray(a, dtype=float)
    z = a - a.mean()
    cross = []
    for i in range(len(z) - 1):
        if z[i] == 0.0 or z[i] * z[i + 1] < 0:
            cross.append(t[i] + (t[i + 1] - t[i]) * z[i] / (z[i] - z[i + 1]))
    if len(cross) >= 2:
        w0 = math.pi / float(np.mean(np.diff(cross)))
    else:
        w0 = math.pi / (t[-1] - t[0])
    A0 = float(a[0] - a.mean()) or float(np.abs(z).max())

    def model(tt, A, g, w, phi, c):
        return A * np.exp(-g * tt) * np.cos(w * tt + phi) + c

    p0 = (A0, 1.0 / (t[-1] - t[0] + 1.0), w0, 0.0, float(a.mean()))
    p, cov = curve_fit(model, t, a, p0=p0, maxfev=20000)
    resid = a - model(t, *p)
    A, g, w, phi, c = (float(v) for v in p)
    if A < 0:
        A, phi = -A, phi + math.pi
    return {"omega": abs(w), "gamma": g, "amplitude": A, "phase": phi, "offset": c,
            "crossings": len(cross), "omega_crossings": w0,
            "rms_residual": float(np.sqrt(np.mean(resid ** 2))),
            "omega_stderr": float(math.sqrt(max(cov[2, 2], 0.0))) if np.all(np.isfinite(cov)) else None}


def cosine_fit_given_decay(t: np.ndarray, a: np.ndarray, gamma: float, offset: float, A0: float, omega0: float,
                           phase0: float) -> float:
    """omega of a(t) = A exp(-gamma t) cos(omega t + phi) + offset with gamma
    and offset given (A, omega, phi fitted from the starting values): over
    less than one period, decay, offset and frequency trade off against each
    other in the free fit, so histories of one wave in several precisions are
    compared at the decay and offset of a reference fit."""
    from scipy.optimize import curve_fit

    t = np.asarray(t, dtype=float)
    a = np.asarray(a, dtype=float)

    def model(tt, A, w, phi):
        return A * np.exp(-gamma * tt) * np.cos(w * tt + phi) + offset

    p, _ = curve_fit(model, t, a, p0=(A0, omega0, phase0), maxfev=20000)
    return abs(float(p[1]))


def capillary_omega(sigma: float, wavelength: float, rho_l: float, rho_v: float) -> float:
    """Linear inviscid deep-layer capillary frequency sqrt(sigma k^3 / (rho_l + rho_v))."""
    k = 2.0 * math.pi / wavelength
    return math.sqrt(sigma * k ** 3 / (rho_l + rho_v))


def track_standing_wave(lattice, run, wavelength: int, steps: int, every: int,
                        rho_mid: float) -> dict:
    """Advance `lattice` by `steps` steps and record the standing-wave amplitude
    a(t) = (h(0) - h(lambda/2)) / 2 every `every` steps, h from the density
    columns at a crest and a trough (read through the library).  `run` is one
    run index or a list of them (all advanced together); with a list, "a" and
    "final_column" are lists in the same order."""
    many = not isinstance(run, (int, np.integer))
    ids = list(run) if many else [int(run)]
    ts: List[int] = []
    amp: List[List[float]] = [[] for _ in ids]
    t = 0
    while True:
        for k, i in enumerate(ids):
            h0 = interface_height(lattice.density_column(i, 0), rho_mid)
            h1 = interface_height(lattice.density_column(i, wavelength // 2), rho_mid)
            amp[k].append(0.5 * (h0 - h1))
        ts.append(t)
        if t >= steps:
            break
        n = min(every, steps - t)
        lattice.step(n)
        t += n
    cols = [lattice.density_column(i, wavelength // 4) for i in ids]
    a = [np.asarray(v) for v in amp]
    return {"t": np.asarray(ts, dtype=float), "a": a if many else a[0],
            "final_column": cols if many else cols[0]}


def crossing_period(t: np.ndarray, a: np.ndarray) -> float:
    """Oscillation period from the sign changes of a(t): twice the mean spacing
    of the linearly interpolated zero crossings (NaN with fewer than two)."""
    z = [t[i] + (t[i + 1] - t[i]) * a[i] / (a[i] - a[i + 1]) for i in range(len(a) - 1)
         if a[i] * a[i + 1] < 0]
    return 2.0 * float(np.mean(np.diff(z))) if len(z) >= 2 else float("nan")


def laplace_sigma(lbm, T_over_Tc: float, epsilon: float, kappa: float = 0.0,
                  radii: Sequence[float] = (20.0, 28.0, 40.0), n: int = 192, steps: int = 20000,
                  precision: str = "fp64") -> dict:
    """Surface tension from the Laplace law: a batch of periodic droplets of the
    given radii stepped on the GPU, then the slope of dp against 1/R_eq."""
    from . import workloads as W

    runs = [W.droplet_run(n, R, T_over_Tc, kappa, epsilon, label="laplace_R%g" % R) for R in radii]
    L = lbm.Lattice(runs, precision=precision)
    try:
        L.init_all()
        L.step(steps)
        diags = L.diagnostics([(r.cx, r.cy, *r.diag_radii()) for r in runs])
    finally:
        L.close()
    fit = laplace_fit(diags, runs, key=lambda r: 0)
    if 0 not in fit:
        raise RuntimeError("Laplace fit failed: %s" % [d["status"] for d in diags])
    # curvature-corrected tension: dp R = sigma_flat (1 - delta / R) to first
    # order in 1/R (Tolman length delta), so the intercept of dp R against 1/R
    # is the tension of a flat interface
    inv = np.array([1.0 / d["r_eq"] for d in diags])
    prod = np.array([d["dp"] * d["r_eq"] for d in diags])
    slope_t, sigma_flat = np.polyfit(inv, prod, 1)
    return {"sigma": fit[0][0], "intercept": fit[0][1], "sigma_flat": float(sigma_flat),
            "tolman_length": float(-slope_t / sigma_flat),
            "rho_l": float(np.mean([d["rho_in"] for d in diags])),
            "rho_v": float(np.mean([d["rho_out"] for d in diags])), "r_eq": [d["r_eq"] for d in diags],
            "dp": [d["dp"] for d in diags]}


def capillary_experiment(lbm, run, precisions: Sequence[str], wavelength: int, steps: int,
                         every: int, graph_steps: int = 16) -> dict:
    """Standing capillary wave of `run` (liquid below, vapour above, crest at
    x = 0) advanced in each precision; per precision the amplitude history,
    its damped-cosine fit and the final density at a quarter wavelength."""
    out = {}
    rl0, rv0 = bulk_densities(run.rho[:, wavelength // 4])
    rho_mid = 0.5 * (rl0 + rv0)
    for prec in precisions:
        L = lbm.Lattice([run], precision=prec, graph_steps=graph_steps)
        try:
            L.init_all()
            tr = track_standing_wave(L, 0, wavelength, steps, every, rho_mid)
            st = int(L.status()[0])
        finally:
            L.close()
        fit = damped_cosine_fit(tr["t"], tr["a"]) if st == 0 and np.all(np.isfinite(tr["a"])) else None
        rl, rv = bulk_densities(tr["final_column"])
        out[prec] = {"t": tr["t"], "a": tr["a"], "fit": fit, "status": st, "rho_l": rl, "rho_v": rv,
                     "final_column": tr["final_column"]}
    return out


DROPLET_CLASSES = ("ok", "unsettled", "evaporated", "mixed", "diverged")


def classify_droplet(d: dict, run, min_ratio: float = 2.0, min_radius_frac: float = 0.5,
                     max_speed: float = 0.02) -> str:
    """'ok', 'diverged' (status flag), 'mixed' (no phase separation: rho_in /
    rho_out below min_ratio), 'evaporated' (R_eq below min_radius_frac R0) or
    'unsettled' (still moving: max |v| above max_speed, or a non-positive
    pressure jump)."""
    if d["status"] != 0 or not np.isfinite(d["rho_in"]):
        return "diverged"
    if not (d["rho_out"] > 0 and d["rho_in"] / d["rho_out"] >= min_ratio):
        return "mixed"
    if not (d["r_eq"] >= min_radius_frac * run.R0):
        return "evaporated"
    if not (d["max_speed"] <= max_speed and d["dp"] > 0):
        return "unsettled"
    return "ok"


def spread_radius(rho: np.ndarray, y: int, rho_mid: float, xc: float, outermost: bool = False) -> float:
    """Spreading radius of the lamella in row y just above the film: half the
    width of the liquid run (rho > rho_mid) that contains the impact column xc
    (NaN if xc is not liquid), or, with outermost, the largest |x - xc| of any
    liquid node of the row (once the impact column has drained)."""
    row = np.asarray(rho)[int(y)]
    liq = row > rho_mid
    i = int(round(xc))
    if outermost:
        xs = np.nonzero(liq)[0]
        return float(np.abs(xs - xc).max()) if xs.size else float("nan")
    if not liq[i]:
        return float("nan")
    lo = i
    while lo > 0 and liq[lo - 1]:
        lo -= 1
    hi = i
    while hi < len(row) - 1 and liq[hi + 1]:
        hi += 1
    return 0.5 * (hi - lo + 1)


def splash_history(lattice, run: int, times: Sequence[int], y: int, rho_mid: float, xc: float,
                   outermost: bool = False) -> dict:
    """Advance the lattice to each of `times` (steps, increasing) and record
    the spread radius (row y), the mass and the largest speed there."""
    out = {"t": [], "r": [], "mass": [], "max_speed": [], "rho": None}
    t = lattice.steps_taken
    for tt in times:
        if tt > t:
            lattice.step(tt - t)
            t = tt
        rho, ux, uy = lattice.moments(run, allow_diverged=True)
        out["t"].append(t)
        out["r"].append(spread_radius(rho, y, rho_mid, xc, outermost))
        out["mass"].append(float(rho.sum()))
        out["max_speed"].append(float(np.sqrt(ux ** 2 + uy ** 2).max()))
        out["rho"] = rho
    return out
