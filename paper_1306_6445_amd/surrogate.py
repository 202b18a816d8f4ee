"""Surrogate-guided choice of model parameters for a target fluid.

The model's free parameters x = (T/T_c, kappa, epsilon) set the coexistence
densities (Eq. 16: T/T_c and epsilon; kappa leaves them unchanged, Section IV)
and the surface tension (Section IV: the source term C scales it by
1 - kappa).  Picking x for a target density ratio and tension by running the
solver is a root search over expensive lattice Boltzmann runs.  This module:

* generates training data with the solver itself: droplet ensembles (surface
  tension from the Laplace law, sigma = dp R_eq in two dimensions) and flat
  liquid slabs (coexistence densities), all stepped on the GPU in batches;
* trains the library's 3-64-64-3 network (include/lbm_mlp.h) on them, inputs
  scaled to [-1, 1] over the parameter box, outputs (rho_l, log rho_v,
  log sigma) standardised;
* selects x for a target (ratio, sigma) at a given epsilon by searching the
  network over a dense (T/T_c, kappa) grid, checking the pick with one solve
  of the reference measurement ("verifier") and, on a miss, correcting the
  network by the observed error at that point and searching again;
* and, as the method without the network, a bisection sweep: bisection on
  T/T_c (density ratio, at kappa = 0) and then on kappa (tension).

Host-side orchestration only: every lattice update, every network evaluation
and every training step runs in the library's HIP kernels.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Sequence

import numpy as np

from . import analysis as A
from . import workloads as W

BOX_LO = np.array([0.55, 0.0, 1.0])   # T/T_c, kappa, epsilon
BOX_HI = np.array([0.85, 0.99, 2.0])


def init_params(seed: int) -> np.ndarray:
    """Glorot-uniform weights and zero biases (float32, layout of lbm_mlp.h)."""
    rng = np.random.default_rng(seed)
    out = []
    for fan_in, fan_out in ((3, 64), (64, 64), (64, 3)):
        a = math.sqrt(6.0 / (fan_in + fan_out))
        out.append(rng.uniform(-a, a, fan_out * fan_in))
        out.append(np.zeros(fan_out))
    return np.concatenate(out).astype(np.float32)


def encode_inputs(P: np.ndarray) -> np.ndarray:
    """(T/T_c, kappa, epsilon) -> [-1, 1]^3 over the parameter box."""
    P = np.atleast_2d(np.asarray(P, dtype=np.float64))
    return 2.0 * (P - BOX_LO) / (BOX_HI - BOX_LO) - 1.0


def encode_targets(rho_l, rho_v, sigma) -> np.ndarray:
    """Network outputs: (rho_l, log rho_v, log sigma); non-positive values -> NaN."""
    rho_l, rho_v, sigma = (np.asarray(v, dtype=np.float64) for v in (rho_l, rho_v, sigma))
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.stack([rho_l, np.where(rho_v > 0, np.log(rho_v), np.nan),
                         np.where(sigma > 0, np.log(sigma), np.nan)], axis=-1)


@dataclasses.dataclass
class Scaler:
    mean: np.ndarray
    std: np.ndarray

    @classmethod
    def fit(cls, Y: np.ndarray, M: np.ndarray) -> "Scaler":
        mean = np.array([np.mean(Y[M[:, k] > 0, k]) for k in range(3)])
        std = np.array([np.std(Y[M[:, k] > 0, k]) for k in range(3)])
        return cls(mean, np.where(std > 0, std, 1.0))

    def encode(self, Y):
        return (Y - self.mean) / self.std

    def decode(self, Z):
        return Z * self.std + self.mean


# ------------------------------------------------------------------ data

@dataclasses.dataclass
class Sample:
    params: tuple          # (T/T_c, kappa, epsilon)
    rho_l: float = float("nan")
    rho_v: float = float("nan")
    sigma: float = float("nan")
    kind: str = ""         # "slab" or "droplet"
    cls: str = ""          # analysis.classify_droplet or classify_slab


def slab_run(T_over_Tc: float, kappa: float, epsilon: float, ny: int = 256, nx: int = 4,
             nu: float = 0.1, label: str = "") -> W.Run:
    """Flat liquid slab of thickness ny/2 centred in a periodic nx x ny box,
    seeded between the Eq. (16) table densities."""
    rl, rv = W.coexistence_seed(T_over_Tc, epsilon)
    kind, eos = W.cs_eos(T_over_Tc)
    return W.Run(nx=nx, ny=ny, eos_kind=kind, eos=eos, G=-1.0, rates=W.rates(nu), kappa=kappa,
                 epsilon=epsilon, rho=W.slab(nx, ny, rl, rv, ny / 2), T_over_Tc=T_over_Tc,
                 label=label or "slab_T%.3f_k%.3f_e%.3f" % (T_over_Tc, kappa, epsilon))


def slab_densities(col: np.ndarray) -> tuple:
    """(rho_l, rho_v) of a slab column: the middle eighth and the outer sixteenths."""
    n = len(col)
    liq = col[n // 2 - n // 16: n // 2 + n // 16]
    vap = np.concatenate([col[: n // 16], col[n - n // 16:]])
    return float(np.mean(liq)), float(np.mean(vap))


def classify_slab(rho_l: float, rho_v: float, status: int, min_ratio: float = 2.0,
                  max_ratio: float = 1e4, min_vapour: float = 1e-5) -> str:
    """'ok', 'diverged' (status flag), 'mixed' (no phase separation) or
    'vacuum': at low T/T_c with small epsilon the vapour branch empties
    (rho_v falls towards zero, ratios beyond 1e4), which no target asks for."""
    if status or not (np.isfinite(rho_l) and np.isfinite(rho_v)):
        return "diverged"
    if not (rho_v > 0 and rho_l / rho_v >= min_ratio):
        return "mixed"
    if rho_v < min_vapour or rho_l / rho_v > max_ratio:
        return "vacuum"
    return "ok"


def parameter_draws(n: int, seed: int) -> np.ndarray:
    """n uniform draws of (T/T_c, kappa, epsilon) over the box."""
    rng = np.random.default_rng(seed)
    return BOX_LO + (BOX_HI - BOX_LO) * rng.uniform(0.0, 1.0, (n, 3))


def measure(lbm, runs: Sequence[W.Run], steps: int, window: int, every: int,
            precision: str = "fp32", graph_steps: int = 16) -> List[Sample]:
    """Step `runs` (slabs and droplets, any mix) together for `steps` steps
    and average their measurements over the last `window` steps (sampled
    every `every` steps): late-time acoustic and shape oscillations of large
    periodic boxes average out of the pressure jump."""
    L = lbm.Lattice(runs, precision=precision, graph_steps=graph_steps)
    try:
        L.init_all()
        L.step(max(steps - window, 0))
        regions = [(r.cx, r.cy, *r.diag_radii()) if r.R0 > 0 else (0.0, 0.0, 0.0, 1.0) for r in runs]
        drop = [i for i, r in enumerate(runs) if r.R0 > 0]
        slab = [i for i, r in enumerate(runs) if r.R0 <= 0]
        acc = {i: [] for i in range(len(runs))}
        nsamp = max(1, window // every)
        for k in range(nsamp):
            L.step(every if k else window - every * (nsamp - 1))
            if drop:
                d = L.diagnostics(regions)
                for i in drop:
                    acc[i].append(d[i])
            for i in slab:
                acc[i].append(slab_densities(L.density_column(i, 0)))
        status = L.status()
    finally:
        L.close()
    out = []
    for i, r in enumerate(runs):
        p = (r.T_over_Tc, r.kappa, r.epsilon)
        if r.R0 > 0:
            ds = acc[i]
            avg = {key: float(np.mean([d[key] for d in ds])) for key in ("rho_in", "rho_out", "dp", "r_eq",
                                                                         "max_speed", "mass")}
            avg["status"] = int(status[i])
            cls = A.classify_droplet(avg, r)
            dps = np.array([d["dp"] for d in ds])
            if cls == "ok" and len(dps) > 1 and np.std(dps) > 0.25 * abs(np.mean(dps)):
                cls = "unsettled"
            out.append(Sample(p, avg["rho_in"], avg["rho_out"], avg["dp"] * avg["r_eq"], "droplet", cls))
        else:
            rl, rv = (float(np.mean([v[j] for v in acc[i]])) for j in (0, 1))
            out.append(Sample(p, rl, rv, float("nan"), "slab", classify_slab(rl, rv, int(status[i]))))
    return out


def droplet_ensemble(n: int, seed: int, lmin: int = 64, lmax: int = 512) -> List[W.Run]:
    """Droplet ensemble with the parameter and size draws of the ensemble workload."""
    return W.config4(nruns=n, seed=seed, lmin=lmin, lmax=lmax)


def slab_set(n: int, seed: int) -> List[W.Run]:
    return [slab_run(*p) for p in parameter_draws(n, seed)]


def dataset(samples: Sequence[Sample]) -> tuple:
    """(X, Y, M) for training: slabs give (rho_l, log rho_v), settled droplets
    give log sigma; every other entry is masked."""
    X, Y, Mk = [], [], []
    for s in samples:
        if s.cls != "ok":
            continue
        y = encode_targets(s.rho_l, s.rho_v, s.sigma)
        m = np.array([1.0, 1.0, 0.0]) if s.kind == "slab" else np.array([0.0, 0.0, 1.0])
        m = m * np.isfinite(y)
        if m.sum() == 0:
            continue
        X.append(s.params)
        Y.append(np.nan_to_num(y))
        Mk.append(m)
    return np.array(X), np.array(Y), np.array(Mk)


# ----------------------------------------------------------------- model

@dataclasses.dataclass
class Surrogate:
    net: object            # lbm.Mlp
    scaler: Scaler
    history: list

    def predict(self, P: np.ndarray) -> np.ndarray:
        """(rho_l, rho_v, sigma) for parameter rows P (network on the GPU)."""
        Z = self.net.forward(encode_inputs(P).astype(np.float32))
        Y = self.scaler.decode(Z.astype(np.float64))
        return np.stack([Y[:, 0], np.exp(Y[:, 1]), np.exp(Y[:, 2])], axis=1)


def train(lbm, X, Y, M, seed: int = 7, schedule=((2000, 3e-3), (2000, 1e-3)),
          max_batch: Optional[int] = None) -> Surrogate:
    """Full-batch Adam with a step-wise learning-rate schedule."""
    scaler = Scaler.fit(Y, M)
    Xe = encode_inputs(X).astype(np.float32)
    Ze = np.nan_to_num(scaler.encode(Y)).astype(np.float32)
    net = lbm.Mlp(init_params(seed), max_batch=max_batch or max(64, len(X)))
    hist = []
    for steps, lr in schedule:
        hist.append((steps, lr, net.train(Xe, Ze, M.astype(np.float32), steps, lr)))
    return Surrogate(net, scaler, hist)


def validation_errors(sur: Surrogate, samples: Sequence[Sample]) -> dict:
    """Relative errors of the network on held-out settled samples."""
    slabs = [s for s in samples if s.kind == "slab" and s.cls == "ok"]
    drops = [s for s in samples if s.kind == "droplet" and s.cls == "ok" and s.sigma > 0]
    out = {}
    if slabs:
        pr = sur.predict(np.array([s.params for s in slabs]))
        ratio = np.array([s.rho_l / s.rho_v for s in slabs])
        out["ratio_rel_err_median"] = float(np.median(np.abs(pr[:, 0] / pr[:, 1] / ratio - 1)))
        out["ratio_rel_err_p90"] = float(np.percentile(np.abs(pr[:, 0] / pr[:, 1] / ratio - 1), 90))
    if drops:
        pr = sur.predict(np.array([s.params for s in drops]))
        sg = np.array([s.sigma for s in drops])
        out["sigma_rel_err_median"] = float(np.median(np.abs(pr[:, 2] / sg - 1)))
        out["sigma_rel_err_p90"] = float(np.percentile(np.abs(pr[:, 2] / sg - 1), 90))
    return out


# ------------------------------------------------------------- selection

@dataclasses.dataclass
class Verified:
    T_over_Tc: float
    kappa: float
    epsilon: float
    ratio: float
    sigma: float
    ok: bool


def verify_runs(T_over_Tc: float, kappa: float, epsilon: float) -> List[W.Run]:
    """The reference measurement: a flat slab (density ratio) and a droplet of
    radius 40 in a periodic 128 x 128 box (sigma = dp R_eq, the radius of the
    paper's Tables 2 and 3)."""
    return [slab_run(T_over_Tc, kappa, epsilon),
            W.droplet_run(128, 40.0, T_over_Tc, kappa, epsilon, label="verify_drop")]


class Verifier:
    """Counts solves of the reference measurement."""

    def __init__(self, lbm, steps: int = 16000, window: int = 4000, every: int = 200,
                 precision: str = "fp32"):
        self.lbm, self.steps, self.window, self.every, self.precision = lbm, steps, window, every, precision
        self.solves = 0
        self.log: List[Verified] = []

    def __call__(self, T_over_Tc: float, kappa: float, epsilon: float) -> Verified:
        s, d = measure(self.lbm, verify_runs(T_over_Tc, kappa, epsilon), self.steps, self.window, self.every,
                       self.precision)
        self.solves += 1
        ok = s.cls == "ok" and d.cls == "ok" and d.sigma > 0
        j = Verified(T_over_Tc, kappa, epsilon, s.rho_l / s.rho_v if s.rho_v > 0 else float("nan"), d.sigma, ok)
        self.log.append(j)
        return j


def hit(j: Verified, ratio: float, sigma: float, tol: float) -> bool:
    return j.ok and abs(j.ratio / ratio - 1) < tol and abs(j.sigma / sigma - 1) < tol


def _grid_argmin(sur: Surrogate, epsilon: float, goal: np.ndarray, T_rng, k_rng, nT: int, nk: int):
    Ts = np.linspace(T_rng[0], T_rng[1], nT)
    ks = np.linspace(k_rng[0], k_rng[1], nk)
    TT, KK = np.meshgrid(Ts, ks, indexing="ij")
    P = np.stack([TT.ravel(), KK.ravel(), np.full(TT.size, epsilon)], axis=1)
    pr = sur.predict(P)
    with np.errstate(divide="ignore", invalid="ignore"):
        f = np.stack([np.log(pr[:, 0] / pr[:, 1]), np.log(pr[:, 2])], axis=1)
    cost = np.sum((f - goal) ** 2, axis=1)
    cost[~np.isfinite(cost)] = np.inf
    i = int(np.argmin(cost))
    return P[i, 0], P[i, 1], f[i]


def surrogate_pick(sur: Surrogate, epsilon: float, goal: np.ndarray) -> tuple:
    """argmin over (T/T_c, kappa) of |(log ratio, log sigma)(x) - goal|^2 on a
    coarse grid of the box, then on a fine grid around the coarse pick."""
    T, k, _ = _grid_argmin(sur, epsilon, goal, (BOX_LO[0], BOX_HI[0]), (BOX_LO[1], BOX_HI[1]), 121, 100)
    dT, dk = (BOX_HI[0] - BOX_LO[0]) / 120 * 3, (BOX_HI[1] - BOX_LO[1]) / 99 * 3
    return _grid_argmin(sur, epsilon, goal, (max(BOX_LO[0], T - dT), min(BOX_HI[0], T + dT)),
                        (max(BOX_LO[1], k - dk), min(BOX_HI[1], k + dk)), 121, 121)


def surrogate_select(sur: Surrogate, verifier: Verifier, ratio: float, sigma: float, epsilon: float,
                     tol: float = 0.01, max_solves: int = 12, fallback_solves: int = 60) -> dict:
    """Network pick, one verifier solve per iteration; after a miss the network's
    outputs are shifted by the error it made at the verified point.  When
    max_solves network-guided solves have not hit the target, the full LB
    solve takes over as the fallback: the physics-aware search (physics_select)
    from the last verified point, with up to fallback_solves more solves, all
    counted in `solves`."""
    target = np.array([math.log(ratio), math.log(sigma)])
    shift = np.zeros(2)
    start = verifier.solves
    j = None
    best = None
    while verifier.solves - start < max_solves:
        T, k, f = surrogate_pick(sur, epsilon, target - shift)
        j = verifier(T, k, epsilon)
        if hit(j, ratio, sigma, tol):
            break
        if j.ok:
            shift = np.array([math.log(j.ratio), math.log(j.sigma)]) - f
            best = j
    network = verifier.solves - start
    out = {"solves": network, "network_solves": network, "fallback_solves": 0, "fallback": False,
           "hit": bool(j and hit(j, ratio, sigma, tol)), "final": j}
    if not out["hit"] and fallback_solves > 0:
        seed = best or j
        warm = bool(seed and seed.ok)
        fb = physics_select(verifier, ratio, sigma, epsilon, tol, fallback_solves,
                            T0=seed.T_over_Tc if warm else 0.6, k0=seed.kappa if warm else 0.0,
                            first_step=0.02 if warm else 0.0)
        out.update(solves=network + fb["solves"], fallback_solves=fb["solves"], fallback=True, hit=fb["hit"],
                   final=fb["final"])
    return out


def bisection_select(verifier: Verifier, ratio: float, sigma: float, epsilon: float, tol: float = 0.01,
                     max_solves: int = 60) -> dict:
    """The method without the network: bisection on T/T_c (starting at
    kappa = 0) until the density ratio is within tol (the ratio falls as T
    rises), then bisection on kappa at that T until sigma is within tol
    (sigma falls as kappa rises); if kappa moved the ratio out of tolerance,
    the two phases alternate again.  A run that diverges or does not separate
    counts as 'T too low' in the first phase and 'kappa too high' in the
    second."""
    start = verifier.solves
    T, k, j = 0.5 * (BOX_LO[0] + BOX_HI[0]), 0.0, None

    def left():
        return verifier.solves - start < max_solves

    while left() and not (j is not None and hit(j, ratio, sigma, tol)):
        lo, hi = BOX_LO[0], BOX_HI[0]
        while left():
            T = 0.5 * (lo + hi)
            j = verifier(T, k, epsilon)
            if j.ok and abs(j.ratio / ratio - 1) < tol:
                break
            if not j.ok or j.ratio > ratio:
                lo = T
            else:
                hi = T
        if hit(j, ratio, sigma, tol):
            break
        klo, khi = BOX_LO[1], BOX_HI[1]
        while left():
            k = 0.5 * (klo + khi)
            j = verifier(T, k, epsilon)
            if j.ok and abs(j.sigma / sigma - 1) < tol:
                break
            if j.ok and j.sigma > sigma:
                klo = k
            else:
                khi = k
    return {"solves": verifier.solves - start, "hit": bool(j and hit(j, ratio, sigma, tol)), "final": j}


def physics_select(verifier: Verifier, ratio: float, sigma: float, epsilon: float, tol: float = 0.01,
                   max_solves: int = 60, T0: float = 0.6, k0: float = 0.0, first_step: float = 0.0) -> dict:
    """A baseline that uses what Section IV states, without the network:
    secant steps on log(ratio) against T/T_c at fixed kappa (kappa leaves the
    ratio unchanged), then kappa from sigma proportional to 1 - kappa,
    k <- 1 - (1 - k) sigma_target / sigma_measured, repeated until both hit.
    Starts from (T0, k0): (0.6, 0) on its own, bracketing with T = 0.8; the last
    verified point when it serves as the surrogate's fallback, with a second
    point first_step away in T."""
    start = verifier.solves
    lo, hi = BOX_LO[0], BOX_HI[0]
    pts = []
    j = None
    T = T0
    k = k0
    while verifier.solves - start < max_solves:
        j = verifier(T, k, epsilon)
        if not j.ok:  # unstable or not separated: move towards higher T
            lo = T
            T = 0.5 * (T + hi)
            continue
        f = math.log(j.ratio / ratio)
        if abs(j.ratio / ratio - 1) < tol:
            break
        if f > 0:
            lo = max(lo, T)
        else:
            hi = min(hi, T)
        pts.append((T, f))
        if len(pts) < 2:
            if first_step:
                # warm start: a second point nearby, on the side the ratio has to
                # move to (it falls with T)
                T = min(hi, T + first_step) if f > 0 else max(lo, T - first_step)
                if not lo < T < hi:
                    T = 0.5 * (lo + hi)
            else:
                T = 0.8 if T < 0.8 else 0.6
        else:
            (Ta, fa), (Tb, fb) = pts[-2], pts[-1]
            Tn = Tb - fb * (Tb - Ta) / (fb - fa) if fb != fa else 0.5 * (lo + hi)
            T = Tn if lo < Tn < hi else 0.5 * (lo + hi)
    while verifier.solves - start < max_solves and not hit(j, ratio, sigma, tol):
        if not j.ok:
            k = 0.5 * k
        else:
            k = min(BOX_HI[1], max(BOX_LO[1], 1.0 - (1.0 - k) * sigma / j.sigma))
        j = verifier(T, k, epsilon)
    return {"solves": verifier.solves - start, "hit": bool(j and hit(j, ratio, sigma, tol)), "final": j}


def build(lbm, n_drops: int, n_slabs: int, seed: int, drop_steps: int, slab_steps: int,
          lmax: int = 512, window_frac: float = 0.3, holdout: float = 0.1,
          log: Callable = lambda *a: None) -> tuple:
    """Generate data with the solver, train, and return (surrogate, train
    samples, held-out samples)."""
    drops = droplet_ensemble(n_drops, seed, lmax=lmax)
    slabs = slab_set(n_slabs, seed + 1)
    log("surrogate data: %d droplets (%d steps), %d slabs (%d steps)" % (len(drops), drop_steps, len(slabs),
                                                                          slab_steps))
    wd = int(drop_steps * window_frac)
    ws = int(slab_steps * window_frac)
    samples = measure(lbm, drops, drop_steps, wd, max(wd // 20, 1)) + \
        measure(lbm, slabs, slab_steps, ws, max(ws // 10, 1))
    rng = np.random.default_rng(seed + 2)
    held = rng.uniform(0, 1, len(samples)) < holdout
    train_s = [s for s, h in zip(samples, held) if not h]
    test_s = [s for s, h in zip(samples, held) if h]
    X, Y, M = dataset(train_s)
    log("training on %d rows (%d sigma, %d density targets)" % (len(X), int(M[:, 2].sum()), int(M[:, 0].sum())))
    sur = train(lbm, X, Y, M, seed=seed + 3)
    return sur, train_s, test_s
