"""Seeded synthetic inputs for the D2Q9 pseudopotential MRT-LB path.

This module serves both the HIP library's callers (benchmark, tests) and the
oracle tests.  It holds no lattice-Boltzmann arithmetic: only geometry (tanh
droplet / slab / wave profiles), seeded noise, parameter draws, and the
lattice-unit conversion nu -> tau_v = 3 nu + 1/2.  T_c and the densities that
seed the initial profiles are read from ``workload_params.json`` (tabulated
from Eq. (16) by a script of the oracle).

Parameter conventions (Section II and Eq. (1)):
* EOS kinds: 0 Carnahan-Starling (a, b, R, T), 1 piecewise Eq. (23)
  (thetaV, thetaM, thetaL, rho1, rho2), 2 exponential psi (psi0, rho0);
* rates: s_rho, s_e, s_zeta, s_j, s_q, s_nu = 1/tau of the moment groups;
* epsilon: exponent of the mechanical-stability integral, Eq. (16); the forcing
  constant of Eq. (8) follows from it inside each implementation.
"""
from __future__ import annotations

import dataclasses
import json
import os
from typing import List, Optional

import numpy as np

EOS_CS, EOS_PIECEWISE, EOS_EXP = 0, 1, 2
BC_PERIODIC, BC_WALL = 0, 1

_HERE = os.path.dirname(os.path.abspath(__file__))
with open(os.path.join(_HERE, "workload_params.json")) as _fh:
    TABLES = json.load(_fh)

CS_A, CS_B, CS_R = TABLES["cs"]["a"], TABLES["cs"]["b"], TABLES["cs"]["R"]
T_C = TABLES["cs"]["T_c"]

BASE_SEED = 13066445


def s_nu(nu: float) -> float:
    """Relaxation rate of the stress moments for kinematic viscosity nu (cs^2 = 1/3)."""
    return 1.0 / (3.0 * nu + 0.5)


def rates(nu: float = 0.1, s_rho: float = 1.0, s_e: float = 0.8, s_zeta: float = 0.8,
          s_j: float = 1.0, s_q: float = 1.1) -> tuple:
    """(s_rho, s_e, s_zeta, s_j, s_q, s_nu).  Defaults: the rates printed for the
    splashing case (Section V.C) with s_nu from the viscosity."""
    return (s_rho, s_e, s_zeta, s_j, s_q, s_nu(nu))


def cs_eos(T_over_Tc: float) -> tuple:
    return (EOS_CS, (CS_A, CS_B, CS_R, T_over_Tc * T_C, 0.0, 0.0))


def piecewise_eos() -> tuple:
    """Eq. (23) with the parameters of Section V.A."""
    cs2 = 1.0 / 3.0
    return (EOS_PIECEWISE, (0.49 * cs2, -0.06 * cs2, 1.0 * cs2, 1.49, 94.65, 0.0))


def exp_eos() -> tuple:
    """psi = 4 exp(-200 / rho), Section III.B."""
    return (EOS_EXP, (4.0, 200.0, 0.0, 0.0, 0.0, 0.0))


def coexistence_seed(T_over_Tc: float, epsilon: float) -> tuple:
    """(rho_l, rho_v) to shape an initial profile: an exact table point when one
    exists, else bilinear interpolation of the Eq. (16) table, else Maxwell."""
    for p in TABLES["points"]:
        if abs(p["T_over_Tc"] - T_over_Tc) < 1e-12 and abs(p["epsilon"] - epsilon) < 1e-12:
            return p["rho_l"], p["rho_v"]
    mech = TABLES["mechanical"]
    tr = np.asarray(mech["T_over_Tc"])
    eg = np.asarray(mech["epsilon"])
    gl = np.array([[np.nan if v is None else v for v in row] for row in mech["rho_l"]])
    gv = np.array([[np.nan if v is None else v for v in row] for row in mech["rho_v"]])
    t = float(np.clip(T_over_Tc, tr[0], tr[-1]))
    e = float(np.clip(epsilon, eg[0], eg[-1]))
    i = min(int(np.searchsorted(tr, t, side="right")) - 1, len(tr) - 2)
    j = min(int(np.searchsorted(eg, e, side="right")) - 1, len(eg) - 2)
    u = (t - tr[i]) / (tr[i + 1] - tr[i])
    w = (e - eg[j]) / (eg[j + 1] - eg[j])

    def bil(g):
        return ((1 - u) * (1 - w) * g[i, j] + u * (1 - w) * g[i + 1, j]
                + (1 - u) * w * g[i, j + 1] + u * w * g[i + 1, j + 1])

    rl, rv = bil(gl), bil(gv)
    if np.isfinite(rl) and np.isfinite(rv) and rv > 0:
        return float(rl), float(rv)
    mx = TABLES["maxwell"]
    return (float(np.interp(t, mx["T_over_Tc"], mx["rho_l"])),
            float(np.interp(t, mx["T_over_Tc"], mx["rho_v"])))


def droplet_seed(T_over_Tc: float, epsilon: float, R: float) -> tuple:
    """(rho_l, rho_v) for a droplet of radius R: the curved-interface bulk
    densities rho(R) = a + c / R tabulated for this (T/T_c, epsilon) when
    available (a droplet seeded with flat-interface vapour in a large box must
    evaporate to raise the vapour density, and small droplets vanish), else
    the flat-interface densities of ``coexistence_seed``."""
    for p in TABLES["points"]:
        if (abs(p["T_over_Tc"] - T_over_Tc) < 1e-12 and abs(p["epsilon"] - epsilon) < 1e-12
                and "droplet_vapour" in p):
            l, v = p["droplet_liquid"], p["droplet_vapour"]
            return l["a"] + l["c"] / R, v["a"] + v["c"] / R
    return coexistence_seed(T_over_Tc, epsilon)


# ---------------------------------------------------------------- geometry

def droplet(nx: int, ny: int, R: float, rho_l: float, rho_v: float, W: float = 5.0,
            cx: Optional[float] = None, cy: Optional[float] = None) -> np.ndarray:
    """tanh droplet of radius R (liquid inside), periodic minimum-image distance."""
    cx = nx / 2 if cx is None else cx
    cy = ny / 2 if cy is None else cy
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    dx = (x - cx + nx / 2) % nx - nx / 2
    dy = (y - cy + ny / 2) % ny - ny / 2
    r = np.hypot(dx, dy)
    return (rho_l + rho_v) / 2 - (rho_l - rho_v) / 2 * np.tanh(2 * (r - R) / W)


def slab(nx: int, ny: int, rho_l: float, rho_v: float, thickness: float, W: float = 5.0) -> np.ndarray:
    """Liquid slab of the given thickness centred in y (two flat interfaces)."""
    y = np.arange(ny, dtype=float)[:, None] * np.ones((1, nx))
    d = np.abs(y - ny / 2)
    return (rho_l + rho_v) / 2 - (rho_l - rho_v) / 2 * np.tanh(2 * (d - thickness / 2) / W)


def wave(nx: int, ny: int, rho_l: float, rho_v: float, wavelength: float, amplitude: float,
         W: float = 5.0) -> np.ndarray:
    """Liquid below y = ny/2 + amplitude cos(2 pi x / wavelength), vapour above."""
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    h = ny / 2 + amplitude * np.cos(2 * np.pi * x / wavelength)
    return (rho_l + rho_v) / 2 - (rho_l - rho_v) / 2 * np.tanh(2 * (y - h) / W)


def noise(shape, amplitude: float, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).uniform(-amplitude, amplitude, shape)


# ------------------------------------------------------------------ runs

@dataclasses.dataclass
class Run:
    nx: int
    ny: int
    eos_kind: int
    eos: tuple
    G: float
    rates: tuple
    kappa: float
    epsilon: float
    rho: np.ndarray
    bc_x: int = BC_PERIODIC
    bc_y: int = BC_PERIODIC
    ux: Optional[np.ndarray] = None
    uy: Optional[np.ndarray] = None
    # droplet bookkeeping for diagnostics
    cx: float = 0.0
    cy: float = 0.0
    R0: float = 0.0
    T_over_Tc: float = float("nan")
    label: str = ""
    # step-function viscosity (Section V.C): below rho_nu relax the stress at s_nu_low
    rho_nu: float = 0.0
    s_nu_low: float = 0.0
    # multi-range potential (Eq. 9): G acts on x + e_a, G2 on x + 2 e_a
    G2: float = 0.0

    @property
    def nodes(self) -> int:
        return self.nx * self.ny

    def diag_radii(self, W: float = 5.0) -> tuple:
        """(r_in, r_out) for the droplet diagnostics: the inner quarter of the
        drop and everything beyond three interface widths outside it."""
        return self.R0 / 4.0, self.R0 + 3.0 * W


def droplet_run(n: int, R: float, T_over_Tc: float, kappa: float, epsilon: float,
                nu: float = 0.1, seed: Optional[int] = None, noise_amp: float = 1e-6,
                label: str = "", curved_seed: bool = True) -> Run:
    rl, rv = droplet_seed(T_over_Tc, epsilon, R) if curved_seed else coexistence_seed(T_over_Tc, epsilon)
    rho = droplet(n, n, R, rl, rv)
    if seed is not None:
        rho = rho + noise(rho.shape, noise_amp, seed)
    kind, eos = cs_eos(T_over_Tc)
    return Run(nx=n, ny=n, eos_kind=kind, eos=eos, G=-1.0, rates=rates(nu), kappa=kappa,
               epsilon=epsilon, rho=rho, cx=n / 2, cy=n / 2, R0=R, T_over_Tc=T_over_Tc,
               label=label)


def config1() -> Run:
    """Stationary droplet, 100x100 periodic, CS at T/Tc = 0.7, R = 25, kappa = 0."""
    return droplet_run(100, 25.0, 0.7, 0.0, 1.93, seed=BASE_SEED + 1, label="c1", curved_seed=False)


CONFIG2_RADII = (20.0, 30.0, 40.0, 50.0, 60.0)
CONFIG2_KAPPAS = (0.0, 0.25, 0.5, 0.75, 0.9, 0.95, 0.98, 0.99)


def config2() -> List[Run]:
    """Laplace-law / kappa sweep: 40 runs of 256x256 at T/Tc = 0.7."""
    runs = []
    k = 0
    for kappa in CONFIG2_KAPPAS:
        for R in CONFIG2_RADII:
            runs.append(droplet_run(256, R, 0.7, kappa, 1.93, seed=BASE_SEED + 2 + 1000 * k,
                                    label="c2_R%g_k%g" % (R, kappa)))
            k += 1
    return runs


def config3(wavelength: int = 256, nx: int = 4096, ny: int = 2048, amp_frac: float = 0.01,
            kappa: float = 0.0) -> Run:
    """Capillary wave: periodic x, walls in y, T/Tc = 0.6, nu = 0.01."""
    rl, rv = coexistence_seed(0.6, 1.93)
    rho = wave(nx, ny, rl, rv, wavelength, amp_frac * wavelength)
    kind, eos = cs_eos(0.6)
    return Run(nx=nx, ny=ny, eos_kind=kind, eos=eos, G=-1.0, rates=rates(0.01), kappa=kappa,
               epsilon=1.93, rho=rho, bc_y=BC_WALL, T_over_Tc=0.6,
               label="c3_lambda%d" % wavelength)


def config4(nruns: int = 512, seed: int = BASE_SEED + 4, lmin: int = 64, lmax: int = 512) -> List[Run]:
    """Ensemble of periodic droplets on uneven square grids with drawn parameters."""
    rng = np.random.default_rng(seed)
    runs = []
    for i in range(nruns):
        L = int(rng.integers(lmin, lmax + 1))
        tr = float(rng.uniform(0.55, 0.85))
        kappa = float(rng.uniform(0.0, 0.99))
        eps = float(rng.uniform(1.0, 2.0))
        R = float(rng.uniform(0.15, 0.3)) * L
        runs.append(droplet_run(L, R, tr, kappa, eps, seed=seed + 1 + i, label="c4_%d" % i))
    return runs


# ------------------------------------------- set-ups of Sections III.B and V

PIECEWISE_SIGMA = 0.087  # forcing constant of Eq. (8) used with Eq. (23), Section V.A


def paper_droplet_run(kind: str, kappa: float, n: int = 120, R: float = 40.0, nu: float = 0.1) -> Run:
    """Stationary droplet of Sections III.B / V.A: R = 40 centred in a periodic
    120 x 120 box.  kind 'exp': psi = 4 exp(-200 / rho), G = -40, no sigma
    forcing, seeded between 514.6 and 79.7 (near the Maxwell densities);
    kind 'pw': Eq. (23), G = -1, sigma = 0.087, seeded between 100 and 1."""
    if kind == "exp":
        ek, eos = exp_eos()
        G, eps, rl, rv = -40.0, 0.0, 514.6, 79.7
    elif kind == "pw":
        ek, eos = piecewise_eos()
        G, eps, rl, rv = -1.0, 16.0 * PIECEWISE_SIGMA, 100.0, 1.0
    else:
        raise ValueError(kind)
    return Run(nx=n, ny=n, eos_kind=ek, eos=eos, G=G, rates=rates(nu), kappa=kappa, epsilon=eps,
               rho=droplet(n, n, R, rl, rv), cx=n / 2, cy=n / 2, R0=R, label="%s_R%g_k%g" % (kind, R, kappa))


def paper_wave_run(kappa: float, L: int = 160, nu: float = 0.01) -> Run:
    """Capillary wave of Section V.B: Eq. (23) EOS, width L (one wavelength,
    periodic), height 3.5 L between walls, interface at mid-height displaced by
    0.125 L cos(2 pi x / L), seeded between 100.13 and 1.012."""
    ek, eos = piecewise_eos()
    H = int(3.5 * L)
    return Run(nx=L, ny=H, eos_kind=ek, eos=eos, G=-1.0, rates=rates(nu), kappa=kappa,
               epsilon=16.0 * PIECEWISE_SIGMA, rho=wave(L, H, 100.13, 1.012, L, 0.125 * L),
               bc_y=BC_WALL, label="pw_wave_L%d_k%g" % (L, kappa))


# ----------------------------------------------------- droplet splashing

def splash_field(nx: int, ny: int, film: float, R: float, U: float, rho_l: float, rho_v: float,
                 gap: float = 1.0, W: float = 5.0) -> tuple:
    """Liquid film of height `film` on the bottom wall and a droplet of radius R
    whose lowest point is `gap` above the film, centred in x, moving down at U:
    (rho, ux, uy).  Liquid fractions are tanh profiles of width W; the
    droplet's velocity is weighted by its own liquid fraction."""
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    phi_film = 0.5 * (1.0 - np.tanh(2.0 * (y - film) / W))
    cy = film + gap + R
    phi_drop = 0.5 * (1.0 - np.tanh(2.0 * (np.hypot(x - nx / 2, y - cy) - R) / W))
    phi = np.maximum(phi_film, phi_drop)
    rho = rho_v + (rho_l - rho_v) * phi
    return rho, np.zeros_like(rho), -U * phi_drop


def paper_splash_run(kappa: float, nx: int = 600, ny: int = 225, film: float = 25.0, R: float = 50.0,
                     U: float = 0.125, Re: float = 1000.0, visc_ratio: float = 20.0) -> Run:
    """Section V.C: Eq. (23) EOS (rho_L/rho_V = 100, sigma = 0.087), film of 25
    on a no-slip bottom wall, droplet R = 50 at U = 0.125, Re = U D / nu_L =
    1000, nu_V / nu_L = 20, nu = nu_V below rho1 = 1.49 and nu_L above, rates
    of the section.  The paper's open top and sides are replaced by a wall on
    top and periodic sides."""
    ek, eos = piecewise_eos()
    nu_l = U * 2 * R / Re
    rho, ux, uy = splash_field(nx, ny, film, R, U, 100.0, 1.0)
    return Run(nx=nx, ny=ny, eos_kind=ek, eos=eos, G=-1.0, rates=rates(nu_l), kappa=kappa,
               epsilon=16.0 * PIECEWISE_SIGMA, rho=rho, ux=ux, uy=uy, bc_y=BC_WALL, cx=nx / 2, R0=R,
               label="pw_splash_k%g" % kappa, rho_nu=1.49, s_nu_low=s_nu(visc_ratio * nu_l))


def config5(T_over_Tc: float, kappa: float, epsilon: float, nx: int = 2048, ny: int = 1024,
            R: float = 100.0, U: float = 0.05, Re: float = 1000.0, visc_ratio: float = 20.0) -> Run:
    """Droplet splashing on a film of 0.1 H: CS EOS at the chosen (T/T_c, kappa,
    epsilon), periodic x, walls at bottom and top, droplet R = 100 at U = 0.05,
    Re = U D / nu_L = 1000, nu_V / nu_L = 20 switched at the mean of the seed
    densities."""
    rl, rv = coexistence_seed(T_over_Tc, epsilon)
    kind, eos = cs_eos(T_over_Tc)
    nu_l = U * 2 * R / Re
    rho, ux, uy = splash_field(nx, ny, 0.1 * ny, R, U, rl, rv)
    return Run(nx=nx, ny=ny, eos_kind=kind, eos=eos, G=-1.0, rates=rates(nu_l), kappa=kappa,
               epsilon=epsilon, rho=rho, ux=ux, uy=uy, bc_y=BC_WALL, cx=nx / 2, R0=R, T_over_Tc=T_over_Tc,
               label="c5_splash", rho_nu=0.5 * (rl + rv), s_nu_low=s_nu(visc_ratio * nu_l))


# Section III.B: the four multi-range cases, (G1, G2) in units of G = -40,
# all with G1 + 2 G2 = G (same EOS)
MULTIRANGE_CASES = {"A": (1.0, 0.0), "B": (1.15, -0.075), "C": (1.3, -0.15), "D": (1.33, -0.165)}


def paper_multirange_run(case: str, n: int = 120, R: float = 40.0, nu: float = 0.1) -> Run:
    """Stationary droplet of Section III.B with the multi-range potential:
    psi = 4 exp(-200 / rho), G = -40, R = 40 in a periodic 120 x 120 box,
    seeded between 514.6 and 79.7 (near the Maxwell densities)."""
    a, b = MULTIRANGE_CASES[case]
    ek, eos = exp_eos()
    G = -40.0
    return Run(nx=n, ny=n, eos_kind=ek, eos=eos, G=a * G, rates=rates(nu), kappa=0.0, epsilon=0.0,
               rho=droplet(n, n, R, 514.6, 79.7), cx=n / 2, cy=n / 2, R0=R, label="mr_%s" % case, G2=b * G)


# --------------------------------------------------------------- 3D (D3Q19)

def rates3(nu: float = 0.1, s_rho: float = 1.0, s_e: float = 0.8, s_eps: float = 0.8, s_j: float = 1.0,
           s_q: float = 1.1, s_pi: float = 1.1, s_m: float = 1.1) -> tuple:
    """(s_rho, s_e, s_eps, s_j, s_q, s_nu, s_pi, s_m) of the D3Q19 moment groups:
    the 2D defaults for the groups both lattices have, s_q for the two extra
    kinetic groups, s_nu from the viscosity."""
    return (s_rho, s_e, s_eps, s_j, s_q, s_nu(nu), s_pi, s_m)


@dataclasses.dataclass
class Run3:
    nx: int
    ny: int
    nz: int
    eos_kind: int
    eos: tuple
    G: float
    rates: tuple
    kappa: float
    epsilon: float
    rho: np.ndarray  # [nz][ny][nx]
    bc_x: int = BC_PERIODIC
    bc_y: int = BC_PERIODIC
    bc_z: int = BC_PERIODIC
    ux: Optional[np.ndarray] = None
    uy: Optional[np.ndarray] = None
    uz: Optional[np.ndarray] = None
    cx: float = 0.0
    cy: float = 0.0
    cz: float = 0.0
    R0: float = 0.0
    label: str = ""

    @property
    def nodes(self) -> int:
        return self.nx * self.ny * self.nz


def sphere(nx: int, ny: int, nz: int, R: float, rho_l: float, rho_v: float, W: float = 5.0) -> np.ndarray:
    """tanh profile of a drop of radius R centred in the box, [nz][ny][nx]."""
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx].astype(float)
    r = np.sqrt((x - nx / 2) ** 2 + (y - ny / 2) ** 2 + (z - nz / 2) ** 2)
    return (rho_l + rho_v) / 2 - (rho_l - rho_v) / 2 * np.tanh(2 * (r - R) / W)


def cylinder(nx: int, ny: int, nz: int, R: float, rho_l: float, rho_v: float, W: float = 5.0) -> np.ndarray:
    """tanh profile of a liquid column of radius R along z, centred in x and y."""
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    r = np.hypot(x - nx / 2, y - ny / 2)
    return np.broadcast_to((rho_l + rho_v) / 2 - (rho_l - rho_v) / 2 * np.tanh(2 * (r - R) / W),
                           (nz, ny, nx)).copy()


def droplet3_run(n: int, R: float, T_over_Tc: float = 0.7, kappa: float = 0.0, epsilon: float = 1.93,
                 nu: float = 0.1, seed: Optional[int] = None, noise_amp: float = 1e-6, label: str = "",
                 shape: Optional[tuple] = None) -> Run3:
    """A periodic 3D drop of the CS fluid (seed densities of the flat interface)."""
    nx, ny, nz = shape or (n, n, n)
    rl, rv = coexistence_seed(T_over_Tc, epsilon)
    rho = sphere(nx, ny, nz, R, rl, rv)
    if seed is not None:
        rho = rho * (1 + noise(rho.shape, noise_amp, seed))
    kind, eos = cs_eos(T_over_Tc)
    return Run3(nx=nx, ny=ny, nz=nz, eos_kind=kind, eos=eos, G=-1.0, rates=rates3(nu), kappa=kappa,
                epsilon=epsilon, rho=rho, cx=nx / 2, cy=ny / 2, cz=nz / 2, R0=R,
                label=label or "d3q19_drop_%dx%dx%d" % (nx, ny, nz))


def config3d(n: int = 256) -> Run3:
    """3D drop of radius n/5 in a periodic n^3 box, CS at T/Tc = 0.7, kappa = 0.5,
    epsilon = 1.93 (the Section VI extension at a grid that fills the GPU)."""
    return droplet3_run(n, n / 5, 0.7, 0.5, 1.93, seed=BASE_SEED + 7, label="d3q19_%d" % n)


# ------------------------------------------------- two components (binary mixture)

@dataclasses.dataclass
class RunMC:
    """A two-component run: densities of A and B, cross interaction G > 0."""
    nx: int
    ny: int
    G: float
    kappa: float
    rates: tuple
    rhoA: np.ndarray
    rhoB: np.ndarray
    bc_x: int = BC_PERIODIC
    bc_y: int = BC_PERIODIC
    ux: Optional[np.ndarray] = None
    uy: Optional[np.ndarray] = None
    cx: float = 0.0
    cy: float = 0.0
    R0: float = 0.0
    label: str = ""

    @property
    def nodes(self) -> int:
        return self.nx * self.ny

    def diag_radii(self, W: float = 4.0) -> tuple:
        return self.R0 / 4.0, self.R0 + 2.0 * W


def mc_drop_run(n: int, R: float, kappa: float, G: float = 1.0, rich: float = 1.0, lean: float = 0.05,
                nu: float = 0.1, W: float = 4.0, shape: Optional[tuple] = None, seed: Optional[int] = None,
                noise_amp: float = 1e-6, label: str = "") -> RunMC:
    """A drop of A (radius R, tanh profile of width W) in B, each component
    between its rich and lean densities, in a periodic box."""
    nx, ny = shape or (n, n)
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    dx = (x - nx / 2 + nx / 2) % nx - nx / 2
    dy = (y - ny / 2 + ny / 2) % ny - ny / 2
    prof = 0.5 * (1 - np.tanh(2 * (np.hypot(dx, dy) - R) / W))
    rhoA = lean + (rich - lean) * prof
    rhoB = lean + (rich - lean) * (1 - prof)
    if seed is not None:
        rhoA = rhoA * (1 + noise((ny, nx), noise_amp, seed))
        rhoB = rhoB * (1 + noise((ny, nx), noise_amp, seed + 1))
    return RunMC(nx=nx, ny=ny, G=G, kappa=kappa, rates=rates(nu), rhoA=rhoA, rhoB=rhoB, cx=nx / 2, cy=ny / 2,
                 R0=R, label=label or "mc_drop_%d_R%g_k%g" % (nx, R, kappa))


def mc_spinodal_run(n: int = 2048, kappa: float = 0.5, G: float = 1.0, rho: float = 1.05, amp: float = 0.01,
                    nu: float = 0.1, seed: int = BASE_SEED + 11) -> RunMC:
    """Spinodal decomposition of a 50/50 mixture of total density rho in a
    periodic n x n box (G rho = 1.05 > 2/3: unstable), seeded with uniform
    composition noise of relative amplitude amp."""
    d = noise((n, n), amp, seed)
    rhoA = 0.5 * rho * (1 + d)
    rhoB = 0.5 * rho * (1 - d)
    return RunMC(nx=n, ny=n, G=G, kappa=kappa, rates=rates(nu), rhoA=rhoA, rhoB=rhoB,
                 label="mc_spinodal_%d_k%g" % (n, kappa))
