"""Plain FP64 CPU oracle for the D2Q9 pseudopotential MRT-LB step with the
surface-tension source term (Li & Luo, arXiv:1306.6445).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the HIP library (``paper_1306_6445_amd``) and never imports it.

The time stepper lives in ``lbm_oracle.c`` (plain C, FP64, dense 9x9 moment
products, two-array streaming); this module is a ctypes wrapper around it plus
the parameter conventions of the paper:

* ``rates(...)``   -- the diagonal of Lambda in moment order, Eq. (1).
* ``sigma_from_epsilon`` -- the reading that ties the Eq. (8) constant sigma to
  the exponent epsilon of the mechanical-stability integral, Eq. (16):
  epsilon = -16 G sigma.  It follows from the Eq. (8) term shifting the energy
  equilibrium by 12 sigma |F|^2 / psi^2 (Section II, Eq. 8 together with Eq. 16).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
# the D3Q19 extension (lbm3d_oracle.c, wrapped by oracle.d3q19) and the two-component
# extension (lbm_mc_oracle.c, wrapped by oracle.binary) are built into the same library
_SRCS = [_SRC, os.path.join(_HERE, "lbm3d_oracle.c"), os.path.join(_HERE, "lbm_mc_oracle.c")]
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

EOS_CS, EOS_PIECEWISE, EOS_EXP = 0, 1, 2
BC_PERIODIC, BC_WALL = 0, 1

# D2Q9 velocities in the order the oracle uses (Section II).
EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
OPP = np.array([0, 3, 4, 1, 2, 7, 8, 5, 6])


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no FP contraction, OpenMP over nodes)."""
    stale = not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(f)
                                            for f in _SRCS + [os.path.join(_HERE, "lbm3d_oracle.h"),
                                                              os.path.join(_HERE, "lbm_oracle.h"),
                                                              os.path.join(_HERE, "lbm_mc_oracle.h")])
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-o", tmp] + _SRCS + ["-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("bc_x", ctypes.c_int),
                ("bc_y", ctypes.c_int), ("eos_kind", ctypes.c_int),
                ("eos", ctypes.c_double * 6), ("G", ctypes.c_double),
                ("s", ctypes.c_double * 9), ("kappa", ctypes.c_double),
                ("sigma", ctypes.c_double), ("rho_nu", ctypes.c_double), ("s_nu_low", ctypes.c_double),
                ("G2", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        dp = ctypes.POINTER(ctypes.c_double)
        P = ctypes.POINTER(_Params)
        L = ctypes.c_long
        sigs = {
            "orc_matrices": (None, [dp, dp]),
            "orc_eos_array": (ctypes.c_int, [P, L, dp, dp, dp]),
            "orc_force_and_q": (None, [P, dp, dp, dp]),
            "orc_force_multirange": (None, [P, dp, dp, dp, dp]),
            "orc_forcing_moments": (None, [P, dp, dp, ctypes.c_double, dp]),
            "orc_source_moments": (None, [P, dp, dp]),
            "orc_collide_node": (None, [P, dp, dp, dp, ctypes.c_double, dp]),
            "orc_init": (ctypes.c_int, [P, dp, dp, dp, dp]),
            "orc_step": (ctypes.c_int, [P, dp, dp]),
            "orc_run": (ctypes.c_int, [P, dp, L]),
            "orc_step_sampled": (ctypes.c_int, [P, dp, L, ctypes.POINTER(ctypes.c_long), dp]),
            "orc_moments": (ctypes.c_int, [P, dp, dp, dp, dp]),
            "orc_diagnostics": (ctypes.c_int, [P, dp, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_double, dp]),
            "orc_threads": (ctypes.c_int, []),
        }
        for name, (res, args) in sigs.items():
            fn = getattr(_lib, name)
            fn.restype = res
            fn.argtypes = args
    return _lib


def rates(s_rho=1.0, s_e=0.8, s_zeta=0.8, s_j=1.0, s_q=1.1, s_nu=1.25):
    """Diagonal of Lambda in moment order (rho, e, zeta, jx, qx, jy, qy, pxx, pxy), Eq. (1)."""
    return (s_rho, s_e, s_zeta, s_j, s_q, s_j, s_q, s_nu, s_nu)


def s_nu_from_viscosity(nu: float) -> float:
    """Kinematic viscosity nu = cs^2 (tau_v - 1/2) in lattice units, cs^2 = 1/3."""
    return 1.0 / (3.0 * nu + 0.5)


def sigma_from_epsilon(epsilon: float, G: float) -> float:
    """Reading of Eq. (8) vs Eq. (16): epsilon = -16 G sigma."""
    return -epsilon / (16.0 * G)


@dataclasses.dataclass
class Params:
    nx: int
    ny: int
    eos_kind: int
    eos: Sequence[float]
    G: float
    s: Sequence[float] = dataclasses.field(default_factory=rates)
    kappa: float = 0.0
    sigma: float = 0.0
    bc_x: int = BC_PERIODIC
    bc_y: int = BC_PERIODIC
    rho_nu: float = 0.0     # step-function viscosity (Section V.C): below rho_nu ...
    s_nu_low: float = 0.0   # ... the stress moments relax at s_nu_low
    G2: float = 0.0         # multi-range potential, Eq. (9) (G acts as G1)

    def c(self) -> _Params:
        p = _Params()
        p.nx, p.ny, p.bc_x, p.bc_y, p.eos_kind = self.nx, self.ny, self.bc_x, self.bc_y, self.eos_kind
        e = list(self.eos) + [0.0] * (6 - len(self.eos))
        for i in range(6):
            p.eos[i] = float(e[i])
        p.G = float(self.G)
        for i in range(9):
            p.s[i] = float(self.s[i])
        p.kappa = float(self.kappa)
        p.sigma = float(self.sigma)
        p.rho_nu = float(self.rho_nu)
        p.s_nu_low = float(self.s_nu_low)
        p.G2 = float(self.G2)
        return p

    def replace(self, **kw) -> "Params":
        return dataclasses.replace(self, **kw)


def params_from_run(run) -> Params:
    """Oracle parameters of a workload run (fields nx, ny, bc_x, bc_y, eos_kind,
    eos, G, rates = (s_rho, s_e, s_zeta, s_j, s_q, s_nu), kappa, epsilon)."""
    s_rho, s_e, s_zeta, s_j, s_q, s_nu = run.rates
    sigma = sigma_from_epsilon(run.epsilon, run.G) if run.epsilon != 0.0 else 0.0
    return Params(nx=run.nx, ny=run.ny, eos_kind=run.eos_kind, eos=tuple(run.eos)[:6], G=run.G,
                  s=rates(s_rho, s_e, s_zeta, s_j, s_q, s_nu), kappa=run.kappa, sigma=sigma,
                  bc_x=run.bc_x, bc_y=run.bc_y, rho_nu=float(getattr(run, "rho_nu", 0.0)),
                  s_nu_low=float(getattr(run, "s_nu_low", 0.0)), G2=float(getattr(run, "G2", 0.0)))


class OracleError(RuntimeError):
    pass


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc: int, what: str):
    if rc != 0:
        raise OracleError("%s failed with code %d" % (what, rc))


def _f64(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        a = a.reshape(shape)
    return a


def matrices():
    M = np.zeros(81)
    Mi = np.zeros(81)
    lib().orc_matrices(_dp(M), _dp(Mi))
    return M.reshape(9, 9), Mi.reshape(9, 9)


def eos(P: Params, rho) -> tuple:
    """(p_EOS, psi) for an array of densities; NaN where psi is undefined."""
    r = _f64(np.atleast_1d(rho))
    p = np.empty_like(r)
    psi = np.empty_like(r)
    lib().orc_eos_array(ctypes.byref(P.c()), r.size, _dp(r), _dp(p), _dp(psi))
    return p.reshape(np.shape(rho)), psi.reshape(np.shape(rho))


def force_and_q(P: Params, psi9) -> tuple:
    psi9 = _f64(psi9)
    F = np.zeros(2)
    Q = np.zeros(3)
    lib().orc_force_and_q(ctypes.byref(P.c()), _dp(psi9), _dp(F), _dp(Q))
    return F, Q


def force_multirange(P: Params, psi9, psi2) -> tuple:
    """Eq. (9) force (G as G1, P.G2) from psi at x + e_a and x + 2 e_a; and Q."""
    psi9, psi2 = _f64(psi9), _f64(psi2)
    F = np.zeros(2)
    Q = np.zeros(3)
    lib().orc_force_multirange(ctypes.byref(P.c()), _dp(psi9), _dp(psi2), _dp(F), _dp(Q))
    return F, Q


def forcing_moments(P: Params, v, F, psi) -> np.ndarray:
    v, F = _f64(v), _f64(F)
    S = np.zeros(9)
    lib().orc_forcing_moments(ctypes.byref(P.c()), _dp(v), _dp(F), float(psi), _dp(S))
    return S


def source_moments(P: Params, Q) -> np.ndarray:
    Q = _f64(Q)
    C = np.zeros(9)
    lib().orc_source_moments(ctypes.byref(P.c()), _dp(Q), _dp(C))
    return C


def collide_node(P: Params, f9, F, Q, psi) -> np.ndarray:
    f9, F, Q = _f64(f9), _f64(F), _f64(Q)
    out = np.zeros(9)
    lib().orc_collide_node(ctypes.byref(P.c()), _dp(f9), _dp(F), _dp(Q), float(psi), _dp(out))
    return out


def init(P: Params, rho, ux=None, uy=None) -> np.ndarray:
    """f = M^-1 m_eq(rho, u) on every node; returns f[9, ny, nx]."""
    shape = (P.ny, P.nx)
    rho = _f64(rho, shape)
    ux = None if ux is None else _f64(ux, shape)
    uy = None if uy is None else _f64(uy, shape)
    f = np.zeros((9, P.ny, P.nx))
    _check(lib().orc_init(ctypes.byref(P.c()), _dp(rho), None if ux is None else _dp(ux),
                          None if uy is None else _dp(uy), _dp(f)), "orc_init")
    return f


def step(P: Params, f) -> np.ndarray:
    fin = _f64(f, (9, P.ny, P.nx))
    fout = np.empty_like(fin)
    _check(lib().orc_step(ctypes.byref(P.c()), _dp(fin), _dp(fout)), "orc_step")
    return fout


def run(P: Params, f, nsteps: int) -> np.ndarray:
    g = _f64(f, (9, P.ny, P.nx)).copy()
    _check(lib().orc_run(ctypes.byref(P.c()), _dp(g), int(nsteps)), "orc_run")
    return g


def step_sampled(P: Params, f, idx) -> np.ndarray:
    """f(t+1) at the nodes idx (flat y*nx+x) computed from the full f(t); shape (n, 9)."""
    fin = _f64(f, (9, P.ny, P.nx))
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.zeros((idx.size, 9))
    _check(lib().orc_step_sampled(ctypes.byref(P.c()), _dp(fin), idx.size,
                                  idx.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _dp(out)),
           "orc_step_sampled")
    return out


def moments(P: Params, f) -> tuple:
    """(rho, ux, uy) with the velocity of Eq. (6) (includes F/2)."""
    fin = _f64(f, (9, P.ny, P.nx))
    rho = np.zeros((P.ny, P.nx))
    ux = np.zeros_like(rho)
    uy = np.zeros_like(rho)
    _check(lib().orc_moments(ctypes.byref(P.c()), _dp(fin), _dp(rho), _dp(ux), _dp(uy)),
           "orc_moments")
    return rho, ux, uy


DIAG_KEYS = ("mass", "rho_in", "rho_out", "p_in", "p_out", "dp", "r_eq", "max_speed")


def diagnostics(P: Params, f, cx, cy, r_in, r_out) -> dict:
    fin = _f64(f, (9, P.ny, P.nx))
    out = np.zeros(8)
    _check(lib().orc_diagnostics(ctypes.byref(P.c()), _dp(fin), float(cx), float(cy),
                                 float(r_in), float(r_out), _dp(out)), "orc_diagnostics")
    return dict(zip(DIAG_KEYS, out.tolist()))


def threads() -> int:
    return int(lib().orc_threads())
