"""FP64 CPU oracle of the two-component extension (ctypes wrapper of lbm_mc_oracle.c).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``: only the test suite,
the smoke check and the benchmark's CPU-baseline leg may import it; it shares
no code with the HIP library.

The two-component form is a reading (Section VI leaves multicomponent models
as future work): components A and B with psi_s = rho_s and a cross interaction
of strength G > 0 (Eq. 7 with the other component's psi), the source tensor
Q_s of Eq. (19) likewise, each component relaxed by Eq. (17) with m_eq of
Eq. (3) at its own density and the mixture velocity u, S of Eq. (5) with u and
its own force, and C of Eq. (18) with its own Q.  The total flux shift is then
(kappa G / 6) sum_s (psi_s lap psi_o I - psi_s grad grad psi_o), the
two-component form of Eq. (22).  Arrays are f[2, 9, ny, nx] (A first).
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Sequence

import numpy as np

from . import BC_PERIODIC, EX, EY, OPP, OracleError, lib as _lib2d  # noqa: F401


class _PMC(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("bc_x", ctypes.c_int), ("bc_y", ctypes.c_int),
                ("G", ctypes.c_double), ("s", ctypes.c_double * 9), ("kappa", ctypes.c_double)]


_ready = False


def lib():
    global _ready
    L = _lib2d()
    if not _ready:
        dp = ctypes.POINTER(ctypes.c_double)
        P = ctypes.POINTER(_PMC)
        Lg = ctypes.c_long
        sigs = {
            "orcmc_matrices": (None, [dp, dp]),
            "orcmc_force_and_q": (None, [P, ctypes.c_double, dp, dp, dp]),
            "orcmc_collide_node": (None, [P, dp, dp, dp, dp, dp]),
            "orcmc_init": (ctypes.c_int, [P, dp, dp, dp, dp, dp]),
            "orcmc_step": (ctypes.c_int, [P, dp, dp]),
            "orcmc_run": (ctypes.c_int, [P, dp, Lg]),
            "orcmc_step_sampled": (ctypes.c_int, [P, dp, Lg, ctypes.POINTER(ctypes.c_long), dp]),
            "orcmc_moments": (ctypes.c_int, [P, dp, dp, dp, dp, dp]),
            "orcmc_diagnostics": (ctypes.c_int, [P, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                                 ctypes.c_double, dp]),
        }
        for name, (res, args) in sigs.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _ready = True
    return L


@dataclasses.dataclass
class ParamsMC:
    nx: int
    ny: int
    G: float
    s: Sequence[float]  # Lambda in moment order (rho, e, zeta, jx, qx, jy, qy, pxx, pxy)
    kappa: float = 0.0
    bc_x: int = BC_PERIODIC
    bc_y: int = BC_PERIODIC

    @property
    def shape(self):
        return (self.ny, self.nx)

    def c(self) -> _PMC:
        p = _PMC()
        p.nx, p.ny, p.bc_x, p.bc_y = self.nx, self.ny, self.bc_x, self.bc_y
        p.G, p.kappa = float(self.G), float(self.kappa)
        for i, v in enumerate(self.s):
            p.s[i] = float(v)
        return p

    def replace(self, **kw) -> "ParamsMC":
        return dataclasses.replace(self, **kw)


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a.reshape(shape) if shape is not None and a.shape != shape else a


def _check(rc, what):
    if rc != 0:
        raise OracleError("%s failed with code %d" % (what, rc))


def matrices():
    M, Mi = np.zeros(81), np.zeros(81)
    lib().orcmc_matrices(_dp(M), _dp(Mi))
    return M.reshape(9, 9), Mi.reshape(9, 9)


def force_and_q(P: ParamsMC, psi_s: float, psi_o9):
    """(F, Q) on one component: Eq. (7) and Eq. (19) with the other component's
    psi at x + e_a (psi_o9[0] at x itself); Q = (xx, yy, xy)."""
    F, Q = np.zeros(2), np.zeros(3)
    lib().orcmc_force_and_q(ctypes.byref(P.c()), float(psi_s), _dp(_f64(psi_o9)), _dp(F), _dp(Q))
    return F, Q


def collide_node(P: ParamsMC, f9, u, F, Q):
    out = np.zeros(9)
    lib().orcmc_collide_node(ctypes.byref(P.c()), _dp(_f64(f9)), _dp(_f64(u)), _dp(_f64(F)), _dp(_f64(Q)), _dp(out))
    return out


def init(P: ParamsMC, rhoA, rhoB, ux=None, uy=None):
    rA, rB = _f64(rhoA, P.shape), _f64(rhoB, P.shape)
    us = [None if u is None else _f64(u, P.shape) for u in (ux, uy)]
    f = np.zeros((2, 9) + P.shape)
    _check(lib().orcmc_init(ctypes.byref(P.c()), _dp(rA), _dp(rB), *[None if u is None else _dp(u) for u in us],
                            _dp(f)), "orcmc_init")
    return f


def step(P: ParamsMC, f):
    fin = _f64(f, (2, 9) + P.shape)
    fout = np.empty_like(fin)
    _check(lib().orcmc_step(ctypes.byref(P.c()), _dp(fin), _dp(fout)), "orcmc_step")
    return fout


def run(P: ParamsMC, f, nsteps: int):
    g = _f64(f, (2, 9) + P.shape).copy()
    _check(lib().orcmc_run(ctypes.byref(P.c()), _dp(g), int(nsteps)), "orcmc_run")
    return g


def step_sampled(P: ParamsMC, f, idx):
    """f(t+1) at nodes idx (flat y nx + x) from the full f(t); shape (n, 2, 9)."""
    fin = _f64(f, (2, 9) + P.shape)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.zeros((idx.size, 2, 9))
    _check(lib().orcmc_step_sampled(ctypes.byref(P.c()), _dp(fin), idx.size,
                                    idx.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _dp(out)),
           "orcmc_step_sampled")
    return out


def moments(P: ParamsMC, f):
    """(rhoA, rhoB, ux, uy), u the mixture velocity of Eq. (6) with both forces."""
    fin = _f64(f, (2, 9) + P.shape)
    out = [np.zeros(P.shape) for _ in range(4)]
    _check(lib().orcmc_moments(ctypes.byref(P.c()), _dp(fin), *[_dp(o) for o in out]), "orcmc_moments")
    return tuple(out)


DIAG_KEYS = ("massA", "massB", "rhoA_in", "rhoA_out", "rhoB_in", "rhoB_out", "p_in", "p_out", "dp", "r_eq",
             "max_speed")


def diagnostics(P: ParamsMC, f, cx, cy, r_in, r_out) -> dict:
    fin = _f64(f, (2, 9) + P.shape)
    out = np.zeros(11)
    _check(lib().orcmc_diagnostics(ctypes.byref(P.c()), _dp(fin), float(cx), float(cy), float(r_in), float(r_out),
                                   _dp(out)), "orcmc_diagnostics")
    return dict(zip(DIAG_KEYS, out.tolist()))


def rates(s_rho=1.0, s_e=0.8, s_zeta=0.8, s_j=1.0, s_q=1.1, s_nu=1.25):
    """Diagonal of Lambda in moment order, both components (Eq. 1)."""
    return (s_rho, s_e, s_zeta, s_j, s_q, s_j, s_q, s_nu, s_nu)
