"""FP64 CPU oracle of the D3Q19 extension (ctypes wrapper of lbm3d_oracle.c).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``: only the test suite,
the smoke check and the benchmark's CPU-baseline leg may import it; it shares
no code with the HIP library.

The 3D form of the method is a reading (Section VI leaves it as future work):
the source term is Lambda M df with df the second-order equilibrium change for
the momentum-flux shift (3/5) tr(Q) I - Q, the Eq. (8) term the same for the
shift 2 sigma |F|^2 / psi^2 I, m_eq = M f_eq and S = M F_Guo; the interaction
weights are 1/6 (axes) and 1/12 (face diagonals).  Arrays are f[19, nz, ny, nx].
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Sequence

import numpy as np

from . import BC_PERIODIC, EOS_CS, EOS_EXP, EOS_PIECEWISE, OracleError, lib as _lib2d  # noqa: F401

# velocities in the oracle's order: rest, +-x, +-y, +-z, then the face diagonals in opposite pairs
E = np.array([(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
              (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1),
              (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)])
OPP = np.array([0] + [a + 1 if a % 2 else a - 1 for a in range(1, 19)])


class _P3(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("bc_x", ctypes.c_int), ("bc_y", ctypes.c_int), ("bc_z", ctypes.c_int),
                ("eos_kind", ctypes.c_int), ("eos", ctypes.c_double * 6), ("G", ctypes.c_double),
                ("s", ctypes.c_double * 19), ("kappa", ctypes.c_double), ("sigma", ctypes.c_double)]


_ready = False


def lib():
    global _ready
    L = _lib2d()
    if not _ready:
        dp = ctypes.POINTER(ctypes.c_double)
        P = ctypes.POINTER(_P3)
        Lg = ctypes.c_long
        sigs = {
            "orc3_matrices": (None, [dp, dp]),
            "orc3_feq": (None, [ctypes.c_double, dp, dp]),
            "orc3_guo": (None, [dp, dp, dp]),
            "orc3_flux_shift": (None, [dp, dp]),
            "orc3_force_and_q": (None, [P, dp, dp, dp]),
            "orc3_collide_node": (None, [P, dp, dp, dp, ctypes.c_double, dp]),
            "orc3_init": (ctypes.c_int, [P, dp, dp, dp, dp, dp]),
            "orc3_step": (ctypes.c_int, [P, dp, dp]),
            "orc3_run": (ctypes.c_int, [P, dp, Lg]),
            "orc3_step_sampled": (ctypes.c_int, [P, dp, Lg, ctypes.POINTER(ctypes.c_long), dp]),
            "orc3_moments": (ctypes.c_int, [P, dp, dp, dp, dp, dp]),
            "orc3_diagnostics": (ctypes.c_int, [P, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                                ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]),
        }
        for name, (res, args) in sigs.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _ready = True
    return L


def rates(s_rho=1.0, s_e=0.8, s_eps=0.8, s_j=1.0, s_q=1.1, s_nu=1.25, s_pi=1.1, s_m=1.1):
    """Diagonal of Lambda in moment order (rho, e, eps, jx, qx, jy, qy, jz, qz,
    3pxx, 3pixx, pww, piww, pxy, pyz, pxz, mx, my, mz)."""
    return (s_rho, s_e, s_eps, s_j, s_q, s_j, s_q, s_j, s_q, s_nu, s_pi, s_nu, s_pi, s_nu, s_nu, s_nu,
            s_m, s_m, s_m)


@dataclasses.dataclass
class Params3:
    nx: int
    ny: int
    nz: int
    eos_kind: int
    eos: Sequence[float]
    G: float
    s: Sequence[float] = dataclasses.field(default_factory=rates)
    kappa: float = 0.0
    sigma: float = 0.0
    bc_x: int = BC_PERIODIC
    bc_y: int = BC_PERIODIC
    bc_z: int = BC_PERIODIC

    def c(self) -> _P3:
        p = _P3()
        p.nx, p.ny, p.nz = self.nx, self.ny, self.nz
        p.bc_x, p.bc_y, p.bc_z, p.eos_kind = self.bc_x, self.bc_y, self.bc_z, self.eos_kind
        e = list(self.eos) + [0.0] * (6 - len(self.eos))
        for i in range(6):
            p.eos[i] = float(e[i])
        p.G = float(self.G)
        for i in range(19):
            p.s[i] = float(self.s[i])
        p.kappa, p.sigma = float(self.kappa), float(self.sigma)
        return p

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def replace(self, **kw) -> "Params3":
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
    M, Mi = np.zeros(361), np.zeros(361)
    lib().orc3_matrices(_dp(M), _dp(Mi))
    return M.reshape(19, 19), Mi.reshape(19, 19)


def feq(rho, v):
    out = np.zeros(19)
    lib().orc3_feq(float(rho), _dp(_f64(v)), _dp(out))
    return out


def guo(v, F):
    out = np.zeros(19)
    lib().orc3_guo(_dp(_f64(v)), _dp(_f64(F)), _dp(out))
    return out


def flux_shift(dPi):
    """df for a momentum-flux shift dPi = (xx, yy, zz, xy, yz, xz)."""
    out = np.zeros(19)
    lib().orc3_flux_shift(_dp(_f64(dPi)), _dp(out))
    return out


def force_and_q(P: Params3, psi19):
    F, Q = np.zeros(3), np.zeros(6)
    lib().orc3_force_and_q(ctypes.byref(P.c()), _dp(_f64(psi19)), _dp(F), _dp(Q))
    return F, Q


def collide_node(P: Params3, f19, F, Q, psi):
    out = np.zeros(19)
    lib().orc3_collide_node(ctypes.byref(P.c()), _dp(_f64(f19)), _dp(_f64(F)), _dp(_f64(Q)), float(psi), _dp(out))
    return out


def init(P: Params3, rho, ux=None, uy=None, uz=None):
    rho = _f64(rho, P.shape)
    us = [None if u is None else _f64(u, P.shape) for u in (ux, uy, uz)]
    f = np.zeros((19,) + P.shape)
    _check(lib().orc3_init(ctypes.byref(P.c()), _dp(rho), *[None if u is None else _dp(u) for u in us], _dp(f)),
           "orc3_init")
    return f


def step(P: Params3, f):
    fin = _f64(f, (19,) + P.shape)
    fout = np.empty_like(fin)
    _check(lib().orc3_step(ctypes.byref(P.c()), _dp(fin), _dp(fout)), "orc3_step")
    return fout


def run(P: Params3, f, nsteps: int):
    g = _f64(f, (19,) + P.shape).copy()
    _check(lib().orc3_run(ctypes.byref(P.c()), _dp(g), int(nsteps)), "orc3_run")
    return g


def step_sampled(P: Params3, f, idx):
    """f(t+1) at nodes idx (flat (z ny + y) nx + x) from the full f(t); shape (n, 19)."""
    fin = _f64(f, (19,) + P.shape)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.zeros((idx.size, 19))
    _check(lib().orc3_step_sampled(ctypes.byref(P.c()), _dp(fin), idx.size,
                                   idx.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _dp(out)),
           "orc3_step_sampled")
    return out


def moments(P: Params3, f):
    """(rho, ux, uy, uz) with the Eq. (6) velocity."""
    fin = _f64(f, (19,) + P.shape)
    out = [np.zeros(P.shape) for _ in range(4)]
    _check(lib().orc3_moments(ctypes.byref(P.c()), _dp(fin), *[_dp(o) for o in out]), "orc3_moments")
    return tuple(out)


DIAG_KEYS = ("mass", "rho_in", "rho_out", "p_in", "p_out", "dp", "r_eq", "max_speed")


def diagnostics(P: Params3, f, dims, cx, cy, cz, r_in, r_out) -> dict:
    fin = _f64(f, (19,) + P.shape)
    out = np.zeros(8)
    _check(lib().orc3_diagnostics(ctypes.byref(P.c()), _dp(fin), int(dims), float(cx), float(cy), float(cz),
                                  float(r_in), float(r_out), _dp(out)), "orc3_diagnostics")
    return dict(zip(DIAG_KEYS, out.tolist()))
