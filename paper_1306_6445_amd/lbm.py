"""ctypes binding of the HIP library (C ABI in include/lbm.h).

Argument marshalling only: every step of the lattice Boltzmann path runs in the
HIP kernels of ``liblbm_mi355x.so``.  PyTorch supplies device memory (the
workspace) and the stream.  There is no CPU fallback: loading fails loudly when
the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblbm_mi355x.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EDIVERGED, LBM_ESTATE = 0, -1, -2, -3, -4, -5
BC_PERIODIC, BC_BOUNCEBACK = 0, 1
EOS_CS, EOS_PIECEWISE, EOS_SC_EXP = 0, 1, 2
FP64, FP32, FP32_BF16STORE = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": FP32_BF16STORE}

STATUS_NAMES = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EDEVICE",
                -4: "LBM_EDIVERGED", -5: "LBM_ESTATE"}


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32)]


class Eos(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32), ("p", ctypes.c_double * 6)]


class Rates(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("s_rho", "s_e", "s_zeta", "s_j", "s_q", "s_nu")]


class RunDesc(ctypes.Structure):
    _fields_ = [("grid", Grid), ("eos", Eos), ("G", ctypes.c_double), ("rates", Rates),
                ("kappa", ctypes.c_double), ("epsilon", ctypes.c_double)]


class Grid3(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32), ("bc_z", ctypes.c_int32)]


class Rates3(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("s_rho", "s_e", "s_eps", "s_j", "s_q", "s_nu", "s_pi", "s_m")]


class Diag(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("mass", "rho_in", "rho_out", "p_in", "p_out", "dp", "r_eq", "max_speed")] + \
               [("status", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class McParams(ctypes.Structure):
    _fields_ = [("G", ctypes.c_double), ("kappa", ctypes.c_double), ("rates", Rates)]


class McDiag(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("massA", "massB", "rhoA_in", "rhoA_out", "rhoB_in", "rhoB_out", "p_in", "p_out", "dp", "r_eq",
                 "max_speed")] + [("status", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Region(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("cx", "cy", "r_in", "r_out")]


class LbmError(RuntimeError):
    def __init__(self, code: int, what: str, msg: str):
        super().__init__("%s: %s (%s)" % (what, STATUS_NAMES.get(code, code), msg))
        self.code = code


_lib = None

# name -> (restype, argtypes); the set of exported entry points of include/lbm.h
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_F = ctypes.POINTER(ctypes.c_float)
_I32 = ctypes.c_int32
SIGNATURES = {
    "lbm_validate_run": (_I32, [ctypes.POINTER(RunDesc)]),
    "lbm_validate": (_I32, [ctypes.POINTER(Grid), ctypes.POINTER(Eos), ctypes.c_double,
                            ctypes.POINTER(Rates), ctypes.c_double, ctypes.c_double]),
    "lbm_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Grid), _I32]),
    "lbm_create": (_I32, [ctypes.POINTER(Grid), ctypes.POINTER(Eos), ctypes.c_double,
                          ctypes.POINTER(Rates), ctypes.c_double, ctypes.c_double, _I32, _P,
                          ctypes.c_size_t, _P, ctypes.POINTER(_P)]),
    "lbm_init_density": (_I32, [_P, _D, _D, _D]),
    "lbm_step": (_I32, [_P, ctypes.c_int64]),
    "lbm_moments": (_I32, [_P, _D, _D, _D]),
    "lbm_diagnostics": (_I32, [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.POINTER(Diag)]),
    "lbm_get_populations": (_I32, [_P, _D]),
    "lbm_set_populations": (_I32, [_P, _D]),
    "lbm_steps_taken": (ctypes.c_int64, [_P]),
    "lbm_state_bytes": (ctypes.c_size_t, [_P]),
    "lbm_save_state": (_I32, [_P, _P, ctypes.c_size_t]),
    "lbm_load_state": (_I32, [_P, _P, ctypes.c_size_t]),
    "lbm_destroy": (None, [_P]),
    "lbm_last_error": (ctypes.c_char_p, []),
    "lbm_batch_workspace_bytes": (ctypes.c_size_t, [_I32, ctypes.POINTER(RunDesc), _I32]),
    "lbm_batch_create": (_I32, [_I32, ctypes.POINTER(RunDesc), _I32, _P, ctypes.c_size_t, _P,
                                ctypes.POINTER(_P)]),
    "lbm_num_runs": (_I32, [_P]),
    "lbm_run_init_density": (_I32, [_P, _I32, _D, _D, _D]),
    "lbm_run_moments": (_I32, [_P, _I32, _D, _D, _D]),
    "lbm_run_get_populations": (_I32, [_P, _I32, _D]),
    "lbm_run_density_column": (_I32, [_P, _I32, _I32, _D]),
    "lbm_run_set_populations": (_I32, [_P, _I32, _D]),
    "lbm_batch_diagnostics": (_I32, [_P, ctypes.POINTER(Region), ctypes.POINTER(Diag)]),
    "lbm_run_status": (_I32, [_P, ctypes.POINTER(_I32)]),
    "lbm_run_pressure": (_I32, [_P, _I32, _D]),
    "lbm_run_get_window": (_I32, [_P, _I32, _I32, _I32, _I32, _I32, _D]),
    "lbm_run_set_reference_density": (_I32, [_P, _I32, ctypes.c_double]),
    "lbm_run_set_viscosity_step": (_I32, [_P, _I32, ctypes.c_double, ctypes.c_double]),
    "lbm_run_set_multirange": (_I32, [_P, _I32, ctypes.c_double, ctypes.c_double]),
    "lbm_set_graph_steps": (_I32, [_P, _I32]),
    "lbm_set_tile": (_I32, [_P, _I32, _I32]),
    "lbm_autotune": (_I32, [_P, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "lbm_set_xcd_order": (_I32, [_P, _I32]),
    "lbm_set_fused": (_I32, [_P, _I32]),
    "lbm_time_kernels": (_I32, [_P, ctypes.c_int64, _D, _D]),
    "lbm_stream_copy": (_I32, [_P, _P, ctypes.c_size_t, _I32, _P, _D]),
    # D3Q19 extension, include/lbm3d.h
    "lbm3d_validate": (_I32, [ctypes.POINTER(Grid3), ctypes.POINTER(Eos), ctypes.c_double, ctypes.POINTER(Rates3),
                              ctypes.c_double, ctypes.c_double]),
    "lbm3d_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Grid3), _I32]),
    "lbm3d_create": (_I32, [ctypes.POINTER(Grid3), ctypes.POINTER(Eos), ctypes.c_double, ctypes.POINTER(Rates3),
                            ctypes.c_double, ctypes.c_double, _I32, _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)]),
    "lbm3d_init_density": (_I32, [_P, _D, _D, _D, _D]),
    "lbm3d_step": (_I32, [_P, ctypes.c_int64]),
    "lbm3d_moments": (_I32, [_P, _D, _D, _D, _D]),
    "lbm3d_get_populations": (_I32, [_P, _D]),
    "lbm3d_set_populations": (_I32, [_P, _D]),
    "lbm3d_state_bytes": (ctypes.c_size_t, [_P]),
    "lbm3d_save_state": (_I32, [_P, _P, ctypes.c_size_t]),
    "lbm3d_load_state": (_I32, [_P, _P, ctypes.c_size_t]),
    "lbm3d_diagnostics": (_I32, [_P, _I32, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.POINTER(Diag)]),
    "lbm3d_time_kernels": (_I32, [_P, ctypes.c_int64, _D, _D]),
    "lbm3d_steps_taken": (ctypes.c_int64, [_P]),
    "lbm3d_set_schedule": (_I32, [_P, _I32, _I32, _I32, _I32]),
    "lbm3d_autotune": (_I32, [_P, _I32] + [ctypes.POINTER(_I32)] * 4),
    "lbm3d_set_graph_steps": (_I32, [_P, _I32]),
    "lbm_mc_validate": (_I32, [ctypes.POINTER(Grid), ctypes.POINTER(McParams)]),
    "lbm_mc_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Grid), _I32]),
    "lbm_mc_create": (_I32, [ctypes.POINTER(Grid), ctypes.POINTER(McParams), _I32, _P, ctypes.c_size_t, _P,
                             ctypes.POINTER(_P)]),
    "lbm_mc_init_density": (_I32, [_P, _D, _D, _D, _D]),
    "lbm_mc_step": (_I32, [_P, ctypes.c_int64]),
    "lbm_mc_moments": (_I32, [_P, _D, _D, _D, _D]),
    "lbm_mc_get_populations": (_I32, [_P, _D]),
    "lbm_mc_set_populations": (_I32, [_P, _D]),
    "lbm_mc_state_bytes": (ctypes.c_size_t, [_P]),
    "lbm_mc_save_state": (_I32, [_P, _P, ctypes.c_size_t]),
    "lbm_mc_load_state": (_I32, [_P, _P, ctypes.c_size_t]),
    "lbm_mc_diagnostics": (_I32, [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                  ctypes.POINTER(McDiag)]),
    "lbm_mc_set_tile": (_I32, [_P, _I32, _I32, _I32]),
    "lbm_mc_autotune": (_I32, [_P, _I32] + [ctypes.POINTER(_I32)] * 3),
    "lbm_mc_set_graph_steps": (_I32, [_P, _I32]),
    "lbm_mc_time_kernels": (_I32, [_P, ctypes.c_int64, _D]),
    "lbm_mc_steps_taken": (ctypes.c_int64, [_P]),
    "lbm_mc_destroy": (None, [_P]),
    "lbm3d_destroy": (None, [_P]),
    "lbm_step_noalloc": (_I32, [ctypes.POINTER(Grid), ctypes.POINTER(Eos), ctypes.c_double, ctypes.POINTER(Rates),
                                ctypes.c_double, ctypes.c_double, _P, ctypes.c_int64, ctypes.c_int64, _P, _P]),
    # surrogate network, include/lbm_mlp.h
    "lbm_mlp_workspace_bytes": (ctypes.c_size_t, [_I32]),
    "lbm_mlp_create": (_I32, [_I32, _F, _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)]),
    "lbm_mlp_set_params": (_I32, [_P, _F]),
    "lbm_mlp_get_params": (_I32, [_P, _F]),
    "lbm_mlp_forward": (_I32, [_P, _P, _I32, _P]),
    "lbm_mlp_loss_grad": (_I32, [_P, _P, _P, _P, _I32, _D, _F]),
    "lbm_mlp_train": (_I32, [_P, _P, _P, _P, _I32, _I32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                             ctypes.c_float, _D]),
    "lbm_mlp_steps_taken": (ctypes.c_int64, [_P]),
    "lbm_mlp_destroy": (None, [_P]),
}


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load liblbm_mi355x.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError("HIP library %s is not built; run `python -m paper_1306_6445_amd.build`"
                               % path)
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def last_error() -> str:
    return load_library().lbm_last_error().decode()


def _check(rc: int, what: str, allow=()):
    if rc != LBM_OK and rc not in allow:
        raise LbmError(rc, what, last_error())
    return rc


def _dp(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_D)


def run_desc(run) -> RunDesc:
    """RunDesc from any object with nx, ny, bc_x, bc_y, eos_kind, eos, G, rates, kappa, epsilon."""
    d = RunDesc()
    d.grid.nx, d.grid.ny = int(run.nx), int(run.ny)
    d.grid.bc_x, d.grid.bc_y = int(run.bc_x), int(run.bc_y)
    d.eos.kind = int(run.eos_kind)
    e = list(run.eos) + [0.0] * (6 - len(run.eos))
    for i in range(6):
        d.eos.p[i] = float(e[i])
    d.G = float(run.G)
    (d.rates.s_rho, d.rates.s_e, d.rates.s_zeta, d.rates.s_j, d.rates.s_q,
     d.rates.s_nu) = [float(v) for v in run.rates]
    d.kappa = float(run.kappa)
    d.epsilon = float(run.epsilon)
    return d


def validate(run) -> int:
    """Host-only parameter check; returns the lbm_status code."""
    d = run_desc(run)
    return int(load_library().lbm_validate_run(ctypes.byref(d)))


def workspace_bytes(runs: Sequence, precision: str) -> int:
    arr = (RunDesc * len(runs))(*[run_desc(r) for r in runs])
    return int(load_library().lbm_batch_workspace_bytes(len(runs), arr, PRECISIONS[precision]))


class Lattice:
    """One or more independent runs stepped together on one GPU.

    ``runs``: objects carrying the run parameters (see ``run_desc``), e.g.
    ``workloads.Run``.  The workspace is a torch uint8 tensor on ``device`` and
    the work goes to a dedicated torch stream of default priority.
    """

    def __init__(self, runs: Sequence, precision: str = "fp32", device: str = "cuda",
                 tile: Optional[tuple] = None, graph_steps: Optional[int] = None,
                 fused=None):
        import torch

        self._lib = load_library()
        self.runs = list(runs)
        self.precision = precision
        self.device = torch.device(device)
        descs = (RunDesc * len(self.runs))(*[run_desc(r) for r in self.runs])
        nbytes = int(self._lib.lbm_batch_workspace_bytes(len(self.runs), descs, PRECISIONS[precision]))
        if nbytes == 0:
            _check(LBM_EINVAL, "lbm_batch_workspace_bytes")
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.Stream(device=self.device)
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        ctx = _P()
        with torch.cuda.device(self.device):
            _check(self._lib.lbm_batch_create(len(self.runs), descs, PRECISIONS[precision],
                                              _P(aligned), nbytes, _P(self.stream.cuda_stream),
                                              ctypes.byref(ctx)), "lbm_batch_create")
        self._ctx = ctx
        if tile is not None:
            self.set_tile(*tile)
        if graph_steps is not None:
            self.set_graph_steps(graph_steps)
        if fused is not None:
            self.set_fused(fused)
        for i, r in enumerate(self.runs):
            if getattr(r, "rho_nu", 0.0) > 0.0:
                self.set_viscosity_step(i, r.rho_nu, r.s_nu_low)
            if getattr(r, "G2", 0.0) != 0.0:
                self.set_multirange(i, r.G, r.G2)

    # -- lifecycle
    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.lbm_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def nruns(self) -> int:
        return int(self._lib.lbm_num_runs(self._ctx))

    @property
    def steps_taken(self) -> int:
        return int(self._lib.lbm_steps_taken(self._ctx))

    def shape(self, run: int) -> tuple:
        return int(self.runs[run].ny), int(self.runs[run].nx)

    # -- state
    def init_density(self, run: int, rho, ux=None, uy=None):
        shape = self.shape(run)
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(shape)
        ux = None if ux is None else np.ascontiguousarray(ux, dtype=np.float64).reshape(shape)
        uy = None if uy is None else np.ascontiguousarray(uy, dtype=np.float64).reshape(shape)
        _check(self._lib.lbm_run_init_density(self._ctx, run, _dp(rho), _dp(ux), _dp(uy)),
               "lbm_run_init_density")

    def init_all(self):
        """Initialise every run from its ``rho`` (and optional ``ux``/``uy``) field."""
        for i, r in enumerate(self.runs):
            self.init_density(i, r.rho, getattr(r, "ux", None), getattr(r, "uy", None))

    def reset_steps(self):
        """Re-initialise run 0 through lbm_init_density (resets the step counter)."""
        r = self.runs[0]
        shape = self.shape(0)
        rho = np.ascontiguousarray(r.rho, dtype=np.float64).reshape(shape)
        _check(self._lib.lbm_init_density(self._ctx, _dp(rho), None, None), "lbm_init_density")

    def step(self, n: int = 1):
        _check(self._lib.lbm_step(self._ctx, int(n)), "lbm_step")

    def synchronize(self):
        self.stream.synchronize()

    def populations(self, run: int = 0) -> np.ndarray:
        ny, nx = self.shape(run)
        f = np.empty((9, ny, nx))
        _check(self._lib.lbm_run_get_populations(self._ctx, run, _dp(f)), "lbm_run_get_populations")
        return f

    def set_populations(self, run: int, f):
        ny, nx = self.shape(run)
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(9, ny, nx)
        _check(self._lib.lbm_run_set_populations(self._ctx, run, _dp(f)), "lbm_run_set_populations")

    def density_column(self, run: int, x: int) -> np.ndarray:
        """Density of column x of one run (FP64)."""
        out = np.empty(int(self.runs[run].ny))
        _check(self._lib.lbm_run_density_column(self._ctx, run, int(x), _dp(out)), "lbm_run_density_column")
        return out

    def set_multirange(self, run: int, G1: float, G2: float):
        """Eq. (9): G1 on the neighbours at e_a, G2 on those at 2 e_a."""
        _check(self._lib.lbm_run_set_multirange(self._ctx, run, float(G1), float(G2)), "lbm_run_set_multirange")

    def set_viscosity_step(self, run: int, rho_threshold: float, s_nu_low: float):
        """nu(rho) = nu_V below rho_threshold (rate s_nu_low), nu_L above (Section V.C)."""
        _check(self._lib.lbm_run_set_viscosity_step(self._ctx, run, float(rho_threshold), float(s_nu_low)),
               "lbm_run_set_viscosity_step")

    def set_reference_density(self, run: int, rho_ref: float):
        """Base density of the deviation storage (FP32, bf16) of one run."""
        _check(self._lib.lbm_run_set_reference_density(self._ctx, run, float(rho_ref)),
               "lbm_run_set_reference_density")

    def moments(self, run: int = 0, allow_diverged: bool = False):
        ny, nx = self.shape(run)
        rho, ux, uy = np.empty((ny, nx)), np.empty((ny, nx)), np.empty((ny, nx))
        _check(self._lib.lbm_run_moments(self._ctx, run, _dp(rho), _dp(ux), _dp(uy)),
               "lbm_run_moments", allow=(LBM_EDIVERGED,) if allow_diverged else ())
        return rho, ux, uy

    def window(self, run: int, x0: int, y0: int, w: int, h: int) -> np.ndarray:
        """Populations [9][h][w] (FP64) of the window at (x0, y0), wrapped on periodic axes."""
        out = np.empty((9, h, w))
        _check(self._lib.lbm_run_get_window(self._ctx, int(run), int(x0), int(y0), int(w), int(h), _dp(out)),
               "lbm_run_get_window")
        return out

    def pressure(self, run: int = 0, allow_diverged: bool = False) -> np.ndarray:
        """Bulk pressure p_EOS(rho) of every node, [ny][nx] FP64."""
        out = np.empty(self.shape(run))
        _check(self._lib.lbm_run_pressure(self._ctx, int(run), _dp(out)), "lbm_run_pressure",
               allow=(LBM_EDIVERGED,) if allow_diverged else ())
        return out

    def diagnostics(self, regions: Iterable, allow_diverged: bool = True) -> List[dict]:
        regs = list(regions)
        arr = (Region * len(regs))(*[Region(*map(float, r)) for r in regs])
        out = (Diag * len(regs))()
        if len(regs) != self.nruns:
            raise ValueError("one region per run is required")
        _check(self._lib.lbm_batch_diagnostics(self._ctx, arr, out), "lbm_batch_diagnostics",
               allow=(LBM_EDIVERGED,) if allow_diverged else ())
        keys = ("mass", "rho_in", "rho_out", "p_in", "p_out", "dp", "r_eq", "max_speed", "status")
        return [{k: getattr(d, k) for k in keys} for d in out]

    def status(self) -> np.ndarray:
        st = (_I32 * self.nruns)()
        _check(self._lib.lbm_run_status(self._ctx, st), "lbm_run_status", allow=(LBM_EDIVERGED,))
        return np.array(st[:], dtype=np.int32)

    def save_state(self) -> bytes:
        n = int(self._lib.lbm_state_bytes(self._ctx))
        buf = ctypes.create_string_buffer(n)
        _check(self._lib.lbm_save_state(self._ctx, ctypes.cast(buf, _P), n), "lbm_save_state")
        return buf.raw

    def load_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(self._lib.lbm_load_state(self._ctx, ctypes.cast(buf, _P), len(blob)), "lbm_load_state")

    # -- measurement
    def time_kernels(self, n: int) -> tuple:
        """Advance n steps with per-kernel HIP events; (psi_ms, collide_ms) means."""
        a, b = ctypes.c_double(), ctypes.c_double()
        _check(self._lib.lbm_time_kernels(self._ctx, int(n), ctypes.byref(a), ctypes.byref(b)),
               "lbm_time_kernels")
        return a.value, b.value

    # -- tuning
    def set_tile(self, tx: int, ty: int):
        _check(self._lib.lbm_set_tile(self._ctx, int(tx), int(ty)), "lbm_set_tile")

    def autotune(self, steps: int = 64) -> dict:
        """Pick the fastest schedule and tile shape for this context (advances the state)."""
        tx, ty, fu = _I32(), _I32(), _I32()
        _check(self._lib.lbm_autotune(self._ctx, int(steps), ctypes.byref(tx), ctypes.byref(ty),
                                      ctypes.byref(fu)), "lbm_autotune")
        return {"tile": (tx.value, ty.value), "fused": fu.value}

    def set_fused(self, rows):
        """One out-of-place fused kernel per step with `rows` nodes per thread
        (1, 2 or 4; True = 1) or the two in-place kernels (0 / False); every
        storage precision."""
        rows = 1 if rows is True else (0 if not rows else int(rows))
        _check(self._lib.lbm_set_fused(self._ctx, rows), "lbm_set_fused")

    def set_xcd_order(self, on: bool):
        _check(self._lib.lbm_set_xcd_order(self._ctx, int(bool(on))), "lbm_set_xcd_order")

    def set_graph_steps(self, k: int):
        _check(self._lib.lbm_set_graph_steps(self._ctx, int(k)), "lbm_set_graph_steps")


def step_noalloc(run, f_ptr: int, t0: int, n: int, status_ptr: int = 0, stream: int = 0) -> None:
    """lbm_step_noalloc: n FP64 steps of `run` in place on the device array at
    f_ptr ([9][ny][nx] doubles at step t0, in the in-place layout of parity
    t0 mod 2); status_ptr: device int32 or 0; stream: hipStream_t handle or 0.
    Enqueues only."""
    d = run_desc(run)
    lib = load_library()
    _check(lib.lbm_step_noalloc(ctypes.byref(d.grid), ctypes.byref(d.eos), d.G, ctypes.byref(d.rates), d.kappa,
                                d.epsilon, _P(f_ptr), int(t0), int(n), _P(status_ptr or None), _P(stream or None)),
           "lbm_step_noalloc")


def run3_args(run):
    """(Grid3, Eos, G, Rates3, kappa, epsilon) of a 3D run (fields nx, ny, nz,
    bc_x, bc_y, bc_z, eos_kind, eos, G, rates = (s_rho, s_e, s_eps, s_j, s_q,
    s_nu, s_pi, s_m), kappa, epsilon)."""
    g = Grid3(int(run.nx), int(run.ny), int(run.nz), int(run.bc_x), int(run.bc_y), int(run.bc_z))
    e = Eos()
    e.kind = int(run.eos_kind)
    p = list(run.eos) + [0.0] * (6 - len(run.eos))
    for i in range(6):
        e.p[i] = float(p[i])
    r = Rates3(*[float(v) for v in run.rates])
    return g, e, float(run.G), r, float(run.kappa), float(run.epsilon)


class Lattice3:
    """One D3Q19 run on the GPU (include/lbm3d.h): FP64 or FP32 storage, two
    kernels per step.  Arrays are [z][y][x]; populations [19][nz][ny][nx]."""

    def __init__(self, run, precision: str = "fp32", device: str = "cuda"):
        import torch

        if precision not in ("fp64", "fp32"):
            raise ValueError("3D runs store FP64 or FP32")
        self._lib = load_library()
        self.run = run
        self.precision = precision
        self.device = torch.device(device)
        g, e, G, r, kappa, eps = run3_args(run)
        self._args = (g, e, r)
        nbytes = int(self._lib.lbm3d_workspace_bytes(ctypes.byref(g), PRECISIONS[precision]))
        if nbytes == 0:
            _check(LBM_EINVAL, "lbm3d_workspace_bytes")
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.Stream(device=self.device)
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.workspace.data_ptr() + 255) & ~255
        ctx = _P()
        with torch.cuda.device(self.device):
            _check(self._lib.lbm3d_create(ctypes.byref(g), ctypes.byref(e), G, ctypes.byref(r), kappa, eps,
                                          PRECISIONS[precision], _P(aligned), nbytes, _P(self.stream.cuda_stream),
                                          ctypes.byref(ctx)), "lbm3d_create")
        self._ctx = ctx

    @property
    def shape(self):
        return (self.run.nz, self.run.ny, self.run.nx)

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.lbm3d_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def steps_taken(self) -> int:
        return int(self._lib.lbm3d_steps_taken(self._ctx))

    def init_density(self, rho, ux=None, uy=None, uz=None):
        f = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(self.shape)
        rho, ux, uy, uz = f(rho), f(ux), f(uy), f(uz)
        _check(self._lib.lbm3d_init_density(self._ctx, _dp(rho), _dp(ux), _dp(uy), _dp(uz)), "lbm3d_init_density")

    def init_all(self):
        self.init_density(self.run.rho, getattr(self.run, "ux", None), getattr(self.run, "uy", None),
                          getattr(self.run, "uz", None))

    def step(self, n: int = 1):
        _check(self._lib.lbm3d_step(self._ctx, int(n)), "lbm3d_step")

    def synchronize(self):
        self.stream.synchronize()

    def populations(self) -> np.ndarray:
        out = np.empty((19,) + self.shape)
        _check(self._lib.lbm3d_get_populations(self._ctx, _dp(out)), "lbm3d_get_populations")
        return out

    def set_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape((19,) + self.shape)
        _check(self._lib.lbm3d_set_populations(self._ctx, _dp(f)), "lbm3d_set_populations")

    def save_state(self) -> bytes:
        """Checkpoint of the current state (raw buffer; bit-exact restore)."""
        n = int(self._lib.lbm3d_state_bytes(self._ctx))
        buf = ctypes.create_string_buffer(n)
        _check(self._lib.lbm3d_save_state(self._ctx, ctypes.cast(buf, _P), n), "lbm3d_save_state")
        return buf.raw

    def load_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(self._lib.lbm3d_load_state(self._ctx, ctypes.cast(buf, _P), len(blob)), "lbm3d_load_state")

    def moments(self, allow_diverged: bool = False):
        out = [np.empty(self.shape) for _ in range(4)]
        _check(self._lib.lbm3d_moments(self._ctx, *[_dp(o) for o in out]), "lbm3d_moments",
               allow=(LBM_EDIVERGED,) if allow_diverged else ())
        return tuple(out)

    def diagnostics(self, dims: int, cx: float, cy: float, cz: float, r_in: float, r_out: float) -> dict:
        d = Diag()
        _check(self._lib.lbm3d_diagnostics(self._ctx, int(dims), float(cx), float(cy), float(cz), float(r_in),
                                           float(r_out), ctypes.byref(d)), "lbm3d_diagnostics",
               allow=(LBM_EDIVERGED,))
        return {k: getattr(d, k) for k in ("mass", "rho_in", "rho_out", "p_in", "p_out", "dp", "r_eq",
                                           "max_speed", "status")}

    def time_kernels(self, n: int) -> tuple:
        """Advance n steps with per-launch HIP events; (psi_ms, collide_ms)
        means (fused schedule: 0 and the fused kernel)."""
        a, b = ctypes.c_double(), ctypes.c_double()
        _check(self._lib.lbm3d_time_kernels(self._ctx, int(n), ctypes.byref(a), ctypes.byref(b)),
               "lbm3d_time_kernels")
        return a.value, b.value

    def set_schedule(self, fused: int = 1, tile_x: int = 64, tile_y: int = 8, z_chunk: int = 64):
        """fused = 1: one launch per step marching x-y tiles along z; 0: psi
        pass + collide pass (same bits)."""
        _check(self._lib.lbm3d_set_schedule(self._ctx, int(fused), int(tile_x), int(tile_y), int(z_chunk)),
               "lbm3d_set_schedule")

    def set_graph_steps(self, k: int):
        """step() replays HIP graphs of 2k steps (0: one launch per step)."""
        _check(self._lib.lbm3d_set_graph_steps(self._ctx, int(k)), "lbm3d_set_graph_steps")

    def autotune(self, steps: int = 8) -> tuple:
        """Pick the fastest schedule for this context (advances the state);
        returns (fused, tile_x, tile_y, z_chunk)."""
        v = [_I32() for _ in range(4)]
        _check(self._lib.lbm3d_autotune(self._ctx, int(steps), *[ctypes.byref(x) for x in v]), "lbm3d_autotune")
        return tuple(x.value for x in v)


def mc_args(run):
    """(Grid, McParams) of a two-component run description (workloads.RunMC)."""
    g = Grid(int(run.nx), int(run.ny), int(run.bc_x), int(run.bc_y))
    p = McParams(float(run.G), float(run.kappa), Rates(*[float(v) for v in run.rates]))
    return g, p


class LatticeMC:
    """One two-component (binary mixture) run on the GPU (include/lbm_mc.h):
    FP64 or FP32 storage, one fused launch per step.  Fields are [ny][nx];
    populations [2][9][ny][nx] (component A first)."""

    def __init__(self, run, precision: str = "fp32", device: str = "cuda"):
        import torch

        if precision not in ("fp64", "fp32"):
            raise ValueError("two-component runs store FP64 or FP32")
        self._lib = load_library()
        self.run = run
        self.precision = precision
        self.device = torch.device(device)
        g, p = mc_args(run)
        self._args = (g, p)
        nbytes = int(self._lib.lbm_mc_workspace_bytes(ctypes.byref(g), PRECISIONS[precision]))
        if nbytes == 0:
            _check(LBM_EINVAL, "lbm_mc_workspace_bytes")
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.Stream(device=self.device)
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.workspace.data_ptr() + 255) & ~255
        ctx = _P()
        with torch.cuda.device(self.device):
            _check(self._lib.lbm_mc_create(ctypes.byref(g), ctypes.byref(p), PRECISIONS[precision], _P(aligned),
                                           nbytes, _P(self.stream.cuda_stream), ctypes.byref(ctx)), "lbm_mc_create")
        self._ctx = ctx

    @property
    def shape(self):
        return (self.run.ny, self.run.nx)

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.lbm_mc_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def steps_taken(self) -> int:
        return int(self._lib.lbm_mc_steps_taken(self._ctx))

    def init_density(self, rhoA, rhoB, ux=None, uy=None):
        f = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(self.shape)
        rhoA, rhoB, ux, uy = f(rhoA), f(rhoB), f(ux), f(uy)
        _check(self._lib.lbm_mc_init_density(self._ctx, _dp(rhoA), _dp(rhoB), _dp(ux), _dp(uy)),
               "lbm_mc_init_density")

    def init_all(self):
        self.init_density(self.run.rhoA, self.run.rhoB, getattr(self.run, "ux", None), getattr(self.run, "uy", None))

    def step(self, n: int = 1):
        _check(self._lib.lbm_mc_step(self._ctx, int(n)), "lbm_mc_step")

    def synchronize(self):
        self.stream.synchronize()

    def set_tile(self, tx: int, ty: int, rows: int):
        _check(self._lib.lbm_mc_set_tile(self._ctx, int(tx), int(ty), int(rows)), "lbm_mc_set_tile")

    def set_graph_steps(self, k: int):
        """step() replays HIP graphs of 2k steps (0: one launch per step)."""
        _check(self._lib.lbm_mc_set_graph_steps(self._ctx, int(k)), "lbm_mc_set_graph_steps")

    def autotune(self, steps: int = 20) -> tuple:
        """Pick the fastest tile for this context (advances the state); returns (tx, ty, rows)."""
        v = [_I32() for _ in range(3)]
        _check(self._lib.lbm_mc_autotune(self._ctx, int(steps), *[ctypes.byref(x) for x in v]), "lbm_mc_autotune")
        return tuple(x.value for x in v)

    def populations(self) -> np.ndarray:
        out = np.empty((2, 9) + self.shape)
        _check(self._lib.lbm_mc_get_populations(self._ctx, _dp(out)), "lbm_mc_get_populations")
        return out

    def set_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape((2, 9) + self.shape)
        _check(self._lib.lbm_mc_set_populations(self._ctx, _dp(f)), "lbm_mc_set_populations")

    def save_state(self) -> bytes:
        """Checkpoint of the current state (raw buffer; bit-exact restore)."""
        n = int(self._lib.lbm_mc_state_bytes(self._ctx))
        buf = ctypes.create_string_buffer(n)
        _check(self._lib.lbm_mc_save_state(self._ctx, ctypes.cast(buf, _P), n), "lbm_mc_save_state")
        return buf.raw

    def load_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(self._lib.lbm_mc_load_state(self._ctx, ctypes.cast(buf, _P), len(blob)), "lbm_mc_load_state")

    def moments(self, allow_diverged: bool = False):
        """(rhoA, rhoB, ux, uy), u the mixture velocity of Eq. (6)."""
        out = [np.empty(self.shape) for _ in range(4)]
        _check(self._lib.lbm_mc_moments(self._ctx, *[_dp(o) for o in out]), "lbm_mc_moments",
               allow=(LBM_EDIVERGED,) if allow_diverged else ())
        return tuple(out)

    def diagnostics(self, cx: float, cy: float, r_in: float, r_out: float, allow_diverged: bool = True) -> dict:
        d = McDiag()
        _check(self._lib.lbm_mc_diagnostics(self._ctx, float(cx), float(cy), float(r_in), float(r_out),
                                            ctypes.byref(d)), "lbm_mc_diagnostics",
               allow=(LBM_EDIVERGED,) if allow_diverged else ())
        return {k: getattr(d, k) for k, _ in McDiag._fields_ if k != "reserved"}

    def time_kernels(self, n: int) -> float:
        """Advance n steps with HIP events around each launch; mean ms per step kernel."""
        t = ctypes.c_double()
        _check(self._lib.lbm_mc_time_kernels(self._ctx, int(n), ctypes.byref(t)), "lbm_mc_time_kernels")
        return t.value


def stream_copy_ms(dst, src, nbytes: int, reps: int, stream=None) -> float:
    """Mean ms of the library's plain copy kernel over nbytes (device pointers)."""
    ms = ctypes.c_double()
    _check(load_library().lbm_stream_copy(_P(dst), _P(src), int(nbytes), int(reps),
                                          _P(stream) if stream else None, ctypes.byref(ms)),
           "lbm_stream_copy")
    return ms.value


MLP_PARAMS = 4611


class Mlp:
    """The surrogate network of include/lbm_mlp.h (3-64-64-3, tanh, FP32).

    Inputs, targets and weights are numpy or torch arrays of shape [n, 3]; they
    are copied to the device as FP32 once per call.  Training and inference
    run in the library's kernels on a dedicated torch stream.
    """

    def __init__(self, params: np.ndarray, max_batch: int = 4096, device: str = "cuda"):
        import torch

        self._lib = load_library()
        self.device = torch.device(device)
        self.max_batch = int(max_batch)
        nbytes = int(self._lib.lbm_mlp_workspace_bytes(self.max_batch))
        if nbytes == 0:
            _check(LBM_EINVAL, "lbm_mlp_workspace_bytes")
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.Stream(device=self.device)
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.workspace.data_ptr() + 255) & ~255
        p = self._params_array(params)
        h = _P()
        with torch.cuda.device(self.device):
            _check(self._lib.lbm_mlp_create(self.max_batch, p.ctypes.data_as(_F), _P(aligned), nbytes,
                                            _P(self.stream.cuda_stream), ctypes.byref(h)), "lbm_mlp_create")
        self._h = h

    @staticmethod
    def _params_array(params) -> np.ndarray:
        p = np.ascontiguousarray(params, dtype=np.float32).ravel()
        if p.size != MLP_PARAMS:
            raise ValueError("expected %d parameters, got %d" % (MLP_PARAMS, p.size))
        return p

    def _dev(self, a):
        import torch

        t = torch.as_tensor(np.asarray(a, dtype=np.float32) if not isinstance(a, torch.Tensor) else a)
        t = t.to(device=self.device, dtype=torch.float32).contiguous()
        if t.dim() != 2 or t.shape[1] != 3:
            raise ValueError("expected an [n, 3] array")
        return t

    def close(self):
        if getattr(self, "_h", None):
            self._lib.lbm_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def params(self) -> np.ndarray:
        out = np.empty(MLP_PARAMS, dtype=np.float32)
        _check(self._lib.lbm_mlp_get_params(self._h, out.ctypes.data_as(_F)), "lbm_mlp_get_params")
        return out

    @params.setter
    def params(self, value):
        p = self._params_array(value)
        _check(self._lib.lbm_mlp_set_params(self._h, p.ctypes.data_as(_F)), "lbm_mlp_set_params")

    @property
    def steps_taken(self) -> int:
        return int(self._lib.lbm_mlp_steps_taken(self._h))

    def forward(self, X) -> np.ndarray:
        import torch

        x = self._dev(X)
        n = x.shape[0]
        y = torch.empty((n, 3), dtype=torch.float32, device=self.device)
        torch.cuda.current_stream(self.device).synchronize()
        for i in range(0, n, self.max_batch):
            m = min(self.max_batch, n - i)
            _check(self._lib.lbm_mlp_forward(self._h, _P(x[i:].data_ptr()), m, _P(y[i:].data_ptr())),
                   "lbm_mlp_forward")
        self.stream.synchronize()
        return y.cpu().numpy()

    def loss_grad(self, X, T, M) -> tuple:
        import torch

        x, t, m = self._dev(X), self._dev(T), self._dev(M)
        torch.cuda.current_stream(self.device).synchronize()
        loss = ctypes.c_double()
        g = np.empty(MLP_PARAMS, dtype=np.float32)
        _check(self._lib.lbm_mlp_loss_grad(self._h, _P(x.data_ptr()), _P(t.data_ptr()), _P(m.data_ptr()),
                                           x.shape[0], ctypes.byref(loss), g.ctypes.data_as(_F)),
               "lbm_mlp_loss_grad")
        return loss.value, g

    def train(self, X, T, M, steps: int, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8) -> float:
        """Full-batch Adam; returns the loss before the last update."""
        import torch

        x, t, m = self._dev(X), self._dev(T), self._dev(M)
        torch.cuda.current_stream(self.device).synchronize()
        loss = ctypes.c_double()
        _check(self._lib.lbm_mlp_train(self._h, _P(x.data_ptr()), _P(t.data_ptr()), _P(m.data_ptr()),
                                       x.shape[0], int(steps), lr, beta1, beta2, eps,
                                       ctypes.byref(loss) if steps > 0 else None), "lbm_mlp_train")
        return loss.value if steps > 0 else float("nan")
