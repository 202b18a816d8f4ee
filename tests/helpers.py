"""Test-side glue: oracle parameters from a workload run, and small seeded runs."""
import numpy as np

import oracle as O
from paper_1306_6445_amd import workloads as WL


def oracle_params(run) -> "O.Params":
    return O.params_from_run(run)


def small_run(nx, ny, kind="cs", kappa=0.3, epsilon=None, bc_x=WL.BC_PERIODIC, bc_y=WL.BC_PERIODIC,
              seed=1, R=None, noise=1e-3, nu=0.1, label=""):
    """A droplet (or slab when nx == 1) with seeded noise so that every term is active."""
    R = R if R is not None else max(1.0, min(nx, ny) / 4)
    if kind == "cs":
        eos_kind, eos = WL.cs_eos(0.7)
        rl, rv = WL.coexistence_seed(0.7, 1.93)
        eps = 1.93 if epsilon is None else epsilon
        G = -1.0
    elif kind == "pw":
        eos_kind, eos = WL.piecewise_eos()
        rl, rv = 100.0, 1.0
        eps = 16 * 0.087 if epsilon is None else epsilon
        G = -1.0
    else:
        eos_kind, eos = WL.exp_eos()
        rl, rv = 514.6, 79.7
        eps = 0.0 if epsilon is None else epsilon
        G = -40.0
    if nx == 1:
        rho = WL.slab(nx, ny, rl, rv, ny / 2)
    else:
        rho = WL.droplet(nx, ny, R, rl, rv)
    rho = rho * (1 + WL.noise(rho.shape, noise, seed))
    return WL.Run(nx=nx, ny=ny, eos_kind=eos_kind, eos=eos, G=G, rates=WL.rates(nu), kappa=kappa,
                  epsilon=eps, rho=rho, bc_x=bc_x, bc_y=bc_y, cx=nx / 2, cy=ny / 2, R0=R,
                  label=label or "%s_%dx%d" % (kind, nx, ny))


def rel_err(f_test, f_ref) -> float:
    """max over nodes and directions of |df_a(x)| / rho_ref(x)."""
    f_test = np.asarray(f_test, dtype=np.float64)
    f_ref = np.asarray(f_ref, dtype=np.float64)
    rho = np.abs(f_ref.sum(axis=0))
    return float((np.abs(f_test - f_ref) / rho[None]).max())


def rel_err_scaled(f_test, f_ref, scale: float) -> float:
    """max of |df_a(x)| / max(rho_ref(x), scale): reduced-precision storage keeps
    deviations from the rest state at a per-run base density, so its rounding is
    bounded relative to that base density rather than to the local one."""
    f_test = np.asarray(f_test, dtype=np.float64)
    f_ref = np.asarray(f_ref, dtype=np.float64)
    rho = np.maximum(np.abs(f_ref.sum(axis=0)), scale)
    return float((np.abs(f_test - f_ref) / rho[None]).max())


def oracle3_params(run):
    """D3Q19 oracle parameters of a 3D workload run."""
    from oracle import d3q19 as D

    s_rho, s_e, s_eps, s_j, s_q, s_nu, s_pi, s_m = run.rates
    sigma = O.sigma_from_epsilon(run.epsilon, run.G) if run.epsilon != 0.0 else 0.0
    return D.Params3(nx=run.nx, ny=run.ny, nz=run.nz, eos_kind=run.eos_kind, eos=tuple(run.eos)[:6], G=run.G,
                     s=D.rates(s_rho, s_e, s_eps, s_j, s_q, s_nu, s_pi, s_m), kappa=run.kappa, sigma=sigma,
                     bc_x=run.bc_x, bc_y=run.bc_y, bc_z=run.bc_z)


def small_run3(nx, ny, nz, kind="cs", kappa=0.6, bc=(0, 0, 0), seed=1, noise=1e-3, R=None):
    """A 3D drop (or, with one of the sizes 1, a column or slab) with seeded noise."""
    import dataclasses

    R = R if R is not None else max(1.0, min(v for v in (nx, ny, nz) if v > 1) / 4)
    run = WL.droplet3_run(0, R, 0.7, kappa, 1.93, shape=(nx, ny, nz), label="%s_%dx%dx%d" % (kind, nx, ny, nz))
    if kind == "pw":
        k, eos = WL.piecewise_eos()
        run = dataclasses.replace(run, eos_kind=k, eos=eos, epsilon=16 * 0.087,
                                  rho=WL.sphere(nx, ny, nz, R, 100.0, 1.0))
    elif kind == "exp":
        k, eos = WL.exp_eos()
        run = dataclasses.replace(run, eos_kind=k, eos=eos, G=-40.0, epsilon=0.0,
                                  rho=WL.sphere(nx, ny, nz, R, 514.6, 79.7))
    rho = run.rho * (1 + WL.noise(run.rho.shape, noise, seed))
    return dataclasses.replace(run, rho=rho, kappa=kappa, bc_x=bc[0], bc_y=bc[1], bc_z=bc[2])


def oracle_mc_params(run):
    """Two-component oracle parameters of a workload run (workloads.RunMC)."""
    from oracle import binary as B

    s_rho, s_e, s_zeta, s_j, s_q, s_nu = run.rates
    return B.ParamsMC(nx=run.nx, ny=run.ny, G=run.G, s=B.rates(s_rho, s_e, s_zeta, s_j, s_q, s_nu),
                      kappa=run.kappa, bc_x=run.bc_x, bc_y=run.bc_y)


def small_mc_run(nx, ny, bc=(0, 0), kappa=0.6, G=1.1, seed=1, R=None, noise=2e-2):
    """A drop of A in B (or a slab when nx == 1) with seeded composition noise
    so that every term is active."""
    import dataclasses

    R = R if R is not None else max(1.0, min(v for v in (nx, ny) if v > 1) / 4)
    run = WL.mc_drop_run(0, R, kappa, G=G, shape=(nx, ny), W=3.0)
    rng = np.random.default_rng(seed)
    rhoA = run.rhoA * (1 + noise * rng.uniform(-1, 1, run.rhoA.shape))
    rhoB = run.rhoB * (1 + noise * rng.uniform(-1, 1, run.rhoB.shape))
    return dataclasses.replace(run, rhoA=rhoA, rhoB=rhoB, bc_x=bc[0], bc_y=bc[1],
                               label="mc_%dx%d_bc%d%d" % (nx, ny, bc[0], bc[1]))


def rel_err_mc(f_test, f_ref) -> float:
    """max over components, directions and nodes of |df| / (rho_A + rho_B)(x)."""
    f_test = np.asarray(f_test, dtype=np.float64)
    f_ref = np.asarray(f_ref, dtype=np.float64)
    rho = np.abs(f_ref.sum(axis=(0, 1)))
    return float((np.abs(f_test - f_ref) / rho[None, None]).max())
