"""Writes paper_1306_6445_amd/workload_params.json (run by hand; calls only oracle/).

The synthetic workloads need numbers the paper does not print:
* T_c of the Carnahan-Starling EOS (a = 0.25, b = 4, R = 1), because the
  configurations are stated in T / T_c;
* liquid / vapour densities to shape the initial tanh profiles.  These come from
  the mechanical-stability condition, Eq. (16) with G2 = 0 and exponent
  epsilon, on a (T/T_c, epsilon) grid; Maxwell densities are stored beside them
  for grid points where Eq. (16) has no root;
* the curvature dependence of the droplet's bulk densities, rho(R) = a + c/R,
  fitted from two oracle droplets (R = 20 and 30 on a 100 x 100 periodic grid,
  6000 steps) for the (T/T_c, epsilon) points of the droplet workloads.  In a
  large periodic box a droplet seeded with flat-interface vapour has to
  evaporate part of its mass to raise the vapour to its own (higher)
  equilibrium density, and small droplets vanish; seeding with rho(R) avoids
  that transfer.

The initial profile only seeds the run: the droplet relaxes to the model's own
coexistence, and parity tests feed the same array to both sides.

Usage:  python oracle/gen_workload_params.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from oracle import theory  # noqa: E402

OUT = os.path.join(ROOT, "paper_1306_6445_amd", "workload_params.json")

A, B, R_GAS = 0.25, 4.0, 1.0
TR_GRID = [round(0.55 + 0.025 * i, 3) for i in range(13)]        # 0.55 .. 0.85
EPS_GRID = [round(1.0 + 0.1 * i, 2) for i in range(11)]           # 1.0 .. 2.0
POINTS = [(0.7, 1.93), (0.6, 1.93)]


def cs_params(tr, T_c):
    return O.Params(nx=1, ny=1, eos_kind=O.EOS_CS, eos=(A, B, R_GAS, tr * T_c), G=-1.0)


def droplet_bulk(tr, eps, T_c, R, rl, rv, n=100, steps=6000):
    """(rho_in, rho_out, r_eq) of an oracle droplet (tanh seed of width 5)."""
    P = O.Params(nx=n, ny=n, eos_kind=O.EOS_CS, eos=(A, B, R_GAS, tr * T_c), G=-1.0,
                 sigma=O.sigma_from_epsilon(eps, -1.0), s=O.rates())
    y, x = np.mgrid[0:n, 0:n].astype(float)
    r = np.hypot(x - n / 2, y - n / 2)
    rho = (rl + rv) / 2 - (rl - rv) / 2 * np.tanh(2 * (r - R) / 5.0)
    f = O.run(P, O.init(P, rho), steps)
    d = O.diagnostics(P, f, n / 2, n / 2, R / 4, R + 15)
    return d["rho_in"], d["rho_out"], d["r_eq"]


def main():
    rho_c, T_c = theory.critical_point(A, B, R_GAS)
    out = {"cs": {"a": A, "b": B, "R": R_GAS, "rho_c": rho_c, "T_c": T_c}}
    mx_l, mx_v = [], []
    for tr in TR_GRID:
        rl, rv, _ = theory.maxwell(cs_params(tr, T_c))
        mx_l.append(rl)
        mx_v.append(rv)
    out["maxwell"] = {"T_over_Tc": TR_GRID, "rho_l": mx_l, "rho_v": mx_v}
    gl = np.full((len(TR_GRID), len(EPS_GRID)), np.nan)
    gv = np.full_like(gl, np.nan)
    for i, tr in enumerate(TR_GRID):
        for j, eps in enumerate(EPS_GRID):
            try:
                rl, rv, _ = theory.coexistence(cs_params(tr, T_c), eps)
                gl[i, j], gv[i, j] = rl, rv
            except ValueError:
                pass
        print("T/Tc", tr, "done", flush=True)
    out["mechanical"] = {"T_over_Tc": TR_GRID, "epsilon": EPS_GRID,
                         "rho_l": [[None if np.isnan(v) else v for v in row] for row in gl],
                         "rho_v": [[None if np.isnan(v) else v for v in row] for row in gv]}
    pts = []
    for tr, eps in POINTS:
        rl, rv, _ = theory.coexistence(cs_params(tr, T_c), eps)
        entry = {"T_over_Tc": tr, "epsilon": eps, "rho_l": rl, "rho_v": rv}
        # curved-interface bulk densities rho(R) = a + c / R from two droplets
        d1 = droplet_bulk(tr, eps, T_c, 20.0, rl, rv)
        d2 = droplet_bulk(tr, eps, T_c, 30.0, rl, rv)
        inv = np.array([1.0 / d1[2], 1.0 / d2[2]])
        for key, i in (("liquid", 0), ("vapour", 1)):
            c = (d1[i] - d2[i]) / (inv[0] - inv[1])
            entry["droplet_" + key] = {"a": d1[i] - c * inv[0], "c": c}
        print("point", tr, eps, entry, flush=True)
        pts.append(entry)
    out["points"] = pts
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
