#!/usr/bin/env python3
"""Benchmark: MLUPS and HBM roofline of the MI355X lattice Boltzmann path.

Workload (one "step" = one time step of every run): the Laplace-law / kappa
sweep of 40 periodic 256x256 droplets (radii 20..60 x 8 kappa values in
[0, 0.99]), Carnahan-Starling EOS at T/Tc = 0.7, stepped together in one
batched FP32 context.  Reported next to it:
  * the plain FP64 path (one run per context, 256x256) and FP64 batched;
  * roofline of the dominant kernel (the fused step kernel in the workload's
    default shape; the collide-stream kernel when the two-kernel schedule is
    chosen with --fused 0 or by --tile auto), timed with HIP events on the
    library's stream, and the two-kernel schedule timed beside it;
  * accuracy of FP32 vs FP64 after the full 20,000 steps: surface tension from
    the Laplace fit (pressure jump vs 1/R) per kappa, rho_l/rho_v, per-node rho;
  * the FP64 CPU oracle timed on the host cores on a bounded sample.
Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS and % HBM roofline, FP32/batched vs plain FP64, at sigma err <0.5%"
HBM_PEAK_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_1306_6445_amd", "csrc", "lbm_kernels.hip")
# HBM traffic per dispatch of the dominant kernel, written from rocprofv3 counter runs
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_%s_%s_%s.json")

# step schedule per workload (threads per tile, nodes per thread of the fused
# kernel), the fastest of an FP32 sweep on MI355X: 256-wide tiles (of 512
# threads) suit the one large grid, 64-wide ones the batches of small runs
DEFAULT_SHAPE = {"config2": ((64, 4), 2), "config3": ((256, 2), 4), "config4": ((128, 2), 4),
                 "config5": ((64, 4), 2)}
# algorithmic bytes per lattice update of the collide-stream kernel of the
# two-kernel schedule: every population read and written once plus one psi read
COLLIDE_BYTES = {"fp64": 9 * 8 * 2 + 8, "fp32": 9 * 4 * 2 + 4, "bf16": 9 * 2 * 2 + 4}
# ... and of the fused step: every population read once and written once
STEP_BYTES_ALG = {"fp64": 9 * 8 * 2, "fp32": 9 * 4 * 2, "bf16": 9 * 2 * 2}
# bf16 storage also reads and writes one FP32 writer density per node
WRITER_BYTES = 8
STORE_BYTES = {"fp64": 8, "fp32": 4, "bf16": 2}
KERNEL_TYPE = {"fp64": "double", "fp32": "float", "bf16": "bf16_t"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def ensure_built():
    from paper_1306_6445_amd import lbm
    if not os.path.exists(lbm.LIB_PATH):
        from paper_1306_6445_amd import build
        build.build(verbose=False)


def launch_ms(fused, t_region, k, dispatch_ms):
    """Mean duration of one launch of the step kernel.  The fused schedule is
    one launch per step, so the timed region (HIP events on the library's
    stream) over its k launches gives it directly, launch gaps included; the
    two-kernel schedule needs the per-dispatch events to separate its kernels."""
    return 1e3 * t_region / k if fused else dispatch_ms


def timed_steps(L, k, torch):
    torch.cuda.synchronize()
    L.synchronize()
    t0 = time.perf_counter()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(L.stream)
    L.step(k)
    stop.record(L.stream)
    L.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(stop) / 1e3, wall


def accuracy_block(runs, steps, lbm, window=8000, every=100):
    """Droplet sweep: FP32 and bf16 vs FP64 after `steps` steps of every run
    (GPU all three).  sigma comes from Laplace fits of the pressure jump
    averaged over the last `window` steps (the drops still ring acoustically
    at 20,000 steps); the fits of the final snapshot are reported beside."""
    from paper_1306_6445_amd.analysis import averaged_diagnostics, laplace_fit

    res = {}
    regions = [(r.cx, r.cy, *r.diag_radii()) for r in runs]
    for prec in ("fp64", "fp32", "bf16"):
        L = lbm.Lattice(runs, precision=prec)
        L.init_all()
        snap, mean = averaged_diagnostics(L, regions, steps, window, every)
        rhos = [L.moments(i, allow_diverged=True)[0] for i in range(len(runs))]
        res[prec] = (mean, rhos, snap)
        L.close()
    d64, r64, s64 = res["fp64"]
    d32, r32, s32 = res["fp32"]
    d16, _, s16 = res["bf16"]

    def sigma_errors(da, db):
        fa, fb = laplace_fit(da, runs), laplace_fit(db, runs)
        return fa, {k: abs(fa[k][0] - fb[k][0]) / abs(fb[k][0]) for k in fb if k in fa}

    def ratio_error(da, db):
        return max(abs(a["rho_in"] / a["rho_out"] - b["rho_in"] / b["rho_out"]) / (b["rho_in"] / b["rho_out"])
                   for a, b in zip(da, db))

    f64 = laplace_fit(d64, runs)
    f32, sig_err = sigma_errors(d32, d64)
    f16, sig_err16 = sigma_errors(d16, d64)
    _, snap_err = sigma_errors(s32, s64)
    _, snap_err16 = sigma_errors(s16, s64)
    ratio_err, ratio_err16 = ratio_error(d32, d64), ratio_error(d16, d64)
    # kappa leaves the density ratio unchanged (Section IV): spread over kappa
    # at each radius (the ratio itself depends on R through the curvature)
    spread = []
    for R in sorted(set(r.R0 for r in runs)):
        rs = [b["rho_in"] / b["rho_out"] for b, r in zip(d64, runs) if r.R0 == R and b["status"] == 0]
        if len(rs) > 1:
            spread.append((max(rs) - min(rs)) / np.mean(rs))
    node_err = max(float(np.abs(a - b).max() / b.max()) for a, b in zip(r32, r64))
    sig0 = abs(f64[min(f64)][0]) if f64 else float("nan")
    return {
        "steps": steps,
        "sigma_estimator": "Laplace fit of dp averaged over the last %d steps (every %d)" % (window, every),
        "sigma_fp64_by_kappa": {"%g" % k: v[0] for k, v in f64.items()},
        "sigma_fp32_by_kappa": {"%g" % k: v[0] for k, v in f32.items()},
        "sigma_rel_err_by_kappa": {"%g" % k: v for k, v in sig_err.items()},
        "sigma_rel_err_max": max(sig_err.values()) if sig_err else None,
        "sigma_abs_err_over_sigma_kappa0_max": max(abs(f32[k][0] - f64[k][0]) for k in sig_err) / sig0
        if sig_err else None,
        "sigma_ratio_to_kappa0_fp64": {"%g" % k: v[0] / f64[min(f64)][0] for k, v in f64.items()},
        "rho_ratio_rel_err_max": ratio_err,
        "rho_node_rel_err_max": node_err,
        "rho_ratio_fp64_spread_over_kappa_max_per_radius": max(spread) if spread else None,
        "diverged_fp32": int(sum(d["status"] for d in d32)),
        "pass_0.5pct": bool(sig_err and max(sig_err.values()) < 5e-3 and ratio_err < 5e-3),
        "snapshot_sigma_rel_err_by_kappa": {"%g" % k: v for k, v in snap_err.items()},
        "bf16": {"sigma_by_kappa": {"%g" % k: v[0] for k, v in f16.items()},
                 "sigma_rel_err_by_kappa": {"%g" % k: v for k, v in sig_err16.items()},
                 "sigma_abs_err_over_sigma_kappa0_max": max(abs(f16[k][0] - f64[k][0]) for k in sig_err16) / sig0
                 if sig_err16 else None,
                 "snapshot_sigma_rel_err_by_kappa": {"%g" % k: v for k, v in snap_err16.items()},
                 "rho_ratio_rel_err_max": ratio_err16,
                 "diverged": int(sum(d["status"] for d in d16))},
    }


def capillary_block(steps, lbm, wavelengths=(256, 512, 1024), every=100):
    """Capillary waves on the full 4096 x 2048 grid, one run per wavelength:
    omega from the amplitude history in FP64, FP32 and bf16 storage, against
    the linear dispersion relation with sigma from an FP64 Laplace fit at the
    same temperature (GPU droplets).  `periods_in_run` says how much of the
    theoretical period the run covers (lambda = 1024 needs about 118,000
    steps: over fewer than one period the damped-cosine fit is loose)."""
    from paper_1306_6445_amd import analysis as A
    from paper_1306_6445_amd import workloads as WL

    T, eps = 0.6, 1.93
    lap = A.laplace_sigma(lbm, T, eps)
    out = {"steps": steps, "sample_every": every, "grid": [4096, 2048],
           "sigma_laplace_slope_fp64": lap["sigma"], "sigma_flat_fp64": lap["sigma_flat"],
           "laplace_r_eq": lap["r_eq"], "wavelengths": {}}
    for lam in wavelengths:
        log("  capillary lambda %d, %d steps" % (lam, steps))
        run = WL.config3(wavelength=lam)
        assert run.T_over_Tc == T and run.epsilon == eps
        exp = A.capillary_experiment(lbm, run, ("fp64", "fp32", "bf16"), lam, steps, every)
        ref = exp["fp64"]
        w = {"wavelength": lam}
        out["wavelengths"][str(lam)] = w
        if ref["fit"] is None:
            w["error"] = "fp64 wave diverged or lost its interface"
            continue
        # theory with the flat-interface tension (curvature-corrected Laplace fit)
        w_th = A.capillary_omega(lap["sigma_flat"], lam, ref["rho_l"], ref["rho_v"])
        w.update(omega_theory=w_th, period_theory_steps=2 * np.pi / w_th, periods_in_run=steps * w_th / (2 * np.pi),
                 omega_theory_laplace_slope=A.capillary_omega(lap["sigma"], lam, ref["rho_l"], ref["rho_v"]))
        a0 = abs(ref["a"][0])
        for prec, e in exp.items():
            d = {"status": e["status"], "rho_l": e["rho_l"], "rho_v": e["rho_v"]}
            if e["fit"] is not None:
                d.update(omega=e["fit"]["omega"], gamma=e["fit"]["gamma"], fit_rms=e["fit"]["rms_residual"],
                         crossings=e["fit"]["crossings"],
                         omega_rel_err_vs_theory=e["fit"]["omega"] / w_th - 1.0,
                         omega_rel_err_vs_fp64=e["fit"]["omega"] / ref["fit"]["omega"] - 1.0,
                         amplitude_max_dev_over_a0=float(np.nanmax(np.abs(e["a"] - ref["a"])) / a0),
                         ratio_rel_err_vs_fp64=(e["rho_l"] / e["rho_v"]) / (ref["rho_l"] / ref["rho_v"]) - 1.0,
                         column_rel_err_max=float(np.max(np.abs(e["final_column"] - ref["final_column"]))
                                                  / np.max(ref["final_column"])))
            w[prec] = d
        key = "omega_rel_err_vs_fp64"
        if w["periods_in_run"] < 1.0:
            # less than one period: the free fit trades decay and offset
            # against frequency, so the precisions are compared at the
            # FP64 fit's decay and offset
            f64 = ref["fit"]
            key = "omega_rel_err_vs_fp64_given_decay"
            w["comparison"] = "omega at the FP64 fit's decay and offset (run shorter than one period)"
            for prec in ("fp32", "bf16"):
                e = exp[prec]
                if e["fit"] is not None:
                    wg = A.cosine_fit_given_decay(e["t"], e["a"], f64["gamma"], f64["offset"], f64["amplitude"],
                                                  f64["omega"], f64["phase"])
                    w[prec][key] = wg / f64["omega"] - 1.0
        errs = [abs(w[p].get(key, np.inf)) for p in ("fp32", "bf16")]
        rerr = [abs(w[p].get("ratio_rel_err_vs_fp64", np.inf)) for p in ("fp32", "bf16")]
        w["pass_0.5pct_fp32"] = bool(errs[0] < 5e-3 and rerr[0] < 5e-3)
        w["pass_0.5pct_bf16"] = bool(errs[1] < 5e-3 and rerr[1] < 5e-3)
    return out


def ensemble_block(runs, steps, lbm, graph_steps, dump=None, window=2000, every=100):
    """Ensemble: per-run (rho_l, rho_v, sigma = dp R_eq) in FP32 against FP64
    after `steps` steps; runs are classified ok / mixed / evaporated / diverged
    on the final state; the per-run values are averaged over the last
    `window` steps (the final snapshot's sigma error is reported beside)."""
    from paper_1306_6445_amd.analysis import DROPLET_CLASSES, averaged_diagnostics, classify_droplet

    regions = [(r.cx, r.cy, *r.diag_radii()) for r in runs]
    res, snap = {}, {}
    for prec in ("fp64", "fp32"):
        L = lbm.Lattice(runs, precision=prec, graph_steps=graph_steps)
        L.init_all()
        snap[prec], res[prec] = averaged_diagnostics(L, regions, steps, window, every)
        L.close()
    cls = {p: [classify_droplet(d, r) for d, r in zip(snap[p], runs)] for p in res}
    both = [i for i in range(len(runs)) if cls["fp64"][i] == "ok" and cls["fp32"][i] == "ok"]

    def rel(key_fn, src=res):
        return max((abs(key_fn(src["fp32"][i]) / key_fn(src["fp64"][i]) - 1.0) for i in both), default=None)

    out = {"steps": steps, "runs": len(runs),
           "classes_fp64": {c: cls["fp64"].count(c) for c in DROPLET_CLASSES},
           "classes_fp32": {c: cls["fp32"].count(c) for c in DROPLET_CLASSES},
           "class_disagreements": int(sum(a != b for a, b in zip(cls["fp64"], cls["fp32"]))),
           "rho_l_rel_err_max": rel(lambda d: d["rho_in"]),
           "rho_v_rel_err_max": rel(lambda d: d["rho_out"]),
           "ratio_rel_err_max": rel(lambda d: d["rho_in"] / d["rho_out"]),
           "sigma_single_rel_err_max": rel(lambda d: d["dp"] * d["r_eq"]),
           "snapshot_sigma_single_rel_err_max": rel(lambda d: d["dp"] * d["r_eq"], snap),
           "estimator": "settled runs: values averaged over the last %d steps (every %d)" % (window, every)}
    if dump:
        cols = ("rho_in", "rho_out", "dp", "r_eq", "mass", "max_speed", "status")
        np.savez(dump, T_over_Tc=np.array([r.T_over_Tc for r in runs]), kappa=np.array([r.kappa for r in runs]),
                 epsilon=np.array([r.epsilon for r in runs]), L=np.array([r.nx for r in runs]),
                 R0=np.array([r.R0 for r in runs]),
                 **{"%s_%s" % (p, c): np.array([d[c] for d in res[p]]) for p in res for c in cols},
                 **{"class_%s" % p: np.array(cls[p]) for p in res})
        out["dump"] = dump
    return out


def surrogate_block(lbm, torch):
    """Surrogate-guided parameter selection: solver-generated data (the
    ensemble's parameter draws on grids of 64..192, plus flat slabs), GPU
    training of the network, then LB solves needed to hit targets measured
    at hidden parameter points, against bisection and a physics-aware search."""
    from paper_1306_6445_amd import surrogate as S, workloads as WL

    t0 = time.perf_counter()
    sur, tr, te = S.build(lbm, n_drops=512, n_slabs=1200, seed=WL.BASE_SEED + 4, drop_steps=12000,
                          slab_steps=12000, lmax=192, log=log)
    t_build = time.perf_counter() - t0
    out = {"data": "ensemble draws (T/Tc, kappa, epsilon, R/L) on grids 64..192, 12000 steps, late-window "
                   "averages; 1200 flat slabs 4x256",
           "departure_from_ensemble": "not trained on the 512-droplet ensemble itself (L 64..512, 10000 "
                                      "steps): its parameter draws are rerun on grids of at most 192 for "
                                      "12000 steps, because most drops with L above 192 still ring "
                                      "acoustically at 10000 steps (pressure jump varying by more than 25% "
                                      "over the averaging window), which makes their tension unusable as a "
                                      "label; flat slabs add the density-ratio data",
           "samples": len(tr) + len(te),
           "classes": {c: sum(s.cls == c for s in tr + te)
                       for c in ("ok", "unsettled", "evaporated", "mixed", "vacuum", "diverged")},
           "loss_schedule": [list(h) for h in sur.history], "data_and_training_s": t_build,
           "heldout": S.validation_errors(sur, te)}
    # training and inference speed of the network kernels alone
    X, Y, M = S.dataset(tr)
    Xe = S.encode_inputs(X).astype(np.float32)
    Ze = np.nan_to_num(sur.scaler.encode(Y)).astype(np.float32)
    with lbm.Mlp(S.init_params(1), max_batch=len(X)) as net:
        net.train(Xe, Ze, M.astype(np.float32), 10, 1e-3)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        net.train(Xe, Ze, M.astype(np.float32), 1000, 1e-3)
        out["train_step_us"] = (time.perf_counter() - t1) * 1e3
    grid = np.stack(np.meshgrid(np.linspace(0.55, 0.85, 512), np.linspace(0, 0.99, 512), [1.9],
                                indexing="ij"), -1).reshape(-1, 3)
    sur.predict(grid[:1024])
    t1 = time.perf_counter()
    sur.predict(grid)
    out["inference_per_s"] = len(grid) / (time.perf_counter() - t1)
    sel = []
    for hidden in ((0.56, 0.5, 1.9), (0.62, 0.7, 1.6), (0.66, 0.45, 1.85), (0.72, 0.3, 1.95)):
        ref = S.Verifier(lbm)
        t = ref(*hidden)
        row = {"hidden": hidden, "ratio": t.ratio, "sigma": t.sigma}
        for name, fn in (("network", lambda j: S.surrogate_select(sur, j, t.ratio, t.sigma, hidden[2])),
                         ("bisection", lambda j: S.bisection_select(j, t.ratio, t.sigma, hidden[2])),
                         ("physics_aware", lambda j: S.physics_select(j, t.ratio, t.sigma, hidden[2]))):
            j = S.Verifier(lbm)
            r = fn(j)
            row[name] = {"solves": r["solves"], "hit": r["hit"],
                         "found": [r["final"].T_over_Tc, r["final"].kappa] if r["final"] else None}
            if "fallback" in r:
                row[name].update(network_solves=r["network_solves"], fallback_solves=r["fallback_solves"])
        log("selection", row)
        sel.append(row)
    out["selection"] = sel
    out["verifier"] = "slab 4x256 (ratio) + droplet R=40 in 128x128 (sigma = dp R_eq), FP32, 16000 steps, " \
                   "last 4000 averaged; hit = both within 1%"
    sur.net.close()
    return out


SPLASH_TARGET = {"ratio": 300.0, "sigma": 0.002, "epsilon": 1.7}


def splash_selection(lbm):
    """Parameters of the splash: the surrogate (trained here on solver data)
    picks (T/Tc, kappa) at epsilon for a target density ratio and tension; one
    verifier solve per iteration until both are within 1%."""
    from paper_1306_6445_amd import surrogate as S, workloads as WL

    t0 = time.perf_counter()
    sur, tr, te = S.build(lbm, n_drops=512, n_slabs=1200, seed=WL.BASE_SEED + 4, drop_steps=12000,
                          slab_steps=12000, lmax=192, log=log)
    j = S.Verifier(lbm)
    sel = S.surrogate_select(sur, j, SPLASH_TARGET["ratio"], SPLASH_TARGET["sigma"], SPLASH_TARGET["epsilon"])
    f = sel["final"]
    sur.net.close()
    return {"target": SPLASH_TARGET, "solves": sel["solves"], "hit": sel["hit"],
            "network_solves": sel["network_solves"], "fallback_solves": sel["fallback_solves"],
            "T_over_Tc": f.T_over_Tc, "kappa": f.kappa, "epsilon": f.epsilon,
            "verified_ratio": f.ratio, "verified_sigma": f.sigma, "seconds": time.perf_counter() - t0}


def splash_block(run, steps, lbm, every=1000):
    """Splash in FP32 and bf16 against the plain FP64 rerun (the verifier): spread
    radius three rows above the film, mass, and the final fields;
    plus the Table 5 set-up (Eq. 23, kappa = 0) as a coarse check."""
    from paper_1306_6445_amd import analysis as A, workloads as WL

    D, U = 2 * run.R0, 0.05
    film = int(0.1 * run.ny)
    times = list(range(0, steps + 1, every))
    res = {}
    for prec in ("fp64", "fp32", "bf16"):
        with lbm.Lattice([run], precision=prec) as L:
            L.init_all()
            h = A.splash_history(L, 0, times, film + 3, run.rho_nu, run.nx / 2, outermost=True)
            h["status"] = int(L.status()[0])
        res[prec] = h
    ref = res["fp64"]
    out = {"steps": steps, "t_star": [U * t / D for t in times], "r_over_D_fp64": [r / D for r in ref["r"]]}
    for prec in ("fp32", "bf16"):
        h = res[prec]
        a, b = h["rho"], ref["rho"]
        out[prec] = {"status": h["status"],
                     "r_over_D": [r / D for r in h["r"]],
                     "r_max_dev_nodes": float(np.nanmax(np.abs(np.array(h["r"]) - np.array(ref["r"])))),
                     "mass_drift": h["mass"][-1] / h["mass"][0] - 1.0,
                     "final_phase_disagreement": float(np.mean((a > run.rho_nu) != (b > run.rho_nu))),
                     "final_rho_L1_rel": float(np.abs(a - b).sum() / np.abs(b).sum())}
    out["fp64_mass_drift"] = ref["mass"][-1] / ref["mass"][0] - 1.0
    # Table 5 set-up, coarse (the paper's open boundaries are replaced by a wall and periodic sides)
    pr = WL.paper_splash_run(0.0)
    ts = [0.05, 0.25, 0.75, 1.0, 1.5]
    with lbm.Lattice([pr], precision="fp32") as L:
        L.init_all()
        h = A.splash_history(L, 0, [int(round(t * 100 / 0.125)) for t in ts], 28, 50.5, pr.nx / 2)
    out["table5_kappa0"] = {"t_star": ts, "r_over_D": [r / 100 for r in h["r"]],
                            "paper": [0.3100, 0.6728, 1.1708, 1.3317, 1.6034],
                            "power_law_1.3sqrt": [1.3 * np.sqrt(t) for t in ts]}
    return out


def graph_plan(steps, graph_steps):
    """Graph length for a timed region of `steps` steps: the library replays
    captured graphs of 2k steps, so k is lowered to steps // 2 when the region
    is shorter than 2k steps (then at least one replay is timed)."""
    k = graph_steps
    if k > 0 and steps < 2 * k:
        k = max(1, steps // 2)
    replays = steps // (2 * k) if k > 0 else 0
    return k, replays, steps - 2 * k * replays


def graph_timed(L, steps, warmup, graph_steps, torch):
    """GPU seconds of `steps` steps from the initial state, graph-replayed as
    graph_plan chooses, after warm_graph's untimed steps."""
    k, _, _ = graph_plan(steps, graph_steps)
    L.set_graph_steps(k)
    L.init_all()
    if warm_graph(L, warmup, k):
        L.init_all()
    return timed_steps(L, steps, torch)[0]


def warm_graph(L, warmup, k):
    """Untimed steps: the requested warm-up, at least one whole graph (so the
    capture happens here, not in the timed region), rounded up to whole graphs
    so that the timed region starts on the buffer the graph was captured from."""
    n = max(warmup, 2 * k if k > 0 else 0)
    if k > 0:
        n = -(-n // (2 * k)) * (2 * k)
    if n:
        L.step(n)
        L.synchronize()
    return n


# HBM-resident workloads timed beside the cache-resident headline: the
# capillary grid (2 x 302 MB of FP32 populations) and the 512-run ensemble
# (2 x 1.9 GB); both exceed the 256 MB Infinity Cache
HBM_LEGS = (("config3", "capillary wave 4096x2048 (lambda 256), FP32"),
            ("config4", "ensemble of 512 droplets, L ~ U{64..512}, FP32"))


def hbm_resident_block(lbm, torch, graph_steps, steps=256, skip=()):
    """FP32 step kernel of each HBM-resident workload in its default shape:
    graph-replayed steps timed with HIP events on the library's stream (one
    launch per step), algorithmic 72 B per node over the launch duration;
    then plain FP64 on the 4096 x 2048 grid (one run, same steps), so the FP32
    vs FP64 comparison is made on a grid that fills the GPU."""
    from paper_1306_6445_amd import workloads as WL

    out = []
    big = None
    for name, desc in HBM_LEGS:
        if name in skip:
            continue
        runs = [WL.config3(256)] if name == "config3" else WL.config4()
        ntot = sum(r.nodes for r in runs)
        (tx, ty), fused = DEFAULT_SHAPE[name]
        k, reps, eager = graph_plan(steps, graph_steps)
        L = lbm.Lattice(runs, precision="fp32", graph_steps=k)
        L.set_tile(tx, ty)
        L.set_fused(fused)
        L.init_all()
        warm_graph(L, 0, k)
        L.init_all()
        t, _ = timed_steps(L, steps, torch)
        L.close()
        ms = 1e3 * t / steps
        ach = STEP_BYTES_ALG["fp32"] * ntot / (ms * 1e-3) / 1e9
        wset = 2 * 9 * 4 * ntot
        leg = {"workload": desc, "nodes": ntot, "mlups": ntot * steps / t / 1e6, "tile": [tx, ty],
               "fused": fused, "steps": steps, "graph_replays": reps, "eager_steps": eager,
               "kernel": "fused_kernel<float>", "kernel_ms": ms, "achieved": ach, "peak": HBM_PEAK_GBS,
               "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "working_set_bytes": wset,
               "cache_resident": False,
               "traffic": traffic_from_profile(ntot, "fused", name, "fp32")}
        if leg["traffic"]:
            leg["traffic_frac"] = leg["traffic"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS
        log("hbm-resident %s: %.1f MLUPS, %.4f ms per launch, %.3f of HBM" % (name, leg["mlups"], ms, leg["frac"]))
        out.append(leg)
        if name == "config3":
            big = runs
    if big is not None:
        k, reps, eager = graph_plan(steps, graph_steps)
        P = lbm.Lattice(big, precision="fp64", graph_steps=k)
        P.init_all()
        warm_graph(P, 0, k)
        P.init_all()
        t, _ = timed_steps(P, steps, torch)
        P.close()
        n = big[0].nodes
        ms = 1e3 * t / steps
        fp64 = {"workload": "capillary wave 4096x2048, FP64, one run", "nodes": n, "mlups": n * steps / t / 1e6,
                "steps": steps, "kernel_ms": ms,
                "achieved": STEP_BYTES_ALG["fp64"] * n / (ms * 1e-3) / 1e9}
        fp64["frac"] = fp64["achieved"] / HBM_PEAK_GBS
        fp64["fp32_over_fp64_same_grid"] = out[0]["mlups"] / fp64["mlups"]
        log("fp64 plain 4096x2048: %.1f MLUPS" % fp64["mlups"])
        return out, fp64
    return out, None


def d3q19_block(lbm, torch, steps=32, n=256):
    """The D3Q19 extension on an n^3 periodic drop (CS, T/Tc 0.7, kappa 0.5),
    FP32 and FP64.  Main figures: the default fused schedule (one launch per
    step; 64 x 8 x-y tiles marching along z through 64 planes in FP32, 128 in
    FP64, psi of each plane in LDS), MLUPS over `steps` steps between stream
    synchronisations (replayed from HIP graphs of 16 steps where `steps`
    allows, as lbm3d_step does by default, after a warm-up that captures the
    graph) and the fused kernel's mean launch duration from per-dispatch HIP
    events;
    algorithmic bytes 2 x 19 s per node (every population read and written
    once; s = 4 FP32, 8 FP64).  Beside it the two-pass schedule (psi pass 19 s
    + s per node, collide pass 2 x 19 s + s, the 18 neighbour psi values from
    cache), which gives the same bits."""
    from paper_1306_6445_amd import workloads as WL

    run = WL.config3d(n)
    out = {"workload": "D3Q19 drop %d^3 (R %g), periodic, CS EOS T/Tc=0.7, kappa 0.5, epsilon 1.93" % (n, run.R0),
           "nodes": run.nodes, "schedule": "fused: 64x8 x-y tiles, z chunks of 64 planes (FP32) / 128 (FP64)"}

    def timed(L):
        L.step(16)  # warm-up: one graph block (2 x 8 steps), so the graph is captured before the timed region
        L.synchronize()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(L.stream)
        L.step(steps)
        b.record(L.stream)
        L.synchronize()
        return a.elapsed_time(b) / 1e3

    for prec, s in (("fp32", 4), ("fp64", 8)):
        with lbm.Lattice3(run, precision=prec) as L:
            L.init_all()
            t = timed(L)
            _, fused_ms = L.time_kernels(10)
            L.set_schedule(0)
            t2 = timed(L)
            psi_ms, col_ms = L.time_kernels(10)
        step_alg = 2 * 19 * s
        leg = {"mlups": run.nodes * steps / t / 1e6, "steps": steps, "ms_per_step": 1e3 * t / steps,
               "kernel": "fused3_kernel<%s, 64, 8>" % ("float" if s == 4 else "double"), "kernel_ms": fused_ms,
               "achieved_GBs": step_alg * run.nodes / (fused_ms * 1e-3) / 1e9,
               "two_pass": {"mlups": run.nodes * steps / t2 / 1e6, "psi_ms": psi_ms, "collide_ms": col_ms,
                            "collide_GBs": (2 * 19 * s + s) * run.nodes / (col_ms * 1e-3) / 1e9,
                            "psi_GBs": (19 * s + s) * run.nodes / (psi_ms * 1e-3) / 1e9}}
        leg["frac"] = leg["achieved_GBs"] / HBM_PEAK_GBS
        leg["two_pass"]["collide_frac"] = leg["two_pass"]["collide_GBs"] / HBM_PEAK_GBS
        # counted HBM bytes per launch of the fused kernel (committed counter runs, current source only)
        leg["traffic"] = traffic_from_profile(run.nodes, "fused3", "d3q19", prec,
                                              os.path.join(ROOT, "paper_1306_6445_amd", "csrc", "lbm3d_kernels.hip"))
        if leg["traffic"]:
            leg["traffic_frac"] = leg["traffic"] / (fused_ms * 1e-3) / 1e9 / HBM_PEAK_GBS
        log("d3q19 %s: fused %.1f MLUPS (kernel %.4f ms, %.0f GB/s); two-pass %.1f MLUPS" %
            (prec, leg["mlups"], fused_ms, leg["achieved_GBs"], leg["two_pass"]["mlups"]))
        out[prec] = leg
    return out


def mc_block(lbm, torch, steps=64, n=2048):
    """The two-component extension: spinodal decomposition of a 50/50 mixture
    in a periodic n x n box (G = 1, total density 1.05, kappa 0.5), FP32 and
    FP64 in their default tiles, one fused launch per step.  MLUPS over
    `steps` steps between stream synchronisations (replayed from HIP graphs of
    16 steps, as lbm_mc_step does by default, after a warm-up that captures
    the graph); the kernel's mean launch
    duration from per-dispatch HIP events; algorithmic bytes 2 x 18 s per node
    (both components' populations read and written once; s = 4 FP32, 8 FP64)."""
    from paper_1306_6445_amd import workloads as WL

    run = WL.mc_spinodal_run(n)
    out = {"workload": "two-component spinodal decomposition %dx%d periodic, G=1, rho=1.05, kappa=0.5" % (n, n),
           "nodes": run.nodes}
    for prec, s in (("fp32", 4), ("fp64", 8)):
        with lbm.LatticeMC(run, precision=prec) as L:
            L.init_all()
            L.step(16)  # warm-up: one graph block (2 x 8 steps), captured before the timed region
            L.synchronize()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(L.stream)
            L.step(steps)
            b.record(L.stream)
            L.synchronize()
            t = a.elapsed_time(b) / 1e3
            k_ms = L.time_kernels(10)
        alg = 36 * s
        leg = {"mlups": run.nodes * steps / t / 1e6, "steps": steps, "ms_per_step": 1e3 * t / steps,
               "kernel": "mc_fused_kernel<%s>" % ("float" if s == 4 else "double"), "kernel_ms": k_ms,
               "achieved_GBs": alg * run.nodes / (k_ms * 1e-3) / 1e9}
        leg["frac"] = leg["achieved_GBs"] / HBM_PEAK_GBS
        leg["traffic"] = traffic_from_profile(run.nodes, "mcfused", "mc", prec,
                                              os.path.join(ROOT, "paper_1306_6445_amd", "csrc", "lbm_mc_kernels.hip"))
        if leg["traffic"]:
            leg["traffic_frac"] = leg["traffic"] / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS
        log("two-component %s: %.1f MLUPS (kernel %.4f ms, %.0f GB/s)" % (prec, leg["mlups"], k_ms, leg["achieved_GBs"]))
        out[prec] = leg
    return out


def traffic_from_profile(ntot, kernel, workload, precision="fp32", src=None):
    """HBM bytes per launch of the dominant kernel from committed rocprofv3
    counter runs, if they were taken on the current kernel source (src: the
    kernel's source file, the 2D kernels by default)."""
    path = TRAFFIC_FILE % (kernel, precision, workload)
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            t = json.load(fh)
        sha = hashlib.sha256(open(src or KERNEL_SRC, "rb").read()).hexdigest()
        if t.get("kernel_source_sha256") != sha or t.get("nodes") != ntot:
            return None
        return float(t["bytes_per_dispatch"])
    except Exception:
        return None


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}


def cpu_baseline(run, budget_s):
    """The FP64 oracle on the host: OpenMP over rows on all its threads (the
    reported value), then one thread (a third of the budget)."""
    import ctypes
    import oracle as O

    Pa = O.params_from_run(run)
    f0 = O.init(Pa, run.rho)

    def sample(budget):
        # a few untimed steps (the first one also starts the thread pool), then
        # chunks of steps until `budget` seconds have passed; each chunk is
        # sized from the rate measured so far (first-touch and spin-up make a
        # short first calibration pessimistic), aiming at about a quarter of
        # the remaining time
        f = O.run(Pa, f0, 2)
        n, dt, chunk = 0, 0.0, 10
        while dt < budget:
            t0 = time.perf_counter()
            f = O.run(Pa, f, chunk)
            dt += time.perf_counter() - t0
            n += chunk
            per_step = dt / n
            chunk = max(5, int(max(budget - dt, 0.0) / 4.0 / max(per_step, 1e-6)))
        return n, dt

    cores = O.threads()
    n, dt = sample(budget_s)
    out = {"value": run.nodes * n / dt / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
           "sample": "FP64 oracle, run '%s' of the workload (%dx%d), %d steps, %.1f s"
                     % (run.label, run.nx, run.ny, n, dt), "host": host_cpu()}
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
        gomp.omp_set_num_threads(1)
        if O.threads() == 1:
            n1, dt1 = sample(budget_s / 3)
            out["single_thread"] = {"value": run.nodes * n1 / dt1 / 1e6, "steps": n1, "seconds": dt1}
        gomp.omp_set_num_threads(cores)
    except OSError:
        pass
    return out


def jsonl_records(out: dict, workload: str) -> list:
    """One flat record per measured leg of a bench result (the headline, the
    HBM-resident and FP64 legs, bf16, the two-kernel schedule, the extensions,
    the accuracy check, the oracle's CPU sample): workload id, precision,
    nodes, steps, MLUPS, achieved GB/s and fraction of 8 TB/s where measured,
    plus the leg's own fields."""
    import socket

    base = {"host": socket.gethostname(), "time": time.strftime("%Y-%m-%dT%H:%M:%S"), "workload_id": workload}

    def rec(leg, fields, **kw):
        r = dict(base)
        r.update(fields)
        r.update(kw, leg=leg)
        return r

    cfg = out.get("config", {})
    roof = out.get("roofline", {})
    recs = [rec("headline", {}, workload=cfg.get("workload"), precision=cfg.get("precision"),
                nodes=cfg.get("nodes_per_step"), steps=out.get("steps"), mlups=out.get("value"),
                achieved_GBs=roof.get("achieved"), frac=roof.get("frac"), traffic=roof.get("traffic"),
                cache_resident=roof.get("cache_resident"), kernel=roof.get("kernel"),
                diverged_runs=cfg.get("diverged_runs"), tile=cfg.get("tile"), fused=cfg.get("fused"))]
    for leg in roof.get("hbm_resident", []):
        recs.append(rec("hbm_resident", leg, precision="fp32"))
    for key, prec in (("fp32_two_kernel", "fp32"), ("bf16_batched", "bf16"), ("fp64_plain", "fp64"),
                      ("fp64_batched", "fp64"), ("fp64_plain_large", "fp64")):
        if key in out:
            v = dict(out[key])
            if "value" in v:
                v["mlups"] = v.pop("value")
            recs.append(rec(key, v, precision=prec))
    for ext in ("d3q19", "mc"):
        for prec in ("fp32", "fp64"):
            if ext in out and isinstance(out[ext].get(prec), dict):
                recs.append(rec(ext, out[ext][prec], precision=prec, workload=out[ext].get("workload")))
    if "accuracy" in out:
        recs.append(rec("accuracy", out["accuracy"]))
    if "cpu_baseline" in out:
        recs.append(rec("cpu_baseline", out["cpu_baseline"], precision="fp64"))
    return recs


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--accuracy-steps", type=int, default=-1,
                    help="steps of the accuracy check (0 = skip; default 20000 for the droplet sweep, "
                         "50000 for each of the capillary waves at lambda 256, 512 and 1024, 10000 for the ensemble, "
                         "20000 for the splash)")
    ap.add_argument("--dump-ensemble", type=str, default="",
                    help="ensemble workload: write per-run inputs and diagnostics (npz) to this path")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the oracle sample (0 = skip)")
    ap.add_argument("--workload", choices=("config2", "config3", "config4", "config5", "d3q19", "mc"), default="config2",
                    help="config2: 40 x 256^2 droplet sweep (default); config3: 4096x2048 capillary wave; "
                         "config4: 512-droplet ensemble; config5: 2048x1024 droplet splash; d3q19: only the 3D "
                         "extension leg (256^3 drop; profiling runs); mc: only the two-component leg (2048^2 "
                         "mixture; profiling runs)")
    ap.add_argument("--tile", type=str, default="default",
                    help="'default' (the workload's shape below), 'auto' (autotune during warm-up) or e.g. 64x4")
    ap.add_argument("--fused", type=int, default=2,
                    help="schedule when --tile is given: nodes per thread of the fused kernel (1, 2, 4), "
                         "0 = two kernels per step")
    ap.add_argument("--graph-steps", type=int, default=16)
    ap.add_argument("--timing-steps", type=int, default=200, help="steps timed per kernel with HIP events")
    ap.add_argument("--quick", action="store_true", help="profiling run: no accuracy / CPU / FP64 legs")
    ap.add_argument("--precision", choices=("fp32", "fp64", "bf16"), default="fp32",
                    help="storage precision of the main timed leg (fp32: the benchmark; the others for "
                         "profiling, with --tile)")
    ap.add_argument("--splash-params", type=str, default="",
                    help="splash workload: 'T/Tc,kappa,epsilon' instead of the surrogate's selection "
                         "(profiling runs; the selection trains the network first)")
    ap.add_argument("--no-hbm-legs", dest="hbm_legs", action="store_false",
                    help="skip the HBM-resident roofline legs (capillary grid, ensemble) and plain FP64 on "
                         "the 4096x2048 grid")
    ap.add_argument("--no-d3q19", dest="d3q19", action="store_false",
                    help="skip the extension legs (D3Q19 256^3 drop and two-component 2048^2 mixture, FP32 and FP64)")
    ap.add_argument("--no-surrogate", dest="surrogate", action="store_false",
                    help="ensemble workload: skip the surrogate training and selection leg")
    ap.add_argument("--jsonl", type=str, default="",
                    help="also append one JSON record per measured leg to this file (run log)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (requested %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    ensure_built()
    import torch
    from paper_1306_6445_amd import lbm, workloads as WL

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.workload == "mc":
        d = mc_block(lbm, torch, steps=args.steps)
        print(json.dumps({"metric": "two-component extension MLUPS (not the headline metric)",
                          "value": d["fp32"]["mlups"], "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
                          "warmup": 16, "ms_per_step": d["fp32"]["ms_per_step"], "higher_is_better": True,
                          "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                          "config": {"workload": d["workload"]}, "mc": d}), flush=True)
        return
    if args.workload == "d3q19":
        d = d3q19_block(lbm, torch, steps=args.steps)
        print(json.dumps({"metric": "D3Q19 extension MLUPS (not the headline metric)", "value": d["fp32"]["mlups"],
                          "unit": "MLUPS", "n_gpus": 1, "steps": args.steps, "warmup": 16,
                          "ms_per_step": d["fp32"]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
                          "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                          "config": {"workload": d["workload"]}, "d3q19": d}), flush=True)
        return
    if args.workload == "config2":
        runs = WL.config2()
        wl_name = ("Laplace-law/kappa sweep: 40 periodic 256x256 droplets (R 20..60 x kappa 0..0.99), "
                   "CS EOS T/Tc=0.7, batched FP32")
    elif args.workload == "config3":
        runs = [WL.config3(256)]
        wl_name = "capillary wave 4096x2048 (lambda 256), periodic x, bounce-back y, CS EOS T/Tc=0.6, FP32"
    elif args.workload == "config4":
        runs = WL.config4()
        wl_name = "ensemble of 512 periodic droplets, L ~ U{64..512}, drawn (T/Tc, kappa, epsilon), FP32"
    else:
        log("splash: surrogate selection of (T/Tc, kappa)")
        if args.splash_params:
            t, k, e = (float(v) for v in args.splash_params.split(","))
            selection = {"given": True, "T_over_Tc": t, "kappa": k, "epsilon": e}
        else:
            selection = splash_selection(lbm)
        log("selected", selection)
        runs = [WL.config5(selection["T_over_Tc"], selection["kappa"], selection["epsilon"])]
        wl_name = ("droplet splash 2048x1024, film 0.1H, R=100, U=0.05, Re=1000, nu_V/nu_L=20, CS EOS at "
                   "%s (T/Tc, kappa, epsilon), FP32" % ("given" if args.splash_params else "surrogate-selected"))
    if args.accuracy_steps < 0:
        args.accuracy_steps = {"config2": 20000, "config3": 50000, "config4": 10000, "config5": 20000}[args.workload]
    ntot = sum(r.nodes for r in runs)

    # ---- FP32 batched: the headline number
    log("%s batched: %d runs, %d nodes" % (args.precision, len(runs), ntot))
    prec = args.precision
    wbytes = WRITER_BYTES if prec == "bf16" else 0
    if prec != "fp32":
        wl_name = wl_name.replace("FP32", {"fp64": "FP64", "bf16": "bf16 storage"}[prec])
    gk, g_replays, g_eager = graph_plan(args.steps, args.graph_steps)
    L = lbm.Lattice(runs, precision=prec, graph_steps=gk)
    L.init_all()
    if args.tile == "auto":
        choice = L.autotune(64)
        tx, ty = choice["tile"]
        fused = choice["fused"]
        log("autotune:", choice)
    else:
        if args.tile == "default":
            (tx, ty), fused = DEFAULT_SHAPE[args.workload]
        else:
            tx, ty = (int(v) for v in args.tile.split("x"))
            fused = args.fused
        L.set_tile(tx, ty)
        L.set_fused(fused)
    L.init_all()
    warm_run = warm_graph(L, args.warmup, gk)
    if warm_run:
        L.init_all()  # timed region starts from the initial state again
    t_gpu, t_wall = timed_steps(L, args.steps, torch)
    mlups = ntot * args.steps / t_gpu / 1e6
    log("%s batched: %.1f MLUPS (%.3f ms/step)" % (prec, mlups, 1e3 * t_gpu / args.steps))
    # spread: five more timed regions of a fifth of the steps each (the state
    # runs on; `value` stays the single region of exactly K steps above)
    rep_k = max(2 * gk if gk else 2, (args.steps // 5) // max(2 * gk, 2) * max(2 * gk, 2))
    reps = sorted(ntot * rep_k / timed_steps(L, rep_k, torch)[0] / 1e6 for _ in range(5))
    repeats = {"n": 5, "steps": rep_k, "median": reps[2], "min": reps[0], "max": reps[4]}
    # dominant kernel: the timed region per launch (fused), or per-dispatch HIP
    # events on the same stream and workload (two kernels; also reported beside)
    psi_ms, ev_ms = L.time_kernels(args.timing_steps)
    col_ms = launch_ms(fused, t_gpu, args.steps, ev_ms)
    st = L.status()
    two = None
    if fused:
        # the in-place two-kernel schedule (psi pass + collide-stream) on the
        # same workload and tiles, for comparison
        L.set_fused(0)
        k2 = min(args.steps, 5000)
        t2 = graph_timed(L, k2, args.warmup, args.graph_steps, torch)
        p2, c2 = L.time_kernels(min(args.timing_steps, 100))
        two = {"value": ntot * k2 / t2 / 1e6, "unit": "MLUPS", "steps": k2, "tile": [tx, ty],
               "psi_ms": p2, "collide_ms": c2,
               "collide_GBs": (COLLIDE_BYTES[prec] + wbytes) * ntot / (c2 * 1e-3) / 1e9,
               "psi_GBs": (9 * STORE_BYTES[prec] + STORE_BYTES[prec if prec == "fp64" else "fp32"]) * ntot
               / (p2 * 1e-3) / 1e9,
               "step_alg_frac": ntot * k2 / t2 * (STEP_BYTES_ALG[prec] + wbytes) / 1e9 / HBM_PEAK_GBS}
    L.close()
    # algorithmic bytes of the dominant kernel: collide reads and writes every
    # population and reads psi once; the fused kernel is the whole step (72 B)
    kbytes = (STEP_BYTES_ALG if fused else COLLIDE_BYTES)[prec] + wbytes
    achieved = kbytes * ntot / (col_ms * 1e-3) / 1e9
    kname = ("fused_kernel<%s>" if fused else "collide_kernel<%s>") % KERNEL_TYPE[prec]
    roof = {"bound": "hbm", "kernel": kname, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic_from_profile(ntot, "fused" if fused else "collide", args.workload, prec),
            "kernel_ms": col_ms, "kernel_ms_source": "timed region / launches" if fused else "per-dispatch events",
            "kernel_ms_dispatch_events": ev_ms, "psi_ms": psi_ms,
            "psi_achieved_GBs": (9 * STORE_BYTES[prec] + STORE_BYTES[prec if prec == "fp64" else "fp32"]) * ntot
            / (psi_ms * 1e-3) / 1e9 if psi_ms > 0 else None,
            "step_alg_frac": mlups * 1e6 * (STEP_BYTES_ALG[prec] + wbytes) / 1e9 / HBM_PEAK_GBS,
            # the two population buffers the step streams through
            "working_set_bytes": 2 * 9 * STORE_BYTES[prec] * ntot,
            "cache_resident": 2 * 9 * STORE_BYTES[prec] * ntot <= 256 * 2 ** 20}
    log("%s %.4f ms per launch -> %.0f GB/s (per-dispatch events %.4f ms); psi %.4f ms"
        % (kname, col_ms, achieved, ev_ms, psi_ms))
    # reference: the library's plain copy kernel over the same bytes as one collide launch
    nbytes = (kbytes * ntot // 2) & ~15
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    copy_ms = lbm.stream_copy_ms(dst.data_ptr(), src.data_ptr(), nbytes, 50)
    big = 1 << 31
    src2 = torch.empty(big, dtype=torch.uint8, device="cuda")
    dst2 = torch.empty_like(src2)
    copy_big_ms = lbm.stream_copy_ms(dst2.data_ptr(), src2.data_ptr(), big, 10)
    del src, dst, src2, dst2
    roof["copy_same_bytes_GBs"] = 2 * nbytes / (copy_ms * 1e-3) / 1e9
    roof["copy_2GiB_GBs"] = 2 * big / (copy_big_ms * 1e-3) / 1e9

    out = {"metric": METRIC, "value": mlups, "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * t_gpu / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64" if prec == "fp64" else "f32",
           "data": "synthetic",
           "config": {"workload": wl_name, "runs": len(runs), "nodes_per_step": ntot, "precision": prec,
                      "tile": [tx, ty], "fused": fused, "graph_steps": gk, "graph_replays": g_replays,
                      "eager_steps": g_eager, "warmup_steps_run": warm_run,
                      "wall_s_timed": t_wall, "diverged_runs": int(st.sum())},
           "roofline": roof, "repeats": repeats}
    if roof["traffic"]:
        # the same kernel's HBM traffic from the counters, over its duration
        roof["traffic_GBs"] = roof["traffic"] / (col_ms * 1e-3) / 1e9
        roof["traffic_frac"] = roof["traffic_GBs"] / HBM_PEAK_GBS
    if two:
        out["fp32_two_kernel"] = two
    if args.workload == "config5":
        out["surrogate_selection"] = selection
    if args.hbm_legs and prec == "fp32":
        legs, fp64_big = hbm_resident_block(lbm, torch, args.graph_steps,
                                            skip=(args.workload,) if not roof["cache_resident"] else ())
        if not roof["cache_resident"]:
            # the main workload is itself HBM-resident: its leg is the headline
            legs.insert(0, {"workload": wl_name, "nodes": ntot, "mlups": mlups, "kernel_ms": col_ms,
                            "achieved": achieved, "frac": achieved / HBM_PEAK_GBS, "cache_resident": False,
                            "same_as_headline": True})
        roof["hbm_resident"] = legs
        if fp64_big:
            out["fp64_plain_large"] = fp64_big

    if not args.quick:
        # ---- bf16 deviation storage, same workload
        log("bf16 batched")
        Bf = lbm.Lattice(runs, precision="bf16", graph_steps=args.graph_steps)
        Bf.init_all()
        bfch = Bf.autotune(32)
        kbf = min(args.steps, 10000)
        tbf = graph_timed(Bf, kbf, args.warmup, args.graph_steps, torch)
        p_ms, c_ms = Bf.time_kernels(100)
        c_ms = launch_ms(bfch["fused"], tbf, kbf, c_ms)
        Bf.close()
        bbytes = (STEP_BYTES_ALG if bfch["fused"] else COLLIDE_BYTES)["bf16"] + WRITER_BYTES
        out["bf16_batched"] = {"value": ntot * kbf / tbf / 1e6, "unit": "MLUPS", "steps": kbf, "schedule": bfch,
                               "step_kernel_GBs": bbytes * ntot / (c_ms * 1e-3) / 1e9, "kernel_ms": c_ms,
                               "psi_ms": p_ms}
        # ---- plain FP64: one run per context
        if args.workload != "config4":
            log("fp64 plain")
            P = lbm.Lattice([runs[0]], precision="fp64", graph_steps=args.graph_steps)
            P.init_all()
            pch = P.autotune(32)
            k64 = min(args.steps, 5000)
            t64 = graph_timed(P, k64, args.warmup, args.graph_steps, torch)
            p_ms, c_ms = P.time_kernels(100)
            c_ms = launch_ms(pch["fused"], t64, k64, c_ms)
            P.close()
            out["fp64_plain"] = {"value": runs[0].nodes * k64 / t64 / 1e6, "unit": "MLUPS", "steps": k64,
                                 "config": "one %dx%d run per context" % (runs[0].nx, runs[0].ny),
                                 "schedule": pch,
                                 "step_kernel_GBs": (STEP_BYTES_ALG if pch["fused"] else COLLIDE_BYTES)["fp64"]
                                 * runs[0].nodes / (c_ms * 1e-3) / 1e9}
            out["fp32_batched_over_fp64_plain"] = mlups / out["fp64_plain"]["value"]
        # ---- FP64 batched
        if len(runs) > 1:
            log("fp64 batched")
            B = lbm.Lattice(runs, precision="fp64", graph_steps=args.graph_steps)
            B.init_all()
            bch = B.autotune(32)
            kb = min(args.steps, 5000)
            tb = graph_timed(B, kb, args.warmup, args.graph_steps, torch)
            p_ms, c_ms = B.time_kernels(100)
            c_ms = launch_ms(bch["fused"], tb, kb, c_ms)
            B.close()
            out["fp64_batched"] = {"value": ntot * kb / tb / 1e6, "unit": "MLUPS", "steps": kb,
                                   "schedule": bch,
                                   "step_kernel_GBs": (STEP_BYTES_ALG if bch["fused"] else COLLIDE_BYTES)["fp64"]
                                   * ntot / (c_ms * 1e-3) / 1e9}
        if args.accuracy_steps:
            log("accuracy: %d steps" % args.accuracy_steps)
            if args.workload == "config2":
                out["accuracy"] = accuracy_block(runs, args.accuracy_steps, lbm)
            elif args.workload == "config3":
                out["accuracy"] = capillary_block(args.accuracy_steps, lbm)
            elif args.workload == "config5":
                out["accuracy"] = splash_block(runs[0], args.accuracy_steps, lbm)
            else:
                out["accuracy"] = ensemble_block(runs, args.accuracy_steps, lbm, args.graph_steps,
                                                 args.dump_ensemble or None)
        if args.d3q19:
            log("d3q19")
            out["d3q19"] = d3q19_block(lbm, torch)
            log("two-component")
            out["mc"] = mc_block(lbm, torch)
        if args.workload == "config4" and args.surrogate:
            log("surrogate")
            out["surrogate"] = surrogate_block(lbm, torch)
        if args.cpu_seconds > 0:
            log("cpu baseline")
            out["cpu_baseline"] = cpu_baseline(runs[0], args.cpu_seconds)
    if args.jsonl:
        with open(args.jsonl, "a") as fh:
            for rec in jsonl_records(out, args.workload):
                fh.write(json.dumps(rec, default=float) + "\n")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
