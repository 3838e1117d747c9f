#!/usr/bin/env python3
"""Benchmark of the SEM Schwarz / p-multigrid solver on one MI355X.

A step is one complete solve with the multigrid-preconditioned CG (Algorithm 4,
one V-cycle of Algorithm 3 per iteration) from the seeded initial guess to a
residual reduction of 1e-10: it runs every part of the hot path (residual,
Schwarz smoother, restriction, prolongation, coarse solve, V-cycle, CG).

Default workload: Poisson on [0,1]^2, 128x128 elements, p = 16 (4.19M
unknowns), FP64, the paper's weights (quintic) and overlaps ceil(p_l/8),
MGCG(1,0) -- the largest configuration that the method runs at the paper's
precision.

Printed JSON line (one):
  value        DOF/s per V-cycle over the timed solves: finest-level unknowns
               times V-cycles done, divided by the wall time of the solves
  ms_per_step  time to 1e-10 of one solve
  roofline     the finest level's dominant kernel (largest summed time over
               the timed solves); durations come from HIP events that the
               kernel dispatch records at the kernels' start and end
  kernels      the same figures for every timed kernel kind of that level
  comparisons  the metric's "mixed/learned vs plain FP64": time to 1e-10,
               iterations and the true FP64 residual of the plain FP64 solve
               and of the mixed-precision / learned-parameter solves, on the
               128x128 p = 16 Poisson workload and on the 48x48 p = 32
               variable-diffusion workload
  cpu_baseline the CPU oracle: one full MGCG solve of the same workload

Usage: python bench.py [--steps K] [--warmup W] [--workload c3]
                       [--precision fp64|mixed|bf16|fp16] [--weights paper|learned]
                       [--no-compare] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP64_PEAK_TFS = 78.6         # MI355X FP64 vector
FP32_PEAK_TFS = 157.3        # MI355X FP32 vector
BF16_PEAK_TFS = 2500.0       # MI355X dense BF16 / FP16 matrix cores
RIDGE = {"f64": FP64_PEAK_TFS * 1e3 / HBM_PEAK_GBS, "f32": FP32_PEAK_TFS * 1e3 / HBM_PEAK_GBS,
         "mfma": BF16_PEAK_TFS * 1e3 / HBM_PEAK_GBS}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = ("fdm_impl.h", "fdm_mfma.hip", "residual_impl.h", "transfer_impl.h", "kernels.h",
                  "common.h")


def _code_only(text: str) -> str:
    """Source text without comments and blank space (string literals in these
    files hold no comment markers)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash(texts=None) -> str:
    """Hash of the level kernels' code (comments and layout ignored): recorded
    HBM traffic is reported only while it matches."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        if texts is None:
            with open(os.path.join(ROOT, "paper_1512_02390_amd", "csrc", f)) as fh:
                t = fh.read()
        else:
            t = texts[f]
        h.update(_code_only(t).encode())
    return h.hexdigest()[:16]


RULES = {"fixed": 0, "ceil8": 1, "floor8": 2, "ceil2": 3}
PRECISIONS = ("fp64", "mixed", "bf16", "fp16")


def progress(msg: str):
    """One progress line on stderr (stdout carries only the result line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_problem(name: str, precision: str = "fp64", n_o: int = 1, rule=None, overlaps=None,
                 net=None, learned_mode: str = "level", ell=None, local: str = "mean",
                 wf: int = 5):
    """Solver, right-hand side, nodal source, initial guess and nu of a
    workload; with a trained network `net` the Schwarz parameters are the
    learned ones (the paper's when the prediction is unusable).  ell: the
    random field's correlation length instead of the workload's; local:
    "mean" (the paper's local solves) or "separable" (separable local
    coefficients); wf: the weight function (-3: multiplicative Schwarz)."""
    import torch
    from paper_1512_02390_amd import sem as S
    from paper_1512_02390_amd import workloads as W

    prec = {"fp64": S.FP64, "mixed": S.MIXED_FP32, "bf16": S.MIXED_BF16,
            "fp16": S.MIXED_FP16}[precision]
    cfg = W.config(name, n_o)
    if rule is not None:
        cfg.overlap_rule = RULES[rule]
    if overlaps is not None:
        cfg.overlaps = overlaps
    NU = None
    if cfg.variable_nu:
        nu = W.GaussianFieldNu() if ell is None else W.GaussianFieldNu(ell=ell)
        probe = S.Solver(cfg.xb, cfg.yb, cfg.p, cfg.bc, cfg.overlap_rule, cfg.n_o, 5)
        xc, yc = probe.node_coords()
        probe.close()
        NU = W.nodal(nu.nu, xc, yc)
    learned_params = None
    if net is not None:
        from paper_1512_02390_amd import learned as LW
        s, learned_params = LW.solver_with_learned(cfg.xb, cfg.yb, cfg.p, cfg.bc, NU, net, prec,
                                                   learned_mode)
    else:
        s = S.Solver(cfg.xb, cfg.yb, cfg.p, cfg.bc, cfg.overlap_rule, cfg.n_o, wf, nu=NU,
                     precision=prec, overlaps=cfg.overlaps,
                     local_solve=S.LOCAL_SEPARABLE if local == "separable" else S.LOCAL_MEAN)
    s.learned_params = learned_params
    shape = s.shape()
    if name == "c1":
        xc, yc = s.node_coords()
        fn = W.nodal(lambda x, y: -W.SineSolution().laplacian(x, y), xc, yc)
    else:
        fn = W.random_nodal(shape, cfg.bc, W.SEED_RHS)
    b = s.zeros()
    s.mass(torch.tensor(fn, dtype=torch.float64, device="cuda"), b)
    u0 = torch.tensor(W.random_guess(shape, cfg.bc, W.SEED_U0), dtype=torch.float64,
                      device="cuda")
    return cfg, s, b, u0, fn, NU


def schedule(cfg, L: int, cycle=None):
    cycle = cycle or ("mg11" if cfg.variable_nu else "mg10")
    if cycle == "mg10":
        return cycle, [1] * (L + 1), [0] * (L + 1)
    if cycle == "mg11":
        return cycle, [1] * (L + 1), [1] * (L + 1)
    s = [2 ** (L - l) for l in range(L + 1)]
    return cycle, s, list(s)


def n_unknowns(cfg) -> int:
    if cfg.bc == 0:
        return (cfg.nx * cfg.p - 1) * (cfg.ny * cfg.p - 1)
    return cfg.nx * cfg.ny * cfg.p ** 2


def timed_solves(s, b, u0, steps: int, warmup: int, ns1, ns2, imax: int, time_level=None):
    """Warm-up solves, then `steps` timed solves (one private copy of the
    initial guess each, made before the timed region).  Returns the wall time
    per solve, iterations, residual history, convergence, the last iterate and,
    with time_level, the kernel timing record of that level."""
    import torch
    for _ in range(max(warmup, 1)):
        u = u0.clone()
        it, hist, ok = s.pcg_solve(u, b, imax, 1e-10, ns1, ns2)
    us = [u0.clone() for _ in range(steps)]
    if time_level is not None:
        s.timing_enable(time_level, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cycles = 0
    for k in range(steps):
        it_k, _, _ = s.pcg_solve(us[k], b, imax, 1e-10, ns1, ns2)
        cycles += it_k
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rec = None
    if time_level is not None:
        rec = s.timing_read_all()
        s.timing_enable(time_level, False)
    return {"s_per_solve": dt / steps, "cycles": cycles, "iterations": it, "hist": hist,
            "converged": bool(ok), "u": us[-1], "timing": rec}


def true_residual_ratio(s, u, b, u0) -> float:
    """||b - A u||_2 / ||b - A u0||_2 recomputed in FP64 by the library."""
    r = s.zeros()
    s.residual(s.L, u0, b, r)
    r0 = s.norm(r)
    s.residual(s.L, u, b, r)
    return s.norm(r) / r0


def level_work(s, cfg, kind: str, word: int):
    """Algorithmic flops and HBM bytes of one launch of a finest-level kernel.
    Schwarz step: per element 8 m^3 + 3 m^2 flops (four m x m x m contractions,
    eigenvalue scaling, weighting); read r, read and write u.  Residual: per
    element 4 n^3 + 4 n^2 flops (n = p + 1, two sum-factorised directions);
    read u and f, write r (the operator product q = A p reads p, writes q).
    Restriction / prolongation: per element 2 n n_c (n + n_c) flops (n_c the
    coarse n); read the fine array (and the coarse one for the prolongation),
    write the other."""
    pl, no, rows, cols = s.level_info(s.L)
    _, _, rc, cc = s.level_info(s.L - 1)
    n_el = cfg.nx * cfg.ny
    nodes, cnodes = rows * cols, rc * cc
    n, nc = pl + 1, s.level_info(s.L - 1)[0] + 1
    m = pl + 1 + 2 * no
    if kind == "schwarz":
        return n_el * (8.0 * m ** 3 + 3.0 * m ** 2), 3.0 * nodes * word
    if kind == "residual":
        f = n_el * (4.0 * n ** 3 + 4.0 * n ** 2) * (2.0 if cfg.variable_nu else 1.0)
        return f, (3.0 + (1.0 if cfg.variable_nu else 0.0)) * nodes * word
    if kind == "apply":
        f = n_el * (4.0 * n ** 3 + 4.0 * n ** 2) * (2.0 if cfg.variable_nu else 1.0)
        return f, (2.0 + (1.0 if cfg.variable_nu else 0.0)) * nodes * word
    if kind == "restrict":
        return n_el * 2.0 * n * nc * (n + nc), (nodes + cnodes) * word
    if kind == "prolong":
        return n_el * 2.0 * n * nc * (n + nc), (2.0 * nodes + cnodes) * word
    raise ValueError(kind)


def kernel_table(s, cfg, precision: str, rec: dict):
    """Per timed kernel kind: launches, average duration, algorithmic work,
    achieved rate and the fraction of the binding roof."""
    from paper_1512_02390_amd.sem import MIXED_BF16, MIXED_FP16
    word = 8 if precision == "fp64" else 4
    pl, no, _, _ = s.level_info(s.L)
    m = pl + 1 + 2 * no
    out = {}
    for kind, (cnt, ms) in rec.items():
        if cnt == 0:
            continue
        flops, nbytes = level_work(s, cfg, kind, word)
        avg = ms / cnt
        ai = flops / nbytes
        mfma = kind == "schwarz" and precision in ("bf16", "fp16") and m >= 17
        ridge = RIDGE["mfma"] if mfma else RIDGE["f64" if word == 8 else "f32"]
        if ai < ridge:
            bound, ach, peak, unit = "hbm", nbytes / (avg * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s"
        elif mfma:
            bound, ach, peak, unit = "mfma", flops / (avg * 1e-3) / 1e12, BF16_PEAK_TFS, "TFLOP/s"
        else:
            peak = FP64_PEAK_TFS if word == 8 else FP32_PEAK_TFS
            bound, ach, unit = "alu", flops / (avg * 1e-3) / 1e12, "TFLOP/s"
        out[kind] = {"bound": bound, "achieved": ach, "peak": peak, "unit": unit,
                     "frac": ach / peak, "launches": cnt, "avg_launch_ms": avg,
                     "total_ms": ms, "algorithmic_flops": flops, "algorithmic_bytes": nbytes,
                     "achieved_gbs": nbytes / (avg * 1e-3) / 1e9,
                     "achieved_tflops": flops / (avg * 1e-3) / 1e12}
    return out


KERNEL_NAMES = {  # rocprofv3 names of the finest-level kernels, for the traffic record
    "schwarz": "k_fdm", "residual": "k_residual", "apply": "k_residual",
    "restrict": "k_restrict", "prolong": "k_prolong"}


def recorded_traffic(key: str):
    """HBM bytes per launch measured with rocprofv3 counters, if the record
    matches the current kernel sources."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("per_launch", {}).get(key)


def cpu_baseline(cfg, fn, NU, ns1, ns2, budget_s: float = 15.0):
    """Oracle MGCG solves of the same workload (at least one full solve, more
    while the budget lasts); DOF/s per V-cycle like the GPU value."""
    from oracle.mgcg import mgcg
    from oracle.multigrid import Multigrid
    from paper_1512_02390_amd import workloads as W
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    mg = Multigrid(cfg.xb, cfg.yb, cfg.p, cfg.bc, cfg.overlap_rule, cfg.n_o, 5, NU=NU,
                   overlaps=cfg.overlaps)
    sp = mg.spaces[-1]
    F = sp.mass(fn)
    U0 = W.random_guess(sp.shape, cfg.bc, W.SEED_U0)
    n = int(sp.mask.sum())
    t0 = time.perf_counter()
    solves, cycles, its = 0, 0, 0
    while True:
        _, hist, it = mgcg(mg, U0, F, 200, 1e-10, ns1, ns2)
        solves += 1
        cycles += it
        its = it
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": n * cycles / dt, "unit": "DOF/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{solves} full MGCG solve(s) to 1e-10 of the same workload "
                      f"({its} iterations each) in {dt:.1f} s: "
                      f"{1e3 * dt / solves:.0f} ms per solve"}


def compare_run(name: str, precision: str, net, steps: int, warmup: int, imax: int,
                plain_ms=None, learned_mode: str = "level", ell=None, local: str = "mean",
                wf: int = 5):
    """One comparison entry: time to 1e-10, iterations and the true FP64
    residual of a solve configuration (or the breakdown, when the iteration
    meets a non-finite residual)."""
    from paper_1512_02390_amd.sem import SemError
    progress(f"comparison {name} {precision} {'learned ' + learned_mode if net is not None else 'paper'}"
             f" local={local} wf={wf}" + (f" length={ell}" if ell is not None else ""))
    t0 = time.perf_counter()
    cfg, s, b, u0, _, _ = make_problem(name, precision, net=net, learned_mode=learned_mode,
                                       ell=ell, local=local, wf=wf)
    setup_s = time.perf_counter() - t0
    cycle, ns1, ns2 = schedule(cfg, s.L)
    entry = {"workload": cfg.description, "precision": precision,
             "weights": "learned" if net is not None else "paper", "solver": f"MGCG {cycle}",
             "smoother": "multiplicative" if wf == -3 else f"additive w_{wf}",
             "local_solve": local, "setup_s": setup_s,
             "overlap": [s.level_info(l)[1] for l in range(1, s.L + 1)]}
    if ell is not None:
        entry["correlation_length"] = ell
    try:
        res = timed_solves(s, b, u0, steps, warmup, ns1, ns2, imax)
    except SemError as e:
        if e.status != -6:
            raise
        entry.update({"time_to_1e-10_ms": None, "converged": False,
                      "breakdown": "non-finite residual"})
        s.close()
        return entry
    entry.update({"time_to_1e-10_ms": 1e3 * res["s_per_solve"] if res["converged"] else None,
                  "iterations": res["iterations"], "converged": res["converged"],
                  "true_residual_ratio": true_residual_ratio(s, res["u"], b, u0)})
    if net is not None:
        entry["learned_mode"] = learned_mode
        entry["learned_fallback_to_paper"] = s.learned_params is None
        if s.learned_params is not None:
            ep = s.learned_params
            entry["learned_alpha_range"] = [float(ep[:, 0].min()), float(ep[:, 0].max())]
            entry["learned_rho_range"] = [float(ep[:, 1].min()), float(ep[:, 1].max())]
    if plain_ms is not None and entry["time_to_1e-10_ms"]:
        entry["speedup_vs_plain_fp64"] = plain_ms / entry["time_to_1e-10_ms"]
    s.close()
    return entry


def compare_3d(n: int, p: int, n_o: int, steps: int, warmup: int, imax: int):
    """3-D Poisson on the unit cube with n^3 elements of order p (the 3-D
    extension, sem3_*): time to 1e-10 of MGCG(1,0), iterations, the true
    residual and DOF/s per V-cycle."""
    import torch
    from paper_1512_02390_amd import workloads as W
    from paper_1512_02390_amd.sem import Solver3
    progress(f"comparison 3-D {n}^3 elements p={p} n_o={n_o}")
    b = W.uniform_breaks(n, 1.0)
    t0 = time.perf_counter()
    s = Solver3(b, b, b, p, 0, n_o, 5)
    setup_s = time.perf_counter() - t0
    shape = s.level_info(s.L)[2]
    g = W.rng(W.SEED_RHS)
    f = g.uniform(-1.0, 1.0, size=shape)
    f[[0, -1], :, :] = 0.0
    f[:, [0, -1], :] = 0.0
    f[:, :, [0, -1]] = 0.0
    fb = torch.tensor(f, dtype=torch.float64, device="cuda")
    u0 = torch.zeros(shape, dtype=torch.float64, device="cuda")
    for _ in range(max(warmup, 1)):
        s.pcg_solve(u0.clone(), fb, imax, 1e-10)
    us = [u0.clone() for _ in range(steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    cycles = 0
    for k in range(steps):
        it, hist, ok = s.pcg_solve(us[k], fb, imax, 1e-10)
        cycles += it
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t1) / steps
    r = s.zeros()
    s.residual(s.L, us[-1], fb, r)
    true_ratio = float(torch.linalg.norm(r)) / float(hist[0])
    dof = int(np.prod([x - 2 for x in shape]))
    s.close()
    return {"workload": f"3-D Poisson [0,1]^3, {n}^3 elements, p={p}, Dirichlet, n_o={n_o}",
            "precision": "fp64", "solver": "MGCG mg10, w_5", "dof": dof, "setup_s": setup_s,
            "time_to_1e-10_ms": 1e3 * dt if ok else None, "iterations": it, "converged": bool(ok),
            "true_residual_ratio": true_ratio, "dof_per_s_per_vcycle": dof * cycles / (dt * steps)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--n-o", type=int, default=1)
    ap.add_argument("--rule", default=None, choices=sorted(RULES),
                    help="overlap rule per level (default: the workload's)")
    ap.add_argument("--overlaps", default=None,
                    help="explicit overlaps of levels 1..L, comma separated")
    ap.add_argument("--precision", default="fp64", choices=PRECISIONS,
                    help="fp64; mixed: FP32 V-cycle in FP64 MGCG; bf16 / fp16: as mixed with "
                         "the subdomain solves of wide tiles on BF16 / FP16 matrix cores")
    ap.add_argument("--imax", type=int, default=200)
    ap.add_argument("--cycle", default=None, choices=["mg10", "mg11", "var11"],
                    help="smoothing schedule (default: mg10; mg11 for variable nu)")
    ap.add_argument("--weights", default="paper", choices=["paper", "learned"],
                    help="Schwarz parameters: the paper's, or predicted by a network trained "
                         "on the solver's own sweeps before the timed region")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the mixed / learned vs plain FP64 comparison runs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-3d", action="store_true",
                    help="only run the 3-D comparison (16^3 elements, p=8) and print its entry")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (the reference "
                         "kernel for scaling HBM counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 4 * n, "copies": 5}), flush=True)
        return
    if args.only_3d:
        print(json.dumps(compare_3d(16, 8, 1, args.steps, args.warmup, args.imax)), flush=True)
        return

    from paper_1512_02390_amd import metrics as MT
    ovl = None
    if args.overlaps:
        ovl = [0] + [int(v) for v in args.overlaps.split(",")]
    net, learned_info = None, None

    def train():
        from paper_1512_02390_amd import learned as LW
        t0 = time.perf_counter()
        X, T, recs = LW.make_dataset(LW.default_patches())
        trained, lh = LW.train(X, T)
        info = {"patches": len(recs), "samples": int(X.shape[0]),
                "candidates_per_patch": len(recs[0][1]), "train_loss": [lh[0], lh[-1]],
                "sweep_and_training_s": time.perf_counter() - t0}
        return trained, info

    if args.weights == "learned":
        net, learned_info = train()
    progress(f"workload {args.workload} {args.precision}: set-up")
    cfg, s, b, u0, fn, NU = make_problem(args.workload, args.precision, args.n_o, args.rule, ovl,
                                         net)
    progress("timed solves")
    cycle, ns1, ns2 = schedule(cfg, s.L, args.cycle)
    n_dof = n_unknowns(cfg)

    # the value: timed solves without per-launch events
    res = timed_solves(s, b, u0, args.steps, args.warmup, ns1, ns2, args.imax)
    if not res["converged"]:
        raise SystemExit(f"MGCG did not reach 1e-10 in {args.imax} iterations")
    # kernel durations: a second timed pass of the same solves, every finest-
    # level launch bracketed by dispatch events (they slow the solve itself)
    progress("timed solves with dispatch events")
    res_k = timed_solves(s, b, u0, args.steps, 0, ns1, ns2, args.imax, time_level=s.L)
    dt = res["s_per_solve"] * args.steps
    r_bar = MT.rbar(res["hist"])
    ov_levels = [0] + [s.level_info(l)[1] for l in range(1, s.L + 1)]
    w_iter = MT.cycle_cost(cfg.p, ov_levels, [a + c for a, c in zip(ns1, ns2)])
    true_res = true_residual_ratio(s, res["u"], b, u0)

    # bare V-cycle throughput on the iterate, for reference
    uv = u0.clone()
    for _ in range(3):
        s.vcycle(uv, b, ns1, ns2)
    torch.cuda.synchronize()
    nv = 50
    tv0 = time.perf_counter()
    for _ in range(nv):
        s.vcycle(uv, b, ns1, ns2)
    torch.cuda.synchronize()
    tv = (time.perf_counter() - tv0) / nv

    kernels = kernel_table(s, cfg, args.precision, res_k["timing"])
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    roof = {k: kernels[dom][k] for k in ("bound", "achieved", "peak", "unit", "frac")}
    pl, no, _, _ = s.level_info(s.L)
    key = f"{args.workload}_{args.precision}_{dom}"
    roof["traffic"] = recorded_traffic(key)
    roof.update({"kernel": f"{KERNEL_NAMES[dom]} (finest level, p={pl}, m={pl + 1 + 2 * no})",
                 "kind": dom, "avg_launch_ms": kernels[dom]["avg_launch_ms"],
                 "launches": kernels[dom]["launches"],
                 "algorithmic_flops": kernels[dom]["algorithmic_flops"],
                 "algorithmic_bytes": kernels[dom]["algorithmic_bytes"]})

    dtype = {"fp64": "f64", "mixed": "f32+f64", "bf16": "bf16+f32+f64",
             "fp16": "f16+f32+f64"}[args.precision]
    out = {
        "metric": "DOF/s per V-cycle + time to 1e-10 residual, mixed/learned vs plain FP64",
        "value": n_dof * res["cycles"] / dt,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * res["s_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": cfg.description, "name": cfg.name, "elements": [cfg.nx, cfg.ny],
                   "p": cfg.p, "dof": n_dof, "solver": f"MGCG {cycle}, w_5",
                   "overlap": ov_levels[1:], "precision": args.precision,
                   "weights": args.weights, "rtol": 1e-10},
        "time_to_1e-10_ms": 1e3 * res["s_per_solve"],
        "iterations": res["iterations"],
        "true_residual_ratio": true_res,
        "r_bar": r_bar,
        "n10": MT.n10(r_bar),
        "omega": w_iter / r_bar,
        "omega_tables": w_iter / r_bar * (cfg.p + 1) / cfg.p,
        "vcycle_ms": 1e3 * tv,
        "vcycle_dof_per_s": n_dof / tv,
        "roofline": roof,
        "kernels": kernels,
        "kernel_timing_pass_ms_per_solve": 1e3 * res_k["s_per_solve"],
    }
    if learned_info is not None:
        learned_info["fallback_to_paper"] = s.learned_params is None
        out["learned"] = learned_info
    s.close()

    if not args.no_compare:
        cmp = {}
        plain = {}
        for wl in ("c3", "c5"):
            e = compare_run(wl, "fp64", None, 10, 2, args.imax)
            plain[wl] = e["time_to_1e-10_ms"]
            cmp[f"{wl}_fp64_paper"] = e
        cmp["c3_fp16_paper"] = compare_run("c3", "fp16", None, 10, 2, args.imax, plain["c3"])
        cmp["c5_fp16_paper"] = compare_run("c5", "fp16", None, 10, 2, args.imax, plain["c5"])
        if net is None:
            progress("training the parameter network")
            net, learned_info = train()
            cmp["learned_training"] = learned_info
        cmp["c5_fp64_learned"] = compare_run("c5", "fp64", net, 10, 2, args.imax, plain["c5"])
        cmp["c5_fp16_learned"] = compare_run("c5", "fp16", net, 10, 2, args.imax, plain["c5"])
        cmp["c5_fp16_learned_per_element"] = compare_run("c5", "fp16", net, 10, 2, args.imax,
                                                         plain["c5"], "element")
        # variable nu with correlation length 0.1: the paper's element-mean
        # local solves against separable local coefficients; and the separable
        # ones on the p = 32 workload itself
        cmp["c4_len0.1_fp64_paper"] = compare_run("c4", "fp64", None, 5, 1, args.imax, ell=0.1)
        cmp["c4_len0.1_fp64_separable"] = compare_run("c4", "fp64", None, 10, 2, args.imax,
                                                      ell=0.1, local="separable")
        cmp["c5_fp64_separable"] = compare_run("c5", "fp64", None, 10, 2, args.imax, plain["c5"],
                                               local="separable")
        # Algorithm 1 (sequential sweeps in one workgroup) against the additive
        # smoother on the 64 x 64, p = 8 workload
        cmp["c2_fp64_paper"] = compare_run("c2", "fp64", None, 10, 2, args.imax)
        cmp["c2_fp64_multiplicative"] = compare_run("c2", "fp64", None, 2, 1, args.imax,
                                                    cmp["c2_fp64_paper"]["time_to_1e-10_ms"],
                                                    wf=-3)
        cmp["d3_fp64_paper"] = compare_3d(16, 8, 1, 10, 2, args.imax)
        out["comparisons"] = cmp
    if not args.no_cpu_baseline:
        progress("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(cfg, fn, NU, ns1, ns2)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
