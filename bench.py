#!/usr/bin/env python3
"""Benchmark of the SEM Schwarz / p-multigrid solver on one MI355X.

A step is one complete solve of the workload with the multigrid-preconditioned
CG (MGCG(1,0): one pre-smoothing per level) from the seeded initial guess to
a residual reduction of 1e-10: it runs every part of the hot path (residual,
Schwarz smoother, restriction, prolongation, coarse solve, V-cycle, CG).

Printed JSON line (one):
  value        DOF/s per V-cycle over the timed solves: finest-level unknowns
               times V-cycles executed, divided by the wall time of the solves
  ms_per_step  time to 1e-10 per solve
  roofline     the finest-level Schwarz kernel, timed with HIP events on the
               library's stream during the timed solves
  cpu_baseline the CPU oracle on a bounded sample of the same workload

Usage: python bench.py [--steps K] [--warmup W] [--workload c2] [--n-o 1]
                       [--precision fp64|mixed|bf16|fp16] [--weights paper|learned]
                       [--no-cpu-baseline]

With --precision mixed / bf16 / fp16 or --weights learned the line also carries
`plain_fp64_paper`: the plain method (FP64, the paper's parameters) timed on
the same workload, and its speedup ratio.  --weights learned first runs the
parameter sweeps and trains the network (outside the timed region; reported
under `learned`).
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP64_PEAK_TFS = 78.6         # MI355X FP64 vector
FP32_PEAK_TFS = 157.3        # MI355X FP32 vector
RIDGE_FP64 = FP64_PEAK_TFS * 1e12 / (HBM_PEAK_GBS * 1e9)
RIDGE_FP32 = FP32_PEAK_TFS * 1e12 / (HBM_PEAK_GBS * 1e9)
BF16_PEAK_TFS = 2500.0       # MI355X dense BF16 (and FP16) matrix cores
RIDGE_BF16 = BF16_PEAK_TFS * 1e12 / (HBM_PEAK_GBS * 1e9)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fdm_traffic.json")


def _code_only(text: str) -> str:
    """Source text without comments and blank space (string literals in these
    files hold no comment markers)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash(texts=None) -> str:
    """Hash of the Schwarz kernels' code (comments and layout ignored): the
    recorded HBM traffic is reported only while it matches."""
    h = hashlib.sha256()
    for f in ("fdm_impl.h", "fdm_mfma.hip", "kernels.h", "common.h"):
        if texts is None:
            with open(os.path.join(ROOT, "paper_1512_02390_amd", "csrc", f)) as fh:
                t = fh.read()
        else:
            t = texts[f]
        h.update(_code_only(t).encode())
    return h.hexdigest()[:16]


RULES = {"fixed": 0, "ceil8": 1, "floor8": 2, "ceil2": 3}


def make_problem(name: str, n_o: int, precision: int, rule=None, overlaps=None, net=None):
    """Solver, right-hand side and initial guess of a workload; with a trained
    network `net` the Schwarz parameters are the learned ones (the paper's
    when the prediction is unusable)."""
    import numpy as np
    import torch
    from paper_1512_02390_amd import workloads as W
    from paper_1512_02390_amd.sem import Solver

    cfg = W.config(name, n_o)
    if rule is not None:
        cfg.overlap_rule = RULES[rule]
    if overlaps is not None:
        cfg.overlaps = overlaps
    nu = None
    NU = None
    if cfg.variable_nu:
        nu = W.GaussianFieldNu()
    if nu is not None:
        # node coordinates from a constant-coefficient handle of the same mesh
        probe = Solver(cfg.xb, cfg.yb, cfg.p, cfg.bc, cfg.overlap_rule, cfg.n_o, 5)
        xc, yc = probe.node_coords()
        probe.close()
        NU = W.nodal(nu.nu, xc, yc)
    learned_params = None
    if net is not None:
        from paper_1512_02390_amd import learned as LW
        s, learned_params = LW.solver_with_learned(cfg.xb, cfg.yb, cfg.p, cfg.bc, NU, net,
                                                   precision)
    else:
        s = Solver(cfg.xb, cfg.yb, cfg.p, cfg.bc, cfg.overlap_rule, cfg.n_o, 5, nu=NU,
                   precision=precision, overlaps=cfg.overlaps)
    s.learned_params = learned_params
    shape = s.shape()
    if name == "c1":
        xc, yc = s.node_coords()
        fn = W.nodal(lambda x, y: -W.SineSolution().laplacian(x, y), xc, yc)
    else:
        fn = W.random_nodal(shape, cfg.bc, W.SEED_RHS)
    f_nodal = torch.tensor(fn, dtype=torch.float64, device="cuda")
    b = s.zeros()
    s.mass(f_nodal, b)
    u0 = torch.tensor(W.random_guess(shape, cfg.bc, W.SEED_U0), dtype=torch.float64,
                      device="cuda")
    return cfg, s, b, u0, fn, NU


def fdm_work(s, cfg):
    """Algorithmic flops and bytes of one finest-level Schwarz-kernel launch:
    per element 8 m^3 + 3 m^2 flops (four m x m x m contractions, eigenvalue
    scaling, weighting); bytes: read r, read and write u (3 words per node)."""
    pl, no, rows, cols = s.level_info(s.L)
    m = pl + 1 + 2 * no
    n_el = cfg.nx * cfg.ny
    flops = n_el * (8.0 * m ** 3 + 3.0 * m ** 2)
    return flops, m


def cpu_baseline(cfg, fn, NU, ns1, ns2, budget_s: float = 12.0):
    """Oracle MGCG(1,0) solves of the same workload until the budget is used
    (at least one); DOF/s per V-cycle like the GPU value."""
    import numpy as np
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
                      f"({its} iterations each), {dt:.1f} s; time to 1e-10 "
                      f"{1e3 * dt / solves:.0f} ms per solve"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--n-o", type=int, default=1)
    ap.add_argument("--rule", default=None, choices=sorted(RULES),
                    help="overlap rule per level (default: the workload's)")
    ap.add_argument("--overlaps", default=None,
                    help="explicit overlaps of levels 1..L, comma separated")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed", "bf16", "fp16"],
                    help="fp64; mixed: FP32 V-cycle in FP64 MGCG; bf16 / fp16: as mixed with "
                         "the subdomain solves of wide tiles on BF16 / FP16 matrix cores")
    ap.add_argument("--imax", type=int, default=200)
    ap.add_argument("--cycle", default=None, choices=["mg10", "mg11", "var11"],
                    help="smoothing schedule (default: mg10; mg11 for variable nu)")
    ap.add_argument("--weights", default="paper", choices=["paper", "learned"],
                    help="Schwarz parameters: the paper's, or predicted by a network trained "
                         "on the solver's own sweeps before the timed region")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (the reference "
                         "kernel for scaling HBM counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1512_02390_amd.sem import FP64, MIXED_BF16, MIXED_FP16, MIXED_FP32

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
    prec = {"fp64": FP64, "mixed": MIXED_FP32, "bf16": MIXED_BF16,
            "fp16": MIXED_FP16}[args.precision]
    ovl = None
    if args.overlaps:
        ovl = [0] + [int(v) for v in args.overlaps.split(",")]
    net, learned_info = None, None
    if args.weights == "learned":
        from paper_1512_02390_amd import learned as LW
        t0 = time.perf_counter()
        X, T, recs = LW.make_dataset(LW.default_patches())
        net, lh = LW.train(X, T)
        learned_info = {"patches": len(recs), "samples": int(X.shape[0]),
                        "candidates_per_patch": len(recs[0][1]),
                        "train_loss": [lh[0], lh[-1]],
                        "sweep_and_training_s": time.perf_counter() - t0}
    cfg, s, b, u0, fn, NU = make_problem(args.workload, args.n_o, prec, args.rule, ovl, net)
    if learned_info is not None:
        learned_info["fallback_to_paper"] = s.learned_params is None
        if s.learned_params is not None:
            ax, ay = s.learned_params[1], s.learned_params[2]
            learned_info["alpha_range"] = [float(min(ax.min(), ay.min())),
                                           float(max(ax.max(), ay.max()))]
    cycle = args.cycle or ("mg11" if cfg.variable_nu else "mg10")
    L = s.L
    if cycle == "mg10":
        ns1, ns2 = [1] * (L + 1), [0] * (L + 1)
    elif cycle == "mg11":
        ns1, ns2 = [1] * (L + 1), [1] * (L + 1)
    else:
        ns1 = [2 ** (L - l) for l in range(L + 1)]
        ns2 = list(ns1)
    pl, no, rows, cols = s.level_info(s.L)
    n_dof = (cfg.nx * cfg.p - 1) * (cfg.ny * cfg.p - 1) if cfg.bc == 0 else cfg.nx * cfg.ny * cfg.p ** 2

    # warm-up solves (also the convergence record)
    for _ in range(max(args.warmup, 1)):
        u = u0.clone()
        it, hist, ok = s.pcg_solve(u, b, args.imax, 1e-10, ns1, ns2)
    if not ok and learned_info is not None and s.learned_params is not None:
        # the learned parameters failed on this problem: the paper's take over
        s.close()
        cfg, s, b, u0, fn, NU = make_problem(args.workload, args.n_o, prec, args.rule, ovl)
        learned_info["fallback_to_paper"] = "learned parameters did not converge"
        for _ in range(max(args.warmup, 1)):
            u = u0.clone()
            it, hist, ok = s.pcg_solve(u, b, args.imax, 1e-10, ns1, ns2)
    if not ok:
        raise SystemExit(f"MGCG did not reach 1e-10 in {args.imax} iterations")
    from paper_1512_02390_amd import metrics as MT
    r_bar = MT.rbar(hist)
    ov_levels = [0] + [s.level_info(l)[1] for l in range(1, s.L + 1)]
    w_iter = MT.cycle_cost(cfg.p, ov_levels, [a + c for a, c in zip(ns1, ns2)])

    # one private copy of the initial guess per timed step: no copies inside
    us = [u0.clone() for _ in range(args.steps)]
    s.timing_enable(s.L, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cycles = 0
    for k in range(args.steps):
        it_k, _, ok_k = s.pcg_solve(us[k], b, args.imax, 1e-10, ns1, ns2)
        cycles += it_k
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nk, kms = s.timing_read()
    s.timing_enable(s.L, False)
    dt = t1 - t0

    # pure V-cycle throughput (MG(1,0) cycles on the iterate), for reference
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

    # the plain method (FP64, the paper's parameters) on the same workload, for
    # the mixed / learned comparison at equal accuracy
    plain = None
    if prec != FP64 or net is not None:
        _, s0, b0, _, _, _ = make_problem(args.workload, args.n_o, FP64, args.rule, ovl)
        for _ in range(max(args.warmup, 1)):
            u = u0.clone()
            it0, _, ok0 = s0.pcg_solve(u, b0, args.imax, 1e-10, ns1, ns2)
        us0 = [u0.clone() for _ in range(args.steps)]
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        for k in range(args.steps):
            s0.pcg_solve(us0[k], b0, args.imax, 1e-10, ns1, ns2)
        torch.cuda.synchronize()
        tp = (time.perf_counter() - tp0) / args.steps
        plain = {"time_to_1e-10_ms": 1e3 * tp if ok0 else None, "iterations": it0,
                 "converged": bool(ok0),
                 "overlap": [s0.level_info(l)[1] for l in range(1, s0.L + 1)],
                 "speedup": (tp / (dt / args.steps)) if ok0 else None}
        s0.close()

    flops, m = fdm_work(s, cfg)
    word = 8 if prec == FP64 else 4
    nbytes = 3.0 * rows * cols * word
    avg_ms = kms / max(nk, 1)
    ai = flops / nbytes
    mfma = prec in (MIXED_BF16, MIXED_FP16) and m >= 17
    ridge = RIDGE_FP64 if prec == FP64 else (RIDGE_BF16 if mfma else RIDGE_FP32)
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        try:
            rec = json.load(open(TRAFFIC_FILE))
            key = f"{args.workload}_n{args.n_o}_{args.precision}"
            if rec.get("source_hash") == kernel_source_hash() and key in rec.get("per_launch", {}):
                traffic = rec["per_launch"][key]
        except Exception:
            traffic = None
    if ai < ridge:
        roof = {"bound": "hbm", "achieved": nbytes / (avg_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s"}
    else:
        peak = FP64_PEAK_TFS if prec == FP64 else FP32_PEAK_TFS
        roof = {"bound": "alu", "achieved": flops / (avg_ms * 1e-3) / 1e12, "peak": peak,
                "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = traffic
    word_t = "double" if prec == FP64 else "float"
    # the library's dispatch: two wavefronts per work item from m = 9, for
    # FP64 only while a factor row fits 256 bytes
    two_waves = m >= 9 and m * (8 if prec == FP64 else 4) <= 256
    kname = (f"k_fdm_mfma<{(m + 15) // 16}> (m={m})" if mfma
             else f"k_fdm{'2' if two_waves else ''}<{word_t},{m}>")
    roof.update({"kernel": kname,
                 "avg_launch_ms": avg_ms, "launches": nk,
                 "algorithmic_flops": flops, "algorithmic_bytes": nbytes,
                 "achieved_tflops": flops / (avg_ms * 1e-3) / 1e12})

    out = {
        "metric": "DOF/s per V-cycle + time to 1e-10 residual, mixed/learned vs plain FP64",
        "value": n_dof * cycles / dt,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {FP64: "f64", MIXED_FP32: "f32+f64", MIXED_BF16: "bf16+f32+f64",
                  MIXED_FP16: "f16+f32+f64"}[prec],
        "data": "synthetic",
        "config": {"workload": cfg.description, "name": cfg.name, "elements": [cfg.nx, cfg.ny],
                   "p": cfg.p, "dof": n_dof, "solver": f"MGCG {cycle}, w_5",
                   "overlap": [s.level_info(l)[1] for l in range(1, s.L + 1)],
                   "precision": args.precision, "weights": args.weights, "rtol": 1e-10},
        "time_to_1e-10_ms": 1e3 * dt / args.steps,
        "iterations": it,
        "r_bar": r_bar,
        "n10": MT.n10(r_bar),
        "omega": w_iter / r_bar,
        "omega_tables": w_iter / r_bar * (cfg.p + 1) / cfg.p,
        "vcycle_ms": 1e3 * tv,
        "vcycle_dof_per_s": n_dof / tv,
        "roofline": roof,
    }
    if plain is not None:
        out["plain_fp64_paper"] = plain
    if learned_info is not None:
        out["learned"] = learned_info
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, fn, NU, ns1, ns2)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
