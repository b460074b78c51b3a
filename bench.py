"""Benchmark of the Newton-step CPR-FGMRES path on one MI355X.

A step is one implicit time step of the 200x200x50 (2,000,000-cell)
correlated-permeability model with 25 wells: Newton iterations, each with
assembly, decoupling, potential reordering, block ILU(0)/RAS set-up, AMG
set-up, a CPR-FGMRES(30) solve to 1e-8 and the update.  All inputs are
seeded and synthetic and resident in HBM before the timed region.

Prints one JSON line.  `value` is the mean wall time of one CPR-FGMRES solve
(set-up excluded) in ms; `ms_per_step` the mean time-step wall time.  The
roofline object prices the dominant kernel (the RAS triangular solve) by its
algorithmic bytes per launch over its event-timed duration; cpu_baseline is
the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CPR-GMRES solve ms + HBM GB/s at 2M cells; step time plain vs FP32+learned"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def ras_bytes(P, model, prec_bytes):
    """Algorithmic bytes of one RAS apply (forward + backward sweeps with the
    gather and restricted scatter): every factor block and inverse diagonal
    read once, column/row index data read once, the residual gathered once
    per local row, the local vector written and read twice, the owned rows
    written once."""
    from paper_1701_06254_amd import r2p
    ns = P.ras_info()
    m_tot = nblk = 0
    for s in range(ns):
        import ctypes as C
        a, m, nb, nl = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        r2p.load().r2p_ras_info(P.h, s, C.byref(a), C.byref(m), C.byref(nb), C.byref(nl))
        m_tot += m.value
        nblk += nb.value
    N = model.N
    factors = (4 * prec_bytes) * (nblk + m_tot)           # L/U blocks + inverse diagonals
    index = 4 * nblk + (4 + 4 + 4 + 1) * m_tot             # ecol; glob, eptr, nl, owned
    vectors = 16 * m_tot + 2 * 2 * (2 * prec_bytes) * m_tot + 8 * N
    return factors + index + vectors, m_tot, nblk


def spmv_bytes(model):
    n, nw, nperf = model.n, model.nw, model.nperf
    return 7 * 32 * n + 4 * n + 16 * n + 16 * n + nperf * (16 + 16 + 4 + 4) + nw * (8 + 32)


def time_kernel(fn, reps):
    import torch
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def cpu_baseline(w, gpu_solve_its, sample_its=5):
    """FP64 oracle on a bounded sample of the same workload: CPR set-up plus
    `sample_its` FGMRES iterations on the first Newton system of the first
    step; scaled to one solve with the GPU's iteration count."""
    import oracle
    oracle.build(force=False)
    m = oracle.Model(w)
    x = m.initial_state()
    J, F = m.jacobian(x, x, w["dt"])
    t0 = time.perf_counter()
    Ad, bd = oracle.decouple(J, -F, m.n, oracle.DEC_QI)
    P = oracle.Cpr(Ad, m, x, oracle.cpr_opts())
    t1 = time.perf_counter()
    y, st, its, rr = oracle.fgmres(Ad, bd, P, maxit=sample_its)
    t2 = time.perf_counter()
    per_it = (t2 - t1) / max(its, 1)
    solve_ms = per_it * gpu_solve_its * 1e3
    return dict(value=round(solve_ms, 1), unit="ms", cores=1, kind="oracle",
                sample=f"FP64 oracle, first Newton system of the 2M-cell model: CPR set-up "
                       f"{(t1 - t0):.1f} s (not in value) and {its} FGMRES(30) iterations "
                       f"({per_it * 1e3:.0f} ms each), scaled to the {gpu_solve_its:.1f} "
                       f"iterations of the mean GPU solve", setup_s=round(t1 - t0, 2))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--form", choices=["two-stage", "fpf"], default="two-stage")
    ap.add_argument("--agg-passes", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "decomposition is not built", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    from paper_1701_06254_amd import r2p
    r2p.load()
    w = workloads.make_config(args.config)
    log(f"workload {w['name']}: {w['grid']['n']} cells, {len(w['wells'])} wells")
    model = r2p.Model(w)
    x = model.initial_state()
    prec = r2p.FP32 if args.precision == "fp32" else r2p.FP64
    form = r2p.CPR_FPF if args.form == "fpf" else r2p.CPR_TWO_STAGE
    opts = r2p.newton_opts(cpr=r2p.cpr_opts(precision=prec, form=form,
                                             agg_passes=args.agg_passes))
    for k in range(args.warmup):
        info = model.newton_step(x, w["dt"], opts)
        log(f"warmup step {k}: status {info.status} newton {info.newton_its} linear "
            f"{info.linear_its} {info.ms_total:.1f} ms")
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        info = model.newton_step(x, w["dt"], opts)
        infos.append(info)
        log(f"step {k}: status {info.status} newton {info.newton_its} linear {info.linear_its} "
            f"assemble {info.ms_assemble:.1f} setup {info.ms_setup:.1f} solve "
            f"{info.ms_solve:.1f} total {info.ms_total:.1f} ms")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    n_solves = sum(i.newton_its for i in infos)
    lin_its = sum(i.linear_its for i in infos)
    solve_ms = sum(i.ms_solve for i in infos) / max(n_solves, 1)
    setup_ms = sum(i.ms_setup for i in infos) / max(n_solves, 1)
    asm_ms = sum(i.ms_assemble for i in infos) / max(sum(i.newton_its + 1 for i in infos), 1)
    its_per_solve = lin_its / max(n_solves, 1)

    # kernel timing on the current state's system
    J = r2p.Jacobian(model)
    b = J.assemble(x, x, w["dt"])
    P = r2p.Cpr().setup(J, opts.cpr)
    v = torch.randn(model.N, dtype=torch.float64, device="cuda")
    y = torch.empty_like(v)
    fp = torch.randn(model.n, dtype=torch.float64, device="cuda")
    xp = torch.empty_like(fp)
    t_spmv = time_kernel(lambda: J.spmv(v, y), 50)
    t_ras = time_kernel(lambda: P.ras_apply(v, y), 10)
    t_amg = time_kernel(lambda: P.amg_vcycle(fp, xp), 10)
    t_cpr = time_kernel(lambda: P.apply(v, y), 10)
    pb = 4 if prec == r2p.FP32 else 8
    rb, m_tot, nblk = ras_bytes(P, model, pb)
    sb = spmv_bytes(model)
    ras_gbs = rb / (t_ras * 1e-3) / 1e9
    spmv_gbs = sb / (t_spmv * 1e-3) / 1e9
    log(f"kernels: spmv {t_spmv * 1e3:.1f} us ({spmv_gbs:.0f} GB/s), ras {t_ras * 1e3:.1f} us "
        f"({ras_gbs:.0f} GB/s), vcycle {t_amg * 1e3:.1f} us, cpr {t_cpr * 1e3:.1f} us")

    out = {
        "metric": METRIC, "value": round(solve_ms, 3), "unit": "ms", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == r2p.FP64 else "f64+f32-preconditioner",
        "data": "synthetic",
        "config": {"workload": f"{w['name']} ({w['grid']['n']} cells, {len(w['wells'])} wells), "
                               f"dt {w['dt']} d, CPR {args.form} QI + potential order, RAS 4x4 "
                               f"overlap 1 BILU(0), aggregation AMG V(1,1), FGMRES(30) rtol 1e-8",
                   "cells": w["grid"]["n"], "precision": args.precision, "form": args.form},
        "newton_its_per_step": round(n_solves / args.steps, 2),
        "linear_its_per_solve": round(its_per_solve, 2),
        "setup_ms_per_newton": round(setup_ms, 3), "assemble_ms": round(asm_ms, 3),
        "ms_per_fgmres_iteration": round(solve_ms / max(its_per_solve, 1e-9), 4),
        "kernels_us": {"spmv": round(t_spmv * 1e3, 2), "ras_apply": round(t_ras * 1e3, 2),
                       "amg_vcycle": round(t_amg * 1e3, 2), "cpr_apply": round(t_cpr * 1e3, 2)},
        "spmv_gbs": round(spmv_gbs, 1),
        "roofline": {"bound": "hbm", "kernel": "k_ras_solve", "achieved": round(ras_gbs, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ras_gbs / HBM_PEAK_GBS, 4),
                     "traffic": None, "bytes_per_launch": rb},
    }
    if not args.no_cpu_baseline:
        try:
            out["cpu_baseline"] = cpu_baseline(w, its_per_solve)
        except Exception as e:  # the baseline is reported, never required
            log(f"cpu baseline failed: {e}")
            out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
