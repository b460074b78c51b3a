"""Benchmark of the Newton-step CPR-FGMRES path on one MI355X.

Workload: the 200x200x50 (2,000,000-cell) correlated-permeability model with
25 wells, seeded and synthetic, resident in HBM before any timed region.

A step is one implicit time step: Newton iterations, each with assembly,
decoupling, potential reordering, block ILU(0)/RAS set-up, AMG set-up, a
CPR-FGMRES(30) solve to 1e-8 and the update.  From the cold start the step
length follows a standard controller: it starts at 0.1 day, is halved when
Newton fails (the state is left unchanged by the library) and doubled after a
step that converged in at most 6 Newton iterations, up to the model's 10 days.
The timed steps continue the same controller from the state the warm-up
steps reached.

Prints one JSON line on stdout (progress goes to stderr):
  value            mean wall time of one CPR-FGMRES solve (r2p_solve, per
                   Newton linear system, CPR set-up excluded) in ms;
  ms_per_step      mean wall time of one time step (plain FP64);
  fp32             the same steps with the FP32 preconditioner (FP64 FGMRES),
                   with the field difference against the FP64 run;
  fp32_learned     the same steps with the FP32 preconditioner and the learned
                   warm start (network trained beforehand, untimed, on seeded
                   smaller models of the same family; training time stated);
  roofline         the RAS apply (gather + level-scheduled triangular sweeps +
                   restricted scatter, the largest single kernel of a solve):
                   algorithmic bytes per apply over its HIP-event-timed mean
                   duration on the library's stream, against 8 TB/s;
  cpu_baseline     the FP64 CPU oracle, single-threaded, on a bounded sample
                   of the same workload, scaled to the GPU's iterations.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CPR-GMRES solve ms + HBM GB/s at 2M cells; step time plain vs FP32+learned"
HBM_PEAK_GBS = 8000.0
# HBM traffic of one RAS apply (k_ras_gather + k_ras_sweep + k_ras_scatter) on
# the first Newton system of the 2M-cell cold start, from two rocprofv3 --pmc
# runs of `bench.py --kernels-only` (FETCH_SIZE, then WRITE_SIZE, KiB per
# dispatch, mean of 5).  The same counters read 262,170 / 524,288 KiB for a
# 512 MiB device copy, so FETCH_SIZE is scaled by 2.0 and WRITE_SIZE by 1.0.
# Valid only for the RAS source these were taken on (first 16 hex digits of
# its SHA-256); any change to it reports traffic as null.
RAS_TRAFFIC = {"source_sha256": "398f98a8e42b5c68",
               "fetch_kib": 26517.2 + 366191.1 + 49718.7, "fetch_scale": 2.0,
               "write_kib": 41554.6 + 65801.0 + 31398.4, "write_scale": 1.0}
DT_INIT, DT_MIN = 0.1, 1e-4
GROW_ITS = 6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def ras_bytes(P, model, prec_bytes):
    """Algorithmic bytes of one RAS apply.

    Per local row of every overlapped subdomain: its off-diagonal factor blocks
    (4 values + a column index each) and its inverse diagonal block read once;
    its row lengths and gather index read once; the gathered right-hand side
    read from the global vector (16 B) and written locally; the local vector
    written by the forward sweep, read and rewritten by the backward sweep,
    read by the scatter; the owned flag read once.  The owned rows' results
    (N doubles) are written once.  Neighbour values re-read within a sweep are
    not counted (they are the same bytes)."""
    from paper_1701_06254_amd import r2p
    ns = P.ras_info()
    m_tot = nblk = 0
    for s in range(ns):
        a, m, nb, nl = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        r2p.load().r2p_ras_info(P.h, s, C.byref(a), C.byref(m), C.byref(nb), C.byref(nl))
        m_tot += m.value
        nblk += nb.value
    vb = 2 * prec_bytes                       # one local 2-vector entry
    factors = 4 * prec_bytes * (nblk + m_tot) + 4 * nblk
    per_row = 4 + 4 + 4 + 1                   # n_L, n_U, gather index, owned flag
    vectors = 16 + vb + vb + 2 * vb + vb      # gather read/write, fwd write, bwd read+write, scatter read
    return factors + per_row * m_tot + vectors * m_tot + 8 * model.N, m_tot, nblk


def ras_traffic():
    """Counter-measured HBM bytes per RAS apply, or None when the kernels
    have changed since the counters were taken."""
    import hashlib
    src = os.path.join(ROOT, "paper_1701_06254_amd", "csrc", "ras_solve.hip")
    with open(src, "rb") as f:
        h = hashlib.sha256(f.read()).hexdigest()[:16]
    t = RAS_TRAFFIC
    if h != t["source_sha256"]:
        return None
    return int(1024 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]))


def spmv_bytes(model):
    """Algorithmic bytes of y = J x: 7 stencil blocks (32 B) per cell, x and
    y (16 B each) per cell, and per perforation / well the coupling blocks,
    offsets and vector entries."""
    n, nw, nperf = model.n, model.nw, model.nperf
    return 7 * 32 * n + 16 * n + 16 * n + nperf * (32 + 32 + 4) + nw * (32 + 8 + 16 + 16)


def vcycle_bytes(P, model, prec_bytes=8):
    """Algorithmic bytes of one AMG V-cycle on the pressure system.

    Level 0 (7-slot stencil): pre-smoothing reads the pressure entries of
    the right-hand side (whole 16-byte pairs), d and the 7 coefficients and
    writes x and r (96 B per cell); post-smoothing reads the same plus x and
    writes the result (96 B); the prolongation onto level 0 reads the
    aggregate index and x and writes x (20 B).  CSR level l: per entry the
    value and column, per row the row pointer, b, x and the output (and d on
    the way up), both ways; restriction: member list, fine residual, member
    pointers, b and x of the coarse level; prolongation: aggregate index,
    x read and written.  Coarsest: the dense inverse and two vectors.
    Neighbour values re-read within a kernel are not counted."""
    from paper_1701_06254_amd import r2p
    L = r2p.load()
    nlev, n, nnz = C.c_int(), C.c_int(), C.c_int()
    L.r2p_amg_info(P.h, 0, C.byref(nlev), C.byref(n), C.byref(nnz))
    sizes = []
    for l in range(nlev.value):
        L.r2p_amg_info(P.h, l, C.byref(nlev), C.byref(n), C.byref(nnz))
        sizes.append((n.value, nnz.value))
    b = prec_bytes
    nl = len(sizes)
    if nl == 1:
        nc = sizes[0][0]
        return 8 * nc * nc + 16 * nc
    n0 = sizes[0][0]
    total = n0 * (16 + b + 7 * b + 2 * b) + n0 * (16 + 7 * b + 3 * b) + n0 * (4 + 2 * b)
    for l in range(1, nl):
        nf, nc = sizes[l - 1][0], sizes[l][0]
        smooth = l < nl - 1
        total += nf * (4 + b) + 4 * (nc + 1) + nc * b * (3 if smooth else 1)
        if smooth:
            n_l, z_l = sizes[l]
            row = 4 * (n_l + 1) + 12 * z_l
            total += row + 3 * b * n_l + row + 4 * b * n_l + n_l * (4 + 2 * b)
    nc = sizes[-1][0]
    total += 8 * nc * nc + 2 * b * nc
    return total


def variants_run(model, x, dt, form):
    """Method variants on one Newton system (state x, step dt), each solved
    from scratch with FGMRES(30) to 1e-8: the decoupling x reordering
    ablation of the paper's Table 4 (NONE, PT, ABF, QI, PT-ABF, PT-QI) and
    the RAS variants (overlap 1 or 2; 2x2, 4x4, 8x8 or 16x16 subdomains).  Returns
    iterations, status and set-up / solve ms per variant."""
    import torch
    from paper_1701_06254_amd import r2p
    rows = []
    cases = [("NONE", r2p.DEC_NONE, r2p.ORDER_NATURAL, 4, 1),
             ("PT", r2p.DEC_NONE, r2p.ORDER_POTENTIAL, 4, 1),
             ("ABF", r2p.DEC_ABF, r2p.ORDER_NATURAL, 4, 1),
             ("QI", r2p.DEC_QI, r2p.ORDER_NATURAL, 4, 1),
             ("PT-ABF", r2p.DEC_ABF, r2p.ORDER_POTENTIAL, 4, 1),
             ("PT-QI", r2p.DEC_QI, r2p.ORDER_POTENTIAL, 4, 1),
             ("PT-QI overlap 2", r2p.DEC_QI, r2p.ORDER_POTENTIAL, 4, 2),
             ("PT-QI 2x2 subdomains", r2p.DEC_QI, r2p.ORDER_POTENTIAL, 2, 1),
             ("PT-QI 8x8 subdomains", r2p.DEC_QI, r2p.ORDER_POTENTIAL, 8, 1),
             ("PT-QI 16x16 subdomains", r2p.DEC_QI, r2p.ORDER_POTENTIAL, 16, 1)]
    for name, dec, order, pxy, ov in cases:
        J = r2p.Jacobian(model)
        b = J.assemble(x, x, dt)
        opts = r2p.cpr_opts(decouple=dec, order=order, form=form, px=pxy, py=pxy, overlap=ov)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P = r2p.Cpr().setup(J, opts)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, info = r2p.solve(J, P, b)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        rows.append({"variant": name, "iterations": info.iterations, "status": info.status,
                     "relres": info.relres, "setup_ms": round((t1 - t0) * 1e3, 2),
                     "solve_ms": round((t2 - t1) * 1e3, 2)})
        log(f"variant {name}: {info.iterations} its status {info.status} "
            f"setup {rows[-1]['setup_ms']} ms solve {rows[-1]['solve_ms']} ms")
        del P, J
    return rows


def time_on_stream(fn, reps):
    """Mean ms of fn() over reps calls, from HIP events on the current stream
    (the stream every library call is enqueued on)."""
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


def newton_record(info, dt):
    """One Newton step's counts and stage times as a plain dict."""
    r = dict(dt=dt, status=info.status, newton=info.newton_its, linear=info.linear_its,
             setup_status=info.setup_status)
    for k in ("ms_assemble", "ms_setup", "ms_decouple", "ms_order", "ms_ras_setup",
              "ms_amg_setup", "ms_solve", "ms_update", "ms_total"):
        r[k] = getattr(info, k)
    return r


def run_steps(model, x, dt, nsteps, opts, dt_max, tag, dts=None):
    """nsteps accepted implicit steps on x (in place).  With `dts` given the
    step lengths are replayed instead of controlled: a replayed step whose
    Newton iteration fails is covered by halved sub-steps, so the replay
    reaches the same simulated time.  Returns the next step length and one
    record per attempted Newton step."""
    recs = []
    for k in range(nsteps):
        remaining = dts[k] if dts is not None else None
        if dts is not None:
            dt = remaining
        while True:
            info = model.newton_step(x, dt, opts)
            recs.append(newton_record(info, dt))
            log(f"{tag} step {k}: dt {dt:.4g} d status {info.status} newton {info.newton_its} "
                f"linear {info.linear_its} setup {info.ms_setup:.0f} solve {info.ms_solve:.0f} "
                f"total {info.ms_total:.0f} ms")
            if info.status == 0:
                if dts is None:
                    break
                remaining -= dt
                if remaining <= 1e-9 * dts[k]:
                    break
                dt = min(dt, remaining)
                continue
            dt *= 0.5
            if dt < DT_MIN:
                raise RuntimeError("time step fell below the minimum")
        if dts is None and info.newton_its <= GROW_ITS:
            dt = min(2.0 * dt, dt_max)
    return dt, recs


def summarise(recs):
    solves = sum(r["newton"] for r in recs)
    lin = sum(r["linear"] for r in recs)
    return dict(solves=solves, linear_its=lin,
                solve_ms=sum(r["ms_solve"] for r in recs) / max(solves, 1),
                setup_ms=sum(r["ms_setup"] for r in recs) / max(solves, 1),
                its_per_solve=lin / max(solves, 1))


def cpu_baseline(w, gpu_its_per_solve, dt, sample_its):
    """FP64 oracle, single-threaded, on the first Newton system of the cold
    start at the controller's first step length: CPR set-up (reported, not in
    value) and `sample_its` FGMRES iterations, whose mean iteration time is
    scaled to the GPU's mean iterations per solve."""
    import oracle
    oracle.build(force=False)
    m = oracle.Model(w)
    x = m.initial_state()
    J, F = m.jacobian(x, x, dt)
    t0 = time.perf_counter()
    Ad, bd = oracle.decouple(J, -F, m.n, oracle.DEC_QI)
    P = oracle.Cpr(Ad, m, x, oracle.cpr_opts())
    t1 = time.perf_counter()
    y, st, its, rr = oracle.fgmres(Ad, bd, P, maxit=sample_its)
    t2 = time.perf_counter()
    per_it = (t2 - t1) / max(its, 1)
    return dict(value=round(per_it * gpu_its_per_solve * 1e3, 1), unit="ms", cores=1,
                kind="oracle",
                sample=f"FP64 oracle, one thread: first Newton system of the 2M-cell cold "
                       f"start (dt {dt} d), decoupling + CPR set-up {t1 - t0:.2f} s (not in "
                       f"value) and {its} FGMRES(30) iterations at {per_it * 1e3:.0f} ms each, "
                       f"scaled to the {gpu_its_per_solve:.1f} iterations of the mean GPU solve")


def learned_run(args, model, x0, x64, dts, form, log):
    """FP32 preconditioner plus the learned warm start on the same steps.

    The network is trained first (not timed) on increments of seeded
    200x200x50 models of the workload's family with new permeability fields
    (seeds 1000 + i; the timed workload is seed 1, held out), each run from
    its cold start through the same step-length controller as the timed run,
    every accepted step kept as four random 48x48-column crops over all
    layers (the recipe of paper_1701_06254_amd.learned_study at a smaller
    count).  Each timed step evaluates the scaled residual at the network's
    iterate and at x^n and starts Newton from the smaller (the library's
    default rule); the two norms are reported per step."""
    import numpy as np
    import torch
    from paper_1701_06254_amd import r2p, warmstart, learned_study
    o64 = r2p.newton_opts(cpr=r2p.cpr_opts(form=form))
    t0 = time.perf_counter()
    rng = np.random.default_rng(2024)
    pairs = learned_study.collect(range(1000, 1000 + args.train_models), args.train_steps,
                                  4, o64, rng)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    net = r2p.Cnn(blocks=4)
    net.set_params(warmstart.init_params(np.random.default_rng(7)))
    losses = warmstart.train(net, pairs, (50, learned_study.CROP, learned_study.CROP),
                             args.train_iters, batch=4, lr=1e-3, seed=3, log=log)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    del pairs
    torch.cuda.empty_cache()
    log(f"learned start: {args.train_models} training runs in {t1 - t0:.1f} s, "
        f"{args.train_iters} Adam steps in {t2 - t1:.1f} s, loss {np.mean(losses[:20]):.3e} -> "
        f"{np.mean(losses[-20:]):.3e}")
    # inference throughput on the full grid (algorithmic flops of the
    # unpadded layers: 6->32, 8 x 32->32, 32->2, 3x3x3 taps)
    feat = r2p.cnn_features(model, x0, dts[0])
    g = model.w["grid"]
    shape = (1, g["nz"], g["ny"], g["nx"])
    net.forward(feat, shape)            # sizes the activation buffers for this grid
    t_fwd = time_on_stream(lambda: net.forward(feat, shape), 5)
    flop = 2 * 27 * (6 * 32 + 8 * 32 * 32 + 32 * 2) * model.n
    o = r2p.newton_opts(cpr=r2p.cpr_opts(form=form, precision=r2p.FP32),
                        guess_rule=r2p.GUESS_SCALED_INF)
    xl = x0.clone()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    recs = []
    guesses = []
    for k, dt in enumerate(dts):
        guess = net.warm_start(model, xl, dt)
        guesses.append(guess)
        info = model.newton_step(xl, dt, o, x_guess=guess)
        recs.append(dict(newton_record(info, dt), used=info.used_guess))
        log(f"fp32+learned step {k}: dt {dt:.4g} d status {info.status} newton {info.newton_its} "
            f"linear {info.linear_its} guess {info.used_guess} total {info.ms_total:.0f} ms")
        if info.status != 0:
            break
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t3) * 1e3 / max(len(recs), 1)
    # untimed: the scaled residual at x^n and at the network's iterate of
    # every step (replayed from the same states)
    norms = []
    Jr = r2p.Jacobian(model)
    xr = x0.clone()
    for k, dt in enumerate(dts[:len(recs)]):
        xo = xr.clone()
        n0 = model.residual_norm(Jr.assemble(xr, xo, dt), dt)
        ng = model.residual_norm(Jr.assemble(guesses[k], xo, dt), dt)
        norms.append([n0, ng])
        model.newton_step(xr, dt, o)
    sm = summarise(recs)
    n = model.n
    p64, s64 = x64[0:2 * n:2], x64[1:2 * n:2]
    pl, sl = xl[0:2 * n:2], xl[1:2 * n:2]
    return dict(ms_per_step=round(ms, 3), solve_ms=round(sm["solve_ms"], 3),
                newton_its=sm["solves"], linear_its_per_solve=round(sm["its_per_solve"], 2),
                guess_taken=int(sum(r["used"] for r in recs)), steps=len(recs),
                guess_rule="scaled residual: the smaller of x^n and the network's iterate",
                residual_xn_vs_guess=norms,
                cnn_forward_ms=round(t_fwd, 3),
                cnn_tflops=round(flop / (t_fwd * 1e-3) / 1e12, 1),
                converged=all(r["status"] == 0 for r in recs),
                rel_err_p=float(torch.linalg.norm(pl - p64) / torch.linalg.norm(p64)),
                rel_err_sw=float(torch.linalg.norm(sl - s64) /
                                 max(float(torch.linalg.norm(s64)), 1e-300)),
                training={"runs": args.train_models, "grid": "200x200x50",
                          "crop": [50, learned_study.CROP, learned_study.CROP],
                          "adam_steps": args.train_iters, "data_s": round(t1 - t0, 2),
                          "train_s": round(t2 - t1, 2),
                          "loss_first20": float(np.mean(losses[:20])),
                          "loss_last20": float(np.mean(losses[-20:]))})


def large_run(args, w, log):
    """The 65.5M-cell channelised model: plain FP64 CPR-FGMRES against the
    FP32 preconditioner plus the learned warm start, on one GPU.

    Per-kernel times (SpMV, RAS apply, V-cycle) are taken first on the first
    Newton system, then one warm-up step (0.1 day) and `--steps` timed steps
    of the controller run in FP64; the FP32 + learned form replays the same
    step lengths from the same state.  The network is trained beforehand
    (untimed) on increments of seeded 80x80x40 channelised models (4 wells).
    Device memory in use is reported after each form."""
    import numpy as np
    import torch
    import workloads
    from paper_1701_06254_amd import r2p, warmstart

    def used_gib():
        free, total = torch.cuda.mem_get_info()
        return round((total - free) / 2 ** 30, 1)

    px, py = args.tiles
    model = r2p.Model(w)
    x = model.initial_state()
    # At this size and step length (0.1-0.2 d from the cold start) the AMG
    # cycle costs more than its iterations save: one cycle per stage with the
    # K-cycle on two levels is faster than the 2M-cell default (1.64 against
    # 1.77 s per solve); the options select either.
    cyc = dict(kcycle=2 if args.kcycle is None else args.kcycle,
               amg_cycles=1 if args.amg_cycles is None else args.amg_cycles)
    o64 = r2p.newton_opts(cpr=r2p.cpr_opts(px=px, py=py, **cyc))
    o32 = r2p.newton_opts(cpr=r2p.cpr_opts(px=px, py=py, precision=r2p.FP32, **cyc),
                          guess_rule=r2p.GUESS_SCALED_INF)
    J = r2p.Jacobian(model)
    J.assemble(x, x, DT_INIT)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P = r2p.Cpr().setup(J, o64.cpr)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    v = torch.randn(model.N, dtype=torch.float64, device="cuda")
    y = torch.empty_like(v)
    fp = torch.randn(model.n, dtype=torch.float64, device="cuda")
    xp = torch.empty_like(fp)
    t_spmv = time_on_stream(lambda: J.spmv(v, y), 10)
    t_ras = time_on_stream(lambda: P.ras_apply(v, y), 5)
    t_amg = time_on_stream(lambda: P.amg_vcycle(fp, xp), 5)
    rb, m_tot, nblk = ras_bytes(P, model, 8)
    sb = spmv_bytes(model)
    levels = [g["n"] for g in P.amg_levels()]
    kern = {"spmv_us": round(t_spmv * 1e3, 1), "spmv_gbs": round(sb / (t_spmv * 1e-3) / 1e9, 1),
            "ras_apply_us": round(t_ras * 1e3, 1),
            "ras_gbs": round(rb / (t_ras * 1e-3) / 1e9, 1),
            "amg_cycle_us": round(t_amg * 1e3, 1),
            "cpr_setup_ms": round(setup_ms, 1), "amg_levels": levels,
            "ras_local_rows": m_tot, "ras_offdiag_blocks": nblk}
    log(f"large: kernels {kern}")
    del J, P, v, y, fp, xp
    torch.cuda.empty_cache()

    dt, _ = run_steps(model, x, DT_INIT, args.warmup, o64, float(w["dt"]), "warmup")
    x0 = x.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, recs = run_steps(model, x, dt, args.steps, o64, float(w["dt"]), "fp64")
    torch.cuda.synchronize()
    ms64 = (time.perf_counter() - t0) * 1e3 / args.steps
    mem64 = used_gib()
    s64 = summarise(recs)
    accepted = [r["dt"] for r in recs if r["status"] == 0]
    out = {
        "metric": METRIC, "value": round(s64["solve_ms"], 3), "unit": "ms", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms64, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{w['name']}: {model.n} cells, {len(w['wells'])} wells, "
                               f"channelised permeability; dt from {DT_INIT} d; CPR two-stage, "
                               f"QI + local potential order, RAS {px}x{py} overlap 1 BILU(0), "
                               f"aggregation AMG, {cyc['amg_cycles']} cycle(s) per pressure stage, "
                               f"K-cycle on {cyc['kcycle']} level(s), FGMRES(30) rtol 1e-8",
                   "cells": model.n, "subdomains": px * py},
        "dt_days": accepted,
        "newton_its_per_step": round(s64["solves"] / args.steps, 2),
        "linear_its_per_solve": round(s64["its_per_solve"], 2),
        "setup_ms_per_solve": round(s64["setup_ms"], 3),
        "device_memory_gib": mem64,
        "kernels": kern,
        "fp32_learned": None,
    }
    if args.no_learned:
        return out

    t1 = time.perf_counter()
    pairs = []
    for seed in range(2001, 2001 + 16):
        wt = workloads.make_channels(nx=80, ny=80, nz=40, seed=seed, n_channels=4,
                                     well_pattern=2)
        mt = r2p.Model(wt)
        xs = mt.initial_state()
        warmstart.collect_pairs(mt, xs, [0.1, 0.1, 0.2, 0.4, 0.8], o64, pairs)
        del mt
    net = r2p.Cnn(blocks=4)
    net.set_params(warmstart.init_params(np.random.default_rng(7)))
    losses = warmstart.train(net, pairs, (40, 80, 80), args.train_iters, batch=2, lr=1e-3,
                             seed=3, log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    del pairs
    torch.cuda.empty_cache()

    xl = x0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recsl = []
    for k, dtk in enumerate(accepted):
        guess = net.warm_start(model, xl, dtk)
        info = model.newton_step(xl, dtk, o32, x_guess=guess)
        del guess
        recsl.append(dict(newton_record(info, dtk), used=info.used_guess))
        log(f"fp32+learned step {k}: dt {dtk:.4g} d status {info.status} newton "
            f"{info.newton_its} linear {info.linear_its} guess {info.used_guess} "
            f"total {info.ms_total:.0f} ms")
        if info.status != 0:
            break
    torch.cuda.synchronize()
    msl = (time.perf_counter() - t0) * 1e3 / max(len(recsl), 1)
    meml = used_gib()
    sl = summarise(recsl)
    n = model.n
    p64, s_64 = x[0:2 * n:2], x[1:2 * n:2]
    pl, s_l = xl[0:2 * n:2], xl[1:2 * n:2]
    out["fp32_learned"] = {
            "ms_per_step": round(msl, 3), "solve_ms": round(sl["solve_ms"], 3),
            "newton_its": sl["solves"], "linear_its_per_solve": round(sl["its_per_solve"], 2),
            "guess_taken": int(sum(r["used"] for r in recsl)), "steps": len(recsl),
            "converged": all(r["status"] == 0 for r in recsl),
            "device_memory_gib": meml,
            "rel_err_p": float(torch.linalg.norm(pl - p64) / torch.linalg.norm(p64)),
            "rel_err_sw": float(torch.linalg.norm(s_l - s_64) /
                                max(float(torch.linalg.norm(s_64)), 1e-300)),
            "training": {"models": 16, "adam_steps": args.train_iters,
                         "seconds": round(train_s, 1),
                         "loss_first20": float(np.mean(losses[:20])),
                         "loss_last20": float(np.mean(losses[-20:]))}}
    return out


def stage_summary(recs):
    """Per-step means of the Newton step's stage times (ms), the columns of
    the paper's timing table (Table 5)."""
    keys = ["ms_assemble", "ms_setup", "ms_decouple", "ms_order", "ms_ras_setup",
            "ms_amg_setup", "ms_solve", "ms_update", "ms_total"]
    ok = [r for r in recs if r["status"] == 0] or recs
    return {k: round(sum(r[k] for r in ok) / max(len(ok), 1), 3) for k in keys}


def snapshot_solves(model, states, dt, form, log):
    """Fixed-snapshot solves: for each named state, the first Newton system of
    a step of length dt (J(x, x, dt)), CPR set-up and one CPR-FGMRES(30)
    solve to 1e-8, in FP64 and with the FP32 preconditioner."""
    import torch
    from paper_1701_06254_amd import r2p
    out = []
    for name, x in states:
        row = {"state": name, "dt_days": dt}
        for tag, prec in (("fp64", r2p.FP64), ("fp32", r2p.FP32)):
            J = r2p.Jacobian(model)
            b = J.assemble(x, x, dt)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            P = r2p.Cpr().setup(J, r2p.cpr_opts(form=form, precision=prec))
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, info = r2p.solve(J, P, b)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            row[tag] = {"setup_ms": round((t1 - t0) * 1e3, 2), "solve_ms": round((t2 - t1) * 1e3, 2),
                        "iterations": info.iterations, "relres": info.relres,
                        "status": info.status}
            del P, J
        log(f"snapshot {name} dt {dt}: {row}")
        out.append(row)
    return out


def host_cpu():
    """CPU model name and logical CPU count of the host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=1,
                    help="1: the 2M-cell model (default); 4: the 65.5M-cell channelised model, "
                         "FP64 against FP32 + learned start (its own JSON line)")
    ap.add_argument("--form", choices=["two-stage", "fpf"], default="two-stage")
    ap.add_argument("--amg-cycles", type=int, default=None,
                    help="AMG cycles per pressure stage (default: the library's, 2; 1 for --config 4)")
    ap.add_argument("--kcycle", type=int, default=None,
                    help="AMG levels whose coarse correction is a K-cycle, 0: V-cycle (default 1; "
                         "2 for --config 4)")
    ap.add_argument("--tiles", type=lambda v: tuple(int(t) for t in v.split("x")), default=(16, 16),
                    help="RAS subdomain tiles PXxPY for --config 4 (default 16x16, one subdomain "
                         "per CU; at most 256 in all)")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-its", type=int, default=20)
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the method variants on the last system and the EW-forcing replay")
    ap.add_argument("--budget-s", type=float, default=420.0,
                    help="optional legs that would start after this many seconds are skipped")
    ap.add_argument("--train-models", type=int, default=3,
                    help="seeded 200x200x50 runs of the same family (new permeability fields) "
                         "that give training pairs")
    ap.add_argument("--train-steps", type=int, default=8,
                    help="controller steps per training run")
    ap.add_argument("--train-iters", type=int, default=1500)
    ap.add_argument("--kernels-only", action="store_true",
                    help="for hardware-counter runs: set up the first Newton system of the "
                         "workload, then run 5 RAS applies, 5 AMG cycles, 5 SpMVs and 5 copies "
                         "of 512 MiB (the traffic calibration), then 15 more AMG cycles, and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): this build has no "
              "multi-GPU decomposition", file=sys.stderr)
        sys.exit(2)
    T0 = time.perf_counter()

    import torch
    import workloads
    from paper_1701_06254_amd import r2p
    r2p.load()
    w = workloads.make_config(args.config)
    log(f"workload {w['name']}: {w['grid']['n']} cells, {len(w['wells'])} wells")
    if args.config == 4:
        print(json.dumps(large_run(args, w, log)), flush=True)
        return
    model = r2p.Model(w)
    x = model.initial_state()
    x_init = x.clone()
    form = r2p.CPR_FPF if args.form == "fpf" else r2p.CPR_TWO_STAGE
    ac = {} if args.amg_cycles is None else {"amg_cycles": args.amg_cycles}
    kc = 1 if args.kcycle is None else args.kcycle
    o64 = r2p.newton_opts(cpr=r2p.cpr_opts(form=form, kcycle=kc, **ac))
    o32 = r2p.newton_opts(cpr=r2p.cpr_opts(form=form, precision=r2p.FP32, kcycle=kc, **ac))
    dt_max = float(w["dt"])

    if args.kernels_only:
        J = r2p.Jacobian(model)
        J.assemble(x, x, DT_INIT)
        P = r2p.Cpr().setup(J, o64.cpr)
        v = torch.randn(model.N, dtype=torch.float64, device="cuda")
        y = torch.empty_like(v)
        fp = torch.randn(model.n, dtype=torch.float64, device="cuda")
        xp = torch.empty_like(fp)
        src = torch.ones(64 << 20, dtype=torch.float64, device="cuda")    # 512 MiB
        dst = torch.empty_like(src)
        for _ in range(5):
            P.ras_apply(v, y)
            P.amg_vcycle(fp, xp)
            J.spmv(v, y)
            dst.copy_(src)
        for _ in range(15):                 # more AMG cycles for per-level traces
            P.amg_vcycle(fp, xp)
        torch.cuda.synchronize()
        rb, m_tot, nblk = ras_bytes(P, model, 8)
        print(json.dumps({"kernels_only": True, "ras_bytes_per_apply": rb,
                          "spmv_bytes": spmv_bytes(model), "copy_bytes": 2 * src.numel() * 8}))
        return

    # ---- the timed region: plain FP64 steps of the controller
    dt, _ = run_steps(model, x, DT_INIT, args.warmup, o64, dt_max, "warmup")
    x0 = x.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dt_next, recs = run_steps(model, x, dt, args.steps, o64, dt_max, "fp64")
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    s64 = summarise(recs)
    accepted = [r["dt"] for r in recs if r["status"] == 0]
    n = model.n
    out = {
        "metric": METRIC, "value": round(s64["solve_ms"], 3), "unit": "ms", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{w['name']}: {w['grid']['n']} cells, {len(w['wells'])} wells, "
                               f"adaptive dt from {DT_INIT} d (max {dt_max} d); CPR {args.form}, "
                               "QI + local potential order, RAS 4x4 overlap 1 BILU(0), "
                               "aggregation AMG, two cycles per pressure stage, K-cycle "
                               "on the first coarse level, "
                               "FGMRES(30) rtol 1e-8",
                   "cells": w["grid"]["n"], "form": args.form},
        "dt_days": accepted,
        "newton_its_per_step": round(s64["solves"] / args.steps, 2),
        "linear_its_per_solve": round(s64["its_per_solve"], 2),
        "setup_ms_per_solve": round(s64["setup_ms"], 3),
        "ms_per_fgmres_iteration": round(s64["solve_ms"] / max(s64["its_per_solve"], 1e-9), 4),
        "stage_ms_per_step": stage_summary(recs),
        "step_records": [{k: (round(v, 2) if isinstance(v, float) else v) for k, v in r.items()}
                         for r in recs],
        "errors": {},
    }
    log(f"fp64: {ms_step:.0f} ms per step, {s64['solve_ms']:.1f} ms per solve, "
        f"{s64['its_per_solve']:.1f} iterations per solve")

    def leg(name, fn, required=False):
        """Run an optional leg; its failure is recorded, never fatal."""
        el = time.perf_counter() - T0
        if not required and el > args.budget_s:
            out["errors"][name] = f"skipped: {el:.0f} s elapsed (budget {args.budget_s:.0f} s)"
            log(out["errors"][name])
            return None
        try:
            return fn()
        except Exception as e:   # recorded in the JSON line, the measurement is kept
            out["errors"][name] = f"{type(e).__name__}: {e}"
            log(f"{name} failed: {e}")
            return None

    # ---- FP32 preconditioner replay of the same steps (timed)
    def fp32_leg():
        x32 = x0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, recs32 = run_steps(model, x32, dt, args.steps, o32, dt_max, "fp32", dts=accepted)
        torch.cuda.synchronize()
        ms32 = (time.perf_counter() - t0) * 1e3 / args.steps
        s32 = summarise(recs32)
        p64, s_64 = x[0:2 * n:2], x[1:2 * n:2]
        p32, s_32 = x32[0:2 * n:2], x32[1:2 * n:2]
        return dict(ms_per_step=round(ms32, 3), solve_ms=round(s32["solve_ms"], 3),
                    setup_ms=round(s32["setup_ms"], 3),
                    linear_its_per_solve=round(s32["its_per_solve"], 2),
                    newton_its=s32["solves"], stage_ms_per_step=stage_summary(recs32),
                    rel_err_p=float(torch.linalg.norm(p32 - p64) / torch.linalg.norm(p64)),
                    rel_err_sw=float(torch.linalg.norm(s_32 - s_64) /
                                     max(float(torch.linalg.norm(s_64)), 1e-300)))
    out["fp32"] = None if args.no_fp32 else leg("fp32", fp32_leg)

    # ---- per-kernel timing and the roofline on the last state's first system
    def kernel_leg():
        J = r2p.Jacobian(model)
        J.assemble(x, x, dt_next)
        P = r2p.Cpr().setup(J, o64.cpr)
        v = torch.randn(model.N, dtype=torch.float64, device="cuda")
        y = torch.empty_like(v)
        fp = torch.randn(model.n, dtype=torch.float64, device="cuda")
        xp = torch.empty_like(fp)
        t_spmv = time_on_stream(lambda: J.spmv(v, y), 50)
        t_ras = time_on_stream(lambda: P.ras_apply(v, y), 20)
        t_amg = time_on_stream(lambda: P.amg_vcycle(fp, xp), 20)
        t_cpr = time_on_stream(lambda: P.apply(v, y), 20)
        rb, m_tot, nblk = ras_bytes(P, model, 8)
        sb = spmv_bytes(model)
        J.assemble(x, x, dt_next)
        Pv = r2p.Cpr().setup(J, r2p.cpr_opts(form=form, kcycle=0))
        t_v = time_on_stream(lambda: Pv.amg_vcycle(fp, xp), 20)
        vb = vcycle_bytes(Pv, model, 8)
        ras_gbs = rb / (t_ras * 1e-3) / 1e9
        spmv_gbs = sb / (t_spmv * 1e-3) / 1e9
        vcycle_gbs = vb / (t_v * 1e-3) / 1e9
        log(f"kernels: spmv {t_spmv * 1e3:.1f} us ({spmv_gbs:.0f} GB/s), ras {t_ras * 1e3:.1f} us "
            f"({ras_gbs:.0f} GB/s), K-cycle {t_amg * 1e3:.1f} us, V-cycle {t_v * 1e3:.1f} us "
            f"({vcycle_gbs:.0f} GB/s), cpr {t_cpr * 1e3:.1f} us")
        out.update({
            "kernels_us": {"spmv": round(t_spmv * 1e3, 2), "ras_apply": round(t_ras * 1e3, 2),
                           "amg_kcycle": round(t_amg * 1e3, 2), "amg_vcycle": round(t_v * 1e3, 2),
                           "cpr_apply": round(t_cpr * 1e3, 2)},
            "amg_levels": [g["n"] for g in P.amg_levels()],
            "spmv_gbs": round(spmv_gbs, 1), "spmv_hbm_frac": round(spmv_gbs / HBM_PEAK_GBS, 4),
            "vcycle_bytes": vb, "vcycle_gbs": round(vcycle_gbs, 1),
            "vcycle_hbm_frac": round(vcycle_gbs / HBM_PEAK_GBS, 4),
            "roofline": {"bound": "hbm",
                         "kernel": "ras_apply (k_ras_gather+k_ras_sweep+k_ras_scatter)",
                         "achieved": round(ras_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(ras_gbs / HBM_PEAK_GBS, 4), "traffic": ras_traffic(),
                         "bytes_per_launch": rb, "local_rows": m_tot, "offdiag_blocks": nblk}})
        return True
    leg("kernels", kernel_leg, required=True)

    # ---- fixed-snapshot solves at the 10-day step length
    out["snapshot_solves"] = leg("snapshots", lambda: snapshot_solves(
        model, [("cold start", x_init), (f"after {args.warmup} warm-up steps", x0),
                (f"after {args.warmup + args.steps} steps", x)], dt_max, form, log))

    # ---- why the controller stays below 10 days: one 10-day step from the
    # states the snapshots use
    def ten_day_leg():
        res = []
        for name, xs in (("cold start", x_init), (f"after {args.warmup + args.steps} steps", x)):
            xt = xs.clone()
            info = model.newton_step(xt, dt_max, o64)
            res.append({"state": name, "dt_days": dt_max, "status": info.status,
                        "newton_its": info.newton_its, "linear_its": info.linear_its,
                        "last_scaled_residual": info.res_hist[min(info.newton_its, 31)]})
        log(f"10-day attempts: {res}")
        return res
    out["ten_day_step_attempts"] = leg("ten_day", ten_day_leg)

    # ---- the oracle on the host
    def cpu_leg():
        c = cpu_baseline(w, s64["its_per_solve"], DT_INIT, args.cpu_sample_its)
        cpu_model, ncpu = host_cpu()
        c["sample"] += f"; host: {cpu_model}, {ncpu} logical CPUs, the oracle used 1"
        c["cpu_model"] = cpu_model
        c["host_cpus"] = ncpu
        return c
    out["cpu_baseline"] = None if args.no_cpu_baseline else leg("cpu_baseline", cpu_leg)

    # ---- inexact Newton with Eisenstat-Walker forcing on the timed steps' lengths
    def ew_leg():
        oew = r2p.newton_opts(cpr=r2p.cpr_opts(form=form), forcing=r2p.FORCING_EW)
        xe = x0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, recs_ew = run_steps(model, xe, dt, args.steps, oew, dt_max, "fp64+EW", dts=accepted)
        torch.cuda.synchronize()
        ms_ew = (time.perf_counter() - t0) * 1e3 / args.steps
        sew = summarise(recs_ew)
        p64, s_64 = x[0:2 * n:2], x[1:2 * n:2]
        pe, se = xe[0:2 * n:2], xe[1:2 * n:2]
        return dict(ms_per_step=round(ms_ew, 3), newton_its=sew["solves"],
                    linear_its=sew["linear_its"],
                    linear_its_per_solve=round(sew["its_per_solve"], 2),
                    plain_newton_its=s64["solves"], plain_linear_its=s64["linear_its"],
                    step_failures=sum(1 for r in recs_ew if r["status"] != 0),
                    rel_err_p=float(torch.linalg.norm(pe - p64) / torch.linalg.norm(p64)),
                    rel_err_sw=float(torch.linalg.norm(se - s_64) /
                                     max(float(torch.linalg.norm(s_64)), 1e-300)))
    out["inexact_newton_ew"] = None if args.no_variants else leg("ew", ew_leg)

    # ---- Krylov methods and the method variants on the last Newton system
    def krylov_leg():
        res = {}
        for name, method, kc in (("fgmres", r2p.KRYLOV_FGMRES, 1),
                                 ("fgmres_vcycle", r2p.KRYLOV_FGMRES, 0),
                                 ("bicgstab_vcycle", r2p.KRYLOV_BICGSTAB, 0)):
            J = r2p.Jacobian(model)
            bd = J.assemble(x, x, dt_next)
            P = r2p.Cpr().setup(J, r2p.cpr_opts(form=form, kcycle=kc))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = r2p.solve(J, P, bd, r2p.solve_opts(method=method))
            torch.cuda.synchronize()
            res[name] = {"ms": round((time.perf_counter() - t0) * 1e3, 3),
                         "iterations": info.iterations, "relres": info.relres,
                         "status": info.status}
        log(f"krylov on the last system: {res}")
        return res
    out["krylov_last_system"] = None if args.no_variants else leg("krylov", krylov_leg)
    out["variants_last_system"] = None if args.no_variants else leg(
        "variants", lambda: variants_run(model, x, dt_next, form))

    # ---- FP32 preconditioner + learned warm start
    out["fp32_learned"] = None
    if not args.no_learned and not args.no_fp32:
        out["fp32_learned"] = leg("learned", lambda: learned_run(args, model, x0, x, accepted,
                                                                 form, log))
    out["wall_s"] = round(time.perf_counter() - T0, 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
