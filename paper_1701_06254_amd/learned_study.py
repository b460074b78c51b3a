"""Learned warm start on the 200x200x50 correlated-permeability family.

Training data: seeded runs of 200x200x50 models with new permeability
fields (seeds from 1000), each from its cold start through the step-length
controller of the benchmark (0.1 d doubling up to the model's 10 d, halved
on a failed Newton step), in FP64.  Every accepted step gives one (state,
increment) pair: the network input of the state at the start of the step
and the normalised increment to the converged state.  Each pair is kept as
`crops` random 48x48 (x-y) windows over all 50 layers, the network's
receptive field being 21 cells.  The network (conv 6 -> 32, 4 residual
blocks, conv 32 -> 2, BF16 weights and activations, FP32 accumulation and
master weights) is trained by Adam with the library's own forward and
backward kernels.

Evaluation: held-out seeds (from 9000), each run from its cold start
through the controller without the network, then the same step lengths
replayed with the network's prediction offered as the first Newton iterate
under the library's rules (the scaled-residual rule, and the try rule), and
again with only its water saturation offered (pressure and well unknowns
from x^n); Newton and linear iterations and wall time are reported per form.

Usage: python -m paper_1701_06254_amd.learned_study [--train-seeds 8]
[--steps 12] [--crops 52] [--eval-seeds 10] [--iters 6000] [--out FILE.json]
[--weights FILE.npy].  The defaults give about 5,000 training crops (96
increments of 8 runs, 52 crops each) and evaluate on seeds 9000-9009.  Only the C ABI does arithmetic; this script moves
tensors and records results.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

CROP = 48


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def controller_steps(model, x, nsteps, opts, dt0=0.1, dt_max=10.0, grow_its=6, on_step=None):
    """nsteps accepted steps of the benchmark's controller from x (in place);
    on_step(x_old, dt) is called before each attempt and its result kept
    for accepted steps.  Returns (records, kept)."""
    recs, kept = [], []
    dt = dt0
    for _ in range(nsteps):
        while True:
            x_old = x.clone()
            extra = on_step(x_old, dt) if on_step else None
            info = model.newton_step(x, dt, opts)
            recs.append(dict(dt=dt, status=info.status, newton=info.newton_its,
                             linear=info.linear_its, ms=info.ms_total))
            if info.status == 0:
                kept.append((x_old, x.clone(), dt, extra))
                break
            dt *= 0.5
        if info.newton_its <= grow_its:
            dt = min(2.0 * dt, dt_max)
    return recs, kept


def collect(seeds, nsteps, crops, opts, rng):
    """Training crops (feature tensor [crops,50,48,48,32] bf16, target
    [crops*50*48*48, 2] fp32) from controller runs of the given seeds."""
    import torch
    import workloads
    from . import r2p
    data = []
    for seed in seeds:
        w = workloads.make_gaussian(seed=seed)
        m = r2p.Model(w)
        x = m.initial_state()
        g = w["grid"]
        nz, ny, nx = g["nz"], g["ny"], g["nx"]
        t0 = time.perf_counter()
        recs, kept = controller_steps(m, x, nsteps, opts,
                                      on_step=lambda xo, dt: r2p.cnn_features(m, xo, dt))
        for x_old, x_new, dt, feat in kept:
            tgt = r2p.cnn_targets(m, x_old, x_new)
            f4 = feat.view(nz, ny, nx, 32)
            t4 = tgt.view(nz, ny, nx, 2)
            for _ in range(crops):
                y0 = int(rng.integers(0, ny - CROP + 1))
                x0 = int(rng.integers(0, nx - CROP + 1))
                data.append((f4[:, y0:y0 + CROP, x0:x0 + CROP, :].contiguous().view(-1, 32),
                             t4[:, y0:y0 + CROP, x0:x0 + CROP, :].contiguous().view(-1, 2),
                             dt))
        torch.cuda.synchronize()
        log(f"train seed {seed}: {len(kept)} steps (dt {[round(k[2], 3) for k in kept]}) in "
            f"{time.perf_counter() - t0:.1f} s")
        del m
    return data


def evaluate(net, seeds, nsteps, opts, rules):
    """Plain controller run, then replays of its accepted step lengths with
    the network's first iterate under each rule.  A rule is (name, guess
    rule, part): part "full" offers the network's iterate, "sw" offers x^n
    with only the water saturation of the network's iterate."""
    import torch
    import workloads
    from . import r2p
    out = []
    for seed in seeds:
        w = workloads.make_gaussian(seed=seed)
        m = r2p.Model(w)
        x0 = m.initial_state()
        x = x0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        recs, kept = controller_steps(m, x, nsteps, opts)
        torch.cuda.synchronize()
        plain_s = time.perf_counter() - t0
        dts = [k[2] for k in kept]
        row = {"seed": seed, "dts": dts,
               "plain": {"newton": sum(r["newton"] for r in recs),
                         "linear": sum(r["linear"] for r in recs),
                         "failed_steps": sum(1 for r in recs if r["status"] != 0),
                         "s": round(plain_s, 2)}}
        n = m.n
        for name, rule, part in rules:
            o = r2p.newton_opts(cpr=opts.cpr, lin=opts.lin, guess_rule=rule)
            xl = x0.clone()
            nt = lt = taken = fails = 0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for dt in dts:
                guess = net.warm_start(m, xl, dt)
                if part == "sw":
                    g = xl.clone()
                    g[1:2 * n:2] = guess[1:2 * n:2]
                    guess = g
                info = m.newton_step(xl, dt, o, x_guess=guess)
                nt += info.newton_its
                lt += info.linear_its
                taken += info.used_guess
                if info.status != 0:
                    fails += 1
                    break
            torch.cuda.synchronize()
            s = time.perf_counter() - t0
            dp = float(torch.linalg.norm(xl[0:2 * n:2] - x[0:2 * n:2]) /
                       torch.linalg.norm(x[0:2 * n:2]))
            ds = float(torch.linalg.norm(xl[1:2 * n:2] - x[1:2 * n:2]) /
                       max(float(torch.linalg.norm(x[1:2 * n:2])), 1e-300))
            row[name] = {"newton": nt, "linear": lt, "guess_taken": taken, "failed": fails,
                         "s": round(s, 2), "rel_diff_p": dp, "rel_diff_sw": ds}
        log(f"eval seed {seed}: {row}")
        out.append(row)
        del m
    return out


def main(argv=None):
    import torch
    from . import r2p, warmstart
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-seeds", type=int, default=8)
    ap.add_argument("--eval-seeds", type=int, default=10)
    ap.add_argument("--steps", type=int, default=12)
    ap.add_argument("--crops", type=int, default=52)
    ap.add_argument("--iters", type=int, default=6000)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--out", default=None)
    ap.add_argument("--weights", default=None)
    args = ap.parse_args(argv)
    r2p.load()
    rng = np.random.default_rng(2024)
    opts = r2p.newton_opts()
    t0 = time.perf_counter()
    data = collect(range(1000, 1000 + args.train_seeds), args.steps, args.crops, opts, rng)
    t_data = time.perf_counter() - t0
    net = r2p.Cnn(blocks=4)
    net.set_params(warmstart.init_params(np.random.default_rng(7)))
    t1 = time.perf_counter()
    losses = warmstart.train(net, data, (50, CROP, CROP), args.iters, batch=args.batch,
                             lr=args.lr, seed=3, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    if args.weights:
        np.save(args.weights, net.get_params())
    rules = [("scaled_rule", r2p.GUESS_SCALED_INF, "full"), ("try_rule", r2p.GUESS_TRY, "full"),
             ("sw_scaled_rule", r2p.GUESS_SCALED_INF, "sw"), ("sw_try_rule", r2p.GUESS_TRY, "sw")]
    ev = evaluate(net, range(9000, 9000 + args.eval_seeds), args.steps, opts, rules)
    tot = {k: {"newton": sum(r[k]["newton"] for r in ev), "linear": sum(r[k]["linear"] for r in ev),
               "guess_taken": sum(r[k].get("guess_taken", 0) for r in ev),
               "s": round(sum(r[k]["s"] for r in ev), 2)}
           for k in ("plain",) + tuple(r[0] for r in rules)}
    res = {"train_seeds": [1000, 1000 + args.train_seeds - 1], "pairs": len(data) // args.crops,
           "crops": len(data), "crop": [50, CROP, CROP], "adam_steps": args.iters,
           "data_s": round(t_data, 1), "train_s": round(t_train, 1),
           "loss_first20": float(np.mean(losses[:20])), "loss_last20": float(np.mean(losses[-20:])),
           "eval_seeds": [9000, 9000 + args.eval_seeds - 1], "eval": ev, "totals": tot}
    line = json.dumps(res)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")
    print(line, flush=True)


if __name__ == "__main__":
    main()
