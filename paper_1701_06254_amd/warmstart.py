"""Learned warm start: data collection and training loop around the C ABI.

The network and every arithmetic step (features, targets, forward, backward,
Adam) run in libr2p's kernels; this module only strings the calls together:
it runs implicit steps to collect (features at x^n, increment x^{n+1} - x^n)
pairs, draws minibatches, and calls backward / sgd_step.
"""
from __future__ import annotations

import numpy as np

from . import r2p


def init_params(rng, blocks=4, channels=32, out_scale=0.1):
    """Initial compact parameter vector (layer order of r2p_cnn_set_params):
    He-normal weights (fan-in 27 cin), zero biases; the second convolution of
    every block and the output layer scaled by out_scale so that training
    starts near identity blocks and a small output."""
    parts = []
    dims = [(6, channels)] + [(channels, channels)] * (2 * blocks) + [(channels, 2)]
    for l, (cin, cout) in enumerate(dims):
        std = np.sqrt(2.0 / (27 * cin))
        if l == len(dims) - 1 or (l > 0 and l % 2 == 0):
            std *= out_scale
        parts.append(rng.normal(0.0, std, 27 * cout * cin))
        parts.append(np.zeros(cout))
    return np.concatenate(parts).astype(np.float32)


def collect_pairs(model, x, dts, opts, pairs=None):
    """Run one implicit step per entry of dts from state x (in place) and
    append (features, target, dt) device tensors of every accepted step."""
    pairs = [] if pairs is None else pairs
    infos = []
    for dt in dts:
        x_old = x.clone()
        feat = r2p.cnn_features(model, x, dt)
        info = model.newton_step(x, dt, opts)
        infos.append(info)
        if info.status != 0:
            break
        pairs.append((feat, r2p.cnn_targets(model, x_old, x), dt))
    return pairs, infos


def train(net, pairs, shape, iters, batch, lr, seed=0, log=None):
    """Adam on minibatches of `batch` pairs drawn uniformly (seeded); each
    pair is one crop of the given (nz, ny, nx) shape.  Returns the losses."""
    import torch
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    losses = []
    for it in range(iters):
        idx = rng.choice(len(pairs), size=min(batch, len(pairs)), replace=False)
        feat = torch.cat([pairs[i][0] for i in idx])
        tgt = torch.cat([pairs[i][1] for i in idx])
        losses.append(net.backward(feat, tgt, (len(idx), nz, ny, nx)))
        net.step(lr)
        if log and (it % 100 == 0 or it == iters - 1):
            log(f"train {it}: loss {losses[-1]:.4e}")
    return losses


def run_steps(model, x, dts, opts, net=None):
    """Implicit steps from x (in place); with `net` every step is offered the
    network's first iterate.  Returns the Newton records."""
    infos = []
    for dt in dts:
        guess = net.warm_start(model, x, dt) if net is not None else None
        info = model.newton_step(x, dt, opts, x_guess=guess)
        infos.append(info)
        if info.status != 0:
            break
    return infos
