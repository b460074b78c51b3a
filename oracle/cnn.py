"""FP64 CPU reference of the learned warm start's 3D convolutional network.

TEST INFRASTRUCTURE ONLY: the slow, plain reference that the device network
kernels are checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; it shares no code with the
device library.

The network maps per-cell features of a reservoir state to a Newton-step
increment.  Arrays are channels-last, [batch, nz, ny, nx, C].  A 3x3x3
convolution with zero padding is

    out[v, co] = b[co] + sum_t sum_ci in[v + off_t, ci] * W[t, co, ci],

with taps t = 9 (dz + 1) + 3 (dy + 1) + (dx + 1), off_t = (dz, dy, dx), and
every crop of the batch padded on its own.  The network is

    h_0     = relu(conv(f, W_in, b_in))                       6 -> C
    a_k     = relu(conv(h_k, W_a,k, b_a,k))                   C -> C
    h_{k+1} = h_k + conv(a_k, W_b,k, b_b,k)      k = 0..K-1   C -> C
    out     = conv(h_K, W_out, b_out)                         C -> 2

and training minimises the mean squared error over voxels and both output
channels.  Parameters are one flat vector in the order W_in, b_in, then per
block W_a, b_a, W_b, b_b, then W_out, b_out; each W is [27, Cout, Cin].
"""
from __future__ import annotations

import numpy as np

NIN, NOUT = 6, 2


def taps():
    return [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def layer_shapes(C=32, K=4):
    """(name, W shape, b shape) of every layer in parameter order."""
    out = [("in", (27, C, NIN), (C,))]
    for k in range(K):
        out.append((f"a{k}", (27, C, C), (C,)))
        out.append((f"b{k}", (27, C, C), (C,)))
    out.append(("out", (27, NOUT, C), (NOUT,)))
    return out


def num_params(C=32, K=4):
    return sum(int(np.prod(w)) + int(np.prod(b)) for _, w, b in layer_shapes(C, K))


def unpack(theta, C=32, K=4):
    """Flat parameter vector -> dict name -> (W, b) views."""
    d, o = {}, 0
    for name, ws, bs in layer_shapes(C, K):
        nw, nb = int(np.prod(ws)), int(np.prod(bs))
        d[name] = (theta[o:o + nw].reshape(ws), theta[o + nw:o + nw + nb])
        o += nw + nb
    return d


def init_params(rng, C=32, K=4, out_scale=0.1):
    """He-normal weights (fan-in 27 Cin), zero biases; the last layer and the
    second convolution of every block scaled down so the initial network is
    close to a small perturbation of identity blocks."""
    parts = []
    for name, ws, bs in layer_shapes(C, K):
        std = np.sqrt(2.0 / (27 * ws[2]))
        if name.startswith("b") or name == "out":
            std *= out_scale
        parts.append(rng.normal(0.0, std, int(np.prod(ws))))
        parts.append(np.zeros(int(np.prod(bs))))
    return np.concatenate(parts)


def _pad(x):
    return np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))


def conv(x, W, b=None):
    """3x3x3 convolution, zero padding, channels-last, written as the sum
    over taps of a shifted matrix product."""
    B, nz, ny, nx, _ = x.shape
    xp = _pad(x)
    out = np.zeros((B, nz, ny, nx, W.shape[1]))
    for t, (dz, dy, dx) in enumerate(taps()):
        sl = xp[:, 1 + dz:1 + dz + nz, 1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx, :]
        out += sl @ W[t].T
    if b is not None:
        out += b
    return out


def conv_grad_input(g, W):
    """d(sum g * conv(x, W)) / dx: the transposed convolution."""
    B, nz, ny, nx, _ = g.shape
    gp = _pad(g)
    out = np.zeros((B, nz, ny, nx, W.shape[2]))
    for t, (dz, dy, dx) in enumerate(taps()):
        sl = gp[:, 1 - dz:1 - dz + nz, 1 - dy:1 - dy + ny, 1 - dx:1 - dx + nx, :]
        out += sl @ W[t]
    return out


def conv_grad_weight(g, x):
    """d(sum g * conv(x, W)) / dW, shape [27, Cout, Cin], and d/db."""
    B, nz, ny, nx, _ = x.shape
    xp = _pad(x)
    gf = g.reshape(-1, g.shape[-1])
    dW = np.zeros((27, g.shape[-1], x.shape[-1]))
    for t, (dz, dy, dx) in enumerate(taps()):
        sl = xp[:, 1 + dz:1 + dz + nz, 1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx, :]
        dW[t] = gf.T @ sl.reshape(-1, x.shape[-1])
    return dW, gf.sum(axis=0)


def relu(x):
    return np.maximum(x, 0.0)


def forward(theta, f, C=32, K=4):
    """Network output and the activations the backward pass needs."""
    P = unpack(theta, C, K)
    h = relu(conv(f, *P["in"]))
    acts = {"f": f, "h0": h}
    for k in range(K):
        a = relu(conv(h, *P[f"a{k}"]))
        h = h + conv(a, *P[f"b{k}"])
        acts[f"a{k}"] = a
        acts[f"h{k + 1}"] = h
    out = conv(h, *P["out"])
    return out, acts


def loss(out, target):
    return float(np.mean((out - target) ** 2))


def backward(theta, acts, out, target, C=32, K=4):
    """Gradient of the mean squared error with respect to the flat parameters."""
    P = unpack(theta, C, K)
    grads = {}
    g = 2.0 * (out - target) / out.size
    grads["out"] = conv_grad_weight(g, acts[f"h{K}"])
    gh = conv_grad_input(g, P["out"][0])
    for k in reversed(range(K)):
        a, h = acts[f"a{k}"], acts[f"h{k}"]
        grads[f"b{k}"] = conv_grad_weight(gh, a)
        ga = conv_grad_input(gh, P[f"b{k}"][0]) * (a > 0)
        grads[f"a{k}"] = conv_grad_weight(ga, h)
        gh = gh + conv_grad_input(ga, P[f"a{k}"][0])
    g0 = gh * (acts["h0"] > 0)
    grads["in"] = conv_grad_weight(g0, acts["f"])
    parts = []
    for name, _, _ in layer_shapes(C, K):
        dW, db = grads[name]
        parts.append(dW.ravel())
        parts.append(db.ravel())
    return np.concatenate(parts)


def forward_bf16(theta, f, C=32, K=4):
    """The network with activations stored in bfloat16, as the extension
    specifies (BF16 weights and activations, FP32 accumulation): every
    hidden layer's result, after its bias, residual addend and ReLU, is
    rounded to the nearest bfloat16; the output layer is not.  Sums are in
    FP64 here, so each rounding sees its exact argument."""
    P = unpack(theta, C, K)
    h = bf16_round(relu(conv(f, *P["in"])))
    acts = {"f": f, "h0": h}
    for k in range(K):
        a = bf16_round(relu(conv(h, *P[f"a{k}"])))
        h = bf16_round(conv(a, *P[f"b{k}"]) + h)
        acts[f"a{k}"] = a
        acts[f"h{k + 1}"] = h
    out = conv(h, *P["out"])
    return out, acts


def backward_bf16(theta, acts, out, target, C=32, K=4):
    """Gradient of the mean squared error with the back-propagated signals
    stored in bfloat16 like the activations: the output gradient, and after
    every transposed convolution (with its ReLU mask or residual addend) the
    input gradient; weight and bias gradients are sums of products of those
    bfloat16 values, not rounded."""
    P = unpack(theta, C, K)
    grads = {}
    g = bf16_round(2.0 * (out - target) / out.size)
    grads["out"] = conv_grad_weight(g, acts[f"h{K}"])
    gh = bf16_round(conv_grad_input(g, P["out"][0]))
    for k in reversed(range(K)):
        a, h = acts[f"a{k}"], acts[f"h{k}"]
        grads[f"b{k}"] = conv_grad_weight(gh, a)
        ga = bf16_round(conv_grad_input(gh, P[f"b{k}"][0]) * (a > 0))
        grads[f"a{k}"] = conv_grad_weight(ga, h)
        gh = bf16_round(gh + conv_grad_input(ga, P[f"a{k}"][0]))
    g0 = gh * (acts["h0"] > 0)
    grads["in"] = conv_grad_weight(g0, acts["f"])
    parts = []
    for name, _, _ in layer_shapes(C, K):
        dW, db = grads[name]
        parts.append(dW.ravel())
        parts.append(db.ravel())
    return np.concatenate(parts)


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
