"""Pins of the CPU reference of the warm-start network (oracle/cnn.py).

The convolution is checked against its definition written as plain loops;
the backward pass against central finite differences of the loss; the
bfloat16 rounding against hand-computed bit patterns.
"""
import numpy as np
import pytest

from oracle import cnn


def conv_loops(x, W, b):
    B, nz, ny, nx, ci = x.shape
    co = W.shape[1]
    out = np.zeros((B, nz, ny, nx, co))
    for n in range(B):
        for z in range(nz):
            for y in range(ny):
                for xx in range(nx):
                    for t, (dz, dy, dx) in enumerate(cnn.taps()):
                        zz, yy, x2 = z + dz, y + dy, xx + dx
                        if 0 <= zz < nz and 0 <= yy < ny and 0 <= x2 < nx:
                            out[n, z, y, xx] += W[t] @ x[n, zz, yy, x2]
                    out[n, z, y, xx] += b
    return out


def test_conv_matches_loop_definition():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 3, 4, 5, 3))
    W = rng.normal(size=(27, 4, 3))
    b = rng.normal(size=4)
    assert np.allclose(cnn.conv(x, W, b), conv_loops(x, W, b), rtol=1e-13, atol=1e-12)


def test_conv_input_gradient_is_adjoint():
    # <g, conv(x)> = <conv_grad_input(g), x> for the bias-free convolution
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 3, 4, 5, 3))
    g = rng.normal(size=(2, 3, 4, 5, 4))
    W = rng.normal(size=(27, 4, 3))
    lhs = np.sum(g * cnn.conv(x, W))
    rhs = np.sum(cnn.conv_grad_input(g, W) * x)
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_network_gradient_matches_finite_differences():
    C, K = 4, 2
    rng = np.random.default_rng(2)
    theta = cnn.init_params(rng, C, K, out_scale=1.0)
    theta += rng.normal(0, 0.01, theta.size)          # nonzero biases
    f = rng.normal(size=(2, 3, 4, 5, cnn.NIN))
    target = rng.normal(size=(2, 3, 4, 5, cnn.NOUT))
    out, acts = cnn.forward(theta, f, C, K)
    g = cnn.backward(theta, acts, out, target, C, K)
    idx = rng.choice(theta.size, 40, replace=False)
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        lp = cnn.loss(cnn.forward(tp, f, C, K)[0], target)
        lm = cnn.loss(cnn.forward(tm, f, C, K)[0], target)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_parameter_count_of_the_default_network():
    # 6->32, four blocks of two 32->32 convolutions, 32->2, 3x3x3 taps, biases
    assert cnn.num_params() == 27 * 32 * 6 + 32 + 4 * 2 * (27 * 32 * 32 + 32) + 27 * 2 * 32 + 2


@pytest.mark.parametrize("v, bits", [(1.0, 0x3F80), (-2.5, 0xC020), (1.00390625, 0x3F80),
                                     (1.01171875, 0x3F82), (3.0e38, 0x7F62)])
def test_bf16_rounding(v, bits):
    # 1 + 2^-8 is a tie between 0x3F80 and 0x3F81: to even; 1 + 3*2^-8 ties up to 0x3F82
    r = cnn.bf16_round(np.array([v]))
    u = np.float32(r[0]).view(np.uint32) >> 16
    assert int(u) == bits


def test_bf16_network_reduces_to_the_fp64_network():
    """forward_bf16 / backward_bf16 differ from the FP64 network only by the
    bfloat16 roundings: with every value already representable (rounding is
    then the identity on them) the two agree, and in general they differ by
    about one rounding (2^-8 relative) per layer."""
    from oracle import cnn
    rng = np.random.default_rng(5)
    K = 1
    theta = cnn.bf16_round(cnn.init_params(rng, 8, K, out_scale=1.0))
    f = cnn.bf16_round(rng.normal(size=(1, 3, 4, 5, cnn.NIN)))
    tgt = rng.normal(size=(1, 3, 4, 5, cnn.NOUT))
    o64, a64 = cnn.forward(theta, f, 8, K)
    o16, a16 = cnn.forward_bf16(theta, f, 8, K)
    for k in a16:
        assert np.array_equal(cnn.bf16_round(a16[k]), a16[k])       # stored as bfloat16
    rel = np.linalg.norm(o16 - o64) / np.linalg.norm(o64)
    assert 0 < rel < 2 ** -6
    g64 = cnn.backward(theta, a64, o64, tgt, 8, K)
    g16 = cnn.backward_bf16(theta, a16, o16, tgt, 8, K)
    assert np.linalg.norm(g16 - g64) / np.linalg.norm(g64) < 2 ** -5
