"""Parity of the warm-start network kernels (BF16 operands, FP32 accumulation)
against the FP64 CPU reference in oracle/cnn.py, evaluated on the same
BF16-rounded inputs, and the effect of the trained network on Newton.

Tolerances: a layer's FP32 result against the FP64 reference within 1e-5 of
the largest magnitude (FP32 accumulation of 864 products); BF16 results
within one BF16 rounding (2^-7 relative, plus the FP32 error); the
end-to-end gradient, whose activations are rounded to BF16 at every layer,
within 5% in relative 2-norm.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    from paper_1701_06254_amd import r2p
    r2p.load()
    return r2p


def bf16_bits(a):
    """float array -> (int16 bit patterns on the GPU, float64 rounded values)."""
    from oracle import cnn
    r = cnn.bf16_round(a)
    bits = (np.asarray(r, dtype=np.float32).view(np.uint32) >> 16).astype(np.uint16)
    return torch.from_numpy(bits.view(np.int16).copy()).cuda(), r


def from_bits(t):
    u = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


SHAPES = [(2, 3, 5, 7), (2, 8, 16, 20), (1, 5, 9, 70)]


@pytest.mark.parametrize("shape", SHAPES)
def test_conv_forward_matches_reference(shape):
    from oracle import cnn
    r2p = _dev()
    rng = np.random.default_rng(7)
    nb, nz, ny, nx = shape
    x_t, x = bf16_bits(rng.normal(size=(nb, nz, ny, nx, 32)))
    w_t, W = bf16_bits(rng.normal(0, 0.05, size=(27, 32, 32)))
    b = rng.normal(size=32).astype(np.float32)
    bias = torch.from_numpy(b).cuda()
    V = nb * nz * ny * nx
    outf = torch.empty(V * 32, dtype=torch.float32, device="cuda")
    r2p.cnn_conv(x_t, shape, w_t, bias=bias, outf=outf)
    torch.cuda.synchronize()
    ref = cnn.conv(x, W, b.astype(np.float64)).reshape(-1)
    got = outf.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref))
    # epilogue: + addend, ReLU, BF16 result
    a_t, A = bf16_bits(rng.normal(size=(nb, nz, ny, nx, 32)))
    out = torch.empty(V * 32, dtype=torch.int16, device="cuda")
    r2p.cnn_conv(x_t, shape, w_t, bias=bias, addend=a_t, relu=True, out=out)
    torch.cuda.synchronize()
    ref2 = np.maximum(ref + A.reshape(-1), 0.0)
    got2 = from_bits(out)
    scale = np.max(np.abs(ref2))
    assert np.all(np.abs(got2 - ref2) <= 2.0 ** -8 * np.abs(ref2) + 2e-5 * scale)


@pytest.mark.parametrize("shape", SHAPES)
def test_conv_input_gradient_matches_reference(shape):
    from oracle import cnn
    r2p = _dev()
    rng = np.random.default_rng(8)
    nb, nz, ny, nx = shape
    g_t, g = bf16_bits(rng.normal(size=(nb, nz, ny, nx, 32)))
    W = cnn.bf16_round(rng.normal(0, 0.05, size=(27, 32, 32)))
    wt_t, _ = bf16_bits(np.ascontiguousarray(W.transpose(0, 2, 1)))
    m_t, M = bf16_bits(rng.normal(size=(nb, nz, ny, nx, 32)))
    V = nb * nz * ny * nx
    outf = torch.empty(V * 32, dtype=torch.float32, device="cuda")
    r2p.cnn_conv(g_t, shape, wt_t, mask=m_t, flip=True, outf=outf)
    torch.cuda.synchronize()
    ref = (cnn.conv_grad_input(g, W) * (M > 0)).reshape(-1)
    got = outf.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref))


@pytest.mark.parametrize("shape", SHAPES)
def test_conv_weight_gradient_matches_reference(shape):
    from oracle import cnn
    r2p = _dev()
    rng = np.random.default_rng(9)
    nb, nz, ny, nx = shape
    g_t, g = bf16_bits(rng.normal(size=(nb, nz, ny, nx, 32)))
    x_t, x = bf16_bits(rng.normal(size=(nb, nz, ny, nx, 32)))
    dw = torch.empty(27 * 32 * 32, dtype=torch.float32, device="cuda")
    db = torch.empty(32, dtype=torch.float32, device="cuda")
    r2p.cnn_conv_dw(g_t, x_t, shape, dw, db)
    rdw, rdb = cnn.conv_grad_weight(g, x)
    got = dw.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - rdw.reshape(-1))) <= 1e-5 * np.max(np.abs(rdw))
    assert np.max(np.abs(db.cpu().numpy() - rdb)) <= 1e-5 * np.max(np.abs(rdb))


def _net_case(K, shape, seed):
    from oracle import cnn
    rng = np.random.default_rng(seed)
    theta = cnn.init_params(rng, 32, K, out_scale=1.0)
    theta += rng.normal(0, 0.02, theta.size)
    theta = cnn.bf16_round(theta)                        # weights exactly representable
    nb, nz, ny, nx = shape
    f = np.zeros((nb, nz, ny, nx, 32))
    f[..., :cnn.NIN] = rng.normal(size=(nb, nz, ny, nx, cnn.NIN))
    f_t, f = bf16_bits(f)
    tgt = rng.normal(size=(nb, nz, ny, nx, cnn.NOUT))
    return theta, f_t, f[..., :cnn.NIN], tgt


def test_network_forward_and_gradient_match_reference():
    """The whole network against the reference with the device's bfloat16
    rounding points (forward_bf16 / backward_bf16: activations and
    back-propagated signals stored in bfloat16).  The two differ only where
    an FP32 accumulation and the exact sum fall on opposite sides of a
    bfloat16 rounding boundary: about 1e-4 of the elements, each by one
    rounding (2^-8), so the relative 2-norm difference stays near 1e-4;
    bound 1e-3 for the output, the loss and the parameter gradient."""
    from oracle import cnn
    r2p = _dev()
    K, shape = 1, (1, 4, 6, 8)
    theta, f_t, f, tgt = _net_case(K, shape, 11)
    net = r2p.Cnn(blocks=K)
    net.set_params(theta.astype(np.float32))
    out = net.forward(f_t, shape)
    torch.cuda.synchronize()
    ref_out, acts = cnn.forward_bf16(theta, f, 32, K)
    got = out.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(got - ref_out.reshape(-1)) / np.linalg.norm(ref_out)
    print(f"network output: relative difference {rel:.2e}")
    assert rel < 1e-3, rel
    tgt_t = torch.from_numpy(tgt.reshape(-1).astype(np.float32)).cuda()
    loss = net.backward(f_t, tgt_t, shape)
    ref_loss = cnn.loss(ref_out, tgt)
    assert abs(loss - ref_loss) <= 1e-3 * ref_loss
    g = net.get_grads().astype(np.float64)
    rg = cnn.backward_bf16(theta, acts, ref_out, tgt, 32, K)
    rel_g = np.linalg.norm(g - rg) / np.linalg.norm(rg)
    print(f"network gradient: relative difference {rel_g:.2e}")
    assert rel_g < 1e-3, rel_g


def test_training_lowers_the_loss():
    from oracle import cnn
    r2p = _dev()
    K, shape = 2, (2, 6, 8, 8)
    theta, f_t, f, _ = _net_case(K, shape, 12)
    # a learnable target: a smooth function of the features
    tgt = np.stack([np.tanh(f[..., 0] + 0.5 * f[..., 1]), 0.3 * f[..., 2]], axis=-1)
    tgt_t = torch.from_numpy(tgt.reshape(-1).astype(np.float32)).cuda()
    net = r2p.Cnn(blocks=K)
    net.set_params(cnn.init_params(np.random.default_rng(3), 32, K).astype(np.float32))
    first = net.backward(f_t, tgt_t, shape)
    for _ in range(60):
        net.backward(f_t, tgt_t, shape)
        net.step(2e-3)
    last = net.backward(f_t, tgt_t, shape)
    assert last < 0.5 * first, (first, last)
