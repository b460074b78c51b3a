"""The 640x640x160 channelised model (65,536,000 cells, 400 wells) on one GPU:
the library's whole path at the largest configured size, with every array of
the Newton step (Jacobian planes, BILU(0) factors of 16 subdomains of about
4.2 M rows, the AMG hierarchy, the FGMRES(30) basis) resident in HBM.

The oracle's Jacobian and CPR set-up at this size do not fit a test, so the
checks are properties that hold at any size, each against the oracle's own
residual: the assembled right-hand side equals the oracle's -F in full, and
one implicit step (dt 0.1 day from the hydrostatic start) in the FP64 and in
the FP32-preconditioner form converges to the oracle's scaled residual
tolerance at the device's new state, with the two forms' fields within 1e-6
(relative 2-norm) of each other.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

DT = 0.1


def _t(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def _h(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def large():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    from paper_1701_06254_amd import r2p
    oracle.build(force=False)
    r2p.load()
    w = workloads.make_config(4)
    mo = oracle.Model(w)
    x0 = mo.initial_state()
    mg = r2p.Model(w)
    return dict(w=w, mo=mo, x0=x0, mg=mg, dev=r2p)


def test_large_initial_state_and_residual(large):
    dev, mo, mg, x0 = large["dev"], large["mo"], large["mg"], large["x0"]
    assert mg.n == 65_536_000 and mg.nw == 400
    xi = _h(mg.initial_state())
    assert np.abs(xi - x0).max() <= 1e-12 * np.abs(x0).max()
    J = dev.Jacobian(mg)
    b = _h(J.assemble(_t(x0), _t(x0), DT))
    del J
    F = mo.residual(x0, x0, DT)
    assert np.abs(b + F).max() <= 1e-12 * np.abs(F).max()


def test_large_newton_step_fp64_and_fp32(large):
    dev, mo, mg, x0 = large["dev"], large["mo"], large["mg"], large["x0"]
    n = mg.n
    out = {}
    for name, prec in (("fp64", dev.FP64), ("fp32", dev.FP32)):
        x = _t(x0)
        info = mg.newton_step(x, DT, dev.newton_opts(cpr=dev.cpr_opts(precision=prec)))
        assert info.status == 0, name
        x1 = _h(x)
        del x
        nrm = mo.scaled_norm(mo.residual(x1, x0, DT), DT)
        print(f"65.5M cells, {name}: {info.newton_its} Newton, {info.linear_its} linear "
              f"iterations, {info.ms_total:.0f} ms, oracle scaled residual {nrm:.2e}")
        assert nrm <= 1.01e-8, name
        sw = x1[1:2 * n:2]
        assert np.all(np.isfinite(x1)) and sw.min() >= -1e-12 and sw.max() <= 1 + 1e-12
        out[name] = x1
    a, c = out["fp64"], out["fp32"]
    for k in (0, 1):
        ref = a[k:2 * n:2]
        assert np.linalg.norm(c[k:2 * n:2] - ref) <= 1e-6 * np.linalg.norm(ref)
