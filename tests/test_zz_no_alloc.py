"""The allocation-free scaled norm (r2p_residual_norm_noalloc) against
r2p_residual_norm, through the C ABI: two calls in a row, the second on a
smaller model, each equal bit for bit; a non-finite entry gives NaN."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def test_residual_norm_noalloc_matches():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1701_06254_amd import r2p
    r2p.load()
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    for w, dt in ((workloads.make_config(1), 0.1), (workloads.make_small(), 10.0)):
        m = r2p.Model(w)
        x = m.initial_state()
        xs = workloads.random_state(w, np.random.default_rng(3))
        xr = torch.as_tensor(xs, device="cuda")
        J = r2p.Jacobian(m)
        for state in (x, xr):
            b = J.assemble(state, x, dt)
            ref = m.residual_norm(b, dt)
            out.fill_(-1.0)
            m.residual_norm_noalloc(b, dt, out)
            torch.cuda.synchronize()
            got = float(out.cpu()[0])
            print(f"{w['name']}: {ref!r} {got!r}")
            assert np.float64(got).tobytes() == np.float64(ref).tobytes()
        b[7] = float("nan")
        m.residual_norm_noalloc(b, dt, out)
        torch.cuda.synchronize()
        assert np.isnan(float(out.cpu()[0]))
        del J, m
