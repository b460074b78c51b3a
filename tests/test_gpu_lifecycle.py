"""Handles across model lifetimes.

Each model owns its Newton workspace (Jacobian, CPR, vectors), and the
structures a CPR handle caches between set-ups are keyed by a per-process
model serial, not by an address: a model created after another was destroyed
may occupy the destroyed one's host address and still be another model, with
other sizes.  Models of different sizes are created, stepped and destroyed in
turn, and one CPR handle is set up on two models in turn; every result is
checked against the oracle's residual or the solve's true residual.
"""
import gc

import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def libs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    from paper_1701_06254_amd import r2p
    oracle.build(force=False)
    r2p.load()
    return r2p, oracle


def test_newton_steps_on_models_created_in_turn(libs):
    r2p, oracle = libs
    dt = 1.0
    for w in (workloads.make_small(), workloads.make_tiny(), workloads.make_small()):
        m = r2p.Model(w)
        x = m.initial_state()
        x0 = x.cpu().numpy()
        info = m.newton_step(x, dt)
        assert info.status == 0, w["name"]
        mo = oracle.Model(w)
        assert mo.scaled_norm(mo.residual(x.cpu().numpy(), x0, dt), dt) <= 1.01e-8, w["name"]
        del m, x
        gc.collect()


def test_one_cpr_handle_on_two_models(libs):
    r2p, _ = libs
    P = r2p.Cpr()
    for w in (workloads.make_small(), workloads.make_tiny()):
        m = r2p.Model(w)
        x = m.initial_state()
        J = r2p.Jacobian(m)
        b = J.assemble(x, x, 1.0)
        P.setup(J, r2p.cpr_opts())
        _, info = r2p.solve(J, P, b)
        assert info.status == 0 and info.relres <= 1e-8, w["name"]
        del J, m
        gc.collect()


def test_model_destroy_releases_device_memory(libs):
    """Each model's Newton workspace, including the Krylov basis of its CPR
    handle, is freed with the model: after a 2M-cell step (about 2 GB of
    FGMRES(30) basis) and the model's destruction, device memory in use
    returns to its level before the model was created."""
    import torch
    r2p, _ = libs
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free0, _ = torch.cuda.mem_get_info()
    w = workloads.make_config(1)
    m = r2p.Model(w)
    x = m.initial_state()
    info = m.newton_step(x, 0.1)
    assert info.status == 0
    free1, _ = torch.cuda.mem_get_info()
    assert free0 - free1 > 2 * 2 ** 30               # the step's workspace was there
    del m, x
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free2, _ = torch.cuda.mem_get_info()
    assert free0 - free2 <= 64 * 2 ** 20, (free0 - free2) / 2 ** 20
