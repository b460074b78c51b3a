"""Parity at the benchmark's own size: the 200x200x50 (2M-cell, 25-well)
correlated-permeability model, through the same library calls and launch
configuration the benchmark times.

The oracle builds the same Jacobian (about a second), the same CPR set-up
(a few seconds) and applies it once per call, so the assembled system, the
residual, SpMV, AMG V-cycle, RAS and CPR applications are compared in full.
A whole oracle Newton step at this size takes minutes, so the step is
checked by properties that hold at any size: the linear solve's true
relative residual, computed with the oracle's decoupled matrix, and the
oracle's scaled residual at the device's new state.  Tolerances as in the
small-case parity tests.
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
def big():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    from paper_1701_06254_amd import r2p
    oracle.build(force=False)
    r2p.load()
    w = workloads.make_config(1)
    mo = oracle.Model(w)
    x0 = mo.initial_state()
    # a second state with a rough potential field: seeded, from the generator
    x1 = workloads.random_state(w, np.random.default_rng(21))
    # a third shaped like a later one: pressure mounds and sinks around the
    # wells and water plumes around the injectors on the oracle's start
    x2 = workloads.developed_state(w, x0, np.random.default_rng(22))
    return dict(w=w, mo=mo, x0=x0, x1=x1, x2=x2, orc=oracle, dev=r2p)


def _assert_vec_close(g, o, rtol, nwell_rows=0):
    """Element by element: every |g_i - o_i| <= rtol max|o|, the 2-norm of the
    difference <= rtol ||o||, and the same on the well rows alone."""
    assert np.abs(g - o).max() <= rtol * np.abs(o).max()
    assert np.linalg.norm(g - o) <= rtol * np.linalg.norm(o)
    if nwell_rows:
        gw, ow = g[-nwell_rows:], o[-nwell_rows:]
        assert np.abs(gw - ow).max() <= rtol * max(np.abs(ow).max(), 1e-300)


def _systems(big, x):
    orc, dev, mo, w = big["orc"], big["dev"], big["mo"], big["w"]
    Jo, Fo = mo.jacobian(x, x, DT)
    mg = dev.Model(w)
    J = dev.Jacobian(mg)
    b = J.assemble(_t(x), _t(x), DT)
    return Jo, Fo, mg, J, b


@pytest.mark.parametrize("state", ["x0", "x1"])
def test_fullsize_residual_and_spmv(big, state):
    x = big[state]
    Jo, Fo, mg, J, b = _systems(big, x)
    assert np.abs(_h(b) + Fo).max() <= 1e-12 * np.abs(Fo).max()
    v = np.random.default_rng(3).standard_normal(big["mo"].N)
    yg = _h(J.spmv(_t(v)))
    yo = Jo.matvec(v)
    assert np.abs(yg - yo).max() <= 1e-13 * np.abs(yo).max()


@pytest.mark.parametrize("state", ["x0", "x1", "x2"])
def test_fullsize_preconditioner(big, state):
    """AMG hierarchy structure, one K-cycle, one RAS application and one CPR
    application on the 2M-cell system, each against the oracle element by
    element; x2 (mounds and plumes around the wells) gives the potential
    order its long chains and the hierarchy its well regions."""
    orc, dev, mo = big["orc"], big["dev"], big["mo"]
    x = big[state]
    Jo, Fo, mg, J, b = _systems(big, x)
    Ad, bd = orc.decouple(Jo, -Fo, mo.n, orc.DEC_QI)
    Po = orc.Cpr(Ad, mo, x, orc.cpr_opts())
    P = dev.Cpr().setup(J, dev.cpr_opts())
    lo, lg = Po.amg_levels(), P.amg_levels()
    assert [a["A"].n for a in lo] == [g["n"] for g in lg]
    assert [len(a["A"].col) for a in lo] == [len(g["col"]) for g in lg]
    assert np.array_equal(lo[1]["A"].col, lg[1]["col"])
    assert np.array_equal(lo[0]["agg"], lg[0]["agg"])
    levels = [P.ras_subdomain_info(s)[2] for s in range(P.ras_info())]
    print(f"{state}: AMG levels {[a['A'].n for a in lo]}, RAS levels per subdomain "
          f"{min(levels)}-{max(levels)}")
    rng = np.random.default_rng(5)
    fp = rng.standard_normal(mo.n)
    xg, xo = _h(P.amg_vcycle(_t(fp))), Po.amg_vcycle(fp)
    _assert_vec_close(xg, xo, 1e-10)
    r = rng.standard_normal(mo.N)
    yg, yo = _h(P.ras_apply(_t(r))), Po.ras_apply(r)
    _assert_vec_close(yg, yo, 1e-10, 2 * mo.nw)
    f = rng.standard_normal(mo.N)
    f[2 * mo.n + 1::2] = 0.0
    zg, zo = _h(P.apply(_t(f))), Po.apply(f)
    _assert_vec_close(zg, zo, 1e-10, 2 * mo.nw)


def test_fullsize_one_subdomain_per_cu(big):
    """256 subdomains (16 x 16 tiles of about 12 x 12 x 50 cells), one per
    CU of the device: one RAS and one CPR application at the cold start
    against the oracle (1e-10)."""
    orc, dev, mo = big["orc"], big["dev"], big["mo"]
    x = big["x0"]
    Jo, Fo, mg, J, b = _systems(big, x)
    Ad, bd = orc.decouple(Jo, -Fo, mo.n, orc.DEC_QI)
    Po = orc.Cpr(Ad, mo, x, orc.cpr_opts(px=16, py=16))
    P = dev.Cpr().setup(J, dev.cpr_opts(px=16, py=16))
    assert P.ras_info() == 256
    rng = np.random.default_rng(9)
    r = rng.standard_normal(mo.N)
    yg, yo = _h(P.ras_apply(_t(r))), Po.ras_apply(r)
    _assert_vec_close(yg, yo, 1e-10, 2 * mo.nw)
    f = rng.standard_normal(mo.N)
    f[2 * mo.n + 1::2] = 0.0
    zg, zo = _h(P.apply(_t(f))), Po.apply(f)
    _assert_vec_close(zg, zo, 1e-10, 2 * mo.nw)


def test_fullsize_fp32_preconditioner(big):
    """The FP32 form of the preconditioner (factors, hierarchy and vectors in
    FP32, coarsest inverse FP64) on the 2M-cell system: one CPR application
    within 1e-4 of the FP64 oracle's, and a solve that still reaches a true
    relative residual of 1e-8 on the oracle's decoupled matrix."""
    orc, dev, mo = big["orc"], big["dev"], big["mo"]
    x = big["x0"]
    Jo, Fo, mg, J, b = _systems(big, x)
    Ad, bd = orc.decouple(Jo, -Fo, mo.n, orc.DEC_QI)
    Po = orc.Cpr(Ad, mo, x, orc.cpr_opts())
    P = dev.Cpr().setup(J, dev.cpr_opts(precision=dev.FP32))
    f = np.random.default_rng(7).standard_normal(mo.N)
    f[2 * mo.n + 1::2] = 0.0
    zg, zo = _h(P.apply(_t(f))), Po.apply(f)
    err = np.linalg.norm(zg - zo) / np.linalg.norm(zo)
    print(f"FP32 CPR application at 2M cells: relative difference {err:.2e}")
    assert err <= 1e-4
    y, info = dev.solve(J, P, b)
    assert info.status == 0
    A = Ad.to_scipy()
    assert np.linalg.norm(bd - A @ _h(y)) <= 1.000001e-8 * np.linalg.norm(bd)


@pytest.mark.parametrize("method", ["fgmres", "bicgstab"])
def test_fullsize_linear_solve(big, method):
    """The first Newton system of the benchmark (x0, dt 0.1): the device
    solution's true residual on the oracle's decoupled system <= 1e-8
    (BiCGSTAB with the V-cycle, a fixed preconditioner)."""
    orc, dev, mo = big["orc"], big["dev"], big["mo"]
    Jo, Fo, mg, J, b = _systems(big, big["x0"])
    Ad, bd = orc.decouple(Jo, -Fo, mo.n, orc.DEC_QI)
    P = dev.Cpr().setup(J, dev.cpr_opts(kcycle=0 if method == "bicgstab" else 2))
    m = dev.KRYLOV_FGMRES if method == "fgmres" else dev.KRYLOV_BICGSTAB
    y, info = dev.solve(J, P, b, dev.solve_opts(method=m))
    assert info.status == 0 and info.relres <= 1e-8
    A = Ad.to_scipy()
    assert np.linalg.norm(bd - A @ _h(y)) <= 1.000001e-8 * np.linalg.norm(bd)
    print(f"{method}: {info.iterations} iterations at 2M cells")


def test_fullsize_newton_step(big):
    """One implicit step of the benchmark (dt 0.1 from x0): converged by the
    oracle's own residual and scaled norm at the device's new state."""
    dev, mo = big["dev"], big["mo"]
    x0 = big["x0"]
    mg = dev.Model(big["w"])
    x = _t(x0)
    info = mg.newton_step(x, DT)
    assert info.status == 0
    x1 = _h(x)
    F = mo.residual(x1, x0, DT)
    nrm = mo.scaled_norm(F, DT)
    print(f"Newton: {info.newton_its} iterations, oracle scaled residual {nrm:.2e}")
    assert nrm <= 1.01e-8
    sw = x1[1:2 * mo.n:2]
    assert np.all(np.isfinite(x1)) and sw.min() >= -1e-12 and sw.max() <= 1 + 1e-12


def test_amg_setup_error_reaches_caller(big):
    """The AMG set-up runs on a worker thread and its own stream beside the
    RAS set-up.  A failure there (a one-level hierarchy leaves a 2M-row
    coarsest matrix, above the dense limit: a stalled coarsening) reaches the
    caller as the soft status R2P_NOT_CONVERGED with its message, and the
    same handle then sets up and solves normally."""
    dev, w, x0 = big["dev"], big["w"], big["x0"]
    mg = dev.Model(w)
    J = dev.Jacobian(mg)
    J.assemble(_t(x0), _t(x0), DT)
    P = dev.Cpr()
    with pytest.raises(dev.R2PError, match="AMG coarsening stalled") as e:
        P.setup(J, dev.cpr_opts(max_levels=1))
    assert e.value.code == dev.NOT_CONVERGED
    b = J.assemble(_t(x0), _t(x0), DT)
    P.setup(J, dev.cpr_opts())
    _, info = dev.solve(J, P, b)
    assert info.status == 0 and info.relres <= 1e-8


def test_newton_step_setup_failure_is_not_converged(big):
    """A CPR set-up that fails inside a Newton step (the same stalled
    coarsening) ends the step as not converged with the state unchanged, so
    that the caller can shorten the step; the next call with working options
    converges."""
    dev, w, x0 = big["dev"], big["w"], big["x0"]
    mg = dev.Model(w)
    x = _t(x0)
    info = mg.newton_step(x, DT, dev.newton_opts(cpr=dev.cpr_opts(max_levels=1)))
    assert info.status == dev.NOT_CONVERGED and info.setup_status == dev.NOT_CONVERGED
    assert np.array_equal(_h(x), x0)
    info = mg.newton_step(x, DT)
    assert info.status == 0 and info.setup_status == 0


def test_newton_stage_times_add_up(big):
    """Per-stage host times of a Newton step (Table 5's columns): assembly,
    set-up, solve and update add up to the whole call within a few percent;
    the set-up is the decoupling plus the longer of its two side-by-side
    parts (reordering + block ILU(0), and AMG)."""
    dev, w, x0 = big["dev"], big["w"], big["x0"]
    mg = dev.Model(w)
    x = _t(x0)
    mg.newton_step(x, DT)                       # sizes every buffer
    info = mg.newton_step(x, DT)
    assert info.status == 0
    parts = info.ms_assemble + info.ms_setup + info.ms_solve + info.ms_update
    print(f"total {info.ms_total:.1f} ms: assemble {info.ms_assemble:.1f}, set-up "
          f"{info.ms_setup:.1f} (decouple {info.ms_decouple:.1f}, order {info.ms_order:.1f}, "
          f"BILU {info.ms_ras_setup:.1f}, AMG {info.ms_amg_setup:.1f}), solve "
          f"{info.ms_solve:.1f}, update {info.ms_update:.1f}")
    assert 0.95 * info.ms_total <= parts <= info.ms_total
    inner = info.ms_decouple + max(info.ms_order + info.ms_ras_setup, info.ms_amg_setup)
    assert 0.85 * info.ms_setup <= inner <= 1.001 * info.ms_setup
    assert min(info.ms_decouple, info.ms_order, info.ms_ras_setup, info.ms_amg_setup) > 0
