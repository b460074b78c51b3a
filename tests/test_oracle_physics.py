"""Pins of the CPU oracle's physics and discretisation (no GPU).

Each test checks the oracle against something other than itself: a closed
form, a conservation identity, finite differences, a printed example or a
known special case.
"""
import json
import os

import numpy as np
import pytest

import workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_hydrostatic_initial_state_has_no_flux(oracle_lib):
    """Gravity sign and face density (readings of Eq 5 and Eq 10): the
    oil-hydrostatic state carries no flux, so with no wells and dt large the
    residual is zero to round-off."""
    w = workloads.make_small()
    w["wells"] = []
    m = oracle_lib.Model(w)
    x = m.initial_state()
    F = m.residual(x, x, 1e6)
    # flux scale: beta * T * lambda * (cell pressure) ~ 1e3 STB/day
    assert np.abs(F).max() < 1e-8
    # pressure increases downward by about the oil gradient (46.244/144 psi/ft)
    p = x[0:2 * m.n:2].reshape(5, 20, 20)
    grad = (p[1:, 0, 0] - p[:-1, 0, 0]) / 2.0
    assert np.allclose(grad, 46.244 / 144.0, rtol=1e-3)
    # and the gradient is in the downward direction with the reference point honoured
    assert p[0, 0, 0] < 4800.0 < p[-1, 0, 0] + 200


def test_peaceman_isotropic_closed_form(oracle_lib):
    """Peaceman's equivalent radius for a square isotropic cell is
    r_o = 0.28*sqrt(2)/2 * dx ~= 0.198 dx, so WI = 2 pi beta k dz / ln(r_o/r_w)."""
    w = workloads.make_small()
    m = oracle_lib.Model(w)
    wi, zb = m.well_index()
    c = w["wells"][0]["cells"][0]
    k = w["kx"][c]
    ro = 0.28 * np.sqrt(2.0) / 2.0 * 20.0
    expect = 2 * np.pi * 0.001127 * k * 2.0 / np.log(ro / 0.25)
    assert abs(wi[0] - expect) / expect < 1e-14
    assert zb[0] == 8335.0


@pytest.mark.parametrize("seed", [0, 1])
def test_mass_balance_any_state(oracle_lib, seed):
    """Each face flux enters two cells with opposite sign (Eq 17 with the
    symmetric upstream rule), so summing the cell residuals leaves only
    accumulation minus well rates, for any state."""
    w = workloads.make_tiny(5, 4, 3, seed=seed)
    m = oracle_lib.Model(w)
    rng = np.random.default_rng(seed)
    x = workloads.random_state(w, rng)
    xo = workloads.random_state(w, rng)
    dt = 3.0
    F = m.residual(x, xo, dt)
    ao, aw = m.accumulation(x)
    aon, awn = m.accumulation(xo)
    qo, qw = m.well_rates(x)
    n = m.n
    for ph, (a, an, q) in enumerate([(ao, aon, qo), (aw, awn, qw)]):
        lhs = F[ph:2 * n:2].sum()
        rhs = ((a - an) / dt).sum() - q.sum()
        scale = np.abs(F[ph:2 * n:2]).sum() + np.abs(q).sum()
        assert abs(lhs - rhs) <= 1e-13 * scale


def _tie_free_state(w, rng, h):
    while True:
        x = workloads.random_state(w, rng, p_spread=80.0)
        g = w["grid"]
        p = x[0:2 * g["n"]:2].reshape(g["nz"], g["ny"], g["nx"])
        ok = True
        for ax in range(3):
            d = np.abs(np.diff(p, axis=ax))
            if d.size and d.min() < 10 * h + 5.0:  # gravity term < 1 psi at dz = 2 ft
                ok = False
        if ok:
            return x


def test_jacobian_matches_finite_differences(oracle_lib):
    """Analytic Jacobian (Eq 17 and the well rows) = central differences of
    the residual, column by column (h_p = 1e-3 psi, h_s = 1e-7), on a state
    with no potential ties."""
    w = workloads.make_tiny(4, 3, 2, seed=7)
    # one rate well so its row is nonzero, one BHP well
    m = oracle_lib.Model(w)
    rng = np.random.default_rng(11)
    x = _tie_free_state(w, rng, 1e-3)
    xo = workloads.random_state(w, rng)
    J, F = m.jacobian(x, xo, 4.0)
    D = J.to_dense()
    N = m.N
    for j in range(N):
        h = 1e-3 if j % 2 == 0 else 1e-7
        xp, xm = x.copy(), x.copy()
        xp[j] += h
        xm[j] -= h
        fd = (m.residual(xp, xo, 4.0) - m.residual(xm, xo, 4.0)) / (2 * h)
        scale = max(np.abs(fd).max(), np.abs(D[:, j]).max(), 1e-12)
        assert np.abs(fd - D[:, j]).max() <= 1e-6 * scale, f"column {j}"


def _run_1d(oracle_lib, nx, t_end, nsteps, rate=10.0):
    w = workloads.make_1d(nx=nx, rate=rate)
    m = oracle_lib.Model(w)
    x = m.initial_state()
    dt = t_end / nsteps
    opts = oracle_lib.cpr_opts(px=1, py=1)
    for _ in range(nsteps):
        rc, ni, li, h = m.newton_step(x, dt, opts=opts, ntol=1e-10, rtol=1e-12)
        assert rc == 0
    return w, m, x


def test_darcy_pressure_drop_ahead_of_front(oracle_lib):
    """Eq 1: in the incompressible 1D core only oil moves ahead of the water
    front, and it carries the whole injection rate q, so neighbouring cell
    pressures differ by q mu_o dx / (beta_c k A) (A = dy dz)."""
    nx = 100
    w, m, x = _run_1d(oracle_lib, nx, t_end=2.0, nsteps=2)
    p = x[0:2 * nx:2]
    s = x[1:2 * nx:2]
    q, mu_o, dx, k, A = 10.0, 5.0, 10.0, 100.0, 400.0
    drop = q * mu_o * dx / (0.001127 * k * A)
    ahead = np.arange(nx // 2, nx - 2)
    assert s[ahead].max() < 1e-12
    d = p[ahead] - p[ahead + 1]
    assert np.abs(d - drop).max() <= 1e-10 * drop


def test_buckley_leverett_front(oracle_lib):
    """Buckley-Leverett closed form (M = 5): the front saturation is
    1/sqrt(1+M) and the front travels at f(S_f)/S_f * q/(phi A).  The L1
    error of the simulated profile and the error of the front position both
    fall as the grid is refined (first-order upwinding smears the front over
    a few cells), and at nx = 400 the front is within 2% of the core length."""
    gold = json.load(open(os.path.join(GOLD, "buckley_leverett.json")))
    M, Sf, speed = gold["M"], gold["front_saturation"], gold["shock_speed_factor"]
    L, phi, A = 1000.0, 0.2, 400.0
    q_ft3 = 10.0 * 5.614583
    t_end = 0.5 * L * phi * A / (speed * q_ft3)   # front at half the core

    def exact(xc):
        s = np.linspace(Sf, 1.0, 20001)
        fp = 2 * M * s * (1 - s) / (M * s * s + (1 - s) ** 2) ** 2
        xs = q_ft3 * t_end * fp / (phi * A)       # position of saturation s (decreasing in s)
        out = np.zeros_like(xc)
        xf = q_ft3 * t_end * speed / (phi * A)
        inside = xc < xf
        out[inside] = np.interp(xc[inside], xs[::-1], s[::-1])
        return out, xf

    errs, ferrs = [], []
    for nx in (100, 200, 400):
        w, m, x = _run_1d(oracle_lib, nx, t_end, nsteps=nx)
        s = x[1:2 * nx:2]
        dxc = L / nx
        xc = (np.arange(nx) + 0.5) * dxc
        se, xf = exact(xc)
        errs.append(np.abs(s - se).sum() * dxc / L)
        # numerical front: last cell with s above half the front saturation
        i_front = np.nonzero(s > 0.5 * Sf)[0].max()
        ferrs.append(abs((i_front + 0.5) * dxc - xf))
    assert errs[0] > errs[1] > errs[2]
    assert ferrs[0] > ferrs[1] > ferrs[2]
    assert ferrs[2] < 0.02 * L
