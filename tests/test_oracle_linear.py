"""Pins of the CPU oracle's linear-solve path (no GPU).

Decoupling, potential reordering, block ILU(0), RAS, aggregation AMG, CPR
(Algorithm 2 and its two-stage form), flexible GMRES and Newton, each
checked against the paper's worked example, exact special cases, dense
linear algebra from numpy, or algebraic identities.
"""
import json
import os

import numpy as np
import pytest

import workloads

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _system(oracle_lib, w, steps=1, dt=None):
    """Jacobian and right-hand side at the first Newton iterate of step `steps`."""
    m = oracle_lib.Model(w)
    x = m.initial_state()
    dt = w["dt"] if dt is None else dt
    for _ in range(steps - 1):
        rc, *_ = m.newton_step(x, dt)
        assert rc == 0
    J, F = m.jacobian(x, x, dt)
    return m, x, J, -F


def test_potential_order_worked_example(oracle_lib):
    """Eq 30 worked example: potentials (2.1, 1.3, 4.2, 1) give Pm = (2, 3, 1, 4)."""
    g = json.load(open(os.path.join(GOLD, "potential_order_example.json")))
    perm = oracle_lib.potential_order(np.array(g["potentials"]))
    pm = np.empty(len(perm), int)
    pm[perm] = np.arange(len(perm)) + 1        # Pm(i) = 1-based position of cell i
    assert list(pm) == g["Pm_one_based"]
    assert list(np.array(g["potentials"])[perm]) == g["sorted_potentials"]


def test_potential_order_ties_and_stability(oracle_lib):
    phi = np.array([1.0, 3.0, 1.0, 3.0, 2.0])
    assert list(oracle_lib.potential_order(phi)) == [1, 3, 4, 0, 2]


def test_reordered_blocks_keep_structure(oracle_lib):
    """Eq 32-33: reordering permutes cells in both the p and s_w parts and
    keeps wells last, so each reordered 2x2 block is an original block."""
    w = workloads.make_small()
    m, x, J, b = _system(oracle_lib, w)
    opts = oracle_lib.cpr_opts(px=1, py=1)
    Ad, bd = oracle_lib.decouple(J, b, m.n, oracle_lib.DEC_QI)
    # factors are not the original blocks, so rebuild the local matrix order
    P = oracle_lib.Cpr(Ad, m, x, opts)
    sub = P.subdomains()[0]
    glob = sub["glob"]
    assert list(glob[m.n:]) == list(range(m.n, m.n + m.nw))       # wells last
    phi = m.potential(x)
    ranks = np.argsort(np.argsort(-phi, kind="stable"), kind="stable")
    assert np.all(np.diff(ranks[glob[:m.n]]) == 1)                # cells in Eq 30 order


def test_decoupling_invariants(oracle_lib):
    """Quasi-IMPES leaves saturation and well rows unchanged and removes the
    pressure row's s_w coupling in the diagonal block; ABF turns every cell
    diagonal block into the identity; both keep the solution (Eq 29)."""
    w = workloads.make_tiny()
    m, x, J, b = _system(oracle_lib, w, steps=2, dt=5.0)
    n = m.n
    Aq, bq = oracle_lib.decouple(J, b, n, oracle_lib.DEC_QI)
    for i in range(m.n + m.nw):
        for z in range(J.rp[i], J.rp[i + 1]):
            if i >= n:
                assert np.array_equal(Aq.val[z], J.val[z])
            else:
                assert np.array_equal(Aq.val[z][1], J.val[z][1])
        if i < n:
            d = Aq.val[Aq.find(i, i)]
            assert abs(d[0, 1]) <= 4e-16 * abs(J.val[J.find(i, i)][0, 1])
    assert np.array_equal(bq[1:2 * n:2], b[1:2 * n:2])
    Aa, ba = oracle_lib.decouple(J, b, n, oracle_lib.DEC_ABF)
    for i in range(n):
        assert np.allclose(Aa.val[Aa.find(i, i)], np.eye(2), atol=1e-14, rtol=0)
    y = np.linalg.solve(J.to_dense(), b)
    for A2, b2 in ((Aq, bq), (Aa, ba)):
        y2 = np.linalg.solve(A2.to_dense(), b2)
        assert np.linalg.norm(y2 - y) <= 1e-9 * np.linalg.norm(y)


def test_bilu0_pattern_identity(oracle_lib):
    """ILU(0): (L U)_IJ = A_IJ on every block of A's pattern."""
    w = workloads.make_small()
    m, x, J, b = _system(oracle_lib, w, steps=2)
    Ad, bd = oracle_lib.decouple(J, b, m.n, oracle_lib.DEC_QI)
    P = oracle_lib.Cpr(Ad, m, x, oracle_lib.cpr_opts())
    for sub in P.subdomains()[:4]:
        LU, dinv, glob = sub["LU"], sub["dinv"], sub["glob"]
        mloc = LU.nb
        L = np.eye(2 * mloc)
        U = np.zeros((2 * mloc, 2 * mloc))
        for i in range(mloc):
            for z in range(LU.rp[i], LU.rp[i + 1]):
                j = LU.col[z]
                tgt = L if j < i else U
                tgt[2 * i:2 * i + 2, 2 * j:2 * j + 2] = LU.val[z]
        prod = L @ U
        loc = {g: a for a, g in enumerate(glob)}
        scale = np.abs(Ad.val).max()
        for a, g in enumerate(glob):
            for z in range(Ad.rp[g], Ad.rp[g + 1]):
                c = Ad.col[z]
                if c in loc:
                    blk = prod[2 * a:2 * a + 2, 2 * loc[c]:2 * loc[c] + 2]
                    assert np.abs(blk - Ad.val[z]).max() <= 1e-13 * scale
        # the stored inverse is the inverse of U's diagonal block
        for i in range(0, mloc, 97):
            d = U[2 * i:2 * i + 2, 2 * i:2 * i + 2]
            assert np.allclose(dinv[i] @ d, np.eye(2), atol=1e-12)


def test_no_fill_column_is_exact(oracle_lib):
    """A vertical column without wells has a block-tridiagonal Jacobian, so
    block ILU(0) is an exact LU and one-subdomain RAS makes FGMRES converge
    in one iteration."""
    w = workloads.make_column(nz=30)
    m = oracle_lib.Model(w)
    x = m.initial_state()
    J, F = m.jacobian(x, x, 1.0)
    Ad, bd = oracle_lib.decouple(J, -F, m.n, oracle_lib.DEC_QI)
    P = oracle_lib.Cpr(Ad, m, x, oracle_lib.cpr_opts(px=1, py=1, form=oracle_lib.CPR_FPF))
    y = P.ras_apply(bd)
    yd = np.linalg.solve(Ad.to_dense(), bd)
    assert np.linalg.norm(y - yd) <= 1e-12 * np.linalg.norm(yd)
    y2, st, its, rr = oracle_lib.fgmres(Ad, bd, P)
    assert st == 0 and its == 1


def test_potential_order_makes_saturation_block_lower_triangular(oracle_lib):
    """With no gravity and no capillary pressure both phases share the
    upstream direction, so in potential order the (water equation, s_w)
    entries above the diagonal vanish (the statement after Eq 33)."""
    w = workloads.make_tiny(6, 5, 3, seed=2)
    w["const"]["grav"] = 0.0
    m = oracle_lib.Model(w)
    rng = np.random.default_rng(4)
    x = workloads.random_state(w, rng)
    J, F = m.jacobian(x, x, 1.0)
    phi = m.potential(x)
    perm = oracle_lib.potential_order(phi)
    rank = np.empty(m.n, int)
    rank[perm] = np.arange(m.n)
    upper = lower = 0
    for i in range(m.n):
        for z in range(J.rp[i], J.rp[i + 1]):
            j = J.col[z]
            if j < m.n and j != i:
                if rank[j] > rank[i]:
                    assert J.val[z][1, 1] == 0.0
                    upper += 1
                elif J.val[z][1, 1] != 0.0:
                    lower += 1
    assert upper > 0 and lower > 0


@pytest.mark.parametrize("form", [0, 1])
def test_cpr_exact_stages_is_exact(oracle_lib, form):
    """Algorithm 2 (and its two-stage form) returns A^-1 f when the RAS and
    AMG stages are replaced by exact solves."""
    w = workloads.make_tiny()
    m, x, J, b = _system(oracle_lib, w, steps=2, dt=5.0)
    Ad, bd = oracle_lib.decouple(J, b, m.n, oracle_lib.DEC_QI)
    P = oracle_lib.Cpr(Ad, m, x, oracle_lib.cpr_opts(form=form, exact_stages=1))
    f = np.random.default_rng(1).standard_normal(m.N)
    f[2 * m.n + 1::2] = 0.0
    y = P.apply(f)
    yd = np.linalg.solve(Ad.to_dense(), f)
    assert np.linalg.norm(y - yd) <= 1e-12 * np.linalg.norm(yd)
    # GMRES with the exact preconditioner converges in one iteration
    y2, st, its, rr = oracle_lib.fgmres(Ad, bd, P)
    assert st == 0 and its == 1


def test_cpr_stage_sequence_differs_from_exact(oracle_lib):
    """With the RAS stage exact and the pressure stage approximate, the
    two-stage form is still exact (its last stage is a full solve): a sign
    or ordering mistake in the residual update would break this."""
    w = workloads.make_tiny()
    m, x, J, b = _system(oracle_lib, w, steps=2, dt=5.0)
    Ad, bd = oracle_lib.decouple(J, b, m.n, oracle_lib.DEC_QI)
    P = oracle_lib.Cpr(Ad, m, x, oracle_lib.cpr_opts(px=1, py=1))
    A = Ad.to_dense()
    f = np.random.default_rng(2).standard_normal(m.N)
    f[2 * m.n + 1::2] = 0.0
    xp = P.amg_vcycle(f[0:2 * m.n:2].copy())
    z = np.zeros(m.N)
    z[0:2 * m.n:2] = xp
    y_manual = z + np.linalg.solve(A, f - A @ z)
    yd = np.linalg.solve(A, f)
    assert np.linalg.norm(y_manual - yd) <= 1e-12 * np.linalg.norm(yd)
    y = P.apply(f)
    # the oracle's two-stage apply equals the manual sequence with RAS in place of A^-1
    y_ras = z + P.ras_apply(f - A @ z)
    assert np.linalg.norm(y - y_ras) <= 1e-12 * np.linalg.norm(y_ras)


def test_amg_single_level_is_dense_solve(oracle_lib):
    w = workloads.make_tiny()
    m, x, J, b = _system(oracle_lib, w, steps=2, dt=5.0)
    Ad, bd = oracle_lib.decouple(J, b, m.n, oracle_lib.DEC_QI)
    App = oracle_lib.extract_pressure(Ad, m.n)
    H = oracle_lib.Amg(App, max_coarse=10 ** 6)
    assert H.nlev == 1
    r = np.random.default_rng(0).standard_normal(m.n)
    assert np.allclose(H.vcycle(r), np.linalg.solve(App.to_scipy().toarray(), r), rtol=1e-12,
                       atol=0)


def test_amg_hierarchy_structure(oracle_lib):
    """Matching is symmetric and pairs strong neighbours; aggregates hold at
    most four rows; A_c = P^T A P checked densely.  Strength, from the dense
    matrix: w_ij = -(a_ij + a_ji)/2, strong when w_ij > 0 and it reaches
    0.25 of the largest weight of row i or of row j."""
    w = workloads.make_small()
    m, x, J, b = _system(oracle_lib, w, steps=2)
    Ad, bd = oracle_lib.decouple(J, b, m.n, oracle_lib.DEC_QI)
    App = oracle_lib.extract_pressure(Ad, m.n)
    match = oracle_lib.strength_match(App)
    D = App.to_scipy().toarray()
    W = -(D + D.T) / 2
    np.fill_diagonal(W, 0.0)
    Mx = np.maximum(W.max(axis=1), 0.0)
    pattern = (App.to_scipy().toarray() != 0) | (App.to_scipy().toarray().T != 0)

    def is_strong(i, j):
        return pattern[i, j] and W[i, j] > 0 and (W[i, j] >= 0.25 * Mx[i] or
                                                  W[i, j] >= 0.25 * Mx[j])
    npair = 0
    for i in range(App.n):
        j = match[i]
        if j >= 0:
            npair += 1
            assert match[j] == i and is_strong(i, j)
    assert npair >= App.n // 2
    # one pass: each aggregate is one pair or singleton plus rows that joined
    # it through a strong coupling to one of its paired members
    agg1, nc1 = oracle_lib.aggregate(App)
    assert agg1.max() + 1 == nc1 and len(np.unique(agg1)) == nc1
    for I in range(nc1):
        mem = np.nonzero(agg1 == I)[0]
        paired = [i for i in mem if match[i] >= 0]
        assert len(paired) in (0, 2)
        if not paired:
            assert len(mem) == 1
        else:
            for i in mem:
                if match[i] < 0:
                    assert any(is_strong(i, p) for p in paired)
    # aggregates are numbered by their leader (smaller row of the pair, or the singleton)
    leaders = []
    for I in range(nc1):
        mem = np.nonzero(agg1 == I)[0]
        paired = [i for i in mem if match[i] >= 0]
        leaders.append(min(paired) if paired else mem[0])
    assert np.all(np.diff(leaders) > 0)
    H = oracle_lib.Amg(App, max_coarse=50)
    assert H.nlev >= 3
    for l in range(H.nlev - 1):
        lv, nxt = H.level(l), H.level(l + 1)
        agg = lv["agg"]
        assert nxt["A"].n < lv["A"].n
        Pm = np.zeros((lv["A"].n, nxt["A"].n))
        Pm[np.arange(lv["A"].n), agg] = 1.0
        Af = lv["A"].to_scipy().toarray()
        Ac = nxt["A"].to_scipy().toarray()
        assert np.abs(Pm.T @ Af @ Pm - Ac).max() <= 1e-12 * np.abs(Af).max()
        assert np.allclose(lv["l1"], np.abs(Af).sum(axis=1), rtol=1e-14)


@pytest.mark.parametrize("form", [0, 1])
def test_fgmres_cpr_matches_dense_lu(oracle_lib, form):
    """FGMRES + CPR on a 4x4x2 grid with two wells (66 unknowns) reaches the
    1e-8 relative residual and the dense-LU solution within kappa * 1e-8."""
    w = workloads.make_tiny()
    m, x, J, b = _system(oracle_lib, w, steps=2, dt=5.0)
    assert m.N == 68      # 64 cell unknowns + 2 wells x (p_b, dummy)
    Ad, bd = oracle_lib.decouple(J, b, m.n, oracle_lib.DEC_QI)
    P = oracle_lib.Cpr(Ad, m, x, oracle_lib.cpr_opts(form=form, px=2, py=2))
    y, st, its, rr = oracle_lib.fgmres(Ad, bd, P)
    A = Ad.to_dense()
    assert st == 0
    assert np.linalg.norm(bd - A @ y) <= 1e-8 * np.linalg.norm(bd)
    yd = oracle_lib.dense_lu_solve(A, bd)
    assert np.allclose(yd, np.linalg.solve(A, bd), rtol=1e-10, atol=0)
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(y - yd) <= kappa * 1e-8 * np.linalg.norm(yd)


@pytest.mark.parametrize("form", [0, 1])
def test_bicgstab_cpr_matches_dense_lu(oracle_lib, form):
    """BiCGSTAB + CPR on the same 66-unknown system: true relative residual
    at most 1e-8 and the dense-LU solution within kappa * 1e-8."""
    w = workloads.make_tiny()
    m, x, J, b = _system(oracle_lib, w, steps=2, dt=5.0)
    Ad, bd = oracle_lib.decouple(J, b, m.n, oracle_lib.DEC_QI)
    P = oracle_lib.Cpr(Ad, m, x, oracle_lib.cpr_opts(form=form, px=2, py=2))
    y, st, its, rr = oracle_lib.bicgstab(Ad, bd, P)
    A = Ad.to_dense()
    assert st == 0 and rr <= 1e-8
    assert np.linalg.norm(bd - A @ y) <= 1e-8 * np.linalg.norm(bd)
    yd = np.linalg.solve(A, bd)
    assert np.linalg.norm(y - yd) <= np.linalg.cond(A) * 1e-8 * np.linalg.norm(yd)


def test_bicgstab_with_exact_preconditioner_takes_one_step(oracle_lib):
    """With the CPR stages replaced by exact solves, M = A^-1, BiCGSTAB
    converges in one iteration (the first half-step already solves)."""
    w = workloads.make_tiny()
    m, x, J, b = _system(oracle_lib, w, steps=1, dt=5.0)
    Ad, bd = oracle_lib.decouple(J, b, m.n, oracle_lib.DEC_QI)
    P = oracle_lib.Cpr(Ad, m, x, oracle_lib.cpr_opts(px=2, py=2, exact_stages=1))
    y, st, its, rr = oracle_lib.bicgstab(Ad, bd, P)
    assert st == 0 and its == 1


def test_gmres_residual_monotone_and_identity(oracle_lib):
    w = workloads.make_small()
    m, x, J, b = _system(oracle_lib, w, steps=2)
    Ad, bd = oracle_lib.decouple(J, b, m.n, oracle_lib.DEC_QI)
    P = oracle_lib.Cpr(Ad, m, x, oracle_lib.cpr_opts())
    y, st, its, rr, hist = oracle_lib.fgmres(Ad, bd, P, history=True)
    assert st == 0
    for c0 in range(0, its, 30):
        h = hist[c0:c0 + 30]
        assert np.all(np.diff(h) <= 1e-15)


def test_newton_quadratic_and_iterative_equals_direct(oracle_lib):
    """Newton with exact solves converges quadratically; the CPR-FGMRES
    Newton reaches the same fields within 1e-8."""
    w = workloads.make_tiny(5, 5, 2, seed=8)
    m = oracle_lib.Model(w)
    x0 = m.initial_state()
    xd, xi = x0.copy(), x0.copy()
    for step in range(2):
        rc, ni, li, hist = m.newton_step(xd, 5.0, exact_linear=True, ntol=1e-12)
        assert rc == 0
        tail = hist[hist > 1e-10]          # above the round-off floor
        assert len(tail) >= 3
        ratios = tail[-2:] / tail[-3:-1] ** 2   # last iterations, chop no longer active
        assert ratios.max() < 1e2
        rc, ni2, li2, _ = m.newton_step(xi, 5.0, ntol=1e-12, rtol=1e-10,
                                        opts=oracle_lib.cpr_opts(px=2, py=2))
        assert rc == 0
    n = m.n
    for sl in (slice(0, 2 * n, 2), slice(1, 2 * n, 2)):
        assert np.linalg.norm(xi[sl] - xd[sl]) <= 1e-8 * np.linalg.norm(xd[sl])


def test_newton_failure_leaves_state_unchanged(oracle_lib):
    w = workloads.make_small()
    m = oracle_lib.Model(w)
    x = m.initial_state()
    x0 = x.copy()
    rc, ni, li, hist = m.newton_step(x, 10.0, max_newton=1)
    assert rc == 1
    assert np.array_equal(x, x0)
