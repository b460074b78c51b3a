"""Further pins of the CPU oracle (no GPU).

Each test replays an oracle routine with dense numpy algebra built
independently from the definition the oracle follows, or checks it against a
closed form or a guaranteed property, so that a dropped term, a wrong sign,
a wrong index or a transposed operand in the oracle fails:

- the FPF preconditioner (Algorithm 2) with approximate stages, against its
  five steps replayed densely;
- the multi-level AMG cycle (V-cycle and K-cycle), against a dense replay
  built from the exported level matrices, l1 diagonals and aggregates, and
  the two-stage preconditioner with two and three AMG cycles per pressure
  stage against the same replay;
- RAS on 4x4 tiles at overlap 1 and 2: the overlapped sets against a
  breadth-first search of the block graph from the tile definition, the
  factors against the ILU(0) pattern identity per subdomain, and the apply
  against sum_s R_s^0^T (L_s U_s)^-1 R_s^delta r;
- the Eisenstat-Walker forcing terms (Eq 26), recomputed from the returned
  residual norms;
- the scaled Newton stopping norm and Peaceman's well index (anisotropic
  and rectangular cells) against hand formulas;
- the aggregation's progress on matrices where a one-sided strength rule
  makes none, and the soft failure when coarsening stalls.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads


def _system(orc, w, steps=1, dt=None):
    m = orc.Model(w)
    x = m.initial_state()
    dt = w["dt"] if dt is None else dt
    for _ in range(steps - 1):
        rc, *_ = m.newton_step(x, dt)
        assert rc == 0
    J, F = m.jacobian(x, x, dt)
    return m, x, J, -F


# ------------------------------------------------------------------ FPF
@pytest.mark.parametrize("exact_amg", [False, True])
def test_fpf_approximate_stages_dense_replay(oracle_lib, exact_amg):
    """Algorithm 2: x = R^-1 f; r = f - A x; x += Pi_p M^-1 Pi_r r;
    r = f - A x; x += R^-1 r, with an approximate RAS stage (2x2 tiles) and
    an approximate (multi-level) or exact (one level) pressure stage."""
    w = workloads.make_small()
    m, x, J, b = _system(oracle_lib, w, steps=2)
    n = m.n
    Ad, _ = oracle_lib.decouple(J, b, n, oracle_lib.DEC_QI)
    opts = oracle_lib.cpr_opts(form=oracle_lib.CPR_FPF, px=2, py=2, amg_cycles=1,
                               max_coarse=10 ** 6 if exact_amg else 100)
    P = oracle_lib.Cpr(Ad, m, x, opts)
    A = Ad.to_scipy().tocsr()
    f = np.random.default_rng(5).standard_normal(m.N)
    f[2 * n + 1::2] = 0.0
    x1 = P.ras_apply(f)
    r = f - A @ x1
    xp = P.amg_vcycle(r[0:2 * n:2].copy())
    if exact_amg:
        App = A[0:2 * n:2, 0:2 * n:2].toarray()
        assert np.linalg.norm(xp - np.linalg.solve(App, r[0:2 * n:2])) <= \
            1e-10 * np.linalg.norm(xp)
    x2 = x1.copy()
    x2[0:2 * n:2] += xp
    y = x2 + P.ras_apply(f - A @ x2)
    z = P.apply(f)
    assert np.linalg.norm(z - y) <= 1e-12 * np.linalg.norm(y)
    # the middle stages matter: dropping the second residual update changes the result
    y_bad = x2 + P.ras_apply(r)
    assert np.linalg.norm(z - y_bad) > 1e-6 * np.linalg.norm(y)


# ------------------------------------------------------------- AMG cycle
def _dense_cycle(levels, l, b, kcycle):
    """V(1,1) with l1-Jacobi (zero start), piecewise-constant P; on levels
    l < kcycle the coarse system gets two generalised-conjugate-residual
    steps, each preconditioned by one cycle a level down."""
    A, d = levels[l]["A"], levels[l]["l1"]
    if l == len(levels) - 1:
        return np.linalg.solve(A, b)
    P = levels[l]["P"]
    x = b / d
    bc = P.T @ (b - A @ x)
    Ac = levels[l + 1]["A"]
    if l < kcycle and l + 1 < len(levels) - 1:
        p1 = _dense_cycle(levels, l + 1, bc, kcycle)
        q1 = Ac @ p1
        a1 = (q1 @ bc) / (q1 @ q1)
        rc = bc - a1 * q1
        p2 = _dense_cycle(levels, l + 1, rc, kcycle)
        q2 = Ac @ p2
        beta = (q1 @ q2) / (q1 @ q1)
        p2, q2 = p2 - beta * p1, q2 - beta * q1
        a2 = (q2 @ rc) / (q2 @ q2)
        xc = a1 * p1 + a2 * p2
        # the correction minimises the coarse residual over span{p1, p2}
        B = np.stack([Ac @ p1, Ac @ p2], axis=1)
        coef = np.linalg.lstsq(B, bc, rcond=None)[0]
        assert np.linalg.norm(bc - Ac @ xc) <= np.linalg.norm(bc - B @ coef) * (1 + 1e-9)
    else:
        xc = _dense_cycle(levels, l + 1, bc, kcycle)
    x = x + P @ xc
    return x + (b - A @ x) / d


@pytest.mark.parametrize("kcycle", [0, 1, 2])
def test_amg_cycle_dense_replay(oracle_lib, kcycle):
    w = workloads.make_small()
    m, x, J, b = _system(oracle_lib, w, steps=2)
    Ad, _ = oracle_lib.decouple(J, b, m.n, oracle_lib.DEC_QI)
    App = oracle_lib.extract_pressure(Ad, m.n)
    H = oracle_lib.Amg(App, max_coarse=40, kcycle=kcycle)
    assert H.nlev >= 4
    levels = []
    for l in range(H.nlev):
        lv = H.level(l)
        A = lv["A"].to_scipy().toarray()
        d = np.abs(A).sum(axis=1)
        assert np.array_equal(lv["l1"], d) or np.allclose(lv["l1"], d, rtol=1e-15)
        entry = dict(A=A, l1=d)
        if l < H.nlev - 1:
            P = np.zeros((A.shape[0], H.level(l + 1)["A"].n))
            P[np.arange(A.shape[0]), lv["agg"]] = 1.0
            entry["P"] = P
        levels.append(entry)
    for seed in range(3):
        r = np.random.default_rng(seed).standard_normal(m.n)
        ref = _dense_cycle(levels, 0, r, kcycle)
        got = H.vcycle(r)
        assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


def _dense_levels(H):
    levels = []
    for l in range(H.nlev):
        lv = H.level(l)
        A = lv["A"].to_scipy().toarray()
        entry = dict(A=A, l1=np.abs(A).sum(axis=1))
        if l < H.nlev - 1:
            P = np.zeros((A.shape[0], H.level(l + 1)["A"].n))
            P[np.arange(A.shape[0]), lv["agg"]] = 1.0
            entry["P"] = P
        levels.append(entry)
    return levels


@pytest.mark.parametrize("ncyc", [2, 3])
def test_two_stage_with_several_amg_cycles_dense_replay(oracle_lib, ncyc):
    """Pressure stage of ncyc AMG cycles, each on the last residual:
    x_p = C(r_p), then x_p += C(r_p - A_pp x_p); then x = Pi_p x_p,
    r = f - A x, x += R^-1 r (the two-stage form)."""
    w = workloads.make_small()
    m, x, J, b = _system(oracle_lib, w, steps=2)
    n = m.n
    Ad, _ = oracle_lib.decouple(J, b, n, oracle_lib.DEC_QI)
    kw = dict(px=2, py=2, max_coarse=40, kcycle=1)
    P = oracle_lib.Cpr(Ad, m, x, oracle_lib.cpr_opts(amg_cycles=ncyc, **kw))
    P1 = oracle_lib.Cpr(Ad, m, x, oracle_lib.cpr_opts(amg_cycles=1, **kw))
    App = oracle_lib.extract_pressure(Ad, n)
    H = oracle_lib.Amg(App, max_coarse=40, kcycle=1)
    assert H.nlev >= 4
    levels = _dense_levels(H)
    A = Ad.to_scipy().tocsr()
    Ap = levels[0]["A"]
    f = np.random.default_rng(11).standard_normal(m.N)
    f[2 * n + 1::2] = 0.0
    fp = f[0:2 * n:2]
    xp = _dense_cycle(levels, 0, fp, 1)
    for _ in range(ncyc - 1):
        xp = xp + _dense_cycle(levels, 0, fp - Ap @ xp, 1)
    y = np.zeros(m.N)
    y[0:2 * n:2] = xp
    y = y + P.ras_apply(f - A @ y)
    z = P.apply(f)
    assert np.linalg.norm(z - y) <= 1e-11 * np.linalg.norm(y)
    # the extra cycles matter
    assert np.linalg.norm(P1.apply(f) - z) > 1e-6 * np.linalg.norm(z)


def _fgmres_count(A, b, M, rtol=1e-8, maxit=200):
    """Flexible GMRES without restart from zero (the K-cycle is not a fixed
    linear operator); returns the iterations to reach rtol."""
    bn = np.linalg.norm(b)
    V, Z = [b / bn], []
    H = np.zeros((maxit + 1, maxit))
    for j in range(maxit):
        Z.append(M(V[j]))
        w = A @ Z[j]
        for i in range(j + 1):
            H[i, j] = w @ V[i]
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        V.append(w / H[j + 1, j])
        e = np.zeros(j + 2)
        e[0] = bn
        y = np.linalg.lstsq(H[:j + 2, :j + 1], e, rcond=None)[0]
        if np.linalg.norm(e - H[:j + 2, :j + 1] @ y) <= rtol * bn:
            xk = np.array(Z).T @ y
            assert np.linalg.norm(b - A @ xk) <= 1.01 * rtol * bn
            return j + 1
    return maxit + 1


def test_kcycle_accelerates_pressure_solve(oracle_lib):
    """As a preconditioner of flexible GMRES on A_pp, the K-cycle on the two
    finest levels needs fewer iterations than the V-cycle (the reason it is
    the default)."""
    w = workloads.make_gaussian(nx=40, ny=40, nz=10, seed=3, well_pattern=2)
    m, x, J, b = _system(oracle_lib, w, dt=5.0)
    Ad, _ = oracle_lib.decouple(J, b, m.n, oracle_lib.DEC_QI)
    App = oracle_lib.extract_pressure(Ad, m.n)
    A = App.to_scipy().tocsr()
    rhs = np.random.default_rng(0).standard_normal(m.n)
    its = {}
    for k in (0, 2):
        H = oracle_lib.Amg(App, max_coarse=20, kcycle=k)
        its[k] = _fgmres_count(A, rhs, H.vcycle)
    assert its[2] < its[0] <= 200


# ------------------------------------------------------------------ RAS
def _tile_owner(w, px, py):
    g = w["grid"]
    nx, ny, n = g["nx"], g["ny"], g["n"]
    c = np.arange(n)
    i, j = c % nx, (c // nx) % ny
    own = (i * px) // nx + px * ((j * py) // ny)
    wells = [own[wl["cells"][0]] for wl in w["wells"]]
    return np.concatenate([own, np.array(wells, dtype=own.dtype)])


@pytest.mark.parametrize("overlap", [1, 2])
def test_ras_multi_subdomain_dense_replay(oracle_lib, overlap):
    w = workloads.make_small()
    m, x, J, b = _system(oracle_lib, w, steps=2)
    n, nb = m.n, m.n + m.nw
    Ad, _ = oracle_lib.decouple(J, b, n, oracle_lib.DEC_QI)
    P = oracle_lib.Cpr(Ad, m, x, oracle_lib.cpr_opts(px=4, py=4, overlap=overlap))
    subs = P.subdomains()
    assert len(subs) == 16
    A = Ad.to_scipy().toarray()
    G = sp.csr_matrix((np.ones(len(Ad.col)), Ad.col,
                       Ad.rp), shape=(nb, nb))            # block graph
    owner = _tile_owner(w, 4, 4)
    f = np.random.default_rng(9).standard_normal(m.N)
    f[2 * n + 1::2] = 0.0
    y = np.zeros(m.N)
    for s, S in enumerate(subs):
        own = owner == s
        reach = own.copy()
        for _ in range(overlap):                            # delta layers of neighbours
            reach = reach | (G.T @ reach.astype(float) > 0) | (G @ reach.astype(float) > 0)
        glob = S["glob"]
        assert sorted(glob) == list(np.nonzero(reach)[0])
        assert np.array_equal(S["owned"], own[glob])
        idx = np.ravel(np.stack([2 * glob, 2 * glob + 1], axis=1))
        As = A[np.ix_(idx, idx)]                            # R_s A R_s^T in local order
        LU = S["LU"]
        m_s = len(glob)
        L, U = np.eye(2 * m_s), np.zeros((2 * m_s, 2 * m_s))
        for a in range(m_s):
            for z in range(LU.rp[a], LU.rp[a + 1]):
                c = LU.col[z]
                blk = LU.val[z]
                if c < a:
                    L[2 * a:2 * a + 2, 2 * c:2 * c + 2] = blk
                else:
                    U[2 * a:2 * a + 2, 2 * c:2 * c + 2] = blk
        # ILU(0) pattern identity on the overlapped subdomain matrix
        prod = L @ U
        mask = np.kron((np.abs(As).reshape(m_s, 2, m_s, 2).sum(axis=(1, 3)) > 0) |
                       np.eye(m_s, dtype=bool), np.ones((2, 2), bool))
        scale = np.abs(As).max()
        assert np.abs((prod - As)[mask]).max() <= 1e-12 * scale
        for a in range(m_s):                                # stored inverse diagonal blocks
            d = U[2 * a:2 * a + 2, 2 * a:2 * a + 2]
            assert np.allclose(S["dinv"][a] @ d, np.eye(2), atol=1e-10)
        v = np.linalg.solve(U, np.linalg.solve(L, f[idx]))
        keep = np.repeat(S["owned"], 2)
        y[idx[keep]] = v[keep]                              # restricted prolongation R_s^0^T
    got = P.ras_apply(f)
    assert np.linalg.norm(got - y) <= 1e-11 * np.linalg.norm(y)


# ---------------------------------------------------------------- Newton
def test_ew_forcing_recomputed_from_norms(oracle_lib):
    """Eq 26, second choice, clipped to [0.01, 0.1], eta_0 = 0.1:
    eta_l = | ||F(x_l)|| - ||F(x_{l-1}) + J y_{l-1}|| | / ||F(x_{l-1})||."""
    w = workloads.make_small()
    m = oracle_lib.Model(w)
    x = m.initial_state()
    for _ in range(2):                 # past the cold start's strongly nonlinear first steps
        assert m.newton_step(x, w["dt"])[0] == 0
    x2 = x.copy()
    rc, ni, li, hist, nrm = m.newton_step(x, w["dt"], forcing=1, norms=True)
    assert rc == 0 and ni >= 3
    fn, rn, eta = nrm["fnorm"], nrm["rnorm"], nrm["eta"]
    assert eta[0] == 0.1
    for l in range(1, ni):
        e = min(max(abs(fn[l] - rn[l - 1]) / fn[l - 1], 0.01), 0.1)
        assert eta[l] == pytest.approx(e, rel=1e-15, abs=0)
    # the linear residual of each solve is below ||F||: the solve did reduce it
    assert np.all(rn[:ni] < fn[:ni])
    # standard Newton solves every system to the fixed tolerance
    rc, ni, li, hist, nrm = m.newton_step(x2, w["dt"], norms=True)
    assert rc == 0 and np.all(nrm["eta"] == 1e-8)


def test_scaled_norm_hand_formula(oracle_lib):
    """max over cells of |F| dt / PV with PV = dx dy dz phi / alpha_c (bbl),
    and over rate wells of |F_w| / |target|."""
    w = workloads.make_small()
    m = oracle_lib.Model(w)
    rng = np.random.default_rng(4)
    g = w["grid"]
    pv = g["dx"] * g["dy"] * g["dz"] * w["phi"] / w["const"]["alpha_c"]
    for dt in (0.5, 10.0):
        F = rng.standard_normal(m.N)
        F[2 * m.n + 1::2] = 0.0
        cells = np.maximum(np.abs(F[0:2 * m.n:2]), np.abs(F[1:2 * m.n:2])) * dt / pv
        wells = [abs(F[2 * (m.n + k)]) / abs(wl["target"]) for k, wl in enumerate(w["wells"])]
        expect = max(cells.max(), max(wells))
        assert m.scaled_norm(F, dt) == pytest.approx(expect, rel=1e-14)
        # the largest entry decides: raising one cell raises the norm to it
        c = 123
        F[2 * c + 1] = 1e6 * pv[c] / dt
        assert m.scaled_norm(F, dt) == pytest.approx(1e6, rel=1e-14)


def test_peaceman_anisotropic_and_rectangular(oracle_lib):
    """Peaceman's equivalent radius (Peaceman 1983): for an isotropic cell
    r_o = 0.14 sqrt(dx^2 + dy^2); with k_y = 4 k_x on a 20 ft square cell,
    r_o = 0.28 sqrt(2*400 + 0.5*400) / (sqrt(2) + sqrt(0.5)) = 4.173994 ft and
    the permeability factor is sqrt(k_x k_y) = 2 k_x.  Swapping the x and y
    data leaves the index unchanged."""
    base = workloads.make_small()
    c = base["wells"][0]["cells"][0]
    beta, rw, dz = 0.001127, 0.25, 2.0

    def wi_of(w):
        return oracle_lib.Model(w).well_index()[0][0]

    w = dict(base)
    w["ky"] = 4.0 * base["kx"]
    kx = base["kx"][c]
    ro = 0.28 * np.sqrt(2 * 400 + 0.5 * 400) / (np.sqrt(2) + np.sqrt(0.5))
    assert ro == pytest.approx(4.173994, abs=1e-6)
    assert wi_of(w) == pytest.approx(2 * np.pi * beta * 2 * kx * dz / np.log(ro / rw), rel=1e-13)
    # swap x and y: k_x <-> k_y (dx = dy): same index
    w2 = dict(base)
    w2["kx"], w2["ky"] = 4.0 * base["kx"], base["kx"]
    assert wi_of(w2) == pytest.approx(wi_of(w), rel=1e-14)
    # isotropic rectangular cell, dy = 10 ft
    w3 = dict(base)
    w3["grid"] = dict(base["grid"], dy=10.0)
    ro3 = 0.14 * np.sqrt(20.0 ** 2 + 10.0 ** 2)
    assert wi_of(w3) == pytest.approx(2 * np.pi * beta * kx * dz / np.log(ro3 / rw), rel=1e-13)


# ------------------------------------------------------------ coarsening
def _one_sided_rule_pairs(A, theta=0.25, rounds=4):
    """Handshake matching with the one-sided strength of row i alone
    (strongest -a_ij of the row, ties to the smaller j), written out with
    loops: the rule that gives no pairs on a cyclic non-symmetric matrix."""
    A = A.tocsr()
    n = A.shape[0]
    match = -np.ones(n, int)
    for _ in range(rounds):
        prop = -np.ones(n, int)
        for i in range(n):
            if match[i] >= 0:
                continue
            cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
            vals = A.data[A.indptr[i]:A.indptr[i + 1]]
            off = [(-v, j) for j, v in zip(cols, vals) if j != i]
            mx = max([s for s, _ in off] + [0.0])
            best = None
            for s, j in sorted(off, key=lambda t: (-t[0], t[1])):
                if s > 0 and s >= theta * mx and match[j] < 0:
                    best = j
                    break
            if best is not None:
                prop[i] = best
        for i in range(n):
            j = prop[i]
            if match[i] < 0 and j >= 0 and prop[j] == i:
                match[i] = j
    return match


def _ring(n, seed):
    """Ring with a_{i,i+1} = -2 and a_{i,i-1} = -(1 + u_i), u_i in (0, 0.5):
    every row's strongest coupling points forward."""
    u = np.random.default_rng(seed).uniform(0.05, 0.5, n)
    i = np.arange(n)
    rows = np.concatenate([i, i, i])
    cols = np.concatenate([i, (i + 1) % n, (i - 1) % n])
    vals = np.concatenate([3.5 + u, -2.0 * np.ones(n), -(1.0 + u)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def test_matching_progress_on_cyclic_matrix(oracle_lib):
    A = _ring(400, 0)
    assert np.all(_one_sided_rule_pairs(A) < 0)          # the one-sided rule stalls
    Ao = oracle_lib.CsrMatrix(A.indptr, A.indices, A.data)
    match = oracle_lib.strength_match(Ao)
    assert np.mean(match >= 0) >= 0.6
    agg, nc = oracle_lib.aggregate(Ao)
    assert nc <= 0.5 * 400
    H = oracle_lib.Amg(Ao, max_coarse=20)
    assert H.level(H.nlev - 1)["A"].n <= 20


def test_matching_pairs_every_strong_component_each_round(oracle_lib):
    """One handshake round pairs at least one row of every connected group
    of rows joined by strong couplings (the symmetric weight and tie rule
    make every chain of proposals end in a mutual pair)."""
    from scipy.sparse.csgraph import connected_components
    rng = np.random.default_rng(11)
    for trial in range(5):
        n = 300
        B = sp.random(n, n, density=0.01, random_state=rng, data_rvs=lambda k: rng.uniform(0.1, 2, k))
        B = (B + sp.random(n, n, density=0.005, random_state=rng,
                           data_rvs=lambda k: rng.uniform(0.1, 2, k)).T).tocsr()
        B.setdiag(0)
        B.eliminate_zeros()
        S = B + B.T                                          # symmetric pattern
        A = (-B + sp.diags(np.asarray(abs(S).sum(axis=1)).ravel() + 1.0)).tocsr()
        A = (A + 0 * S).tocsr()
        A.sort_indices()
        Ao = oracle_lib.CsrMatrix(A.indptr, A.indices, A.data)
        D = A.toarray()
        W = -(D + D.T) / 2
        np.fill_diagonal(W, 0)
        Mx = np.maximum(W.max(axis=1), 0)
        strong = (W > 0) & ((W >= 0.25 * Mx[:, None]) | (W >= 0.25 * Mx[None, :]))
        ncomp, lab = connected_components(sp.csr_matrix(strong), directed=False)
        match = oracle_lib.strength_match(Ao, rounds=1)
        for c in range(ncomp):
            mem = lab == c
            if mem.sum() > 1:
                assert np.any(match[mem] >= 0)
        assert np.all(match[match >= 0][match[match[match >= 0]] >= 0] >= 0)


def test_coarsening_stall_is_a_soft_failure(oracle_lib):
    """A matrix without couplings cannot be coarsened: above the dense limit
    (4096 rows) the set-up reports a stall (status 1) instead of solving."""
    n = 5000
    A = sp.diags(np.linspace(1.0, 2.0, n)).tocsr()
    Ao = oracle_lib.CsrMatrix(A.indptr, A.indices, A.data)
    with pytest.raises(ValueError, match="stalled"):
        oracle_lib.Amg(Ao)
    A = sp.diags(np.linspace(1.0, 2.0, 3000)).tocsr()     # below the limit: one dense level
    H = oracle_lib.Amg(oracle_lib.CsrMatrix(A.indptr, A.indices, A.data))
    r = np.random.default_rng(0).standard_normal(3000)
    assert np.allclose(H.vcycle(r), r / np.linspace(1.0, 2.0, 3000), rtol=1e-13)
