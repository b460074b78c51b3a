"""FP64 CPU oracle for the two-phase CPR-FGMRES path (Python binding).

TEST INFRASTRUCTURE ONLY: the plain, slow reference that the device library
is checked against.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  It shares no code
with the device library; the seeded input generators (package `workloads`)
are the only thing both sides use.

The C sources in this folder are compiled with gcc by `build()` into
`oracle/_build/liboracle.so` and loaded with ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["physics.c", "sparse.c", "ras.c", "amg.c", "solver.c", "api.c"]
LIB_PATH = os.path.join(HERE, "_build", "liboracle.so")

DEC_NONE, DEC_QI, DEC_ABF = 0, 1, 2
ORD_NATURAL, ORD_POTENTIAL = 0, 1
CPR_TWO_STAGE, CPR_FPF = 0, 1
AMG_CYCLES = 2      # AMG cycles per pressure stage (the default of both sides)

_lib = None

i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")


def build(force=True):
    """Compile the oracle with gcc (plain C11, no FMA contraction)."""
    os.makedirs(os.path.dirname(LIB_PATH), exist_ok=True)
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    if not force and os.path.exists(LIB_PATH):
        newest = max(os.path.getmtime(s) for s in srcs + [os.path.join(HERE, "oracle.h")])
        if os.path.getmtime(LIB_PATH) >= newest:
            return LIB_PATH
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
           "-D_DEFAULT_SOURCE", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Bsr(C.Structure):
    _fields_ = [("nb", C.c_int), ("nnzb", C.c_int), ("rp", C.POINTER(C.c_int)),
                ("col", C.POINTER(C.c_int)), ("val", C.POINTER(C.c_double))]


class Csr(C.Structure):
    _fields_ = [("n", C.c_int), ("nnz", C.c_int), ("rp", C.POINTER(C.c_int)),
                ("col", C.POINTER(C.c_int)), ("val", C.POINTER(C.c_double))]


class CprOpts(C.Structure):
    _fields_ = [("decouple", C.c_int), ("order", C.c_int), ("form", C.c_int),
                ("px", C.c_int), ("py", C.c_int), ("overlap", C.c_int),
                ("theta", C.c_double), ("max_coarse", C.c_int), ("max_levels", C.c_int),
                ("match_rounds", C.c_int), ("agg_passes", C.c_int), ("kcycle", C.c_int),
                ("amg_cycles", C.c_int), ("exact_stages", C.c_int)]


def cpr_opts(decouple=DEC_QI, order=ORD_POTENTIAL, form=CPR_TWO_STAGE, px=4, py=4, overlap=1,
             theta=0.25, max_coarse=500, max_levels=20, match_rounds=4, agg_passes=2, kcycle=1,
             amg_cycles=AMG_CYCLES, exact_stages=0):
    return CprOpts(decouple, order, form, px, py, overlap, theta, max_coarse, max_levels,
                   match_rounds, agg_passes, kcycle, amg_cycles, exact_stages)


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.om_model_create.argtypes = [C.POINTER(vp), C.c_int, C.c_int, C.c_int, C.c_double,
                                  C.c_double, C.c_double, C.c_double, f64p, f64p, f64p, f64p,
                                  f64p, C.c_int, i32p, i32p, i32p, i32p, f64p, f64p, f64p]
    L.om_model_destroy.argtypes = [vp]
    L.om_initial_state.argtypes = [vp, f64p]
    L.om_residual.argtypes = [vp, f64p, f64p, C.c_double, f64p]
    L.om_scaled_norm.argtypes = [vp, f64p, C.c_double]
    L.om_scaled_norm.restype = C.c_double
    L.om_accumulation.argtypes = [vp, f64p, f64p, f64p]
    L.om_well_rates.argtypes = [vp, f64p, f64p, f64p]
    L.om_potential.argtypes = [vp, f64p, f64p]
    L.om_api_jacobian_nnzb.argtypes = [vp]
    L.om_api_jacobian.argtypes = [vp, f64p, f64p, C.c_double, i32p, i32p, f64p, f64p]
    L.om_api_wells.argtypes = [vp, f64p, f64p]
    L.om_potential_order.argtypes = [C.c_int, f64p, i32p, i32p]
    L.om_decouple.argtypes = [C.POINTER(Bsr), vp, C.c_int, C.c_int]
    L.om_bsr_spmv.argtypes = [C.POINTER(Bsr), f64p, f64p]
    L.om_bilu0.argtypes = [C.POINTER(Bsr), f64p, i32p]
    L.om_bilu0_solve.argtypes = [C.POINTER(Bsr), f64p, i32p, f64p]
    L.om_dense_lu.argtypes = [C.c_int, f64p, i32p]
    L.om_dense_lu_solve.argtypes = [C.c_int, f64p, i32p, f64p]
    L.om_strength_match.argtypes = [C.POINTER(Csr), C.c_double, C.c_int, i32p]
    L.om_coupling_weights.argtypes = [C.POINTER(Csr), f64p, f64p]
    L.om_join_targets.argtypes = [C.POINTER(Csr), C.c_double, i32p, i32p]
    L.om_galerkin.argtypes = [C.POINTER(Csr), i32p, C.c_int, C.POINTER(Csr)]
    L.om_aggregate.argtypes = [C.POINTER(Csr), C.c_double, C.c_int, i32p]
    L.om_csr_free.argtypes = [C.POINTER(Csr)]
    L.om_api_cpr_create.argtypes = [C.POINTER(Bsr), vp, f64p, C.POINTER(CprOpts),
                                    C.POINTER(C.c_int)]
    L.om_api_cpr_create.restype = vp
    L.om_api_cpr_destroy.argtypes = [vp]
    L.om_cpr_apply.argtypes = [vp, f64p, f64p]
    L.om_api_amg_nlev.argtypes = [vp]
    L.om_api_amg_level_size.argtypes = [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.om_api_amg_copy_level.argtypes = [vp, C.c_int, i32p, i32p, f64p, f64p, vp]
    L.om_api_amg_vcycle.argtypes = [vp, f64p, f64p]
    L.om_api_ras_nsub.argtypes = [vp]
    L.om_api_ras_sub_size.argtypes = [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.om_api_ras_copy_sub.argtypes = [vp, C.c_int, i32p, u8p, i32p, i32p, f64p, f64p]
    L.om_api_ras_apply.argtypes = [vp, f64p, f64p]
    L.om_api_amg_create.argtypes = [C.POINTER(Csr), C.c_double, C.c_int, C.c_int, C.c_int,
                                    C.c_int, C.c_int, C.POINTER(C.c_int)]
    L.om_api_amg_create.restype = vp
    L.om_api_amg_destroy.argtypes = [vp]
    L.om_api_amg_h_nlev.argtypes = [vp]
    L.om_api_amg_h_level_size.argtypes = [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.om_api_amg_h_copy_level.argtypes = [vp, C.c_int, i32p, i32p, f64p, f64p, vp]
    L.om_api_amg_h_vcycle.argtypes = [vp, f64p, f64p]
    L.om_fgmres.argtypes = [C.POINTER(Bsr), vp, f64p, f64p, C.c_int, C.c_double, C.c_int,
                            C.POINTER(C.c_int), C.POINTER(C.c_double), vp]
    L.om_bicgstab.argtypes = [C.POINTER(Bsr), vp, f64p, f64p, C.c_double, C.c_int,
                              C.POINTER(C.c_int), C.POINTER(C.c_double)]
    L.om_newton_step.argtypes = [vp, f64p, C.c_double, C.POINTER(CprOpts), C.c_int, C.c_double,
                                 C.c_int, C.c_double, C.c_int, C.c_int, C.c_int, C.c_double,
                                 C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), f64p, f64p,
                                 f64p, f64p]
    _lib = L
    return L


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class BsrMatrix:
    """Block-CSR matrix with 2x2 blocks held in numpy arrays (rp, col, val[nnzb,2,2])."""

    def __init__(self, rp, col, val):
        self.rp = _i32(rp)
        self.col = _i32(col)
        self.val = _f64(val).reshape(-1, 2, 2)
        self.nb = len(self.rp) - 1

    def cstruct(self):
        s = Bsr(self.nb, len(self.col), self.rp.ctypes.data_as(C.POINTER(C.c_int)),
                self.col.ctypes.data_as(C.POINTER(C.c_int)),
                self.val.ctypes.data_as(C.POINTER(C.c_double)))
        s._keep = (self.rp, self.col, self.val)
        return s

    def copy(self):
        return BsrMatrix(self.rp.copy(), self.col.copy(), self.val.copy())

    def to_dense(self):
        N = 2 * self.nb
        D = np.zeros((N, N))
        for i in range(self.nb):
            for z in range(self.rp[i], self.rp[i + 1]):
                j = self.col[z]
                D[2 * i:2 * i + 2, 2 * j:2 * j + 2] = self.val[z]
        return D

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.bsr_matrix((self.val, self.col, self.rp), shape=(2 * self.nb, 2 * self.nb))

    def matvec(self, x):
        y = np.zeros(2 * self.nb)
        lib().om_bsr_spmv(C.byref(self.cstruct()), _f64(x), y)
        return y

    def find(self, i, j):
        for z in range(self.rp[i], self.rp[i + 1]):
            if self.col[z] == j:
                return z
        return -1


class CsrMatrix:
    def __init__(self, rp, col, val, n=None):
        self.rp = _i32(rp)
        self.col = _i32(col)
        self.val = _f64(val)
        self.n = len(self.rp) - 1 if n is None else n

    def cstruct(self):
        s = Csr(self.n, len(self.col), self.rp.ctypes.data_as(C.POINTER(C.c_int)),
                self.col.ctypes.data_as(C.POINTER(C.c_int)),
                self.val.ctypes.data_as(C.POINTER(C.c_double)))
        s._keep = (self.rp, self.col, self.val)
        return s

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.rp), shape=(self.n, self.n))


class Model:
    """The discretised two-phase model built from a `workloads` description."""

    def __init__(self, w):
        from workloads import flat_wells
        L = lib()
        g, c = w["grid"], w["const"]
        fw = flat_wells(w)
        consts = np.array([c["beta_c"], c["alpha_c"], c["rho_o"], c["rho_w"], c["p_ref"],
                           c["z_ref"], c["c_o"], c["c_w"], c["c_r"], c["mu_o"], c["mu_w"],
                           c["grav"]], dtype=np.float64)
        h = C.c_void_p()
        L.om_model_create(C.byref(h), g["nx"], g["ny"], g["nz"], g["dx"], g["dy"], g["dz"],
                          g["top"], _f64(w["kx"]), _f64(w["ky"]), _f64(w["kz"]),
                          _f64(w["phi"]), consts, len(w["wells"]), fw["ptr"], fw["cells"],
                          fw["kind"], fw["ctrl"], fw["target"], fw["rw"], fw["skin"])
        self.h = h
        self.w = w
        self.n = g["n"]
        self.nw = len(w["wells"])
        self.N = 2 * (self.n + self.nw)
        self.nperf = int(fw["ptr"][-1]) if self.nw else 0

    def __del__(self):
        try:
            if self.h:
                lib().om_model_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def initial_state(self):
        x = np.zeros(self.N)
        lib().om_initial_state(self.h, x)
        if "sw0" in self.w:
            x[1:2 * self.n:2] = self.w["sw0"]
        return x

    def residual(self, x, xold, dt):
        F = np.zeros(self.N)
        lib().om_residual(self.h, _f64(x), _f64(xold), float(dt), F)
        return F

    def jacobian(self, x, xold, dt):
        L = lib()
        nnzb = L.om_api_jacobian_nnzb(self.h)
        rp = np.zeros(self.n + self.nw + 1, np.int32)
        col = np.zeros(nnzb, np.int32)
        val = np.zeros(4 * nnzb)
        F = np.zeros(self.N)
        L.om_api_jacobian(self.h, _f64(x), _f64(xold), float(dt), rp, col, val, F)
        return BsrMatrix(rp, col, val), F

    def scaled_norm(self, F, dt):
        return lib().om_scaled_norm(self.h, _f64(F), float(dt))

    def accumulation(self, x):
        ao, aw = np.zeros(self.n), np.zeros(self.n)
        lib().om_accumulation(self.h, _f64(x), ao, aw)
        return ao, aw

    def well_rates(self, x):
        qo, qw = np.zeros(max(self.nperf, 1)), np.zeros(max(self.nperf, 1))
        lib().om_well_rates(self.h, _f64(x), qo, qw)
        return qo[:self.nperf], qw[:self.nperf]

    def well_index(self):
        wi, zb = np.zeros(max(self.nperf, 1)), np.zeros(max(self.nw, 1))
        lib().om_api_wells(self.h, wi, zb)
        return wi[:self.nperf], zb[:self.nw]

    def potential(self, x):
        ph = np.zeros(self.n)
        lib().om_potential(self.h, _f64(x), ph)
        return ph

    def newton_step(self, x, dt, opts=None, restart=30, rtol=1e-8, maxit=300, ntol=1e-8,
                    max_newton=20, exact_linear=False, forcing=0, ds_max=0.2, krylov=0,
                    norms=False):
        """One implicit step in place; returns (status, newton_its, linear_its, hist), and
        with norms=True also a dict of per-iteration ||F||_2, ||b - J y||_2 and the
        linear tolerance used."""
        opts = cpr_opts() if opts is None else opts
        xx = _f64(x).copy()
        ni, li = C.c_int(), C.c_int()
        hist = np.zeros(max_newton + 1)
        fn, rn, eta = (np.full(max_newton + 1, np.nan) for _ in range(3))
        rc = lib().om_newton_step(self.h, xx, float(dt), C.byref(opts), restart, rtol, maxit,
                                  ntol, max_newton, int(exact_linear), int(forcing),
                                  float(ds_max), int(krylov), C.byref(ni), C.byref(li), hist,
                                  fn, rn, eta)
        if rc == 0:
            x[:] = xx
        out = (rc, ni.value, li.value, hist[:ni.value + 1])
        if norms:
            k = ni.value
            return out + (dict(fnorm=fn[:k], rnorm=rn[:k], eta=eta[:k]),)
        return out


def potential_order(phi, cells=None):
    """Eq 30: cells sorted by descending potential (ties by ascending index)."""
    phi = _f64(phi)
    cells = _i32(np.arange(len(phi)) if cells is None else cells)
    perm = np.zeros(len(cells), np.int32)
    rc = lib().om_potential_order(len(cells), phi, cells, perm)
    if rc:
        raise ValueError("non-finite potential")
    return perm


def decouple(A, b, ncell, kind):
    """Return (D^-1 A, D^-1 b) as new arrays (Eq 29)."""
    A2 = A.copy()
    b2 = None if b is None else _f64(b).copy()
    lib().om_decouple(C.byref(A2.cstruct()),
                      None if b2 is None else b2.ctypes.data_as(C.c_void_p), ncell, kind)
    return A2, b2


def bilu0(A):
    """In-place-style block ILU(0) on a copy; returns (LU, dinv, diag)."""
    LU = A.copy()
    dinv = np.zeros(4 * LU.nb)
    diag = np.zeros(LU.nb, np.int32)
    rc = lib().om_bilu0(C.byref(LU.cstruct()), dinv, diag)
    if rc:
        raise ValueError(f"singular pivot block at row {rc - 1}")
    return LU, dinv.reshape(-1, 2, 2), diag


def bilu0_solve(LU, dinv, diag, v):
    out = _f64(v).copy()
    lib().om_bilu0_solve(C.byref(LU.cstruct()), _f64(dinv).reshape(-1), _i32(diag), out)
    return out


def dense_lu_solve(A, b):
    n = A.shape[0]
    lu = _f64(A).copy()
    piv = np.zeros(n, np.int32)
    rc = lib().om_dense_lu(n, lu, piv)
    if rc:
        raise ValueError("singular matrix")
    x = _f64(b).copy()
    lib().om_dense_lu_solve(n, lu, piv, x)
    return x


def extract_pressure(A, ncell):
    rows, cols, vals = [0], [], []
    for i in range(ncell):
        for z in range(A.rp[i], A.rp[i + 1]):
            if A.col[z] < ncell:
                cols.append(A.col[z])
                vals.append(A.val[z, 0, 0])
        rows.append(len(cols))
    return CsrMatrix(rows, cols, vals)


def aggregate(A, theta=0.25, rounds=4):
    """One aggregation pass (matching, joins, numbering): (agg, number of aggregates)."""
    agg = np.zeros(A.n, np.int32)
    nc = lib().om_aggregate(C.byref(A.cstruct()), theta, rounds, agg)
    return agg, nc


def strength_match(A, theta=0.25, rounds=4):
    m = np.zeros(A.n, np.int32)
    lib().om_strength_match(C.byref(A.cstruct()), theta, rounds, m)
    return m


def galerkin(A, agg, nc):
    out = Csr()
    lib().om_galerkin(C.byref(A.cstruct()), _i32(agg), nc, C.byref(out))
    nnz = out.nnz
    R = CsrMatrix(np.ctypeslib.as_array(out.rp, (nc + 1,)).copy(),
                  np.ctypeslib.as_array(out.col, (max(nnz, 1),))[:nnz].copy(),
                  np.ctypeslib.as_array(out.val, (max(nnz, 1),))[:nnz].copy(), n=nc)
    lib().om_csr_free(C.byref(out))
    return R


class Amg:
    """Standalone AMG hierarchy on a scalar CSR matrix."""

    def __init__(self, A, theta=0.25, max_coarse=500, max_levels=20, rounds=4, passes=2,
                 kcycle=2):
        rc = C.c_int()
        self._A = A.cstruct()
        self.h = lib().om_api_amg_create(C.byref(self._A), theta, max_coarse, max_levels,
                                         rounds, passes, kcycle, C.byref(rc))
        self.rc = rc.value
        if rc.value == 1:
            raise ValueError("AMG coarsening stalled above the dense coarsest size")
        if rc.value:
            raise ValueError("coarsest matrix singular")

    def __del__(self):
        try:
            lib().om_api_amg_destroy(self.h)
        except Exception:
            pass

    @property
    def nlev(self):
        return lib().om_api_amg_h_nlev(self.h)

    def level(self, l):
        n, nnz = C.c_int(), C.c_int()
        lib().om_api_amg_h_level_size(self.h, l, C.byref(n), C.byref(nnz))
        n, nnz = n.value, nnz.value
        rp = np.zeros(n + 1, np.int32); col = np.zeros(max(nnz, 1), np.int32)
        val = np.zeros(max(nnz, 1)); l1 = np.zeros(max(n, 1)); agg = np.zeros(max(n, 1), np.int32)
        lib().om_api_amg_h_copy_level(self.h, l, rp, col, val, l1, agg.ctypes.data_as(C.c_void_p))
        return dict(A=CsrMatrix(rp, col[:nnz], val[:nnz], n=n), l1=l1[:n],
                    agg=agg[:n] if l < self.nlev - 1 else None)

    def vcycle(self, b):
        x = np.zeros(len(b))
        lib().om_api_amg_h_vcycle(self.h, _f64(b), x)
        return x


class Cpr:
    """CPR preconditioner (two-stage or FPF) on an already decoupled matrix."""

    def __init__(self, Adec, model, x, opts=None):
        self.opts = cpr_opts() if opts is None else opts
        self.A = Adec
        self._A = Adec.cstruct()
        rc = C.c_int()
        self.h = lib().om_api_cpr_create(C.byref(self._A), model.h, _f64(x), C.byref(self.opts),
                                         C.byref(rc))
        self.rc = rc.value
        if rc.value:
            raise ValueError(f"CPR setup failed ({rc.value})")
        self.model = model

    def __del__(self):
        try:
            lib().om_api_cpr_destroy(self.h)
        except Exception:
            pass

    def apply(self, f):
        x = np.zeros(len(f))
        lib().om_cpr_apply(self.h, _f64(f), x)
        return x

    def amg_levels(self):
        L = lib()
        out = []
        for l in range(L.om_api_amg_nlev(self.h)):
            n, nnz = C.c_int(), C.c_int()
            L.om_api_amg_level_size(self.h, l, C.byref(n), C.byref(nnz))
            n, nnz = n.value, nnz.value
            rp = np.zeros(n + 1, np.int32); col = np.zeros(max(nnz, 1), np.int32)
            val = np.zeros(max(nnz, 1)); l1 = np.zeros(max(n, 1)); agg = np.zeros(max(n, 1), np.int32)
            L.om_api_amg_copy_level(self.h, l, rp, col, val, l1, agg.ctypes.data_as(C.c_void_p))
            out.append(dict(A=CsrMatrix(rp, col[:nnz], val[:nnz], n=n), l1=l1[:n], agg=agg[:n]))
        out[-1]["agg"] = None
        return out

    def amg_vcycle(self, b):
        x = np.zeros(len(b))
        lib().om_api_amg_vcycle(self.h, _f64(b), x)
        return x

    def subdomains(self):
        L = lib()
        out = []
        for s in range(L.om_api_ras_nsub(self.h)):
            m, nnzb = C.c_int(), C.c_int()
            L.om_api_ras_sub_size(self.h, s, C.byref(m), C.byref(nnzb))
            m, nnzb = m.value, nnzb.value
            glob = np.zeros(max(m, 1), np.int32); owned = np.zeros(max(m, 1), np.uint8)
            rp = np.zeros(m + 1, np.int32); col = np.zeros(max(nnzb, 1), np.int32)
            val = np.zeros(4 * max(nnzb, 1)); dinv = np.zeros(4 * max(m, 1))
            L.om_api_ras_copy_sub(self.h, s, glob, owned, rp, col, val, dinv)
            out.append(dict(glob=glob[:m], owned=owned[:m].astype(bool),
                            LU=BsrMatrix(rp, col[:nnzb], val[:4 * nnzb]),
                            dinv=dinv[:4 * m].reshape(-1, 2, 2)))
        return out

    def ras_apply(self, r):
        y = np.zeros(len(r))
        lib().om_api_ras_apply(self.h, _f64(r), y)
        return y


def bicgstab(A, b, P=None, rtol=1e-8, maxit=300):
    """Right-preconditioned BiCGSTAB from zero; returns (x, status, iters, relres)."""
    x = np.zeros(len(b))
    its, rr = C.c_int(), C.c_double()
    st = lib().om_bicgstab(C.byref(A.cstruct()), None if P is None else P.h, _f64(b), x, rtol,
                           maxit, C.byref(its), C.byref(rr))
    return x, st, its.value, rr.value


def fgmres(A, b, P=None, restart=30, rtol=1e-8, maxit=300, history=False):
    """Right-preconditioned FGMRES(restart) from zero; returns (x, status, iters, relres[, hist])."""
    x = np.zeros(len(b))
    its, rr = C.c_int(), C.c_double()
    hist = np.zeros(maxit + 1)
    st = lib().om_fgmres(C.byref(A.cstruct()), None if P is None else P.h, _f64(b), x, restart,
                         rtol, maxit, C.byref(its), C.byref(rr), hist.ctypes.data_as(C.c_void_p))
    if history:
        return x, st, its.value, rr.value, hist[:its.value]
    return x, st, its.value, rr.value
