"""Python binding of libr2p.so (argument marshalling only).

Every numerical step runs in the HIP kernels of the library.  PyTorch is
used for device memory (float64 / int32 tensors on a ROCm device) and for
the current HIP stream.  Importing this module does not touch the GPU; the
library is loaded on first use and a missing build raises RuntimeError.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libr2p.so")

OK, NOT_CONVERGED, BREAKDOWN = 0, 1, 2
DEC_NONE, DEC_QI, DEC_ABF = 0, 1, 2
ORDER_NATURAL, ORDER_POTENTIAL = 0, 1
CPR_TWO_STAGE, CPR_FPF = 0, 1
FP64, FP32 = 0, 1
FORCING_FIXED, FORCING_EW = 0, 1

_lib = None


class R2PError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"r2p error {code}: {msg}")
        self.code = code


class ModelDesc(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double), ("top", C.c_double),
                ("kx", C.c_void_p), ("ky", C.c_void_p), ("kz", C.c_void_p), ("phi", C.c_void_p),
                ("consts", C.c_double * 12), ("nw", C.c_int),
                ("w_ptr", C.c_void_p), ("w_cell", C.c_void_p), ("w_kind", C.c_void_p),
                ("w_ctrl", C.c_void_p), ("w_target", C.c_void_p), ("w_rw", C.c_void_p),
                ("w_skin", C.c_void_p), ("device", C.c_int)]


class CprOpts(C.Structure):
    _fields_ = [("decouple", C.c_int), ("order", C.c_int), ("form", C.c_int),
                ("px", C.c_int), ("py", C.c_int), ("overlap", C.c_int),
                ("theta", C.c_double), ("max_coarse", C.c_int), ("max_levels", C.c_int),
                ("match_rounds", C.c_int), ("agg_passes", C.c_int), ("precision", C.c_int),
                ("kcycle", C.c_int), ("amg_cycles", C.c_int)]


class SolveOpts(C.Structure):
    _fields_ = [("restart", C.c_int), ("maxit", C.c_int), ("rtol", C.c_double),
                ("method", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int), ("status", C.c_int), ("relres", C.c_double),
                ("ms_total", C.c_double), ("reorth", C.c_int)]


class NewtonOpts(C.Structure):
    _fields_ = [("max_newton", C.c_int), ("tol", C.c_double), ("forcing", C.c_int),
                ("ds_max", C.c_double), ("cpr", CprOpts), ("lin", SolveOpts),
                ("guess_rule", C.c_int)]


class NewtonInfo(C.Structure):
    _fields_ = [("status", C.c_int), ("newton_its", C.c_int), ("linear_its", C.c_int),
                ("used_guess", C.c_int), ("res_hist", C.c_double * 32),
                ("ms_assemble", C.c_double), ("ms_setup", C.c_double),
                ("ms_solve", C.c_double), ("ms_total", C.c_double),
                ("ms_decouple", C.c_double), ("ms_order", C.c_double),
                ("ms_ras_setup", C.c_double), ("ms_amg_setup", C.c_double),
                ("ms_update", C.c_double), ("setup_status", C.c_int)]


def cpr_opts(decouple=DEC_QI, order=ORDER_POTENTIAL, form=CPR_TWO_STAGE, px=4, py=4, overlap=1,
             theta=0.25, max_coarse=500, max_levels=20, match_rounds=4, agg_passes=2,
             precision=FP64, kcycle=1, amg_cycles=2):
    return CprOpts(decouple, order, form, px, py, overlap, theta, max_coarse, max_levels,
                   match_rounds, agg_passes, precision, kcycle, amg_cycles)


KRYLOV_FGMRES, KRYLOV_BICGSTAB = 0, 1


def solve_opts(restart=30, maxit=300, rtol=1e-8, method=KRYLOV_FGMRES):
    return SolveOpts(restart, maxit, rtol, method)


GUESS_SCALED_INF, GUESS_L2, GUESS_TRY = 0, 1, 2


def newton_opts(max_newton=20, tol=1e-8, forcing=FORCING_FIXED, ds_max=0.2, cpr=None, lin=None,
                guess_rule=GUESS_SCALED_INF):
    return NewtonOpts(max_newton, tol, forcing, ds_max, cpr or cpr_opts(), lin or solve_opts(),
                      guess_rule)


EXPORTS = ["r2p_model_create", "r2p_model_destroy", "r2p_model_sizes", "r2p_initial_state",
           "r2p_jacobian_create", "r2p_jacobian_destroy", "r2p_assemble_jacobian",
           "r2p_residual_norm", "r2p_residual_norm_noalloc", "r2p_spmv", "r2p_jacobian_export", "r2p_cpr_create",
           "r2p_cpr_destroy", "r2p_setup_cpr", "r2p_cpr_apply", "r2p_amg_vcycle",
           "r2p_ras_apply", "r2p_amg_info", "r2p_amg_export_level", "r2p_ras_info",
           "r2p_ras_export", "r2p_solve", "r2p_newton_step", "r2p_default_newton_opts",
           "r2p_cnn_param_count", "r2p_cnn_create", "r2p_cnn_destroy", "r2p_cnn_set_params",
           "r2p_cnn_get_params", "r2p_cnn_get_grads", "r2p_cnn_forward", "r2p_cnn_backward",
           "r2p_cnn_sgd_step", "r2p_cnn_conv", "r2p_cnn_conv_dw", "r2p_cnn_features",
           "r2p_cnn_targets", "r2p_cnn_warm_start", "r2p_last_error"]


def load(path=LIB_PATH):
    """Load libr2p.so; raises RuntimeError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1701_06254_amd.build.build()")
    L = C.CDLL(path)
    vp, ip, dp = C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_double)
    sig = {
        "r2p_model_create": [C.POINTER(ModelDesc), C.POINTER(vp)],
        "r2p_model_destroy": [vp],
        "r2p_model_sizes": [vp, ip, ip, ip],
        "r2p_initial_state": [vp, vp, vp],
        "r2p_jacobian_create": [vp, C.POINTER(vp)],
        "r2p_jacobian_destroy": [vp],
        "r2p_assemble_jacobian": [vp, vp, vp, C.c_double, vp, vp, vp],
        "r2p_residual_norm": [vp, vp, C.c_double, dp, vp],
        "r2p_residual_norm_noalloc": [vp, vp, C.c_double, vp, vp],
        "r2p_spmv": [vp, vp, vp, vp],
        "r2p_jacobian_export": [vp, ip, vp, vp, vp, vp],
        "r2p_cpr_create": [C.POINTER(vp)],
        "r2p_cpr_destroy": [vp],
        "r2p_setup_cpr": [vp, C.POINTER(CprOpts), vp, vp],
        "r2p_cpr_apply": [vp, vp, vp, vp],
        "r2p_amg_vcycle": [vp, vp, vp, vp],
        "r2p_ras_apply": [vp, vp, vp, vp],
        "r2p_amg_info": [vp, C.c_int, ip, ip, ip],
        "r2p_amg_export_level": [vp, C.c_int, vp, vp, vp, vp, vp, vp],
        "r2p_ras_info": [vp, C.c_int, ip, ip, ip, ip],
        "r2p_ras_export": [vp, C.c_int, vp, vp, vp, vp, vp, vp, vp, vp],
        "r2p_solve": [vp, vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveInfo), vp],
        "r2p_newton_step": [vp, vp, C.c_double, vp, C.POINTER(NewtonOpts),
                            C.POINTER(NewtonInfo), vp],
        "r2p_default_newton_opts": [C.POINTER(NewtonOpts)],
        "r2p_cnn_param_count": [C.c_int, C.POINTER(C.c_long)],
        "r2p_cnn_create": [C.c_int, C.POINTER(vp)],
        "r2p_cnn_destroy": [vp],
        "r2p_cnn_set_params": [vp, vp],
        "r2p_cnn_get_params": [vp, vp],
        "r2p_cnn_get_grads": [vp, vp],
        "r2p_cnn_forward": [vp, vp, C.c_int, C.c_int, C.c_int, C.c_int, vp, vp],
        "r2p_cnn_backward": [vp, vp, vp, C.c_int, C.c_int, C.c_int, C.c_int, dp, vp],
        "r2p_cnn_sgd_step": [vp, C.c_float, vp],
        "r2p_cnn_conv": [vp, C.c_int, C.c_int, C.c_int, C.c_int, vp, vp, vp, vp, C.c_int,
                         C.c_int, vp, vp, vp],
        "r2p_cnn_conv_dw": [vp, vp, C.c_int, C.c_int, C.c_int, C.c_int, vp, vp, vp],
        "r2p_cnn_features": [vp, vp, C.c_double, vp, vp],
        "r2p_cnn_targets": [vp, vp, vp, vp, vp],
        "r2p_cnn_warm_start": [vp, vp, vp, C.c_double, vp, vp],
        "r2p_last_error": [],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    L.r2p_default_newton_opts.restype = None
    L.r2p_last_error.restype = C.c_char_p
    _lib = L
    return L


def _check(rc, soft_ok=False):
    if rc < 0 or (rc > 0 and not soft_ok):
        raise R2PError(rc, load().r2p_last_error().decode())
    return rc


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _np(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class Model:
    """A two-phase model resident on one GPU (r2p_model)."""

    def __init__(self, w, device=0):
        from workloads import flat_wells
        L = load()
        g, c = w["grid"], w["const"]
        fw = flat_wells(w)
        self._keep = [_np(w["kx"], np.float64), _np(w["ky"], np.float64),
                      _np(w["kz"], np.float64), _np(w["phi"], np.float64), fw["ptr"],
                      fw["cells"], fw["kind"], fw["ctrl"], fw["target"], fw["rw"], fw["skin"]]
        k = self._keep
        d = ModelDesc()
        d.nx, d.ny, d.nz = g["nx"], g["ny"], g["nz"]
        d.dx, d.dy, d.dz, d.top = g["dx"], g["dy"], g["dz"], g["top"]
        d.kx, d.ky, d.kz, d.phi = (k[0].ctypes.data, k[1].ctypes.data, k[2].ctypes.data,
                                   k[3].ctypes.data)
        for i, key in enumerate(["beta_c", "alpha_c", "rho_o", "rho_w", "p_ref", "z_ref", "c_o",
                                 "c_w", "c_r", "mu_o", "mu_w", "grav"]):
            d.consts[i] = c[key]
        d.nw = len(w["wells"])
        d.w_ptr, d.w_cell, d.w_kind, d.w_ctrl = (k[4].ctypes.data, k[5].ctypes.data,
                                                 k[6].ctypes.data, k[7].ctypes.data)
        d.w_target, d.w_rw, d.w_skin = k[8].ctypes.data, k[9].ctypes.data, k[10].ctypes.data
        d.device = device
        h = C.c_void_p()
        _check(L.r2p_model_create(C.byref(d), C.byref(h)))
        self.h = h
        self.w = w
        self.device = device
        n, nw, npf = C.c_int(), C.c_int(), C.c_int()
        _check(L.r2p_model_sizes(h, C.byref(n), C.byref(nw), C.byref(npf)))
        self.n, self.nw, self.nperf = n.value, nw.value, npf.value
        self.N = 2 * (self.n + self.nw)

    def __del__(self):
        try:
            if getattr(self, "h", None):
                load().r2p_model_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def tensor(self, n=None):
        import torch
        return torch.zeros(self.N if n is None else n, dtype=torch.float64,
                           device=f"cuda:{self.device}")

    def initial_state(self):
        x = self.tensor()
        _check(load().r2p_initial_state(self.h, _ptr(x), _stream()))
        return x

    def residual_norm(self, b, dt):
        v = C.c_double()
        rc = load().r2p_residual_norm(self.h, _ptr(b), float(dt), C.byref(v), _stream())
        if rc == -4:
            return float("nan")
        _check(rc)
        return v.value

    def residual_norm_noalloc(self, b, dt, out):
        """Scaled norm into the device double `out` (asynchronous; no allocation)."""
        _check(load().r2p_residual_norm_noalloc(self.h, _ptr(b), float(dt), _ptr(out), _stream()))
        return out

    def newton_step(self, x, dt, opts=None, x_guess=None):
        """One implicit step on x in place; returns the NewtonInfo record."""
        info = NewtonInfo()
        o = newton_opts() if opts is None else opts
        rc = load().r2p_newton_step(self.h, _ptr(x), float(dt), _ptr(x_guess), C.byref(o),
                                    C.byref(info), _stream())
        _check(rc, soft_ok=True)
        return info


class Jacobian:
    def __init__(self, model):
        self.model = model
        h = C.c_void_p()
        _check(load().r2p_jacobian_create(model.h, C.byref(h)))
        self.h = h

    def __del__(self):
        try:
            if getattr(self, "h", None):
                load().r2p_jacobian_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def assemble(self, x, x_old, dt, b=None):
        """J <- dF/dx at x; returns b = -F(x) (device tensor)."""
        b = self.model.tensor() if b is None else b
        _check(load().r2p_assemble_jacobian(self.model.h, _ptr(x), _ptr(x_old), float(dt), self.h,
                                            _ptr(b), _stream()))
        return b

    def spmv(self, x, y=None):
        y = self.model.tensor() if y is None else y
        _check(load().r2p_spmv(self.h, _ptr(x), _ptr(y), _stream()))
        return y

    def export(self):
        """Host block-CSR copy: (rp, col, val[nnzb,2,2])."""
        L = load()
        nnzb = C.c_int()
        _check(L.r2p_jacobian_export(self.h, C.byref(nnzb), None, None, None, _stream()))
        nb = self.model.n + self.model.nw
        rp = np.zeros(nb + 1, np.int32)
        col = np.zeros(nnzb.value, np.int32)
        val = np.zeros(4 * nnzb.value)
        _check(L.r2p_jacobian_export(self.h, C.byref(nnzb), rp.ctypes.data_as(C.c_void_p),
                                     col.ctypes.data_as(C.c_void_p),
                                     val.ctypes.data_as(C.c_void_p), _stream()))
        return rp, col, val.reshape(-1, 2, 2)


class Cpr:
    def __init__(self):
        h = C.c_void_p()
        _check(load().r2p_cpr_create(C.byref(h)))
        self.h = h
        self.J = None

    def __del__(self):
        try:
            if getattr(self, "h", None):
                load().r2p_cpr_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def setup(self, J, opts=None):
        self.opts = cpr_opts() if opts is None else opts
        _check(load().r2p_setup_cpr(J.h, C.byref(self.opts), self.h, _stream()))
        self.J = J
        return self

    def apply(self, f, z=None):
        z = self.J.model.tensor() if z is None else z
        _check(load().r2p_cpr_apply(self.h, _ptr(f), _ptr(z), _stream()))
        return z

    def amg_vcycle(self, fp, xp=None):
        xp = self.J.model.tensor(self.J.model.n) if xp is None else xp
        _check(load().r2p_amg_vcycle(self.h, _ptr(fp), _ptr(xp), _stream()))
        return xp

    def ras_apply(self, r, y=None):
        y = self.J.model.tensor() if y is None else y
        _check(load().r2p_ras_apply(self.h, _ptr(r), _ptr(y), _stream()))
        return y

    def amg_levels(self):
        L = load()
        nlev, n, nnz = C.c_int(), C.c_int(), C.c_int()
        _check(L.r2p_amg_info(self.h, 0, C.byref(nlev), C.byref(n), C.byref(nnz)))
        out = []
        for l in range(nlev.value):
            _check(L.r2p_amg_info(self.h, l, C.byref(nlev), C.byref(n), C.byref(nnz)))
            rp = np.zeros(n.value + 1, np.int32)
            col = np.zeros(max(nnz.value, 1), np.int32)
            val = np.zeros(max(nnz.value, 1))
            l1 = np.zeros(max(n.value, 1))
            agg = np.zeros(max(n.value, 1), np.int32)
            last = l == nlev.value - 1
            _check(L.r2p_amg_export_level(self.h, l, rp.ctypes.data_as(C.c_void_p),
                                          col.ctypes.data_as(C.c_void_p),
                                          val.ctypes.data_as(C.c_void_p),
                                          l1.ctypes.data_as(C.c_void_p),
                                          None if last else agg.ctypes.data_as(C.c_void_p),
                                          _stream()))
            out.append(dict(n=n.value, rp=rp, col=col[:nnz.value], val=val[:nnz.value],
                            l1=l1[:n.value], agg=None if last else agg[:n.value]))
        return out

    def ras_info(self):
        ns = C.c_int()
        _check(load().r2p_ras_info(self.h, -1, C.byref(ns), None, None, None))
        return ns.value

    def ras_subdomain_info(self, s):
        """(local rows, off-diagonal factor blocks, dependency levels) of subdomain s."""
        ns, m, nb, nl = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        _check(load().r2p_ras_info(self.h, s, C.byref(ns), C.byref(m), C.byref(nb),
                                   C.byref(nl)))
        return m.value, nb.value, nl.value

    def ras_subdomain(self, s):
        L = load()
        ns, m, nb, nl = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        _check(L.r2p_ras_info(self.h, s, C.byref(ns), C.byref(m), C.byref(nb), C.byref(nl)))
        m, nb = m.value, nb.value
        glob = np.zeros(max(m, 1), np.int32); level = np.zeros(max(m, 1), np.int32)
        owned = np.zeros(max(m, 1), np.uint8); dinv = np.zeros(4 * max(m, 1))
        erow = np.zeros(max(nb, 1), np.int32); ecol = np.zeros(max(nb, 1), np.int32)
        eval_ = np.zeros(4 * max(nb, 1))
        _check(L.r2p_ras_export(self.h, s, *(a.ctypes.data_as(C.c_void_p) for a in
                                             (glob, level, owned, dinv, erow, ecol, eval_)),
                                _stream()))
        return dict(glob=glob[:m], level=level[:m], owned=owned[:m].astype(bool),
                    dinv=dinv[:4 * m].reshape(-1, 2, 2), erow=erow[:nb], ecol=ecol[:nb],
                    eval=eval_[:4 * nb].reshape(-1, 2, 2), nlevels=nl.value)


def solve(J, P, b, opts=None, y=None):
    """Solve J y = b with CPR-FGMRES or CPR-BiCGSTAB (opts.method); returns (y, SolveInfo)."""
    y = J.model.tensor() if y is None else y
    info = SolveInfo()
    o = solve_opts() if opts is None else opts
    rc = load().r2p_solve(J.h, P.h, _ptr(b), _ptr(y), C.byref(o), C.byref(info), _stream())
    _check(rc, soft_ok=True)
    return y, info


def default_newton_opts():
    o = NewtonOpts()
    load().r2p_default_newton_opts(C.byref(o))
    return o


class Cnn:
    """The warm-start network (r2p_cnn): bf16 activations, FP32 master weights."""

    def __init__(self, blocks=4):
        L = load()
        n = C.c_long()
        _check(L.r2p_cnn_param_count(blocks, C.byref(n)))
        self.nparams = n.value
        self.blocks = blocks
        h = C.c_void_p()
        _check(L.r2p_cnn_create(blocks, C.byref(h)))
        self.h = h

    def __del__(self):
        try:
            if getattr(self, "h", None):
                load().r2p_cnn_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def set_params(self, theta):
        a = _np(theta, np.float32)
        assert a.size == self.nparams
        _check(load().r2p_cnn_set_params(self.h, a.ctypes.data_as(C.c_void_p)))

    def get_params(self):
        a = np.zeros(self.nparams, np.float32)
        _check(load().r2p_cnn_get_params(self.h, a.ctypes.data_as(C.c_void_p)))
        return a

    def get_grads(self):
        a = np.zeros(self.nparams, np.float32)
        _check(load().r2p_cnn_get_grads(self.h, a.ctypes.data_as(C.c_void_p)))
        return a

    def forward(self, feat, shape, out=None):
        """feat: int16 device tensor of bf16 bits [V*32]; shape (nb, nz, ny, nx)."""
        import torch
        nb, nz, ny, nx = shape
        V = nb * nz * ny * nx
        out = torch.empty(2 * V, dtype=torch.float32, device="cuda") if out is None else out
        _check(load().r2p_cnn_forward(self.h, _ptr(feat), nb, nz, ny, nx, _ptr(out), _stream()))
        return out

    def backward(self, feat, target, shape):
        nb, nz, ny, nx = shape
        loss = C.c_double()
        _check(load().r2p_cnn_backward(self.h, _ptr(feat), _ptr(target), nb, nz, ny, nx,
                                       C.byref(loss), _stream()))
        return loss.value

    def step(self, lr):
        _check(load().r2p_cnn_sgd_step(self.h, float(lr), _stream()))

    def warm_start(self, model, x, dt, x_guess=None):
        x_guess = model.tensor() if x_guess is None else x_guess
        _check(load().r2p_cnn_warm_start(model.h, self.h, _ptr(x), float(dt), _ptr(x_guess),
                                         _stream()))
        return x_guess


def cnn_conv(x, shape, w, bias=None, addend=None, mask=None, relu=False, flip=False,
             out=None, outf=None):
    nb, nz, ny, nx = shape
    _check(load().r2p_cnn_conv(_ptr(x), nb, nz, ny, nx, _ptr(w), _ptr(bias), _ptr(addend),
                               _ptr(mask), int(relu), int(flip), _ptr(out), _ptr(outf), _stream()))


def cnn_conv_dw(gy, x, shape, dw, db):
    nb, nz, ny, nx = shape
    _check(load().r2p_cnn_conv_dw(_ptr(gy), _ptr(x), nb, nz, ny, nx, _ptr(dw), _ptr(db),
                                  _stream()))


def cnn_features(model, x, dt, feat=None):
    import torch
    feat = torch.empty(model.n * 32, dtype=torch.int16, device="cuda") if feat is None else feat
    _check(load().r2p_cnn_features(model.h, _ptr(x), float(dt), _ptr(feat), _stream()))
    return feat


def cnn_targets(model, x_old, x_new, target=None):
    import torch
    target = torch.empty(2 * model.n, dtype=torch.float32, device="cuda") if target is None else target
    _check(load().r2p_cnn_targets(model.h, _ptr(x_old), _ptr(x_new), _ptr(target), _stream()))
    return target
