// Model set-up, residual and Jacobian assembly, decoupling, SpMV and the
// Newton update for the two-phase oil-water model.
//
// Paper sections: "Two-phase oil-water flow model" (Eq 1-14), "Numerical
// methods" (Eq 15-23), "Matrix decoupling strategy" (Eq 29, D_QI, D_ABF).
// Readings where the paper is silent: depth positive downward with
// Phi_a = p - gamma_a z (Eq 5 and Eq 10); equations divided by reference
// density (b_a = 1 + c_a (p - p_ref), Eq 6); p_c = 0; Corey krw = s^2,
// kro = (1-s)^2; constant viscosity; mobility upwinded per face with the
// geometric factor harmonic (Eq 16-18); mean face density; the upstream cell
// of face (a < b) is b when Phi_b - Phi_a >= 0; producers use phase
// mobilities and injectors the cell's total mobility (Eq 10); Peaceman's
// anisotropic well index; z_b = depth of the top perforation.
//
// This file is compiled without floating-point contraction so the property
// and flux arithmetic (and with it every upstream decision) is reproducible.
#include <atomic>
#include <algorithm>
#include <mutex>
#include <cmath>
#include <cstring>

#include "r2p_impl.h"

int r2p_noalloc_init(int dev);

constexpr int BS = 256;

// --------------------------------------------------------- property laws
__device__ __forceinline__ double bfac(double c, double p, double pref) {
    return 1.0 + c * (p - pref);
}
__device__ __forceinline__ double gamma_of(const Phys &P, double rho, double c, double p) {
    double b = 1.0 + c * (p - P.p_ref);
    return P.grav * rho * b / 144.0;
}
__device__ __forceinline__ double depth_of(const Phys &P, int k) { return P.top + P.dz * k; }

// ------------------------------------------------------------ geometry
__global__ void k_geometry(Phys P, const double *kx, const double *ky, const double *kz,
                           double *tx, double *ty, double *tz) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= P.n) return;
    int nxy = P.nx * P.ny;
    int i = c % P.nx, j = (c / P.nx) % P.ny, k = c / nxy;
    tx[c] = i + 1 < P.nx ? P.dy * P.dz / (P.dx / (2.0 * kx[c]) + P.dx / (2.0 * kx[c + 1])) : 0.0;
    ty[c] = j + 1 < P.ny ? P.dx * P.dz / (P.dy / (2.0 * ky[c]) + P.dy / (2.0 * ky[c + P.nx])) : 0.0;
    tz[c] = k + 1 < P.nz ? P.dx * P.dy / (P.dz / (2.0 * kz[c]) + P.dz / (2.0 * kz[c + nxy])) : 0.0;
}

// Peaceman well index (equivalent radius for an anisotropic cell) and z_b.
__global__ void k_wells_static(Phys P, const double *kx, const double *ky, const int *w_ptr,
                               const int *perf_cell, const double *w_rw, const double *w_skin,
                               double *perf_wi, double *w_zb, int *perf_well) {
    int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= P.nw) return;
    int nxy = P.nx * P.ny;
    w_zb[w] = depth_of(P, perf_cell[w_ptr[w]] / nxy);
    for (int q = w_ptr[w]; q < w_ptr[w + 1]; q++) {
        int c = perf_cell[q];
        double ryx = sqrt(ky[c] / kx[c]), rxy = sqrt(kx[c] / ky[c]);
        double ro = 0.28 * sqrt(ryx * P.dx * P.dx + rxy * P.dy * P.dy) / (sqrt(ryx) + sqrt(rxy));
        perf_wi[q] = 2.0 * M_PI * P.beta * sqrt(kx[c] * ky[c]) * P.dz / (log(ro / w_rw[w]) + w_skin[w]);
        perf_well[q] = w;
    }
}

__global__ void k_fill_int(int *a, int v, long n) {
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

__global__ void k_cell_perf(int nperf, const int *perf_cell, int *cell_perf) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nperf) cell_perf[perf_cell[q]] = q;
}

extern "C" int r2p_model_create(const r2p_model_desc *d, r2p_model **out) {
    if (!d || !out) { r2p_set_error("NULL argument"); return R2P_EINVAL; }
    *out = nullptr;
    long n = (long)d->nx * d->ny * d->nz;
    if (d->nx <= 0 || d->ny <= 0 || d->nz <= 0 || n > (1L << 30) || d->nw < 0 ||
        !(d->dx > 0) || !(d->dy > 0) || !(d->dz > 0) || !d->kx_host || !d->ky_host ||
        !d->kz_host || !d->phi_host) {
        r2p_set_error("invalid grid description");
        return R2P_EINVAL;
    }
    for (long c = 0; c < n; c++) {
        if (!(d->kx_host[c] > 0) || !(d->ky_host[c] > 0) || !(d->kz_host[c] > 0)) {
            r2p_set_error("permeability must be > 0 (cell %ld)", c);
            return R2P_EINVAL;
        }
        if (!(d->phi_host[c] > 0 && d->phi_host[c] < 1)) {
            r2p_set_error("porosity must lie in (0,1) (cell %ld)", c);
            return R2P_EINVAL;
        }
    }
    int nperf = 0;
    std::vector<int> seen;
    if (d->nw > 0) {
        if (!d->w_ptr_host || !d->w_cell_host || !d->w_kind_host || !d->w_ctrl_host ||
            !d->w_target_host || !d->w_rw_host || !d->w_skin_host || d->w_ptr_host[0] != 0) {
            r2p_set_error("invalid well description");
            return R2P_EINVAL;
        }
        nperf = d->w_ptr_host[d->nw];
        seen.assign(n, 0);
        for (int w = 0; w < d->nw; w++) {
            if (d->w_ptr_host[w + 1] <= d->w_ptr_host[w]) {
                r2p_set_error("well %d has no perforation", w);
                return R2P_EINVAL;
            }
            if ((d->w_kind_host[w] != R2P_INJECTOR && d->w_kind_host[w] != R2P_PRODUCER) ||
                d->w_ctrl_host[w] < 0 || d->w_ctrl_host[w] > 3 || !(d->w_rw_host[w] > 0)) {
                r2p_set_error("well %d: bad kind, control or radius", w);
                return R2P_EINVAL;
            }
            for (int q = d->w_ptr_host[w]; q < d->w_ptr_host[w + 1]; q++) {
                int c = d->w_cell_host[q];
                if (c < 0 || c >= n) { r2p_set_error("perforation %d out of range", q); return R2P_EINVAL; }
                if (seen[c]) { r2p_set_error("cell %d perforated twice", c); return R2P_EINVAL; }
                seen[c] = 1;
            }
        }
    }
    R2P_HIP(hipSetDevice(d->device));
    R2P_TRY(r2p_noalloc_init(d->device));
    r2p_model *m = new r2p_model();
    static std::atomic<unsigned long long> next_serial{1};
    m->serial = next_serial++;
    m->dev = d->device;
    Phys &P = m->ph;
    P.nx = d->nx; P.ny = d->ny; P.nz = d->nz; P.n = (int)n; P.nw = d->nw; P.nperf = nperf;
    P.dx = d->dx; P.dy = d->dy; P.dz = d->dz; P.top = d->top;
    P.beta = d->consts[0]; P.alpha = d->consts[1]; P.rho_o = d->consts[2]; P.rho_w = d->consts[3];
    P.p_ref = d->consts[4]; P.z_ref = d->consts[5]; P.c_o = d->consts[6]; P.c_w = d->consts[7];
    P.c_r = d->consts[8]; P.mu_o = d->consts[9]; P.mu_w = d->consts[10]; P.grav = d->consts[11];
    int rc = 0;
    auto fail = [&](int r) { delete m; return r; };
    if ((rc = m->kx.ensure(n)) || (rc = m->ky.ensure(n)) || (rc = m->kz.ensure(n)) ||
        (rc = m->phi.ensure(n)) || (rc = m->tx.ensure(n)) || (rc = m->ty.ensure(n)) ||
        (rc = m->tz.ensure(n)) || (rc = m->cell_perf.ensure(n)) ||
        (rc = m->perf_cell.ensure(nperf)) || (rc = m->perf_well.ensure(nperf)) ||
        (rc = m->perf_wi.ensure(nperf)) || (rc = m->w_ptr.ensure(d->nw + 1)) ||
        (rc = m->w_kind.ensure(d->nw)) || (rc = m->w_ctrl.ensure(d->nw)) ||
        (rc = m->w_target.ensure(d->nw)) || (rc = m->w_zb.ensure(d->nw)) ||
        (rc = m->w_rw.ensure(d->nw)) || (rc = m->w_skin.ensure(d->nw)) ||
        (rc = m->red.ensure(64)) || (rc = m->pin.ensure(4096)))
        return fail(rc);
#define H2D(dst, src, cnt)                                                              \
    if ((cnt) > 0) {                                                                    \
        hipError_t e_ = hipMemcpy(dst, src, sizeof(*(src)) * (size_t)(cnt), hipMemcpyHostToDevice); \
        if (e_ != hipSuccess) return fail(r2p_hip_fail(e_, "H2D", __FILE__, __LINE__));  \
    }
    H2D(m->kx.p, d->kx_host, n);
    H2D(m->ky.p, d->ky_host, n);
    H2D(m->kz.p, d->kz_host, n);
    H2D(m->phi.p, d->phi_host, n);
    if (d->nw > 0) {
        H2D(m->w_ptr.p, d->w_ptr_host, d->nw + 1);
        H2D(m->perf_cell.p, d->w_cell_host, nperf);
        H2D(m->w_kind.p, d->w_kind_host, d->nw);
        H2D(m->w_ctrl.p, d->w_ctrl_host, d->nw);
        H2D(m->w_target.p, d->w_target_host, d->nw);
        H2D(m->w_rw.p, d->w_rw_host, d->nw);
        H2D(m->w_skin.p, d->w_skin_host, d->nw);
        m->h_w_ptr.assign(d->w_ptr_host, d->w_ptr_host + d->nw + 1);
        m->h_w_cell.assign(d->w_cell_host, d->w_cell_host + nperf);
        m->h_w_kind.assign(d->w_kind_host, d->w_kind_host + d->nw);
        m->h_w_ctrl.assign(d->w_ctrl_host, d->w_ctrl_host + d->nw);
        m->h_w_target.assign(d->w_target_host, d->w_target_host + d->nw);
    }
#undef H2D
    k_geometry<<<r2p_blocks(n, BS), BS>>>(P, m->kx.p, m->ky.p, m->kz.p, m->tx.p, m->ty.p, m->tz.p);
    k_fill_int<<<r2p_blocks(n, BS), BS>>>(m->cell_perf.p, -1, n);
    if (d->nw > 0) {
        k_wells_static<<<r2p_blocks(d->nw, 64), 64>>>(P, m->kx.p, m->ky.p, m->w_ptr.p,
                                                      m->perf_cell.p, m->w_rw.p, m->w_skin.p,
                                                      m->perf_wi.p, m->w_zb.p, m->perf_well.p);
        k_cell_perf<<<r2p_blocks(nperf, BS), BS>>>(nperf, m->perf_cell.p, m->cell_perf.p);
    }
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return fail(r2p_hip_fail(e, "model set-up kernels", __FILE__, __LINE__));
    *out = m;
    return 0;
}

extern "C" int r2p_model_destroy(r2p_model *m) {
    if (m) r2p_newton_work_free(m->newton);
    delete m;
    return 0;
}

extern "C" int r2p_model_sizes(const r2p_model *m, int *n, int *nw, int *nperf) {
    if (!m) { r2p_set_error("NULL model"); return R2P_EINVAL; }
    if (n) *n = m->ph.n;
    if (nw) *nw = m->ph.nw;
    if (nperf) *nperf = m->ph.nperf;
    return 0;
}

// ----------------------------------------------------------- initial state
// Layer pressures of the oil-hydrostatic column through (p_ref, z_ref): each
// layer solves p_k = p_{k-1} + (gamma(p_{k-1}) + gamma(p_k))/2 (z_k - z_{k-1})
// by fixed-point iteration, the discrete equilibrium of the face flux.
__global__ void k_hydro_layers(Phys P, double *pl) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double zprev = P.z_ref, pprev = P.p_ref;
    for (int k = 0; k < P.nz; k++) {
        double z = depth_of(P, k);
        double p = pprev;
        for (int it = 0; it < 100; it++) {
            double pn = pprev + 0.5 * (gamma_of(P, P.rho_o, P.c_o, pprev) +
                                       gamma_of(P, P.rho_o, P.c_o, p)) * (z - zprev);
            if (pn == p) break;
            p = pn;
        }
        pl[k] = p;
        pprev = p;
        zprev = z;
    }
}

__global__ void k_initial_state(Phys P, const double *pl, const int *w_ptr, const int *w_ctrl,
                                const double *w_target, const int *perf_cell, double *x) {
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    int nxy = P.nx * P.ny;
    if (i < P.n) {
        x[2 * i] = pl[i / nxy];
        x[2 * i + 1] = 0.0;
    } else if (i < P.n + P.nw) {
        int w = (int)(i - P.n);
        x[2 * i] = w_ctrl[w] == 0 ? w_target[w] : pl[perf_cell[w_ptr[w]] / nxy];
        x[2 * i + 1] = 0.0;
    }
}

extern "C" int r2p_initial_state(r2p_model *m, double *x, void *stream) {
    if (!m || !x) { r2p_set_error("NULL argument"); return R2P_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    DBuf<double> pl;
    R2P_TRY(pl.ensure(m->ph.nz));
    k_hydro_layers<<<1, 64, 0, s>>>(m->ph, pl.p);
    R2P_LAUNCH();
    long tot = m->ph.n + m->ph.nw;
    k_initial_state<<<r2p_blocks(tot, BS), BS, 0, s>>>(m->ph, pl.p, m->w_ptr.p, m->w_ctrl.p,
                                                       m->w_target.p, m->perf_cell.p, x);
    R2P_LAUNCH();
    R2P_HIP(hipStreamSynchronize(s));   // pl is released on return
    return 0;
}

// ---------------------------------------------------------------- assembly
struct FaceTerms {
    double flux, fpa, fsa, fpb, fsb;
};

// Flux of phase `ph` into cell a from cell b (a < b) and its derivatives with
// respect to (p_a, s_a, p_b, s_b) (Eq 16-18 with the readings above).
__device__ __forceinline__ FaceTerms face_phase(const Phys &P, int ph, double pa, double sa,
                                                double pb, double sb, double dz, double tg) {
    double rho = ph == 0 ? P.rho_o : P.rho_w;
    double cc = ph == 0 ? P.c_o : P.c_w;
    double mu = ph == 0 ? P.mu_o : P.mu_w;
    double ga = gamma_of(P, rho, cc, pa), gb = gamma_of(P, rho, cc, pb);
    double dphi = (pb - pa) - 0.5 * (ga + gb) * dz;
    bool up_b = dphi >= 0.0;
    double pu = up_b ? pb : pa, su = up_b ? sb : sa;
    double kr = ph == 0 ? (1.0 - su) * (1.0 - su) : su * su;
    double dkr = ph == 0 ? -2.0 * (1.0 - su) : 2.0 * su;
    double bu = bfac(cc, pu, P.p_ref);
    double lam = kr * bu / mu;
    FaceTerms t;
    t.flux = P.beta * tg * lam * dphi;
    double dg = P.grav * rho * cc / 144.0;
    double ddphi_a = -1.0 - 0.5 * dg * dz;
    double ddphi_b = 1.0 - 0.5 * dg * dz;
    double dlam_p = kr * cc / mu, dlam_s = dkr * bu / mu;
    t.fpa = P.beta * tg * (lam * ddphi_a + (up_b ? 0.0 : dlam_p * dphi));
    t.fsa = P.beta * tg * (up_b ? 0.0 : dlam_s * dphi);
    t.fpb = P.beta * tg * (lam * ddphi_b + (up_b ? dlam_p * dphi : 0.0));
    t.fsb = P.beta * tg * (up_b ? dlam_s * dphi : 0.0);
    return t;
}

struct PerfTerms {
    double qo, qw, qo_p, qo_s, qo_b, qw_p, qw_s, qw_b;
};

// Perforation rates (Eq 10) and their derivatives.
__device__ __forceinline__ PerfTerms perf_terms(const Phys &P, int kind, double WI, double p,
                                                double s, double pbh, double dzb) {
    double bo = bfac(P.c_o, p, P.p_ref), bw = bfac(P.c_w, p, P.p_ref);
    double lo = (1.0 - s) * (1.0 - s) * bo / P.mu_o, lw = s * s * bw / P.mu_w;
    double lo_p = (1.0 - s) * (1.0 - s) * P.c_o / P.mu_o, lw_p = s * s * P.c_w / P.mu_w;
    double lo_s = -2.0 * (1.0 - s) * bo / P.mu_o, lw_s = 2.0 * s * bw / P.mu_w;
    double dgo = P.grav * P.rho_o * P.c_o / 144.0, dgw = P.grav * P.rho_w * P.c_w / 144.0;
    double dpo = pbh - p - gamma_of(P, P.rho_o, P.c_o, p) * dzb;
    double dpw = pbh - p - gamma_of(P, P.rho_w, P.c_w, p) * dzb;
    PerfTerms t;
    if (kind == 0) {
        double lt = lo + lw;
        t.qo = t.qo_p = t.qo_s = t.qo_b = 0.0;
        t.qw = WI * lt * dpw;
        t.qw_p = WI * ((lo_p + lw_p) * dpw + lt * (-1.0 - dgw * dzb));
        t.qw_s = WI * (lo_s + lw_s) * dpw;
        t.qw_b = WI * lt;
    } else {
        t.qo = WI * lo * dpo;
        t.qo_p = WI * (lo_p * dpo + lo * (-1.0 - dgo * dzb));
        t.qo_s = WI * lo_s * dpo;
        t.qo_b = WI * lo;
        t.qw = WI * lw * dpw;
        t.qw_p = WI * (lw_p * dpw + lw * (-1.0 - dgw * dzb));
        t.qw_s = WI * lw_s * dpw;
        t.qw_b = WI * lw;
    }
    return t;
}

struct AsmArgs {
    Phys P;
    const double *phi, *tx, *ty, *tz, *perf_wi, *w_zb;
    const int *cell_perf, *perf_well, *w_kind;
    const double *x, *xold;
    double dt;
    double2 *vp, *vs, *cw;
    double *b, *phi_o;
};

// One thread per cell: accumulation, the six faces in ascending order of the
// neighbour's index, then the perforation, exactly as the residual is summed
// cell by cell.  Writes the 7 slot blocks, b = -F and the oil potential.
__global__ __launch_bounds__(256) void k_assemble_cells(AsmArgs A) {
    const Phys &P = A.P;
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= P.n) return;
    int n = P.n, nx = P.nx, nxy = P.nx * P.ny;
    int i = c % nx, j = (c / nx) % P.ny, k = c / nxy;
    const double *x = A.x;
    double p = x[2 * c], s = x[2 * c + 1], pn = A.xold[2 * c], sn = A.xold[2 * c + 1];
    double dc = depth_of(P, k);
    double vol = P.dx * P.dy * P.dz;
    double coef = vol / (P.alpha * A.dt);
    double phr = A.phi[c];
    double ph = phr * (1.0 + P.c_r * (p - P.p_ref)), phn = phr * (1.0 + P.c_r * (pn - P.p_ref));
    double bo = bfac(P.c_o, p, P.p_ref), bw = bfac(P.c_w, p, P.p_ref);
    double bon = bfac(P.c_o, pn, P.p_ref), bwn = bfac(P.c_w, pn, P.p_ref);
    double F[2], D[4], O[7][4];
    F[0] = coef * (ph * bo * (1.0 - s) - phn * bon * (1.0 - sn));
    F[1] = coef * (ph * bw * s - phn * bwn * sn);
    double dph = phr * P.c_r;
    D[0] = coef * (1.0 - s) * (dph * bo + ph * P.c_o);
    D[1] = -coef * ph * bo;
    D[2] = coef * s * (dph * bw + ph * P.c_w);
    D[3] = coef * ph * bw;
    for (int t = 0; t < 7; t++) O[t][0] = O[t][1] = O[t][2] = O[t][3] = 0.0;
    // faces where c is the higher index (neighbour a = c - stride), then the lower
    const int order[6] = {5, 3, 1, 2, 4, 6};
    for (int oi = 0; oi < 6; oi++) {
        int sl = order[oi];
        bool exists; int nb; double tg;
        switch (sl) {
        case 5: exists = k > 0; nb = c - nxy; tg = exists ? A.tz[nb] : 0.0; break;
        case 3: exists = j > 0; nb = c - nx; tg = exists ? A.ty[nb] : 0.0; break;
        case 1: exists = i > 0; nb = c - 1; tg = exists ? A.tx[nb] : 0.0; break;
        case 2: exists = i + 1 < nx; nb = c + 1; tg = A.tx[c]; break;
        case 4: exists = j + 1 < P.ny; nb = c + nx; tg = A.ty[c]; break;
        default: exists = k + 1 < P.nz; nb = c + nxy; tg = A.tz[c]; break;
        }
        if (!exists) continue;
        double pnb = x[2 * nb], snb = x[2 * nb + 1];
        bool c_is_a = sl == 2 || sl == 4 || sl == 6;
        double dz = c_is_a ? depth_of(P, nb / nxy) - dc : dc - depth_of(P, nb / nxy);
        for (int phs = 0; phs < 2; phs++) {
            FaceTerms t = c_is_a ? face_phase(P, phs, p, s, pnb, snb, dz, tg)
                                 : face_phase(P, phs, pnb, snb, p, s, dz, tg);
            if (c_is_a) {
                F[phs] -= t.flux;
                D[2 * phs] -= t.fpa;
                D[2 * phs + 1] -= t.fsa;
                O[sl][2 * phs] -= t.fpb;
                O[sl][2 * phs + 1] -= t.fsb;
            } else {
                F[phs] += t.flux;
                D[2 * phs] += t.fpb;
                D[2 * phs + 1] += t.fsb;
                O[sl][2 * phs] += t.fpa;
                O[sl][2 * phs + 1] += t.fsa;
            }
        }
    }
    int q = A.cell_perf[c];
    if (q >= 0) {
        int w = A.perf_well[q];
        PerfTerms t = perf_terms(P, A.w_kind[w], A.perf_wi[q], p, s, x[2 * (n + w)], A.w_zb[w] - dc);
        F[0] -= t.qo;
        F[1] -= t.qw;
        D[0] -= t.qo_p; D[1] -= t.qo_s; D[2] -= t.qw_p; D[3] -= t.qw_s;
        double2 cwv;
        cwv.x = 0.0 - t.qo_b;
        cwv.y = 0.0 - t.qw_b;
        A.cw[q] = cwv;
    }
    A.b[2 * c] = -F[0];
    A.b[2 * c + 1] = -F[1];
    for (int t = 0; t < 7; t++) {
        const double *blk = t == 0 ? D : O[t];
        A.vp[(long)t * n + c] = make_double2(blk[0], blk[2]);
        A.vs[(long)t * n + c] = make_double2(blk[1], blk[3]);
    }
    A.phi_o[c] = p - gamma_of(P, P.rho_o, P.c_o, p) * dc;
}

// One thread per well: the constraint equation (Eq 11-14) and its row.
__global__ void k_assemble_wells(Phys P, const int *w_ptr, const int *w_kind, const int *w_ctrl,
                                 const double *w_target, const double *w_zb, const int *perf_cell,
                                 const double *perf_wi, const double *x, double2 *wc, double *wd,
                                 double *b) {
    int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= P.nw) return;
    int n = P.n, nxy = P.nx * P.ny;
    int rw = n + w;
    double pbh = x[2 * rw];
    double sgn = w_kind[w] == 0 ? 1.0 : -1.0;
    int ctrl = w_ctrl[w];
    double sum = 0.0, dsum_pb = 0.0;
    for (int q = w_ptr[w]; q < w_ptr[w + 1]; q++) {
        int c = perf_cell[q];
        PerfTerms t = perf_terms(P, w_kind[w], perf_wi[q], x[2 * c], x[2 * c + 1], pbh,
                                 w_zb[w] - depth_of(P, c / nxy));
        double sel = 0.0, sel_p = 0.0, sel_s = 0.0, sel_b = 0.0;
        if (ctrl == 1) { sel = t.qw; sel_p = t.qw_p; sel_s = t.qw_s; sel_b = t.qw_b; }
        else if (ctrl == 2) { sel = t.qo; sel_p = t.qo_p; sel_s = t.qo_s; sel_b = t.qo_b; }
        else if (ctrl == 3) { sel = t.qo + t.qw; sel_p = t.qo_p + t.qw_p; sel_s = t.qo_s + t.qw_s; sel_b = t.qo_b + t.qw_b; }
        sum += sel;
        dsum_pb += sel_b;
        wc[q] = ctrl != 0 ? make_double2(sel_p, sel_s) : make_double2(0.0, 0.0);
    }
    double F = ctrl == 0 ? pbh - w_target[w] : sum - sgn * w_target[w];
    b[2 * rw] = -F;
    b[2 * rw + 1] = -x[2 * rw + 1];
    wd[w] = ctrl == 0 ? 1.0 : dsum_pb;
}

extern "C" int r2p_jacobian_create(r2p_model *m, r2p_jacobian **out) {
    if (!m || !out) { r2p_set_error("NULL argument"); return R2P_EINVAL; }
    r2p_jacobian *J = new r2p_jacobian();
    J->m = m;
    J->serial = m->serial;
    long n = m->ph.n;
    int rc;
    if ((rc = J->vp.ensure(7 * n)) || (rc = J->vs.ensure(7 * n)) || (rc = J->cw.ensure(m->ph.nperf)) ||
        (rc = J->wc.ensure(m->ph.nperf)) || (rc = J->wd.ensure(m->ph.nw)) ||
        (rc = J->phi_o.ensure(n)) || (rc = J->dec.ensure(n))) {
        delete J;
        return rc;
    }
    *out = J;
    return 0;
}

extern "C" int r2p_jacobian_destroy(r2p_jacobian *J) {
    delete J;
    return 0;
}

extern "C" int r2p_assemble_jacobian(r2p_model *m, const double *x, const double *x_old, double dt,
                                     r2p_jacobian *J, double *b, void *stream) {
    if (!m || !x || !x_old || !J || !b || J->m != m || J->serial != m->serial) {
        r2p_set_error("NULL argument, or a Jacobian created for another model");
        return R2P_EINVAL;
    }
    if (!(dt > 0)) { r2p_set_error("dt must be > 0"); return R2P_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    AsmArgs A;
    A.P = m->ph;
    A.phi = m->phi.p; A.tx = m->tx.p; A.ty = m->ty.p; A.tz = m->tz.p;
    A.perf_wi = m->perf_wi.p; A.w_zb = m->w_zb.p;
    A.cell_perf = m->cell_perf.p; A.perf_well = m->perf_well.p; A.w_kind = m->w_kind.p;
    A.x = x; A.xold = x_old; A.dt = dt;
    A.vp = J->vp.p; A.vs = J->vs.p; A.cw = J->cw.p; A.b = b; A.phi_o = J->phi_o.p;
    k_assemble_cells<<<r2p_blocks(m->ph.n, BS), BS, 0, s>>>(A);
    R2P_LAUNCH();
    if (m->ph.nw > 0) {
        k_assemble_wells<<<r2p_blocks(m->ph.nw, 64), 64, 0, s>>>(
            m->ph, m->w_ptr.p, m->w_kind.p, m->w_ctrl.p, m->w_target.p, m->w_zb.p, m->perf_cell.p,
            m->perf_wi.p, x, J->wc.p, J->wd.p, b);
        R2P_LAUNCH();
    }
    J->state = 1;
    J->dec_kind = 0;
    return 0;
}

// ------------------------------------------------------------ scaled norm
// Non-negative doubles order like their bit patterns, so an unsigned max is
// an exact, order-independent reduction.  NaN is flagged separately.
__global__ void k_resnorm(Phys P, const double *phi, const double *w_target, const double *b,
                          double dt, unsigned long long *red) {
    __shared__ unsigned long long smax[BS / 64];
    __shared__ int snan[BS / 64];
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    double v = 0.0;
    int nan = 0;
    if (i < P.n) {
        double pv = P.dx * P.dy * P.dz * phi[i] / P.alpha;
        double a = fabs(b[2 * i]) * dt / pv, c = fabs(b[2 * i + 1]) * dt / pv;
        nan = (a != a) || (c != c);
        v = a > c ? a : c;
    } else if (i < P.n + P.nw) {
        int w = (int)(i - P.n);
        double t = fabs(w_target[w]);
        v = fabs(b[2 * i]) / (t > 0.0 ? t : 1.0);
        nan = v != v;
    }
    unsigned long long u = nan ? 0ull : (unsigned long long)__double_as_longlong(v);
    for (int d = 32; d > 0; d >>= 1) {
        unsigned long long o = __shfl_xor(u, d, 64);
        u = o > u ? o : u;
        nan |= __shfl_xor(nan, d, 64);
    }
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { smax[wid] = u; snan[wid] = nan; }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long mx = 0; int nn = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); w++) { mx = smax[w] > mx ? smax[w] : mx; nn |= snan[w]; }
        atomicMax(&red[0], mx);
        if (nn) atomicOr(&red[1], 1ull);
    }
}

extern "C" int r2p_residual_norm(r2p_model *m, const double *b, double dt, double *norm,
                                 void *stream) {
    if (!m || !b || !norm) { r2p_set_error("NULL argument"); return R2P_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    R2P_HIP(hipMemsetAsync(m->red.p, 0, 2 * sizeof(unsigned long long), s));
    long tot = m->ph.n + m->ph.nw;
    k_resnorm<<<r2p_blocks(tot, BS), BS, 0, s>>>(m->ph, m->phi.p, m->w_target.p, b, dt, m->red.p);
    R2P_LAUNCH();
    R2P_HIP(hipMemcpyAsync(m->pin.p, m->red.p, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    R2P_HIP(hipStreamSynchronize(s));
    unsigned long long *h = (unsigned long long *)m->pin.p;
    double v;
    memcpy(&v, &h[0], sizeof(double));
    *norm = v;
    if (h[1]) { *norm = NAN; r2p_set_error("non-finite residual"); return R2P_ENAN; }
    return 0;
}

// ----------------------------------------------- allocation-free scaled norm
// For callers that cannot allocate (HIP graph capture, serving loops): the
// per-workgroup partial maxima live in a file-scope device array, one copy
// per GPU, whose address each device resolves once (at model creation, with
// that device current).  Host code uses only that resolved address.
constexpr int NOALLOC_BLOCKS = 1 << 18;     // workgroups of BS rows: at most 2^26 rows
static __device__ __align__(256) unsigned long long scratch[2 * NOALLOC_BLOCKS];
constexpr int NOALLOC_MAX_DEV = 64;
static unsigned long long *noalloc_ptr[NOALLOC_MAX_DEV];
static std::mutex noalloc_mu;

int r2p_noalloc_init(int dev) {
    if (dev < 0 || dev >= NOALLOC_MAX_DEV) { r2p_set_error("device ordinal %d out of range", dev); return R2P_EINVAL; }
    std::lock_guard<std::mutex> g(noalloc_mu);
    if (noalloc_ptr[dev]) return 0;
    void *ptr = nullptr;
    R2P_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    noalloc_ptr[dev] = (unsigned long long *)ptr;
    return 0;
}

// Partial maxima of the scaled residual (the same per-row values as
// k_resnorm) per workgroup: part[blk] = the largest as bits, part[nb + blk]
// = 1 if a row was not finite.  Every entry is written, so nothing needs
// clearing between calls.
__global__ void k_resnorm_part(Phys P, const double *phi, const double *w_target, const double *b,
                               double dt, unsigned long long *part) {
    __shared__ unsigned long long smax[BS / 64];
    __shared__ int snan[BS / 64];
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    double v = 0.0;
    int nan = 0;
    if (i < P.n) {
        double pv = P.dx * P.dy * P.dz * phi[i] / P.alpha;
        double a = fabs(b[2 * i]) * dt / pv, c = fabs(b[2 * i + 1]) * dt / pv;
        nan = (a != a) || (c != c);
        v = a > c ? a : c;
    } else if (i < P.n + P.nw) {
        int w = (int)(i - P.n);
        double t = fabs(w_target[w]);
        v = fabs(b[2 * i]) / (t > 0.0 ? t : 1.0);
        nan = v != v;
    }
    unsigned long long u = nan ? 0ull : (unsigned long long)__double_as_longlong(v);
    for (int d = 32; d > 0; d >>= 1) {
        unsigned long long o = __shfl_xor(u, d, 64);
        u = o > u ? o : u;
        nan |= __shfl_xor(nan, d, 64);
    }
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { smax[wid] = u; snan[wid] = nan; }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long mx = 0;
        int nn = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); w++) { mx = smax[w] > mx ? smax[w] : mx; nn |= snan[w]; }
        part[blockIdx.x] = mx;
        part[gridDim.x + blockIdx.x] = (unsigned long long)nn;
    }
}

// norm = the largest partial, or NaN if any row was not finite.
__global__ __launch_bounds__(1024) void k_resnorm_fin(int nb, const unsigned long long *part,
                                                      double *norm) {
    __shared__ unsigned long long smax[1024 / 64];
    __shared__ int snan[1024 / 64];
    unsigned long long mx = 0;
    int nan = 0;
    for (int k = threadIdx.x; k < nb; k += blockDim.x) {
        unsigned long long v = part[k];
        mx = v > mx ? v : mx;
        nan |= part[nb + k] != 0;
    }
    for (int d = 32; d > 0; d >>= 1) {
        unsigned long long o = __shfl_xor(mx, d, 64);
        mx = o > mx ? o : mx;
        nan |= __shfl_xor(nan, d, 64);
    }
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { smax[wid] = mx; snan[wid] = nan; }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = 0;
        int nn = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); w++) { m = smax[w] > m ? smax[w] : m; nn |= snan[w]; }
        *norm = nn ? __longlong_as_double(0x7ff8000000000000ll) : __longlong_as_double((long long)m);
    }
}

extern "C" int r2p_residual_norm_noalloc(r2p_model *m, const double *b, double dt, double *norm,
                                         void *stream) {
    if (!m || !b || !norm) { r2p_set_error("NULL argument"); return R2P_EINVAL; }
    long tot = (long)m->ph.n + m->ph.nw;
    long nb = (tot + BS - 1) / BS;
    if (nb > NOALLOC_BLOCKS) {
        r2p_set_error("r2p_residual_norm_noalloc: %ld rows exceed its scratch limit of %ld rows",
                      tot, (long)NOALLOC_BLOCKS * BS);
        return R2P_EINVAL;
    }
    if (m->dev < 0 || m->dev >= NOALLOC_MAX_DEV || !noalloc_ptr[m->dev]) {
        r2p_set_error("scratch of device %d not resolved", m->dev);
        return R2P_ESTATE;
    }
    unsigned long long *part = noalloc_ptr[m->dev];
    hipStream_t s = (hipStream_t)stream;
    k_resnorm_part<<<(int)nb, BS, 0, s>>>(m->ph, m->phi.p, m->w_target.p, b, dt, part);
    R2P_LAUNCH();
    k_resnorm_fin<<<1, 1024, 0, s>>>((int)nb, part, norm);
    R2P_LAUNCH();
    return 0;
}

// --------------------------------------------------------------- decoupling
// Row operator D_i^-1 for cell row i (Quasi-IMPES or ABF), applied to all
// blocks of the row (the 7 slots and the well column) and stored for the
// right-hand side.  Well rows are left unchanged.
__global__ void k_decouple(int n, int kind, const int *cell_perf, double2 *vp, double2 *vs,
                           double2 *cw, double4 *dec) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double2 dp = vp[c], ds = vs[c];
    double a0 = dp.x, a1 = ds.x, a2 = dp.y, a3 = ds.y;   // [[a0 a1] [a2 a3]]
    double M0, M1, M2, M3;
    if (kind == R2P_DEC_QI) {
        M0 = 1.0; M1 = -a1 / a3; M2 = 0.0; M3 = 1.0;
    } else {
        double det = a0 * a3 - a1 * a2;
        M0 = a3 / det; M1 = -a1 / det; M2 = -a2 / det; M3 = a0 / det;
    }
    for (int t = 0; t < 7; t++) {
        long z = (long)t * n + c;
        double2 P = vp[z], S = vs[z];
        double b0 = P.x, b1 = S.x, b2 = P.y, b3 = S.y;
        vp[z] = make_double2(M0 * b0 + M1 * b2, M2 * b0 + M3 * b2);
        vs[z] = make_double2(M0 * b1 + M1 * b3, M2 * b1 + M3 * b3);
    }
    int q = cell_perf[c];
    if (q >= 0) {
        double2 w = cw[q];
        // block [[w.x 0] [w.y 0]]
        cw[q] = make_double2(M0 * w.x + M1 * w.y, M2 * w.x + M3 * w.y);
    }
    dec[c] = make_double4(M0, M1, M2, M3);
}

int r2p_decouple_jacobian(r2p_jacobian *J, int kind, hipStream_t s) {
    if (J->state != 1) { r2p_set_error("Jacobian not assembled since its last set-up"); return R2P_ESTATE; }
    if (kind != R2P_DEC_NONE) {
        k_decouple<<<r2p_blocks(J->m->ph.n, BS), BS, 0, s>>>(J->m->ph.n, kind, J->m->cell_perf.p,
                                                            J->vp.p, J->vs.p, J->cw.p, J->dec.p);
        R2P_LAUNCH();
    }
    J->dec_kind = kind;
    J->state = 2;
    return 0;
}

__global__ void k_decouple_rhs(int n, int nw, const double4 *dec, const double *b, double *bd) {
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) {
        double4 M = dec[i];
        double v0 = b[2 * i], v1 = b[2 * i + 1];
        bd[2 * i] = M.x * v0 + M.y * v1;
        bd[2 * i + 1] = M.z * v0 + M.w * v1;
    } else if (i < n + nw) {
        bd[2 * i] = b[2 * i];
        bd[2 * i + 1] = b[2 * i + 1];
    }
}

int r2p_decouple_rhs(r2p_jacobian *J, const double *b, double *bd, hipStream_t s) {
    const Phys &P = J->m->ph;
    if (J->dec_kind == R2P_DEC_NONE) {
        if (b != bd) R2P_HIP(hipMemcpyAsync(bd, b, sizeof(double) * 2 * (size_t)(P.n + P.nw), hipMemcpyDeviceToDevice, s));
        return 0;
    }
    k_decouple_rhs<<<r2p_blocks(P.n + P.nw, BS), BS, 0, s>>>(P.n, P.nw, J->dec.p, b, bd);
    R2P_LAUNCH();
    return 0;
}

// --------------------------------------------------------------------- SpMV
// y = A x, or r = f - A x when f != NULL.  One thread per cell row; blocks
// summed in ascending column order (-z, -y, -x, self, +x, +y, +z, well).
// Well rows and the dummy rows come first, one wavefront per well (lanes
// over the perforations, then a fixed butterfly), in the first nwblk
// workgroups (a multiple of 8, so the cell blocks keep their XCD order).
struct SpmvArgs {
    int n, nx, nxy, nw, ncellblk, nwblk;
    const double2 *vp, *vs, *cw, *wc;
    const double *wd;
    const int *cell_perf, *perf_well, *perf_cell, *w_ptr;
    const double *x, *f;
    double *y;
};

__global__ __launch_bounds__(256) void k_spmv(SpmvArgs A) {
    if ((int)blockIdx.x >= A.nwblk) {
        int c = xcd_block((int)blockIdx.x - A.nwblk, A.ncellblk) * blockDim.x + threadIdx.x;
        if (c >= A.n) return;
        const double2 *xv = (const double2 *)A.x;
        const int order[7] = {5, 3, 1, 0, 2, 4, 6};
        double y0 = 0.0, y1 = 0.0;
#pragma unroll
        for (int oi = 0; oi < 7; oi++) {
            int sl = order[oi];
            int col = c + slot_offset(sl, A.nx, A.nxy);
            col = col < 0 ? 0 : (col >= A.n ? A.n - 1 : col);
            double2 P = ld_stream2(&A.vp[(long)sl * A.n + c]), S = ld_stream2(&A.vs[(long)sl * A.n + c]);
            double2 xc = xv[col];
            y0 += P.x * xc.x + S.x * xc.y;
            y1 += P.y * xc.x + S.y * xc.y;
        }
        int q = A.cell_perf[c];
        if (q >= 0) {
            double2 w = A.cw[q];
            double pb = A.x[2 * (A.n + A.perf_well[q])], dm = A.x[2 * (A.n + A.perf_well[q]) + 1];
            y0 += w.x * pb + 0.0 * dm;
            y1 += w.y * pb + 0.0 * dm;
        }
        if (A.f) {
            y0 = A.f[2 * c] - y0;
            y1 = A.f[2 * c + 1] - y1;
        }
        ((double2 *)A.y)[c] = make_double2(y0, y1);
    } else {
        int lane = threadIdx.x & 63;
        int w = (int)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
        if (w >= A.nw) return;
        // perforated cells' blocks (lanes stride over them, then a fixed
        // butterfly), then the well's own block
        double y0 = 0.0;
        for (int q = A.w_ptr[w] + lane; q < A.w_ptr[w + 1]; q += 64) {
            int c = A.perf_cell[q];
            double2 v = A.wc[q];
            y0 += v.x * A.x[2 * c] + v.y * A.x[2 * c + 1];
        }
        for (int d = 1; d < 64; d <<= 1) y0 += __shfl_xor(y0, d, 64);
        if (lane == 0) {
            long rw = A.n + w;
            y0 += A.wd[w] * A.x[2 * rw] + 0.0 * A.x[2 * rw + 1];
            double y1 = 0.0 * A.x[2 * rw] + 1.0 * A.x[2 * rw + 1];
            if (A.f) {
                y0 = A.f[2 * rw] - y0;
                y1 = A.f[2 * rw + 1] - y1;
            }
            A.y[2 * rw] = y0;
            A.y[2 * rw + 1] = y1;
        }
    }
}

int r2p_spmv_impl(r2p_jacobian *J, const double *x, double *y, const double *f, hipStream_t s) {
    const Phys &P = J->m->ph;
    SpmvArgs A;
    A.n = P.n; A.nx = P.nx; A.nxy = P.nx * P.ny; A.nw = P.nw;
    A.ncellblk = r2p_blocks(P.n, BS);
    A.vp = J->vp.p; A.vs = J->vs.p; A.cw = J->cw.p; A.wc = J->wc.p; A.wd = J->wd.p;
    A.cell_perf = J->m->cell_perf.p; A.perf_well = J->m->perf_well.p;
    A.perf_cell = J->m->perf_cell.p; A.w_ptr = J->m->w_ptr.p;
    A.x = x; A.f = f; A.y = y;
    A.nwblk = (r2p_blocks(P.nw, BS / 64) + 7) & ~7;
    k_spmv<<<A.nwblk + A.ncellblk, BS, 0, s>>>(A);
    R2P_LAUNCH();
    return 0;
}

extern "C" int r2p_spmv(r2p_jacobian *J, const double *x, double *y, void *stream) {
    if (!J || !x || !y) { r2p_set_error("NULL argument"); return R2P_EINVAL; }
    if (J->state == 0) { r2p_set_error("Jacobian not assembled"); return R2P_ESTATE; }
    return r2p_spmv_impl(J, x, y, nullptr, (hipStream_t)stream);
}

// r = f - A (Pi_p xp): only the pressure columns of the cell blocks and of
// the well rows' cell blocks (Eq 35 puts zeros in s_w and p_b).
__global__ __launch_bounds__(256) void k_pcol_residual(SpmvArgs A) {
    if ((int)blockIdx.x >= A.nwblk) {
        int c = xcd_block((int)blockIdx.x - A.nwblk, A.ncellblk) * blockDim.x + threadIdx.x;
        if (c >= A.n) return;
        const int order[7] = {5, 3, 1, 0, 2, 4, 6};
        double y0 = 0.0, y1 = 0.0;
#pragma unroll
        for (int oi = 0; oi < 7; oi++) {
            int sl = order[oi];
            int col = c + slot_offset(sl, A.nx, A.nxy);
            col = col < 0 ? 0 : (col >= A.n ? A.n - 1 : col);
            double2 P = ld_stream2(&A.vp[(long)sl * A.n + c]);
            double xc = A.x[col];
            y0 += P.x * xc;
            y1 += P.y * xc;
        }
        ((double2 *)A.y)[c] = make_double2(A.f[2 * c] - y0, A.f[2 * c + 1] - y1);
    } else {
        int lane = threadIdx.x & 63;
        int w = (int)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
        if (w >= A.nw) return;
        double y0 = 0.0;
        for (int q = A.w_ptr[w] + lane; q < A.w_ptr[w + 1]; q += 64)
            y0 += A.wc[q].x * A.x[A.perf_cell[q]];
        for (int d = 1; d < 64; d <<= 1) y0 += __shfl_xor(y0, d, 64);
        if (lane == 0) {
            long rw = A.n + w;
            A.y[2 * rw] = A.f[2 * rw] - y0;
            A.y[2 * rw + 1] = A.f[2 * rw + 1];
        }
    }
}

int r2p_pcol_residual(r2p_jacobian *J, const double *f, const double *xp, double *r, hipStream_t s) {
    const Phys &P = J->m->ph;
    SpmvArgs A;
    A.n = P.n; A.nx = P.nx; A.nxy = P.nx * P.ny; A.nw = P.nw;
    A.ncellblk = r2p_blocks(P.n, BS);
    A.vp = J->vp.p; A.vs = J->vs.p; A.cw = J->cw.p; A.wc = J->wc.p; A.wd = J->wd.p;
    A.cell_perf = J->m->cell_perf.p; A.perf_well = J->m->perf_well.p;
    A.perf_cell = J->m->perf_cell.p; A.w_ptr = J->m->w_ptr.p;
    A.x = xp; A.f = f; A.y = r;
    A.nwblk = (r2p_blocks(P.nw, BS / 64) + 7) & ~7;
    k_pcol_residual<<<A.nwblk + A.ncellblk, BS, 0, s>>>(A);
    R2P_LAUNCH();
    return 0;
}

// ---------------------------------------------------------------- export
extern "C" int r2p_jacobian_export(r2p_jacobian *J, int *nnzb, int *rp, int *col, double *val,
                                   void *stream) {
    if (!J || !nnzb) { r2p_set_error("NULL argument"); return R2P_EINVAL; }
    if (J->state == 0) { r2p_set_error("Jacobian not assembled"); return R2P_ESTATE; }
    const r2p_model *m = J->m;
    const Phys &P = m->ph;
    int n = P.n, nx = P.nx, ny = P.ny, nz = P.nz, nxy = nx * ny;
    std::vector<int> cperf(n, -1);
    for (int q = 0; q < P.nperf; q++) cperf[m->h_w_cell[q]] = q;
    long cnt = 0;
    for (int c = 0; c < n; c++) {
        int i = c % nx, j = (c / nx) % ny, k = c / nxy;
        cnt += 1 + (i > 0) + (i + 1 < nx) + (j > 0) + (j + 1 < ny) + (k > 0) + (k + 1 < nz) + (cperf[c] >= 0);
    }
    cnt += P.nperf + P.nw;
    *nnzb = (int)cnt;
    if (!rp) return 0;
    hipStream_t s = (hipStream_t)stream;
    std::vector<double2> hvp(7L * n), hvs(7L * n), hcw(P.nperf), hwc(P.nperf);
    std::vector<double> hwd(P.nw);
    R2P_HIP(hipMemcpyAsync(hvp.data(), J->vp.p, sizeof(double2) * 7L * n, hipMemcpyDeviceToHost, s));
    R2P_HIP(hipMemcpyAsync(hvs.data(), J->vs.p, sizeof(double2) * 7L * n, hipMemcpyDeviceToHost, s));
    if (P.nperf) {
        R2P_HIP(hipMemcpyAsync(hcw.data(), J->cw.p, sizeof(double2) * P.nperf, hipMemcpyDeviceToHost, s));
        R2P_HIP(hipMemcpyAsync(hwc.data(), J->wc.p, sizeof(double2) * P.nperf, hipMemcpyDeviceToHost, s));
        R2P_HIP(hipMemcpyAsync(hwd.data(), J->wd.p, sizeof(double) * P.nw, hipMemcpyDeviceToHost, s));
    }
    R2P_HIP(hipStreamSynchronize(s));
    long z = 0;
    rp[0] = 0;
    const int order[7] = {5, 3, 1, 0, 2, 4, 6};
    for (int c = 0; c < n; c++) {
        int i = c % nx, j = (c / nx) % ny, k = c / nxy;
        bool ex[7] = {true, i > 0, i + 1 < nx, j > 0, j + 1 < ny, k > 0, k + 1 < nz};
        for (int oi = 0; oi < 7; oi++) {
            int sl = order[oi];
            if (!ex[sl]) continue;
            double2 pv = hvp[(long)sl * n + c], sv = hvs[(long)sl * n + c];
            col[z] = c + slot_offset(sl, nx, nxy);
            val[4 * z + 0] = pv.x; val[4 * z + 1] = sv.x; val[4 * z + 2] = pv.y; val[4 * z + 3] = sv.y;
            z++;
        }
        if (cperf[c] >= 0) {
            int q = cperf[c];
            int w = 0;
            while (m->h_w_ptr[w + 1] <= q) w++;
            col[z] = n + w;
            val[4 * z + 0] = hcw[q].x; val[4 * z + 1] = 0.0; val[4 * z + 2] = hcw[q].y; val[4 * z + 3] = 0.0;
            z++;
        }
        rp[c + 1] = (int)z;
    }
    for (int w = 0; w < P.nw; w++) {
        std::vector<std::pair<int, int>> cells;
        for (int q = m->h_w_ptr[w]; q < m->h_w_ptr[w + 1]; q++) cells.push_back({m->h_w_cell[q], q});
        std::sort(cells.begin(), cells.end());
        for (auto &cq : cells) {
            col[z] = cq.first;
            val[4 * z + 0] = hwc[cq.second].x; val[4 * z + 1] = hwc[cq.second].y;
            val[4 * z + 2] = 0.0; val[4 * z + 3] = 0.0;
            z++;
        }
        col[z] = n + w;
        val[4 * z + 0] = hwd[w]; val[4 * z + 1] = 0.0; val[4 * z + 2] = 0.0; val[4 * z + 3] = 1.0;
        z++;
        rp[n + w + 1] = (int)z;
    }
    return 0;
}

// ---------------------------------------------------------- Newton update
// x += y with each cell's saturation change limited to ds_max, then s_w
// clipped to [0, 1] (Algorithm 1 update).
__global__ void k_newton_update(long N2n, long N, double ds_max, const double *y, double *x) {
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= N) return;
    double d = y[i];
    bool sat = i < N2n && (i & 1);
    if (sat && ds_max > 0.0) d = d > ds_max ? ds_max : (d < -ds_max ? -ds_max : d);
    double v = x[i] + d;
    if (sat) v = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
    x[i] = v;
}

int r2p_newton_update(r2p_model *m, const double *y, double *x, double ds_max, hipStream_t s) {
    long N = 2L * (m->ph.n + m->ph.nw);
    k_newton_update<<<r2p_blocks(N, BS), BS, 0, s>>>(2L * m->ph.n, N, ds_max, y, x);
    R2P_LAUNCH();
    return 0;
}
