/*
 * Oracle: two-phase oil-water model and its fully implicit discretisation.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Paper sections followed: "Two-phase oil-water flow model" (Eq 1-14) and
 * "Numerical methods" (Eq 15-23).  Readings where the paper is silent:
 *   - depth z is positive downward; potential Phi_a = p_a - gamma_a z with
 *     gamma_a = grav * rho_a / 144 psi/ft (Eq 5 written with depth; Eq 10's
 *     head term is consistent only with this sign);
 *   - equations are divided by the reference density, so b_a = rho_a/rho_a^r
 *     = 1 + c_a (p - p_ref) (Eq 6) and residuals are in STB/day;
 *   - capillary pressure is zero, so p_w = p_o = p (Eq 9 with p_c = 0);
 *   - Corey relative permeabilities krw = s^2, kro = (1-s)^2;
 *   - viscosities are constant (Eq 7 with c_mu = 0);
 *   - face transmissibility = beta_c * Tgeo * (kr b / mu) of the upstream
 *     cell, Tgeo the harmonic geometric factor (Eq 16 split into a geometric
 *     and a mobility part, the mobility upwinded as in Eq 18);
 *   - gravity density on a face is the mean of the two cells' values;
 *   - upstream rule on a face (i < j in natural order): the upstream cell is
 *     j when Phi_j - Phi_i >= 0, else i (Eq 18 made symmetric);
 *   - wells (Eq 10): producers use each phase's mobility; injectors inject
 *     water with the cell's total mobility; Peaceman's anisotropic well
 *     index; z_b is the depth of the top perforated cell.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

static double *dup(const double *a, int n)
{
    double *b = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    if (n > 0) memcpy(b, a, sizeof(double) * n);
    return b;
}

static int *dupi(const int *a, int n)
{
    int *b = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    if (n > 0) memcpy(b, a, sizeof(int) * n);
    return b;
}

/* Peaceman's well index for a vertical perforation in an anisotropic cell. */
static double peaceman_wi(double kx, double ky, double dx, double dy, double dz,
                          double rw, double skin, double beta_c)
{
    double ryx = sqrt(ky / kx), rxy = sqrt(kx / ky);
    double ro = 0.28 * sqrt(ryx * dx * dx + rxy * dy * dy) / (sqrt(ryx) + sqrt(rxy));
    return 2.0 * M_PI * beta_c * sqrt(kx * ky) * dz / (log(ro / rw) + skin);
}

int om_model_create(om_model **out, int nx, int ny, int nz, double dx, double dy, double dz,
                    double top, const double *kx, const double *ky, const double *kz,
                    const double *phi, const double *c, int nw, const int *w_ptr,
                    const int *w_cell, const int *w_kind, const int *w_ctrl,
                    const double *w_target, const double *w_rw, const double *w_skin)
{
    om_model *m = (om_model *)calloc(1, sizeof(om_model));
    int n = nx * ny * nz;
    m->nx = nx; m->ny = ny; m->nz = nz; m->n = n;
    m->dx = dx; m->dy = dy; m->dz = dz; m->top = top;
    m->kx = dup(kx, n); m->ky = dup(ky, n); m->kz = dup(kz, n); m->phi = dup(phi, n);
    m->beta_c = c[0]; m->alpha_c = c[1]; m->rho_o = c[2]; m->rho_w = c[3];
    m->p_ref = c[4]; m->z_ref = c[5]; m->c_o = c[6]; m->c_w = c[7]; m->c_r = c[8];
    m->mu_o = c[9]; m->mu_w = c[10]; m->grav = c[11];
    m->depth = (double *)malloc(sizeof(double) * n);
    m->vol = (double *)malloc(sizeof(double) * n);
    m->tx = (double *)calloc(n, sizeof(double));
    m->ty = (double *)calloc(n, sizeof(double));
    m->tz = (double *)calloc(n, sizeof(double));
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                int cc = i + nx * (j + ny * k);
                m->depth[cc] = top + dz * k;
                m->vol[cc] = dx * dy * dz;
                /* harmonic two-point geometric transmissibility, mD*ft */
                if (i + 1 < nx)
                    m->tx[cc] = dy * dz / (dx / (2.0 * kx[cc]) + dx / (2.0 * kx[cc + 1]));
                if (j + 1 < ny)
                    m->ty[cc] = dx * dz / (dy / (2.0 * ky[cc]) + dy / (2.0 * ky[cc + nx]));
                if (k + 1 < nz)
                    m->tz[cc] = dx * dy / (dz / (2.0 * kz[cc]) + dz / (2.0 * kz[cc + nx * ny]));
            }
    m->nw = nw;
    m->nperf = nw > 0 ? w_ptr[nw] : 0;
    m->w_ptr = dupi(w_ptr, nw + 1);
    m->w_cell = dupi(w_cell, m->nperf);
    m->w_kind = dupi(w_kind, nw);
    m->w_ctrl = dupi(w_ctrl, nw);
    m->w_target = dup(w_target, nw);
    m->w_rw = dup(w_rw, nw);
    m->w_skin = dup(w_skin, nw);
    m->wi = (double *)malloc(sizeof(double) * (m->nperf > 0 ? m->nperf : 1));
    m->perf_well = (int *)malloc(sizeof(int) * (m->nperf > 0 ? m->nperf : 1));
    m->w_zb = (double *)malloc(sizeof(double) * (nw > 0 ? nw : 1));
    for (int w = 0; w < nw; w++)
        for (int q = w_ptr[w]; q < w_ptr[w + 1]; q++) m->perf_well[q] = w;
    om_well_index(m, m->wi, m->w_zb);
    *out = m;
    return 0;
}

void om_model_destroy(om_model *m)
{
    if (!m) return;
    free(m->kx); free(m->ky); free(m->kz); free(m->phi); free(m->depth); free(m->vol);
    free(m->tx); free(m->ty); free(m->tz);
    free(m->w_ptr); free(m->w_cell); free(m->w_kind); free(m->w_ctrl);
    free(m->w_target); free(m->w_rw); free(m->w_skin); free(m->wi); free(m->perf_well);
    free(m->w_zb);
    free(m);
}

void om_well_index(const om_model *m, double *wi, double *zb)
{
    for (int w = 0; w < m->nw; w++) {
        zb[w] = m->depth[m->w_cell[m->w_ptr[w]]];
        for (int q = m->w_ptr[w]; q < m->w_ptr[w + 1]; q++) {
            int c = m->w_cell[q];
            wi[q] = peaceman_wi(m->kx[c], m->ky[c], m->dx, m->dy, m->dz, m->w_rw[w],
                                m->w_skin[w], m->beta_c);
        }
    }
}

/* ------------------------------------------------------- property laws */
/* Eq 6 divided by the reference density. */
static double bfac(const om_model *m, double c, double p) { return 1.0 + c * (p - m->p_ref); }
/* Hydrostatic gradient of a phase, psi/ft. */
static double gam(const om_model *m, double rho, double c, double p)
{
    double b = 1.0 + c * (p - m->p_ref);
    return m->grav * rho * b / 144.0;
}
/* Eq 4 */
static double poro(const om_model *m, int i, double p) { return m->phi[i] * (1.0 + m->c_r * (p - m->p_ref)); }

/* Oil potential per cell (Eq 5 with depth positive downward). */
void om_potential(const om_model *m, const double *x, double *phi_o)
{
    for (int i = 0; i < m->n; i++) {
        double p = x[2 * i];
        phi_o[i] = p - gam(m, m->rho_o, m->c_o, p) * m->depth[i];
    }
}

/* Oil-hydrostatic initial state through (p_ref, z_ref); s_w = 0.
 * Layer pressures satisfy p_{k+1} - p_k = 0.5*(gamma(p_k)+gamma(p_{k+1}))*dz,
 * the discrete equilibrium of the face flux, so the initial flux is zero. */
void om_initial_state(const om_model *m, double *x)
{
    int n = m->n;
    double *pl = (double *)malloc(sizeof(double) * m->nz);
    double zprev = m->z_ref, pprev = m->p_ref;
    for (int k = 0; k < m->nz; k++) {
        double z = m->top + m->dz * k;
        double p = pprev;
        for (int it = 0; it < 100; it++) { /* fixed point on gamma(p) */
            double pn = pprev + 0.5 * (gam(m, m->rho_o, m->c_o, pprev) + gam(m, m->rho_o, m->c_o, p)) * (z - zprev);
            if (pn == p) break;
            p = pn;
        }
        pl[k] = p;
        pprev = p; zprev = z;
    }
    int nxy = m->nx * m->ny;
    for (int i = 0; i < n; i++) { x[2 * i] = pl[i / nxy]; x[2 * i + 1] = 0.0; }
    for (int w = 0; w < m->nw; w++) {
        double pb = m->w_ctrl[w] == 0 ? m->w_target[w] : x[2 * m->w_cell[m->w_ptr[w]]];
        x[2 * (n + w)] = pb;
        x[2 * (n + w) + 1] = 0.0;
    }
    free(pl);
}

/* Per-phase volumes-in-place term phi*b*s per cell scaled to STB: V phi b s / alpha_c. */
void om_accumulation(const om_model *m, const double *x, double *acc_o, double *acc_w)
{
    for (int i = 0; i < m->n; i++) {
        double p = x[2 * i], s = x[2 * i + 1];
        double f = m->vol[i] / m->alpha_c * poro(m, i, p);
        acc_o[i] = f * bfac(m, m->c_o, p) * (1.0 - s);
        acc_w[i] = f * bfac(m, m->c_w, p) * s;
    }
}

/* Well rates per perforation (Eq 10), STB/day, positive into the reservoir. */
void om_well_rates(const om_model *m, const double *x, double *q_o, double *q_w)
{
    int n = m->n;
    for (int w = 0; w < m->nw; w++) {
        double pb = x[2 * (n + w)];
        for (int q = m->w_ptr[w]; q < m->w_ptr[w + 1]; q++) {
            int c = m->w_cell[q];
            double p = x[2 * c], s = x[2 * c + 1];
            double lo = (1.0 - s) * (1.0 - s) * bfac(m, m->c_o, p) / m->mu_o;
            double lw = s * s * bfac(m, m->c_w, p) / m->mu_w;
            double dzb = m->w_zb[w] - m->depth[c];
            double dpw = pb - p - gam(m, m->rho_w, m->c_w, p) * dzb;
            if (m->w_kind[w] == 0) {
                q_o[q] = 0.0;
                q_w[q] = m->wi[q] * (lo + lw) * dpw;
            } else {
                double dpo = pb - p - gam(m, m->rho_o, m->c_o, p) * dzb;
                q_o[q] = m->wi[q] * lo * dpo;
                q_w[q] = m->wi[q] * lw * dpw;
            }
        }
    }
}

/* ------------------------------------------------------------ pattern */
/* Block sparsity of the Jacobian: cell rows hold the cell, its six face
 * neighbours and the well it is perforated by; well rows hold their
 * perforated cells and themselves.  Columns ascending. */
void om_pattern(const om_model *m, om_bsr *J)
{
    int n = m->n, nx = m->nx, ny = m->ny, nz = m->nz, nxy = nx * ny;
    int nb = n + m->nw;
    int *perf_of = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    for (int i = 0; i < n; i++) perf_of[i] = -1;
    for (int q = 0; q < m->nperf; q++) perf_of[m->w_cell[q]] = q;
    J->nb = nb;
    J->rp = (int *)malloc(sizeof(int) * (nb + 1));
    int cap = 7 * n + 2 * m->nperf + m->nw + 1;
    J->col = (int *)malloc(sizeof(int) * cap);
    int z = 0;
    J->rp[0] = 0;
    for (int c = 0; c < n; c++) {
        int i = c % nx, j = (c / nx) % ny, k = c / nxy;
        if (k > 0) J->col[z++] = c - nxy;
        if (j > 0) J->col[z++] = c - nx;
        if (i > 0) J->col[z++] = c - 1;
        J->col[z++] = c;
        if (i + 1 < nx) J->col[z++] = c + 1;
        if (j + 1 < ny) J->col[z++] = c + nx;
        if (k + 1 < nz) J->col[z++] = c + nxy;
        if (perf_of[c] >= 0) J->col[z++] = n + m->perf_well[perf_of[c]];
        J->rp[c + 1] = z;
    }
    for (int w = 0; w < m->nw; w++) {
        int a = m->w_ptr[w], b = m->w_ptr[w + 1];
        int start = z;
        for (int q = a; q < b; q++) J->col[z++] = m->w_cell[q];
        /* sort the perforated cells ascending (insertion sort) */
        for (int u = start + 1; u < z; u++) {
            int v = J->col[u], t = u - 1;
            while (t >= start && J->col[t] > v) { J->col[t + 1] = J->col[t]; t--; }
            J->col[t + 1] = v;
        }
        J->col[z++] = n + w;
        J->rp[n + w + 1] = z;
    }
    J->nnzb = z;
    J->val = (double *)calloc(4 * (size_t)z, sizeof(double));
    free(perf_of);
}

/* ------------------------------------------------ residual and Jacobian */
typedef struct { double v[2]; } ph2;

/* Residual F(x) of Eq 17 plus the well equations (Eq 11-14), interleaved.
 * If J is non-NULL its values (pattern from om_pattern) receive dF/dx. */
static void assemble(const om_model *m, const double *x, const double *xold, double dt,
                     double *F, om_bsr *J)
{
    int n = m->n, nx = m->nx, nxy = m->nx * m->ny;
    const double beta = m->beta_c;
    for (int i = 0; i < 2 * (n + m->nw); i++) F[i] = 0.0;
    if (J) memset(J->val, 0, sizeof(double) * 4 * (size_t)J->nnzb);

    /* accumulation, Eq 15 + left side of Eq 17 */
    for (int i = 0; i < n; i++) {
        double p = x[2 * i], s = x[2 * i + 1], pn = xold[2 * i], sn = xold[2 * i + 1];
        double coef = m->vol[i] / (m->alpha_c * dt);
        double ph = poro(m, i, p), phn = poro(m, i, pn);
        double bo = bfac(m, m->c_o, p), bw = bfac(m, m->c_w, p);
        double bon = bfac(m, m->c_o, pn), bwn = bfac(m, m->c_w, pn);
        F[2 * i] = coef * (ph * bo * (1.0 - s) - phn * bon * (1.0 - sn));
        F[2 * i + 1] = coef * (ph * bw * s - phn * bwn * sn);
        if (J) {
            double dph = m->phi[i] * m->c_r;
            double *D = &J->val[4 * om_bsr_find(J, i, i)];
            D[0] += coef * (1.0 - s) * (dph * bo + ph * m->c_o);
            D[1] += -coef * ph * bo;
            D[2] += coef * s * (dph * bw + ph * m->c_w);
            D[3] += coef * ph * bw;
        }
    }

    /* face fluxes (Eq 16-18); flux into cell a from cell b on face (a < b) */
    for (int a = 0; a < n; a++) {
        int i = a % nx, j = (a / nx) % m->ny, k = a / nxy;
        for (int d = 0; d < 3; d++) {
            int b; double tg;
            if (d == 0) { if (i + 1 >= nx) continue; b = a + 1; tg = m->tx[a]; }
            else if (d == 1) { if (j + 1 >= m->ny) continue; b = a + nx; tg = m->ty[a]; }
            else { if (k + 1 >= m->nz) continue; b = a + nxy; tg = m->tz[a]; }
            double pa = x[2 * a], sa = x[2 * a + 1], pb = x[2 * b], sb = x[2 * b + 1];
            double dz = m->depth[b] - m->depth[a];
            for (int ph = 0; ph < 2; ph++) {
                double rho = ph == 0 ? m->rho_o : m->rho_w;
                double cc = ph == 0 ? m->c_o : m->c_w;
                double mu = ph == 0 ? m->mu_o : m->mu_w;
                double ga = gam(m, rho, cc, pa), gb = gam(m, rho, cc, pb);
                double dphi = (pb - pa) - 0.5 * (ga + gb) * dz;
                int up_b = dphi >= 0.0;
                double pu = up_b ? pb : pa, su = up_b ? sb : sa;
                double kr = ph == 0 ? (1.0 - su) * (1.0 - su) : su * su;
                double dkr = ph == 0 ? -2.0 * (1.0 - su) : 2.0 * su;
                double bu = bfac(m, cc, pu);
                double lam = kr * bu / mu;
                double flux = beta * tg * lam * dphi;
                F[2 * a + ph] -= flux;
                F[2 * b + ph] += flux;
                if (J) {
                    double dg = m->grav * rho * cc / 144.0;
                    double ddphi_a = -1.0 - 0.5 * dg * dz;
                    double ddphi_b = 1.0 - 0.5 * dg * dz;
                    double dlam_p = kr * cc / mu, dlam_s = dkr * bu / mu;
                    /* d flux / d (pa, sa, pb, sb) */
                    double fpa = beta * tg * (lam * ddphi_a + (up_b ? 0.0 : dlam_p * dphi));
                    double fsa = beta * tg * (up_b ? 0.0 : dlam_s * dphi);
                    double fpb = beta * tg * (lam * ddphi_b + (up_b ? dlam_p * dphi : 0.0));
                    double fsb = beta * tg * (up_b ? dlam_s * dphi : 0.0);
                    double *Aaa = &J->val[4 * om_bsr_find(J, a, a)];
                    double *Aab = &J->val[4 * om_bsr_find(J, a, b)];
                    double *Aba = &J->val[4 * om_bsr_find(J, b, a)];
                    double *Abb = &J->val[4 * om_bsr_find(J, b, b)];
                    Aaa[2 * ph] -= fpa; Aaa[2 * ph + 1] -= fsa;
                    Aab[2 * ph] -= fpb; Aab[2 * ph + 1] -= fsb;
                    Aba[2 * ph] += fpa; Aba[2 * ph + 1] += fsa;
                    Abb[2 * ph] += fpb; Abb[2 * ph + 1] += fsb;
                }
            }
        }
    }

    /* wells (Eq 10-14) */
    for (int w = 0; w < m->nw; w++) {
        int rw = n + w;
        double pbh = x[2 * rw];
        double sgn = m->w_kind[w] == 0 ? 1.0 : -1.0;
        int ctrl = m->w_ctrl[w];
        double sum = 0.0, dsum_pb = 0.0;
        for (int q = m->w_ptr[w]; q < m->w_ptr[w + 1]; q++) {
            int c = m->w_cell[q];
            double p = x[2 * c], s = x[2 * c + 1];
            double bo = bfac(m, m->c_o, p), bw = bfac(m, m->c_w, p);
            double lo = (1.0 - s) * (1.0 - s) * bo / m->mu_o, lw = s * s * bw / m->mu_w;
            double lo_p = (1.0 - s) * (1.0 - s) * m->c_o / m->mu_o, lw_p = s * s * m->c_w / m->mu_w;
            double lo_s = -2.0 * (1.0 - s) * bo / m->mu_o, lw_s = 2.0 * s * bw / m->mu_w;
            double dzb = m->w_zb[w] - m->depth[c];
            double dgo = m->grav * m->rho_o * m->c_o / 144.0, dgw = m->grav * m->rho_w * m->c_w / 144.0;
            double dpo = pbh - p - gam(m, m->rho_o, m->c_o, p) * dzb;
            double dpw = pbh - p - gam(m, m->rho_w, m->c_w, p) * dzb;
            double WI = m->wi[q];
            double qo, qw, qo_p, qo_s, qo_b, qw_p, qw_s, qw_b;
            if (m->w_kind[w] == 0) {
                double lt = lo + lw;
                qo = qo_p = qo_s = qo_b = 0.0;
                qw = WI * lt * dpw;
                qw_p = WI * ((lo_p + lw_p) * dpw + lt * (-1.0 - dgw * dzb));
                qw_s = WI * (lo_s + lw_s) * dpw;
                qw_b = WI * lt;
            } else {
                qo = WI * lo * dpo;
                qo_p = WI * (lo_p * dpo + lo * (-1.0 - dgo * dzb));
                qo_s = WI * lo_s * dpo;
                qo_b = WI * lo;
                qw = WI * lw * dpw;
                qw_p = WI * (lw_p * dpw + lw * (-1.0 - dgw * dzb));
                qw_s = WI * lw_s * dpw;
                qw_b = WI * lw;
            }
            F[2 * c] -= qo;
            F[2 * c + 1] -= qw;
            double sel = 0.0, sel_p = 0.0, sel_s = 0.0, sel_b = 0.0;
            if (ctrl == 1) { sel = qw; sel_p = qw_p; sel_s = qw_s; sel_b = qw_b; }
            else if (ctrl == 2) { sel = qo; sel_p = qo_p; sel_s = qo_s; sel_b = qo_b; }
            else if (ctrl == 3) { sel = qo + qw; sel_p = qo_p + qw_p; sel_s = qo_s + qw_s; sel_b = qo_b + qw_b; }
            sum += sel;
            dsum_pb += sel_b;
            if (J) {
                double *Acc = &J->val[4 * om_bsr_find(J, c, c)];
                double *Acw = &J->val[4 * om_bsr_find(J, c, rw)];
                Acc[0] -= qo_p; Acc[1] -= qo_s; Acc[2] -= qw_p; Acc[3] -= qw_s;
                Acw[0] -= qo_b; Acw[2] -= qw_b;
                if (ctrl != 0) {
                    double *Awc = &J->val[4 * om_bsr_find(J, rw, c)];
                    Awc[0] += sel_p; Awc[1] += sel_s;
                }
            }
        }
        if (ctrl == 0) F[2 * rw] = pbh - m->w_target[w];
        else F[2 * rw] = sum - sgn * m->w_target[w];
        F[2 * rw + 1] = x[2 * rw + 1];
        if (J) {
            double *Aww = &J->val[4 * om_bsr_find(J, rw, rw)];
            Aww[0] = ctrl == 0 ? 1.0 : dsum_pb;
            Aww[1] = 0.0; Aww[2] = 0.0; Aww[3] = 1.0;
        }
    }
}

void om_residual(const om_model *m, const double *x, const double *xold, double dt, double *F)
{
    assemble(m, x, xold, dt, F, NULL);
}

int om_jacobian(const om_model *m, const double *x, const double *xold, double dt,
                om_bsr *J, double *F)
{
    if (!J->rp) om_pattern(m, J);
    assemble(m, x, xold, dt, F, J);
    return 0;
}

/* Scaled infinity norm used as the Newton stopping test:
 * max over cells of |R_a| * dt / PV (PV = V*phi_r/alpha_c, bbl) and over
 * wells of |R_w| / |target|. */
double om_scaled_norm(const om_model *m, const double *F, double dt)
{
    double r = 0.0;
    for (int i = 0; i < m->n; i++) {
        double pv = m->vol[i] * m->phi[i] / m->alpha_c;
        double a = fabs(F[2 * i]) * dt / pv, b = fabs(F[2 * i + 1]) * dt / pv;
        if (a > r || a != a) r = a;
        if (b > r || b != b) r = b;
    }
    for (int w = 0; w < m->nw; w++) {
        double t = fabs(m->w_target[w]);
        double a = fabs(F[2 * (m->n + w)]) / (t > 0.0 ? t : 1.0);
        if (a > r || a != a) r = a;
    }
    return r;
}
