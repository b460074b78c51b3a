/*
 * Oracle: CPR preconditioner, flexible GMRES and Newton's method.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Paper sections followed:
 *   - "Multi-stage preconditioner": restriction Pi_r and prolongation Pi_p
 *     (Eq 34-35) and the CPR-FPF preconditioner of Algorithm 2.  The
 *     two-stage form is Algorithm 2 started at its third step with x = 0:
 *       x = Pi_p M(A_pp)^-1 Pi_r f;  r = f - A x;  x = x + R(A)^-1 r.
 *   - Krylov solver: restarted GMRES(m) (Examples 4-5), here right
 *     preconditioned and flexible (the preconditioned basis is stored), with
 *     modified Gram-Schmidt and Givens rotations (Saad's textbook form).
 *     Convergence is decided on the true residual of the decoupled system.
 *   - "Nonlinear methods": Newton's method (standard: fixed linear
 *     tolerance) and the inexact Newton method of Algorithm 1 with the
 *     second forcing term of Eq 26 clipped to [0.01, 0.1].
 *   - Decoupling D^-1 A x = D^-1 b (Eq 29) before the preconditioner setup.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

static double nrm2(int n, const double *a) { return sqrt(om_dot(n, a, a)); }

int om_cpr_setup(om_cpr *P, const om_bsr *A, const om_model *mdl, const double *x,
                 const om_cpr_opts *o)
{
    memset(P, 0, sizeof(*P));
    P->o = *o;
    P->A = A;
    P->ncell = mdl->n;
    int N = 2 * A->nb;
    P->t1 = (double *)malloc(sizeof(double) * N);
    P->t2 = (double *)malloc(sizeof(double) * N);
    P->t3 = (double *)malloc(sizeof(double) * N);
    om_csr App;
    om_extract_pressure(A, mdl->n, &App);
    int rc = 0;
    if (o->exact_stages) {
        P->dense_A = (double *)malloc(sizeof(double) * (size_t)N * N);
        P->piv_A = (int *)malloc(sizeof(int) * N);
        om_bsr_to_dense(A, P->dense_A);
        rc = om_dense_lu(N, P->dense_A, P->piv_A);
        int n = mdl->n;
        P->dense_App = (double *)calloc((size_t)n * n, sizeof(double));
        P->piv_App = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
        for (int i = 0; i < n; i++)
            for (int z = App.rp[i]; z < App.rp[i + 1]; z++)
                P->dense_App[(size_t)i * n + App.col[z]] = App.val[z];
        if (!rc) rc = om_dense_lu(n, P->dense_App, P->piv_App);
    } else {
        rc = om_ras_setup(&P->ras, A, mdl, x, o->px, o->py, o->overlap, o->order);
        if (!rc) rc = om_amg_setup(&P->amg, &App, o->theta, o->max_coarse, o->max_levels,
                                   o->match_rounds, o->agg_passes, o->kcycle);
    }
    om_csr_free(&App);
    return rc;
}

static void stage_ras(const om_cpr *P, const double *r, double *y)
{
    int N = 2 * P->A->nb;
    if (P->o.exact_stages) {
        memcpy(y, r, sizeof(double) * N);
        om_dense_lu_solve(N, P->dense_A, P->piv_A, y);
    } else {
        om_ras_apply(&P->ras, r, y);
    }
}

/* x_p = M(A_pp)^-1 (Pi_r r), M(A_pp)^-1 being amg_cycles AMG cycles */
static void stage_amg(const om_cpr *P, const double *r, double *xp)
{
    int n = P->ncell;
    double *rp = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    for (int i = 0; i < n; i++) rp[i] = r[2 * i];                 /* Pi_r, Eq 34 */
    if (P->o.exact_stages) {
        memcpy(xp, rp, sizeof(double) * n);
        om_dense_lu_solve(n, P->dense_App, P->piv_App, xp);
    } else {
        om_amg_cycles(&P->amg, rp, xp, P->o.amg_cycles);
    }
    free(rp);
}

static void residual(const om_bsr *A, const double *f, const double *x, double *r)
{
    int N = 2 * A->nb;
    om_bsr_spmv(A, x, r);
    for (int i = 0; i < N; i++) r[i] = f[i] - r[i];
}

void om_cpr_apply(const om_cpr *P, const double *f, double *x)
{
    int N = 2 * P->A->nb, n = P->ncell;
    double *r = P->t1, *y = P->t2, *xp = P->t3;
    if (P->o.form == OM_CPR_FPF) {
        stage_ras(P, f, x);                                       /* x = R(A)^-1 f */
        residual(P->A, f, x, r);                                  /* r = f - A x */
        stage_amg(P, r, xp);
        for (int i = 0; i < n; i++) x[2 * i] += xp[i];            /* x += Pi_p xp, Eq 35 */
        residual(P->A, f, x, r);                                  /* r = f - A x */
        stage_ras(P, r, y);
        for (int i = 0; i < N; i++) x[i] += y[i];                 /* x += R(A)^-1 r */
    } else {
        stage_amg(P, f, xp);
        for (int i = 0; i < N; i++) x[i] = 0.0;
        for (int i = 0; i < n; i++) x[2 * i] = xp[i];             /* x = Pi_p xp */
        residual(P->A, f, x, r);
        stage_ras(P, r, y);
        for (int i = 0; i < N; i++) x[i] += y[i];
    }
}

void om_cpr_free(om_cpr *P)
{
    if (P->o.exact_stages) {
        free(P->dense_A); free(P->piv_A); free(P->dense_App); free(P->piv_App);
    } else {
        om_ras_free(&P->ras);
        om_amg_free(&P->amg);
    }
    free(P->t1); free(P->t2); free(P->t3);
    memset(P, 0, sizeof(*P));
}

/* Right-preconditioned flexible GMRES(restart) from x = 0.  P == NULL means
 * no preconditioner.  Returns 0 when the true relative residual reaches
 * rtol, 1 when maxit is exhausted (x holds the last iterate), 2 on breakdown. */
int om_fgmres(const om_bsr *A, const om_cpr *P, const double *b, double *x, int m,
              double rtol, int maxit, int *iters, double *relres, double *hist)
{
    int N = 2 * A->nb;
    double *V = (double *)malloc(sizeof(double) * (size_t)N * (m + 1));
    double *Z = (double *)malloc(sizeof(double) * (size_t)N * m);
    double *H = (double *)calloc((size_t)(m + 1) * m, sizeof(double));
    double *cs = (double *)malloc(sizeof(double) * m), *sn = (double *)malloc(sizeof(double) * m);
    double *g = (double *)malloc(sizeof(double) * (m + 1)), *yv = (double *)malloc(sizeof(double) * m);
    double *r = (double *)malloc(sizeof(double) * N);
    for (int i = 0; i < N; i++) x[i] = 0.0;
    double bnorm = nrm2(N, b);
    int total = 0, status = 1;
    *iters = 0;
    if (bnorm == 0.0) { *relres = 0.0; status = 0; goto done; }
    memcpy(r, b, sizeof(double) * N);
    double beta = bnorm;
    while (total < maxit) {
        for (int i = 0; i < N; i++) V[i] = r[i] / beta;
        for (int i = 0; i <= m; i++) g[i] = 0.0;
        g[0] = beta;
        int j, k = 0;
        for (j = 0; j < m && total < maxit; j++) {
            double *vj = V + (size_t)j * N, *zj = Z + (size_t)j * N, *w = V + (size_t)(j + 1) * N;
            if (P) om_cpr_apply(P, vj, zj); else memcpy(zj, vj, sizeof(double) * N);
            om_bsr_spmv(A, zj, w);
            for (int i = 0; i <= j; i++) {                        /* modified Gram-Schmidt */
                double *vi = V + (size_t)i * N;
                double h = om_dot(N, w, vi);
                H[(size_t)i * m + j] = h;
                for (int t = 0; t < N; t++) w[t] -= h * vi[t];
            }
            double hn = nrm2(N, w);
            H[(size_t)(j + 1) * m + j] = hn;
            if (hn != 0.0) for (int t = 0; t < N; t++) w[t] /= hn;
            for (int i = 0; i < j; i++) {                         /* previous rotations */
                double a = H[(size_t)i * m + j], c = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * c;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
            }
            double a = H[(size_t)j * m + j], c = H[(size_t)(j + 1) * m + j];
            double den = sqrt(a * a + c * c);
            if (den == 0.0) { status = 2; goto done; }
            cs[j] = a / den; sn[j] = c / den;
            H[(size_t)j * m + j] = den;
            H[(size_t)(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            total++;
            k = j + 1;
            if (hist) hist[total - 1] = fabs(g[j + 1]) / bnorm;
            if (fabs(g[j + 1]) <= rtol * bnorm || hn == 0.0) break;
        }
        for (int i = k - 1; i >= 0; i--) {                        /* back substitution */
            double s = g[i];
            for (int t = i + 1; t < k; t++) s -= H[(size_t)i * m + t] * yv[t];
            yv[i] = s / H[(size_t)i * m + i];
        }
        for (int i = 0; i < k; i++) {
            double *zi = Z + (size_t)i * N;
            for (int t = 0; t < N; t++) x[t] += yv[i] * zi[t];
        }
        residual(A, b, x, r);
        beta = nrm2(N, r);
        *relres = beta / bnorm;
        if (beta <= rtol * bnorm) { status = 0; break; }
        if (beta == 0.0) { status = 0; break; }
    }
    *iters = total;
done:
    *iters = total;
    if (status == 0 && bnorm == 0.0) *relres = 0.0;
    free(V); free(Z); free(H); free(cs); free(sn); free(g); free(yv); free(r);
    return status;
}

/* Right-preconditioned BiCGSTAB (van der Vorst's stabilised bi-conjugate
 * gradients, the paper's other Krylov solver), zero initial guess, shadow
 * residual r^ = b.  Converged when the recursive residual is at most rtol
 * ||b||; the true residual b - A x is then checked, and if it is above the
 * target the recurrences restart from it.  One iteration = two
 * preconditioner applications and two products with A. */
int om_bicgstab(const om_bsr *A, const om_cpr *P, const double *b, double *x, double rtol,
                int maxit, int *iters, double *relres)
{
    int N = 2 * A->nb;
    double *r = (double *)malloc(sizeof(double) * N), *rh = (double *)malloc(sizeof(double) * N);
    double *p = (double *)calloc(N, sizeof(double)), *v = (double *)calloc(N, sizeof(double));
    double *ph = (double *)malloc(sizeof(double) * N), *sv = (double *)malloc(sizeof(double) * N);
    double *sh = (double *)malloc(sizeof(double) * N), *t = (double *)malloc(sizeof(double) * N);
    for (int i = 0; i < N; i++) x[i] = 0.0;
    double bnorm = nrm2(N, b);
    int status = 1, it = 0;
    *iters = 0;
    *relres = 0.0;
    if (bnorm == 0.0) { status = 0; goto done; }
    memcpy(r, b, sizeof(double) * N);
    memcpy(rh, b, sizeof(double) * N);
    double rho_prev = 1.0, alpha = 1.0, omega = 1.0;
    int fresh = 1;
    while (it < maxit) {
        double rho = om_dot(N, rh, r);
        if (rho == 0.0) { status = 2; break; }
        if (fresh) {
            memcpy(p, r, sizeof(double) * N);
        } else {
            double beta = (rho / rho_prev) * (alpha / omega);
            for (int i = 0; i < N; i++) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        }
        fresh = 0;
        if (P) om_cpr_apply(P, p, ph); else memcpy(ph, p, sizeof(double) * N);
        om_bsr_spmv(A, ph, v);
        double rv = om_dot(N, rh, v);
        if (rv == 0.0) { status = 2; break; }
        alpha = rho / rv;
        for (int i = 0; i < N; i++) sv[i] = r[i] - alpha * v[i];
        it++;
        int conv = 0;
        if (nrm2(N, sv) <= rtol * bnorm) {
            for (int i = 0; i < N; i++) x[i] += alpha * ph[i];
            conv = 1;
        } else {
            if (P) om_cpr_apply(P, sv, sh); else memcpy(sh, sv, sizeof(double) * N);
            om_bsr_spmv(A, sh, t);
            double tt = om_dot(N, t, t);
            omega = tt > 0.0 ? om_dot(N, t, sv) / tt : 0.0;
            for (int i = 0; i < N; i++) x[i] += alpha * ph[i] + omega * sh[i];
            for (int i = 0; i < N; i++) r[i] = sv[i] - omega * t[i];
            rho_prev = rho;
            if (nrm2(N, r) <= rtol * bnorm) conv = 1;
            else if (omega == 0.0) { status = 2; break; }
        }
        if (conv) {
            om_bsr_spmv(A, x, t);                                  /* true residual */
            for (int i = 0; i < N; i++) r[i] = b[i] - t[i];
            double rn = nrm2(N, r);
            *relres = rn / bnorm;
            if (rn <= rtol * bnorm) { status = 0; break; }
            memcpy(rh, r, sizeof(double) * N);                     /* restart */
            rho_prev = alpha = omega = 1.0;
            fresh = 1;
        }
    }
    if (status != 0) {
        om_bsr_spmv(A, x, t);
        for (int i = 0; i < N; i++) r[i] = b[i] - t[i];
        *relres = nrm2(N, r) / bnorm;
    }
done:
    *iters = it;
    free(r); free(rh); free(p); free(v); free(ph); free(sv); free(sh); free(t);
    return status;
}

/* One implicit time step x^n -> x^{n+1} by Newton's method (in place).
 * forcing 0: every linear solve to rtol; forcing 1: Eisenstat-Walker
 * (second choice of Eq 26, clipped to [0.01, 0.1], starting at 0.1).
 * Per Newton iteration l (NULL allowed): fn_hist[l] = ||F(x_l)||_2,
 * eta_hist[l] = the linear tolerance used, rn_hist[l] = ||b - J y||_2 of the
 * solve (Eq 27).  A CPR set-up that fails (singular pivot, stalled AMG
 * coarsening) ends the step as not converged.
 * exact_linear: solve each Newton system by dense LU instead of CPR-Krylov;
 * krylov 0: FGMRES(restart), 1: BiCGSTAB.
 * ds_max > 0 limits each cell's saturation change per Newton iteration.
 * Returns 0 on convergence (x updated), 1 if Newton or a linear solve
 * failed (x unchanged). */
int om_newton_step(const om_model *m, double *x, double dt, const om_cpr_opts *o, int restart,
                   double rtol, int maxit, double ntol, int max_newton, int exact_linear,
                   int forcing, double ds_max, int krylov, int *newton_its, int *lin_its,
                   double *res_hist, double *fn_hist, double *rn_hist, double *eta_hist)
{
    int n = m->n, N = 2 * (m->n + m->nw);
    double *xo = (double *)malloc(sizeof(double) * N);
    double *xk = (double *)malloc(sizeof(double) * N);
    double *F = (double *)malloc(sizeof(double) * N);
    double *b = (double *)malloc(sizeof(double) * N);
    double *bd = (double *)malloc(sizeof(double) * N);
    double *y = (double *)malloc(sizeof(double) * N);
    double *t = (double *)malloc(sizeof(double) * N);
    memcpy(xo, x, sizeof(double) * N);
    memcpy(xk, x, sizeof(double) * N);
    om_bsr J = {0};
    om_pattern(m, &J);
    int status = 1, lits = 0;
    double eta = 0.1, prev_fn = 0.0, prev_rn = 0.0;
    *newton_its = 0;
    for (int it = 0; it <= max_newton; it++) {
        om_jacobian(m, xk, xo, dt, &J, F);
        double sn = om_scaled_norm(m, F, dt);
        if (res_hist) res_hist[it] = sn;
        if (sn != sn) break;
        if (sn <= ntol) { status = 0; break; }
        if (it == max_newton) break;
        for (int i = 0; i < N; i++) b[i] = -F[i];
        double fn = nrm2(N, b);
        if (forcing == 1 && it > 0) {
            eta = fabs(fn - prev_rn) / prev_fn;                   /* Eq 26, second choice */
            if (eta < 0.01) eta = 0.01;
            if (eta > 0.1) eta = 0.1;
        }
        double tol = forcing == 1 ? eta : rtol;
        if (fn_hist) fn_hist[it] = fn;
        if (eta_hist) eta_hist[it] = tol;
        if (exact_linear) {
            double *D = (double *)malloc(sizeof(double) * (size_t)N * N);
            int *piv = (int *)malloc(sizeof(int) * N);
            om_bsr_to_dense(&J, D);
            int rc = om_dense_lu(N, D, piv);
            memcpy(y, b, sizeof(double) * N);
            if (!rc) om_dense_lu_solve(N, D, piv, y);
            free(D); free(piv);
            if (rc) break;
        } else {
            om_bsr Ad;
            om_bsr_copy(&Ad, &J);
            memcpy(bd, b, sizeof(double) * N);
            om_decouple(&Ad, bd, n, o->decouple);
            om_cpr P;
            int rc = om_cpr_setup(&P, &Ad, m, xk, o);
            int its = 0, lrc = 0;
            double rr = 0.0;
            if (!rc) lrc = krylov == 1 ? om_bicgstab(&Ad, &P, bd, y, tol, maxit, &its, &rr)
                                       : om_fgmres(&Ad, &P, bd, y, restart, tol, maxit, &its, &rr, NULL);
            lits += its;
            om_cpr_free(&P);
            om_bsr_free(&Ad);
            if (rc) break;                                        /* set-up failed */
            if (lrc && forcing == 0) break;
        }
        om_bsr_spmv(&J, y, t);                                    /* r = b - J y, Eq 27 */
        for (int i = 0; i < N; i++) t[i] = b[i] - t[i];
        prev_rn = nrm2(N, t);
        if (rn_hist) rn_hist[it] = prev_rn;
        prev_fn = fn;
        for (int i = 0; i < N; i++) {                             /* Algorithm 1, update */
            double d = y[i];
            if (i < 2 * n && (i & 1) && ds_max > 0.0)             /* saturation chop */
                d = d > ds_max ? ds_max : (d < -ds_max ? -ds_max : d);
            xk[i] += d;
        }
        for (int i = 0; i < n; i++) {
            double s = xk[2 * i + 1];
            xk[2 * i + 1] = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
        }
        *newton_its = it + 1;
    }
    if (status == 0) memcpy(x, xk, sizeof(double) * N);
    *lin_its = lits;
    om_bsr_free(&J);
    free(xo); free(xk); free(F); free(b); free(bd); free(y); free(t);
    return status;
}
