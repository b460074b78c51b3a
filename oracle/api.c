/*
 * Oracle: heap-allocating wrappers and accessors for the Python binding.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 */
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

om_cpr *om_api_cpr_create(const om_bsr *A, const om_model *m, const double *x,
                          const om_cpr_opts *o, int *rc)
{
    om_cpr *P = (om_cpr *)calloc(1, sizeof(om_cpr));
    *rc = om_cpr_setup(P, A, m, x, o);
    return P;
}

void om_api_cpr_destroy(om_cpr *P)
{
    if (!P) return;
    om_cpr_free(P);
    free(P);
}

int om_api_amg_nlev(const om_cpr *P) { return P->amg.nlev; }

void om_api_amg_level_size(const om_cpr *P, int l, int *n, int *nnz)
{
    *n = P->amg.A[l].n;
    *nnz = P->amg.A[l].nnz;
}

void om_api_amg_copy_level(const om_cpr *P, int l, int *rp, int *col, double *val, double *l1,
                           int *agg)
{
    const om_csr *A = &P->amg.A[l];
    memcpy(rp, A->rp, sizeof(int) * (A->n + 1));
    memcpy(col, A->col, sizeof(int) * A->nnz);
    memcpy(val, A->val, sizeof(double) * A->nnz);
    memcpy(l1, P->amg.l1[l], sizeof(double) * A->n);
    if (agg && P->amg.agg[l]) memcpy(agg, P->amg.agg[l], sizeof(int) * A->n);
}

void om_api_amg_vcycle(const om_cpr *P, const double *b, double *x) { om_amg_vcycle(&P->amg, b, x); }

int om_api_ras_nsub(const om_cpr *P) { return P->ras.ns; }

void om_api_ras_sub_size(const om_cpr *P, int s, int *m, int *nnzb)
{
    *m = P->ras.sub[s].m;
    *nnzb = P->ras.sub[s].lu.nnzb;
}

void om_api_ras_copy_sub(const om_cpr *P, int s, int *glob, unsigned char *owned, int *rp,
                         int *col, double *val, double *dinv)
{
    const om_sub *S = &P->ras.sub[s];
    memcpy(glob, S->glob, sizeof(int) * S->m);
    memcpy(owned, S->owned, S->m);
    memcpy(rp, S->lu.rp, sizeof(int) * (S->m + 1));
    memcpy(col, S->lu.col, sizeof(int) * S->lu.nnzb);
    memcpy(val, S->lu.val, sizeof(double) * 4 * S->lu.nnzb);
    memcpy(dinv, S->dinv, sizeof(double) * 4 * S->m);
}

void om_api_ras_apply(const om_cpr *P, const double *r, double *y) { om_ras_apply(&P->ras, r, y); }

om_amg *om_api_amg_create(const om_csr *A, double theta, int max_coarse, int max_levels,
                          int rounds, int passes, int kcycle, int *rc)
{
    om_amg *H = (om_amg *)calloc(1, sizeof(om_amg));
    *rc = om_amg_setup(H, A, theta, max_coarse, max_levels, rounds, passes, kcycle);
    return H;
}

void om_api_amg_destroy(om_amg *H)
{
    if (!H) return;
    om_amg_free(H);
    free(H);
}

int om_api_amg_h_nlev(const om_amg *H) { return H->nlev; }

void om_api_amg_h_level_size(const om_amg *H, int l, int *n, int *nnz)
{
    *n = H->A[l].n;
    *nnz = H->A[l].nnz;
}

void om_api_amg_h_copy_level(const om_amg *H, int l, int *rp, int *col, double *val, double *l1,
                             int *agg)
{
    const om_csr *A = &H->A[l];
    memcpy(rp, A->rp, sizeof(int) * (A->n + 1));
    memcpy(col, A->col, sizeof(int) * A->nnz);
    memcpy(val, A->val, sizeof(double) * A->nnz);
    memcpy(l1, H->l1[l], sizeof(double) * A->n);
    if (agg && H->agg[l]) memcpy(agg, H->agg[l], sizeof(int) * A->n);
}

void om_api_amg_h_vcycle(const om_amg *H, const double *b, double *x) { om_amg_vcycle(H, b, x); }

/* Jacobian into caller arrays: pattern sizes first, then values. */
int om_api_jacobian_nnzb(const om_model *m)
{
    om_bsr J = {0};
    om_pattern(m, &J);
    int z = J.nnzb;
    om_bsr_free(&J);
    return z;
}

void om_api_jacobian(const om_model *m, const double *x, const double *xold, double dt, int *rp,
                     int *col, double *val, double *F)
{
    om_bsr J = {0};
    om_jacobian(m, x, xold, dt, &J, F);
    memcpy(rp, J.rp, sizeof(int) * (J.nb + 1));
    memcpy(col, J.col, sizeof(int) * J.nnzb);
    memcpy(val, J.val, sizeof(double) * 4 * J.nnzb);
    om_bsr_free(&J);
}

void om_api_wells(const om_model *m, double *wi, double *zb)
{
    memcpy(wi, m->wi, sizeof(double) * m->nperf);
    memcpy(zb, m->w_zb, sizeof(double) * m->nw);
}
