/*
 * Oracle: local potential reordering, block ILU(0) and restricted additive
 * Schwarz.  TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Paper sections followed: "Local potential reordering technique" (Eq 30-33)
 * and "Multi-stage preconditioner" (the RAS stage R(A)^-1 of Algorithm 2).
 * Readings where the paper is silent:
 *   - subdomains are px x py tiles of the x-y plane with full columns in z;
 *     a well belongs to the tile holding its first perforation;
 *   - the overlapped subdomain is every block row within block-graph
 *     distance `overlap` of the owned rows; couplings leaving it are dropped;
 *   - the local order sorts the subdomain's cells by descending oil
 *     potential, ties by ascending natural index (Eq 30 on the local cells),
 *     then appends its wells (the well part of Eq 32);
 *   - the subdomain solver is block ILU(0) with 2x2 blocks on that order;
 *   - RAS adds back only the owned rows of each local solution.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

typedef struct { double key; int idx; } kv;

static int cmp_desc(const void *a, const void *b)
{
    const kv *x = (const kv *)a, *y = (const kv *)b;
    if (x->key > y->key) return -1;
    if (x->key < y->key) return 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

/* Eq 30 on a set of cells: perm[pos] = cells[...] sorted by descending
 * potential (ties by ascending cell index).  Returns -1 on a NaN potential. */
int om_potential_order(int m, const double *phi_o, const int *cells, int *perm)
{
    kv *t = (kv *)malloc(sizeof(kv) * (m > 0 ? m : 1));
    for (int a = 0; a < m; a++) {
        t[a].key = phi_o[cells[a]];
        t[a].idx = cells[a];
        if (t[a].key != t[a].key) { free(t); return -1; }
    }
    qsort(t, m, sizeof(kv), cmp_desc);
    for (int a = 0; a < m; a++) perm[a] = t[a].idx;
    free(t);
    return 0;
}

static int cmp_int(const void *a, const void *b)
{
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/* In-place block ILU(0) in row order (IKJ form).  On return the strict lower
 * blocks hold L (unit block diagonal implied), the rest hold U, and dinv
 * holds the inverses of U's diagonal blocks.  Returns 0, or 1+row of a
 * singular pivot block. */
int om_bilu0(om_bsr *A, double *dinv, int *diag)
{
    for (int i = 0; i < A->nb; i++) {
        diag[i] = -1;
        for (int z = A->rp[i]; z < A->rp[i + 1]; z++)
            if (A->col[z] == i) diag[i] = z;
        if (diag[i] < 0) return i + 1;
    }
    for (int i = 0; i < A->nb; i++) {
        for (int z = A->rp[i]; z < A->rp[i + 1] && A->col[z] < i; z++) {
            int k = A->col[z];
            double *a = &A->val[4 * z];
            const double *dk = &dinv[4 * k];
            double l0 = a[0] * dk[0] + a[1] * dk[2];
            double l1 = a[0] * dk[1] + a[1] * dk[3];
            double l2 = a[2] * dk[0] + a[3] * dk[2];
            double l3 = a[2] * dk[1] + a[3] * dk[3];
            a[0] = l0; a[1] = l1; a[2] = l2; a[3] = l3;
            for (int z2 = z + 1; z2 < A->rp[i + 1]; z2++) {
                int j = A->col[z2];
                int zk = -1;
                for (int y = A->rp[k]; y < A->rp[k + 1]; y++)
                    if (A->col[y] == j) { zk = y; break; }
                if (zk < 0) continue;
                const double *u = &A->val[4 * zk];
                double *t = &A->val[4 * z2];
                t[0] -= l0 * u[0] + l1 * u[2];
                t[1] -= l0 * u[1] + l1 * u[3];
                t[2] -= l2 * u[0] + l3 * u[2];
                t[3] -= l2 * u[1] + l3 * u[3];
            }
        }
        const double *d = &A->val[4 * diag[i]];
        double det = d[0] * d[3] - d[1] * d[2];
        if (det == 0.0 || det != det) return i + 1;
        om_block_inv(d, &dinv[4 * i]);
    }
    return 0;
}

/* v <- (LU)^-1 v, forward then backward substitution in row order. */
void om_bilu0_solve(const om_bsr *LU, const double *dinv, const int *diag, double *v)
{
    for (int i = 0; i < LU->nb; i++) {
        double t0 = v[2 * i], t1 = v[2 * i + 1];
        for (int z = LU->rp[i]; z < diag[i]; z++) {
            const double *l = &LU->val[4 * z];
            int k = LU->col[z];
            t0 -= l[0] * v[2 * k] + l[1] * v[2 * k + 1];
            t1 -= l[2] * v[2 * k] + l[3] * v[2 * k + 1];
        }
        v[2 * i] = t0; v[2 * i + 1] = t1;
    }
    for (int i = LU->nb - 1; i >= 0; i--) {
        double t0 = v[2 * i], t1 = v[2 * i + 1];
        for (int z = diag[i] + 1; z < LU->rp[i + 1]; z++) {
            const double *u = &LU->val[4 * z];
            int j = LU->col[z];
            t0 -= u[0] * v[2 * j] + u[1] * v[2 * j + 1];
            t1 -= u[2] * v[2 * j] + u[3] * v[2 * j + 1];
        }
        const double *di = &dinv[4 * i];
        v[2 * i] = di[0] * t0 + di[1] * t1;
        v[2 * i + 1] = di[2] * t0 + di[3] * t1;
    }
}

/* Owner tile of each block row (cells by x-y tile, wells by first perforation). */
static void tile_owner(const om_model *mdl, int px, int py, int *owner)
{
    int nx = mdl->nx, ny = mdl->ny;
    for (int c = 0; c < mdl->n; c++) {
        int i = c % nx, j = (c / nx) % ny;
        int a = (int)(((long)i * px) / nx), b = (int)(((long)j * py) / ny);
        owner[c] = a + px * b;
    }
    for (int w = 0; w < mdl->nw; w++) owner[mdl->n + w] = owner[mdl->w_cell[mdl->w_ptr[w]]];
}

int om_ras_setup(om_ras *R, const om_bsr *A, const om_model *mdl, const double *x,
                 int px, int py, int overlap, int order)
{
    int nb = A->nb, n = mdl->n;
    R->ns = px * py;
    R->sub = (om_sub *)calloc(R->ns, sizeof(om_sub));
    R->owner = (int *)malloc(sizeof(int) * nb);
    R->work = (double *)malloc(sizeof(double) * 2 * nb);
    tile_owner(mdl, px, py, R->owner);
    double *phi = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    om_potential(mdl, x, phi);
    int *mark = (int *)malloc(sizeof(int) * nb);
    int *loc = (int *)malloc(sizeof(int) * nb);
    int *list = (int *)malloc(sizeof(int) * nb);
    for (int s = 0; s < R->ns; s++) {
        om_sub *S = &R->sub[s];
        /* overlapped set: breadth-first layers on the block graph */
        for (int i = 0; i < nb; i++) mark[i] = 0;
        int cnt = 0;
        for (int i = 0; i < nb; i++)
            if (R->owner[i] == s) { mark[i] = 1; list[cnt++] = i; }
        int lo = 0;
        for (int d = 0; d < overlap; d++) {
            int hi = cnt;
            for (int q = lo; q < hi; q++) {
                int i = list[q];
                for (int z = A->rp[i]; z < A->rp[i + 1]; z++) {
                    int j = A->col[z];
                    if (!mark[j]) { mark[j] = 1; list[cnt++] = j; }
                }
            }
            lo = hi;
        }
        qsort(list, cnt, sizeof(int), cmp_int);
        int nc = 0;
        while (nc < cnt && list[nc] < n) nc++;
        S->m = cnt;
        S->glob = (int *)malloc(sizeof(int) * (cnt > 0 ? cnt : 1));
        S->owned = (unsigned char *)malloc(cnt > 0 ? cnt : 1);
        if (order == OM_ORD_POTENTIAL) {
            if (om_potential_order(nc, phi, list, S->glob)) return -1;
        } else {
            memcpy(S->glob, list, sizeof(int) * nc);
        }
        memcpy(S->glob + nc, list + nc, sizeof(int) * (cnt - nc)); /* wells last */
        for (int i = 0; i < nb; i++) loc[i] = -1;
        for (int a = 0; a < cnt; a++) {
            loc[S->glob[a]] = a;
            S->owned[a] = R->owner[S->glob[a]] == s;
        }
        /* local matrix in local order, columns sorted by local index */
        om_bsr *L = &S->lu;
        L->nb = cnt;
        L->rp = (int *)malloc(sizeof(int) * (cnt + 1));
        int nz = 0;
        for (int a = 0; a < cnt; a++) {
            int g = S->glob[a];
            for (int z = A->rp[g]; z < A->rp[g + 1]; z++)
                if (loc[A->col[z]] >= 0) nz++;
        }
        L->nnzb = nz;
        L->col = (int *)malloc(sizeof(int) * (nz > 0 ? nz : 1));
        L->val = (double *)malloc(sizeof(double) * 4 * (nz > 0 ? nz : 1));
        nz = 0;
        L->rp[0] = 0;
        for (int a = 0; a < cnt; a++) {
            int g = S->glob[a];
            int start = nz;
            for (int z = A->rp[g]; z < A->rp[g + 1]; z++) {
                int c = loc[A->col[z]];
                if (c < 0) continue;
                /* insertion by local column */
                int t = nz - 1;
                while (t >= start && L->col[t] > c) {
                    L->col[t + 1] = L->col[t];
                    memcpy(&L->val[4 * (t + 1)], &L->val[4 * t], 4 * sizeof(double));
                    t--;
                }
                L->col[t + 1] = c;
                memcpy(&L->val[4 * (t + 1)], &A->val[4 * z], 4 * sizeof(double));
                nz++;
            }
            L->rp[a + 1] = nz;
        }
        S->dinv = (double *)malloc(sizeof(double) * 4 * (cnt > 0 ? cnt : 1));
        S->diag = (int *)malloc(sizeof(int) * (cnt > 0 ? cnt : 1));
        int rc = om_bilu0(L, S->dinv, S->diag);
        if (rc) { free(phi); free(mark); free(loc); free(list); return rc; }
    }
    free(phi); free(mark); free(loc); free(list);
    return 0;
}

/* y = sum_s R_s^0^T (L_s U_s)^-1 R_s^delta r */
void om_ras_apply(const om_ras *R, const double *r, double *y)
{
    for (int s = 0; s < R->ns; s++) {
        const om_sub *S = &R->sub[s];
        double *v = R->work;
        for (int a = 0; a < S->m; a++) {
            v[2 * a] = r[2 * S->glob[a]];
            v[2 * a + 1] = r[2 * S->glob[a] + 1];
        }
        om_bilu0_solve(&S->lu, S->dinv, S->diag, v);
        for (int a = 0; a < S->m; a++)
            if (S->owned[a]) {
                y[2 * S->glob[a]] = v[2 * a];
                y[2 * S->glob[a] + 1] = v[2 * a + 1];
            }
    }
}

void om_ras_free(om_ras *R)
{
    for (int s = 0; s < R->ns; s++) {
        om_sub *S = &R->sub[s];
        free(S->glob); free(S->owned); om_bsr_free(&S->lu); free(S->dinv); free(S->diag);
    }
    free(R->sub); free(R->owner); free(R->work);
    memset(R, 0, sizeof(*R));
}
