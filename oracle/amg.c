/*
 * Oracle: algebraic multigrid on the pressure block A_pp.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The paper names AMG for the pressure stage M(A_pp)^-1 of Algorithm 2 (the
 * "Multi-stage preconditioner" section) without fixing a variant.  This
 * oracle uses the reading adopted for both sides:
 *   - A_pp = the (pressure-equation, pressure) entry of every decoupled
 *     cell-cell block, restriction Pi_r of Eq 34 applied to rows and columns;
 *   - coupling weight of rows i != j: w_ij = -(a_ij + a_ji) / 2 (a missing
 *     entry counts as 0), the same number seen from either row; M_i = the
 *     largest w_ik of row i (0 when none is positive); the pair is strong
 *     when w_ij > 0 and w_ij >= theta * M_i or w_ij >= theta * M_j, a
 *     relation that is symmetric too;
 *   - pairwise matching by handshakes: in each round every unmatched row
 *     proposes its strongest unmatched strong neighbour (largest w_ij, ties
 *     to the smaller index); mutual proposals become pairs.  Because weight,
 *     relation and tie rule are symmetric, a chain of proposals climbs to a
 *     mutual pair, so every round pairs off at least one row of every group
 *     of unmatched rows joined by strong couplings.  Rows left after the last
 *     round join the pair of their strongest strong neighbour that is in a
 *     pair (same order), or stay singletons when there is none;
 *   - `passes` aggregation passes per level (each on the Galerkin product of
 *     the previous one); aggregates are numbered by their leader (the
 *     smaller row of a pair, or the singleton);
 *   - piecewise-constant prolongation P, Galerkin coarse matrix A_c = P^T A P
 *     summed in ascending fine row, then stored column order;
 *   - l1-Jacobi smoothing (d_i = sum_j |a_ij|), one sweep before and after
 *     the coarse correction, zero initial guess;
 *   - the cycle: on the `kcycle` finest levels the coarse system is solved by
 *     two steps of the generalised conjugate residual method, each
 *     preconditioned by one cycle on the coarser level (a K-cycle); below,
 *     one cycle (a V-cycle);
 *   - coarsest level solved by dense LU with partial pivoting.  Coarsening
 *     stops when a level makes no progress; a coarsest level above 4096
 *     rows is then reported as a soft failure of the set-up.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

/* Pi_r A Pi_p restricted to reservoir rows/columns: scalar CSR of a00. */
void om_extract_pressure(const om_bsr *A, int ncell, om_csr *P)
{
    int nnz = 0;
    for (int i = 0; i < ncell; i++)
        for (int z = A->rp[i]; z < A->rp[i + 1]; z++)
            if (A->col[z] < ncell) nnz++;
    P->n = ncell; P->nnz = nnz;
    P->rp = (int *)malloc(sizeof(int) * (ncell + 1));
    P->col = (int *)malloc(sizeof(int) * (nnz > 0 ? nnz : 1));
    P->val = (double *)malloc(sizeof(double) * (nnz > 0 ? nnz : 1));
    nnz = 0;
    P->rp[0] = 0;
    for (int i = 0; i < ncell; i++) {
        for (int z = A->rp[i]; z < A->rp[i + 1]; z++)
            if (A->col[z] < ncell) {
                P->col[nnz] = A->col[z];
                P->val[nnz] = A->val[4 * z];
                nnz++;
            }
        P->rp[i + 1] = nnz;
    }
}

/* a_ij, or 0 when row i stores no column j. */
static double entry(const om_csr *A, int i, int j)
{
    for (int z = A->rp[i]; z < A->rp[i + 1]; z++)
        if (A->col[z] == j) return A->val[z];
    return 0.0;
}

/* w[z] = -(a_ij + a_ji)/2 for each stored off-diagonal entry z = (i, j)
 * (0 on the diagonal), and M_i = max(0, max_j w_ij). */
void om_coupling_weights(const om_csr *A, double *w, double *M)
{
    for (int i = 0; i < A->n; i++) {
        double mx = 0.0;
        for (int z = A->rp[i]; z < A->rp[i + 1]; z++) {
            int j = A->col[z];
            w[z] = 0.0;
            if (j == i) continue;
            w[z] = -(A->val[z] + entry(A, j, i)) / 2.0;
            if (w[z] > mx) mx = w[z];
        }
        M[i] = mx;
    }
}

static int strong(double wij, double Mi, double Mj, double theta)
{
    return wij > 0.0 && (wij >= theta * Mi || wij >= theta * Mj);
}

void om_strength_match(const om_csr *A, double theta, int rounds, int *match)
{
    int n = A->n;
    int *prop = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    double *w = (double *)malloc(sizeof(double) * (A->nnz > 0 ? A->nnz : 1));
    double *M = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    om_coupling_weights(A, w, M);
    for (int i = 0; i < n; i++) match[i] = -1;
    for (int r = 0; r < rounds; r++) {
        for (int i = 0; i < n; i++) {
            prop[i] = -1;
            if (match[i] >= 0) continue;
            double best = 0.0;
            for (int z = A->rp[i]; z < A->rp[i + 1]; z++) {
                int j = A->col[z];
                if (j == i || match[j] >= 0 || !strong(w[z], M[i], M[j], theta)) continue;
                /* columns ascend, so a strict > keeps the smaller index on ties */
                if (prop[i] < 0 || w[z] > best) { best = w[z]; prop[i] = j; }
            }
        }
        for (int i = 0; i < n; i++) {
            int j = prop[i];
            if (match[i] < 0 && j >= 0 && prop[j] == i) match[i] = j;
        }
    }
    free(prop); free(w); free(M);
}

/* Rows left unmatched after the handshake rounds join the pair of their
 * strongest strong neighbour that is in a pair (ties to the smaller index);
 * a row with no such neighbour stays a singleton.  jt[i] = that neighbour
 * or -1. */
void om_join_targets(const om_csr *A, double theta, const int *match, int *jt)
{
    int n = A->n;
    double *w = (double *)malloc(sizeof(double) * (A->nnz > 0 ? A->nnz : 1));
    double *M = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    om_coupling_weights(A, w, M);
    for (int i = 0; i < n; i++) {
        jt[i] = -1;
        if (match[i] >= 0) continue;
        double best = 0.0;
        for (int z = A->rp[i]; z < A->rp[i + 1]; z++) {
            int j = A->col[z];
            if (j == i || match[j] < 0 || !strong(w[z], M[i], M[j], theta)) continue;
            if (jt[i] < 0 || w[z] > best) { best = w[z]; jt[i] = j; }
        }
    }
    free(w); free(M);
}

/* Aggregates of one pass: pairs, the rows that join them and the remaining
 * singletons, numbered in order of their leader (the smaller row of the
 * pair, or the singleton).  Returns the number of aggregates. */
int om_aggregate(const om_csr *A, double theta, int rounds, int *agg)
{
    int n = A->n;
    int *match = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    int *jt = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    int *lead = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    om_strength_match(A, theta, rounds, match);
    om_join_targets(A, theta, match, jt);
    for (int i = 0; i < n; i++) {
        if (match[i] >= 0) lead[i] = i < match[i] ? i : match[i];
        else if (jt[i] >= 0) {
            int k = jt[i];
            lead[i] = k < match[k] ? k : match[k];
        } else lead[i] = i;
    }
    int nc = 0;
    for (int i = 0; i < n; i++)
        if (lead[i] == i) agg[i] = nc++;
    for (int i = 0; i < n; i++)
        if (lead[i] != i) agg[i] = agg[lead[i]];
    free(match); free(jt); free(lead);
    return nc;
}

static int cmp_int(const void *a, const void *b)
{
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/* A_c = P^T A P for the piecewise-constant P of `agg` (fine row -> aggregate). */
void om_galerkin(const om_csr *A, const int *agg, int nc, om_csr *Ac)
{
    int n = A->n;
    /* members of each aggregate in ascending fine order */
    int *mp = (int *)calloc(nc + 1, sizeof(int));
    int *mem = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    for (int i = 0; i < n; i++) mp[agg[i] + 1]++;
    for (int I = 0; I < nc; I++) mp[I + 1] += mp[I];
    int *fill = (int *)malloc(sizeof(int) * (nc > 0 ? nc : 1));
    memcpy(fill, mp, sizeof(int) * nc);
    for (int i = 0; i < n; i++) mem[fill[agg[i]]++] = i;
    /* sparse accumulator per coarse row */
    int *marker = (int *)malloc(sizeof(int) * (nc > 0 ? nc : 1));
    double *acc = (double *)malloc(sizeof(double) * (nc > 0 ? nc : 1));
    for (int J = 0; J < nc; J++) marker[J] = -1;
    int cap = A->nnz > 0 ? A->nnz : 1;
    Ac->rp = (int *)malloc(sizeof(int) * (nc + 1));
    Ac->col = (int *)malloc(sizeof(int) * cap);
    Ac->val = (double *)malloc(sizeof(double) * cap);
    Ac->n = nc;
    int nz = 0;
    Ac->rp[0] = 0;
    for (int I = 0; I < nc; I++) {
        int start = nz;
        for (int q = mp[I]; q < mp[I + 1]; q++) {
            int i = mem[q];
            for (int z = A->rp[i]; z < A->rp[i + 1]; z++) {
                int J = agg[A->col[z]];
                if (marker[J] != I) { marker[J] = I; acc[J] = 0.0; Ac->col[nz++] = J; }
                acc[J] += A->val[z];
            }
        }
        qsort(Ac->col + start, nz - start, sizeof(int), cmp_int);
        for (int z = start; z < nz; z++) Ac->val[z] = acc[Ac->col[z]];
        Ac->rp[I + 1] = nz;
    }
    Ac->nnz = nz;
    free(mp); free(mem); free(fill); free(marker); free(acc);
}

static void csr_copy(om_csr *d, const om_csr *s)
{
    d->n = s->n; d->nnz = s->nnz;
    d->rp = (int *)malloc(sizeof(int) * (s->n + 1));
    d->col = (int *)malloc(sizeof(int) * (s->nnz > 0 ? s->nnz : 1));
    d->val = (double *)malloc(sizeof(double) * (s->nnz > 0 ? s->nnz : 1));
    memcpy(d->rp, s->rp, sizeof(int) * (s->n + 1));
    memcpy(d->col, s->col, sizeof(int) * s->nnz);
    memcpy(d->val, s->val, sizeof(double) * s->nnz);
}

static double *vec(int n) { return (double *)malloc(sizeof(double) * (n > 0 ? n : 1)); }

int om_amg_setup(om_amg *H, const om_csr *A0, double theta, int max_coarse, int max_levels,
                 int rounds, int passes, int kcycle)
{
    memset(H, 0, sizeof(*H));
    if (max_levels > 24) max_levels = 24;
    csr_copy(&H->A[0], A0);
    int l = 0;
    if (passes < 1) passes = 1;
    while (H->A[l].n > max_coarse && l + 1 < max_levels) {
        int n = H->A[l].n;
        int *agg = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
        for (int i = 0; i < n; i++) agg[i] = i;
        om_csr cur;
        csr_copy(&cur, &H->A[l]);
        int nc = n;
        for (int p = 0; p < passes; p++) {     /* successive passes on Galerkin products */
            int *a = (int *)malloc(sizeof(int) * (cur.n > 0 ? cur.n : 1));
            int m = om_aggregate(&cur, theta, rounds, a);
            om_csr next;
            om_galerkin(&cur, a, m, &next);
            for (int i = 0; i < n; i++) agg[i] = a[agg[i]];
            om_csr_free(&cur);
            cur = next;
            nc = m;
            free(a);
        }
        if (nc >= n) { /* no coarsening progress */
            om_csr_free(&cur);
            free(agg);
            break;
        }
        H->A[l + 1] = cur;
        H->agg[l] = agg;
        l++;
    }
    H->nlev = l + 1;
    H->kcycle = kcycle;
    for (int k = 0; k < H->nlev; k++) {
        const om_csr *A = &H->A[k];
        H->l1[k] = vec(A->n);
        for (int i = 0; i < A->n; i++) {
            double s = 0.0;
            for (int z = A->rp[i]; z < A->rp[i + 1]; z++) s += fabs(A->val[z]);
            H->l1[k][i] = s;
        }
        H->wr[k] = vec(A->n);
        H->wx[k] = vec(A->n);
        H->wb[k] = vec(A->n);
        H->kw[k] = vec(5 * A->n);
    }
    const om_csr *C = &H->A[H->nlev - 1];
    int nc = C->n;
    H->ncoarse = nc;
    if (nc > 4096) return 1;     /* coarsening stalled: no dense solve of that size */
    H->lu = (double *)calloc((size_t)nc * nc > 0 ? (size_t)nc * nc : 1, sizeof(double));
    H->piv = (int *)malloc(sizeof(int) * (nc > 0 ? nc : 1));
    for (int i = 0; i < nc; i++)
        for (int z = C->rp[i]; z < C->rp[i + 1]; z++) H->lu[(size_t)i * nc + C->col[z]] += C->val[z];
    return om_dense_lu(nc, H->lu, H->piv) ? 2 : 0;
}

static void csr_mv(const om_csr *A, const double *x, double *y)
{
    for (int i = 0; i < A->n; i++) {
        double s = 0.0;
        for (int z = A->rp[i]; z < A->rp[i + 1]; z++) s += A->val[z] * x[A->col[z]];
        y[i] = s;
    }
}

static void csr_resid(const om_csr *A, const double *b, const double *x, double *r)
{
    for (int i = 0; i < A->n; i++) {
        double s = b[i];
        for (int z = A->rp[i]; z < A->rp[i + 1]; z++) s -= A->val[z] * x[A->col[z]];
        r[i] = s;
    }
}

static void cycle(const om_amg *H, int l, const double *b, double *x);

/* Coarse correction at level c by two steps of the generalised conjugate
 * residual method on A_c x = b, each preconditioned by one cycle at level c:
 *   p1 = C(b), q1 = A p1, a1 = (q1.b)/(q1.q1), r = b - a1 q1;
 *   p2 = C(r), q2 = A p2, beta = (q1.q2)/(q1.q1), p2 -= beta p1, q2 -= beta q1,
 *   a2 = (q2.r)/(q2.q2);  x = a1 p1 + a2 p2.
 * A zero denominator gives a zero step. */
static void kstep(const om_amg *H, int c, const double *b, double *x)
{
    const om_csr *A = &H->A[c];
    int n = A->n;
    double *p1 = H->kw[c], *p2 = p1 + n, *q1 = p2 + n, *q2 = q1 + n, *r = q2 + n;
    cycle(H, c, b, p1);
    csr_mv(A, p1, q1);
    double qq = om_dot(n, q1, q1);
    double a1 = qq > 0.0 ? om_dot(n, q1, b) / qq : 0.0;
    for (int i = 0; i < n; i++) r[i] = b[i] - a1 * q1[i];
    cycle(H, c, r, p2);
    csr_mv(A, p2, q2);
    double beta = qq > 0.0 ? om_dot(n, q1, q2) / qq : 0.0;
    for (int i = 0; i < n; i++) {
        p2[i] = p2[i] - beta * p1[i];
        q2[i] = q2[i] - beta * q1[i];
    }
    double q22 = om_dot(n, q2, q2);
    double a2 = q22 > 0.0 ? om_dot(n, q2, r) / q22 : 0.0;
    for (int i = 0; i < n; i++) x[i] = a1 * p1[i] + a2 * p2[i];
}

static void cycle(const om_amg *H, int l, const double *b, double *x)
{
    const om_csr *A = &H->A[l];
    int n = A->n;
    if (l == H->nlev - 1) {
        memcpy(x, b, sizeof(double) * n);
        om_dense_lu_solve(n, H->lu, H->piv, x);
        return;
    }
    const double *d = H->l1[l];
    double *r = H->wr[l];
    for (int i = 0; i < n; i++) x[i] = b[i] / d[i];              /* pre-smooth, zero guess */
    csr_resid(A, b, x, r);
    int nc = H->A[l + 1].n;
    double *bc = H->wb[l + 1], *xc = H->wx[l + 1];
    for (int I = 0; I < nc; I++) bc[I] = 0.0;
    for (int i = 0; i < n; i++) bc[H->agg[l][i]] += r[i];       /* restriction P^T r */
    if (l < H->kcycle && l + 1 < H->nlev - 1) kstep(H, l + 1, bc, xc);
    else cycle(H, l + 1, bc, xc);
    for (int i = 0; i < n; i++) x[i] += xc[H->agg[l][i]];       /* prolongation P xc */
    csr_resid(A, b, x, r);
    for (int i = 0; i < n; i++) x[i] += r[i] / d[i];             /* post-smooth */
}

void om_amg_vcycle(const om_amg *H, const double *b, double *x)
{
    cycle(H, 0, b, x);
}

/* ncyc cycles on A_0 x = b from x = 0, each on the residual of the last:
 * x = C(b); then x = x + C(b - A_0 x), ncyc - 1 times (an AMG-preconditioned
 * Richardson iteration on the pressure system; reading B6h). */
void om_amg_cycles(const om_amg *H, const double *b, double *x, int ncyc)
{
    cycle(H, 0, b, x);
    int n = H->A[0].n;
    if (ncyc < 2 || n < 1) return;
    double *r = (double *)malloc(sizeof(double) * n);
    double *c = (double *)malloc(sizeof(double) * n);
    for (int k = 1; k < ncyc; k++) {
        csr_resid(&H->A[0], b, x, r);
        cycle(H, 0, r, c);
        for (int i = 0; i < n; i++) x[i] = x[i] + c[i];
    }
    free(r);
    free(c);
}

void om_amg_free(om_amg *H)
{
    for (int k = 0; k < H->nlev; k++) {
        om_csr_free(&H->A[k]);
        free(H->l1[k]); free(H->agg[k]); free(H->wr[k]); free(H->wx[k]); free(H->wb[k]);
        free(H->kw[k]);
    }
    free(H->lu); free(H->piv);
    memset(H, 0, sizeof(*H));
}
