/*
 * Oracle: block-sparse utilities, decoupling and dense LU.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Decoupling follows the paper's "Matrix decoupling strategy" (Eq 29 and
 * the definitions of D_ABF and D_QI): for each reservoir (cell) block row i
 * with diagonal block [[a00, a01], [a10, a11]],
 *   Quasi-IMPES: D_i^-1 = [[1, -a01/a11], [0, 1]]   (saturation row kept),
 *   ABF:         D_i^-1 = inverse of the diagonal block,
 * applied to every block of the row and to the right-hand side.  Well rows
 * are left unchanged in both.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

void om_bsr_free(om_bsr *A)
{
    free(A->rp); free(A->col); free(A->val);
    A->rp = NULL; A->col = NULL; A->val = NULL; A->nb = A->nnzb = 0;
}

void om_csr_free(om_csr *A)
{
    free(A->rp); free(A->col); free(A->val);
    A->rp = NULL; A->col = NULL; A->val = NULL; A->n = A->nnz = 0;
}

void om_bsr_copy(om_bsr *d, const om_bsr *s)
{
    d->nb = s->nb; d->nnzb = s->nnzb;
    d->rp = (int *)malloc(sizeof(int) * (s->nb + 1));
    d->col = (int *)malloc(sizeof(int) * (s->nnzb > 0 ? s->nnzb : 1));
    d->val = (double *)malloc(sizeof(double) * 4 * (s->nnzb > 0 ? s->nnzb : 1));
    memcpy(d->rp, s->rp, sizeof(int) * (s->nb + 1));
    memcpy(d->col, s->col, sizeof(int) * s->nnzb);
    memcpy(d->val, s->val, sizeof(double) * 4 * s->nnzb);
}

int om_bsr_find(const om_bsr *A, int i, int j)
{
    for (int z = A->rp[i]; z < A->rp[i + 1]; z++)
        if (A->col[z] == j) return z;
    return -1;
}

/* y = A x */
void om_bsr_spmv(const om_bsr *A, const double *x, double *y)
{
    for (int i = 0; i < A->nb; i++) {
        double y0 = 0.0, y1 = 0.0;
        for (int z = A->rp[i]; z < A->rp[i + 1]; z++) {
            const double *a = &A->val[4 * z];
            int j = A->col[z];
            y0 += a[0] * x[2 * j] + a[1] * x[2 * j + 1];
            y1 += a[2] * x[2 * j] + a[3] * x[2 * j + 1];
        }
        y[2 * i] = y0;
        y[2 * i + 1] = y1;
    }
}

void om_block_inv(const double *a, double *inv)
{
    double det = a[0] * a[3] - a[1] * a[2];
    inv[0] = a[3] / det;
    inv[1] = -a[1] / det;
    inv[2] = -a[2] / det;
    inv[3] = a[0] / det;
}

/* The 2x2 row operator D_i^-1 of the chosen decoupling for cell row i. */
static void row_operator(const om_bsr *A, int i, int kind, double *M)
{
    const double *d = &A->val[4 * om_bsr_find(A, i, i)];
    if (kind == OM_DEC_QI) {
        M[0] = 1.0; M[1] = -d[1] / d[3]; M[2] = 0.0; M[3] = 1.0;
    } else if (kind == OM_DEC_ABF) {
        om_block_inv(d, M);
    } else {
        M[0] = 1.0; M[1] = 0.0; M[2] = 0.0; M[3] = 1.0;
    }
}

static void apply2(const double *M, double *v)
{
    double a = v[0], b = v[1];
    v[0] = M[0] * a + M[1] * b;
    v[1] = M[2] * a + M[3] * b;
}

static void apply_block(const double *M, double *B)
{
    double b0 = B[0], b1 = B[1], b2 = B[2], b3 = B[3];
    B[0] = M[0] * b0 + M[1] * b2;
    B[1] = M[0] * b1 + M[1] * b3;
    B[2] = M[2] * b0 + M[3] * b2;
    B[3] = M[2] * b1 + M[3] * b3;
}

/* A <- D^-1 A and b <- D^-1 b (b may be NULL), reservoir rows only (Eq 29). */
void om_decouple(om_bsr *A, double *b, int ncell, int kind)
{
    if (kind == OM_DEC_NONE) return;
    for (int i = 0; i < ncell; i++) {
        double M[4];
        row_operator(A, i, kind, M);
        for (int z = A->rp[i]; z < A->rp[i + 1]; z++) apply_block(M, &A->val[4 * z]);
        if (b) apply2(M, &b[2 * i]);
    }
}

/* b <- D^-1 b using the operator built from the undecoupled matrix. */
void om_decouple_rhs(const om_bsr *Aorig, double *b, int ncell, int kind)
{
    if (kind == OM_DEC_NONE) return;
    for (int i = 0; i < ncell; i++) {
        double M[4];
        row_operator(Aorig, i, kind, M);
        apply2(M, &b[2 * i]);
    }
}

void om_bsr_to_dense(const om_bsr *A, double *D)
{
    int N = 2 * A->nb;
    memset(D, 0, sizeof(double) * (size_t)N * N);
    for (int i = 0; i < A->nb; i++)
        for (int z = A->rp[i]; z < A->rp[i + 1]; z++) {
            int j = A->col[z];
            const double *a = &A->val[4 * z];
            D[(size_t)(2 * i) * N + 2 * j] = a[0];
            D[(size_t)(2 * i) * N + 2 * j + 1] = a[1];
            D[(size_t)(2 * i + 1) * N + 2 * j] = a[2];
            D[(size_t)(2 * i + 1) * N + 2 * j + 1] = a[3];
        }
}

/* Textbook LU with partial pivoting, in place, row-major; returns 0 or the
 * 1-based column of a zero pivot. */
int om_dense_lu(int n, double *a, int *piv)
{
    for (int k = 0; k < n; k++) {
        int p = k;
        double best = fabs(a[(size_t)k * n + k]);
        for (int i = k + 1; i < n; i++) {
            double v = fabs(a[(size_t)i * n + k]);
            if (v > best) { best = v; p = i; }
        }
        piv[k] = p;
        if (best == 0.0) return k + 1;
        if (p != k)
            for (int j = 0; j < n; j++) {
                double t = a[(size_t)k * n + j];
                a[(size_t)k * n + j] = a[(size_t)p * n + j];
                a[(size_t)p * n + j] = t;
            }
        double inv = 1.0 / a[(size_t)k * n + k];
        for (int i = k + 1; i < n; i++) {
            double l = a[(size_t)i * n + k] * inv;
            a[(size_t)i * n + k] = l;
            if (l != 0.0)
                for (int j = k + 1; j < n; j++) a[(size_t)i * n + j] -= l * a[(size_t)k * n + j];
        }
    }
    return 0;
}

void om_dense_lu_solve(int n, const double *lu, const int *piv, double *b)
{
    for (int k = 0; k < n; k++)
        if (piv[k] != k) { double t = b[k]; b[k] = b[piv[k]]; b[piv[k]] = t; }
    for (int i = 0; i < n; i++) {
        double s = b[i];
        for (int j = 0; j < i; j++) s -= lu[(size_t)i * n + j] * b[j];
        b[i] = s;
    }
    for (int i = n - 1; i >= 0; i--) {
        double s = b[i];
        for (int j = i + 1; j < n; j++) s -= lu[(size_t)i * n + j] * b[j];
        b[i] = s / lu[(size_t)i * n + i];
    }
}

double om_dot(int n, const double *a, const double *b)
{
    double s = 0.0;
    for (int i = 0; i < n; i++) s += a[i] * b[i];
    return s;
}
