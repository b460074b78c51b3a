/*
 * FP64 CPU oracle for the fully implicit two-phase (oil-water) simulator of
 * Liu, Shen, Chen, Wang, Yang and Chen, "A Parallel Simulator for Massive
 * Reservoir Models Utilizing Distributed-Memory Parallel Systems"
 * (arXiv 1701.06254).
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the slow, plain reference that the
 * device library is checked against.  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or helper with the device library.
 *
 * Conventions
 *   - Field units: ft, psi, mD, cP, bbl, STB/day, days.
 *   - Cells in natural order c = i + nx*(j + ny*k), k counted downward.
 *   - Unknowns interleaved per cell, x[2c] = p (oil pressure), x[2c+1] = s_w;
 *     then per well x[2(n+w)] = p_b and x[2(n+w)+1] = a dummy unknown that
 *     always solves to 0.  The paper's field-split vector (p; s_w; p_b) of
 *     Eq 20 is the fixed permutation p_c <-> 2c, s_c <-> 2c+1, p_b,w <-> 2(n+w).
 *   - Jacobian in block CSR (BSR) with 2x2 blocks, row-major within a block:
 *     block row = (oil equation, water equation), block column = (d/dp, d/ds_w);
 *     well rows carry (well equation, dummy identity row).  Columns are sorted
 *     ascending within each block row.
 */
#ifndef R2P_ORACLE_H
#define R2P_ORACLE_H

#include <stddef.h>

/* ---------------------------------------------------------------- model */
typedef struct {
    int nx, ny, nz, n;        /* grid and cell count */
    double dx, dy, dz, top;   /* cell sizes, depth of the top-layer centre */
    double *kx, *ky, *kz, *phi, *depth, *vol;
    double *tx, *ty, *tz;     /* geometric transmissibility to the +d neighbour */
    /* constants: Darcy factor, ft^3/bbl, reference densities, reference
       pressure and its depth, compressibilities, viscosities, gravity switch */
    double beta_c, alpha_c, rho_o, rho_w, p_ref, z_ref, c_o, c_w, c_r, mu_o, mu_w, grav;
    int nw, nperf;
    int *w_ptr, *w_cell, *w_kind, *w_ctrl; /* kind: 0 inj 1 prod; ctrl: 0 BHP 1 WRATE 2 ORATE 3 LRATE */
    double *w_target, *w_rw, *w_skin;
    double *wi;               /* per perforation well index */
    int *perf_well;           /* per perforation owning well */
    double *w_zb;             /* per well reference depth (top perforation centre) */
} om_model;

/* ---------------------------------------------------------------- BSR */
typedef struct {
    int nb;       /* block rows (= block columns) */
    int nnzb;
    int *rp;      /* nb+1 */
    int *col;     /* nnzb */
    double *val;  /* 4*nnzb */
} om_bsr;

/* scalar CSR (AMG levels) */
typedef struct {
    int n, nnz;
    int *rp, *col;
    double *val;
} om_csr;

/* ---------------------------------------------------------------- RAS */
typedef struct {
    int m;            /* local block rows (cells of the overlapped set + owned wells) */
    int *glob;        /* local -> global block row */
    unsigned char *owned;
    om_bsr lu;        /* in-place block ILU(0) factors in local order: strict lower = L (unit diag), upper = U */
    double *dinv;     /* 4*m: inverse of U's diagonal blocks */
    int *diag;        /* m: position of the diagonal block */
} om_sub;

typedef struct {
    int ns;
    om_sub *sub;
    int *owner;       /* global block row -> owning subdomain */
    double *work;     /* scratch */
} om_ras;

/* ---------------------------------------------------------------- AMG */
typedef struct {
    int nlev;
    om_csr A[24];
    double *l1[24];   /* l1 row sums of each level */
    int *agg[24];     /* level l row -> level l+1 row (composite of both passes) */
    int ncoarse;      /* rows of the coarsest level */
    double *lu;       /* coarsest dense LU (row-major), with partial pivoting */
    int *piv;
    double *wr[24], *wx[24], *wb[24];
    double *kw[24];   /* K-cycle work vectors of a level: p1, p2, q1, q2, r */
    int kcycle;       /* coarse corrections of levels < kcycle are K-cycles */
} om_amg;

/* ---------------------------------------------------------------- options */
enum { OM_DEC_NONE = 0, OM_DEC_QI = 1, OM_DEC_ABF = 2 };
enum { OM_ORD_NATURAL = 0, OM_ORD_POTENTIAL = 1 };
enum { OM_CPR_TWO_STAGE = 0, OM_CPR_FPF = 1 };

typedef struct {
    int decouple, order, form;
    int px, py, overlap;
    double theta;         /* AMG strength threshold */
    int max_coarse, max_levels, match_rounds, agg_passes;
    int kcycle;           /* AMG levels whose coarse correction is a K-cycle */
    int amg_cycles;       /* AMG cycles per pressure stage, each on the last residual */
    int exact_stages;     /* 1: RAS and V-cycle replaced by dense solves (pin of Alg 2) */
} om_cpr_opts;

typedef struct {
    om_cpr_opts o;
    const om_bsr *A;      /* decoupled matrix (borrowed) */
    int ncell;
    om_ras ras;
    om_amg amg;
    double *dense_A, *dense_App; int *piv_A, *piv_App;  /* exact-stage mode */
    double *t1, *t2, *t3; /* scratch vectors */
} om_cpr;

#ifdef __cplusplus
extern "C" {
#endif

/* physics.c */
int  om_model_create(om_model **out, int nx, int ny, int nz, double dx, double dy, double dz,
                     double top, const double *kx, const double *ky, const double *kz,
                     const double *phi, const double *consts /* 12 */, int nw, const int *w_ptr,
                     const int *w_cell, const int *w_kind, const int *w_ctrl,
                     const double *w_target, const double *w_rw, const double *w_skin);
void om_model_destroy(om_model *m);
void om_well_index(const om_model *m, double *wi_out, double *zb_out);
void om_initial_state(const om_model *m, double *x);
void om_residual(const om_model *m, const double *x, const double *xold, double dt, double *F);
int  om_jacobian(const om_model *m, const double *x, const double *xold, double dt,
                 om_bsr *J, double *F);
void om_pattern(const om_model *m, om_bsr *J);
double om_scaled_norm(const om_model *m, const double *F, double dt);
void om_accumulation(const om_model *m, const double *x, double *acc_o, double *acc_w);
void om_well_rates(const om_model *m, const double *x, double *q_o, double *q_w);
void om_potential(const om_model *m, const double *x, double *phi_o);

/* sparse.c */
void om_bsr_free(om_bsr *A);
void om_bsr_copy(om_bsr *dst, const om_bsr *src);
int  om_bsr_find(const om_bsr *A, int i, int j);
void om_bsr_spmv(const om_bsr *A, const double *x, double *y);
void om_decouple(om_bsr *A, double *b, int ncell, int kind);
void om_decouple_rhs(const om_bsr *Aorig, double *b, int ncell, int kind);
void om_bsr_to_dense(const om_bsr *A, double *D);
int  om_dense_lu(int n, double *a, int *piv);
void om_dense_lu_solve(int n, const double *lu, const int *piv, double *b);
void om_block_inv(const double *a, double *inv);
double om_dot(int n, const double *a, const double *b);
void om_csr_free(om_csr *A);

/* ras.c */
int  om_potential_order(int m, const double *phi_o, const int *cells, int *perm);
int  om_ras_setup(om_ras *R, const om_bsr *A, const om_model *mdl, const double *x,
                  int px, int py, int overlap, int order);
void om_ras_apply(const om_ras *R, const double *r, double *y);
void om_ras_free(om_ras *R);
int  om_bilu0(om_bsr *A, double *dinv, int *diag);
void om_bilu0_solve(const om_bsr *LU, const double *dinv, const int *diag, double *v);

/* amg.c */
/* Returns 0, 1 when coarsening stalled above the dense coarsest size (soft
 * failure), or 2 when the coarsest matrix is singular. */
int  om_amg_setup(om_amg *H, const om_csr *A0, double theta, int max_coarse, int max_levels,
                  int rounds, int passes, int kcycle);
void om_amg_vcycle(const om_amg *H, const double *b, double *x);
void om_amg_cycles(const om_amg *H, const double *b, double *x, int ncyc);
void om_amg_free(om_amg *H);
void om_extract_pressure(const om_bsr *A, int ncell, om_csr *App);
void om_strength_match(const om_csr *A, double theta, int rounds, int *match);
void om_galerkin(const om_csr *A, const int *agg, int nc, om_csr *Ac);
void om_join_targets(const om_csr *A, double theta, const int *match, int *jt);
void om_coupling_weights(const om_csr *A, double *w, double *M);
int  om_aggregate(const om_csr *A, double theta, int rounds, int *agg);

/* solver.c */
int  om_cpr_setup(om_cpr *P, const om_bsr *Adec, const om_model *mdl, const double *x,
                  const om_cpr_opts *o);
void om_cpr_apply(const om_cpr *P, const double *f, double *x);
void om_cpr_free(om_cpr *P);
int  om_fgmres(const om_bsr *A, const om_cpr *P, const double *b, double *x, int restart,
               double rtol, int maxit, int *iters, double *relres, double *hist);
int  om_bicgstab(const om_bsr *A, const om_cpr *P, const double *b, double *x, double rtol,
                 int maxit, int *iters, double *relres);
/* krylov: 0 FGMRES(restart), 1 BiCGSTAB */
int  om_newton_step(const om_model *m, double *x, double dt, const om_cpr_opts *o, int restart,
                    double rtol, int maxit, double ntol, int max_newton, int exact_linear,
                    int forcing, double ds_max, int krylov, int *newton_its, int *lin_its,
                    double *res_hist, double *fn_hist, double *rn_hist, double *eta_hist);

#ifdef __cplusplus
}
#endif
#endif
