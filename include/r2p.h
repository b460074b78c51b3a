/*
 * r2p: MI355X (gfx950) library for the Newton-step linear solve of a fully
 * implicit two-phase (oil-water) finite-difference reservoir model.
 *
 * Method: Liu, Shen, Chen, Wang, Yang, Chen, "A Parallel Simulator for Massive
 * Reservoir Models Utilizing Distributed-Memory Parallel Systems",
 * arXiv 1701.06254.  Citations below name the paper's sections and
 * equations.
 *
 * Conventions (all entry points)
 *   - Return value: 0 = success, > 0 = soft failure (see each entry point),
 *     < 0 = error (R2P_E*).  r2p_last_error() gives a message for the last
 *     non-zero status on the calling thread.  No C++ exception crosses this
 *     interface.
 *   - Pointers whose name ends in _host point to host memory; every other
 *     array pointer is device memory on the model's device, owned by the
 *     caller unless stated otherwise.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on it; calls that must read scalars back synchronise
 *     that stream and say so.
 *   - Field units: ft, psi, mD, cP, bbl, STB/day, days.
 *   - Cells are in natural order c = i + nx*(j + ny*k), k counted downward
 *     from the top layer.  A state vector has N = 2*(n + nw) doubles,
 *     interleaved per cell: x[2c] = oil pressure p, x[2c+1] = water
 *     saturation s_w; then per well x[2(n+w)] = bottom-hole pressure p_b and
 *     x[2(n+w)+1] = a dummy unknown that is always 0.  This is the paper's
 *     unknown vector (p; s_w; p_b) of Eq 19-23 under a fixed permutation
 *     (p_c -> 2c, s_c -> 2c+1, p_b,w -> 2(n+w)).
 *   - Handles are not thread safe; one handle is used by one thread at a time.
 */
#ifndef R2P_H
#define R2P_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    R2P_OK = 0,
    R2P_NOT_CONVERGED = 1,   /* iterative method stopped at its iteration limit */
    R2P_BREAKDOWN = 2,       /* Krylov breakdown before convergence */
    R2P_EINVAL = -1,         /* invalid argument */
    R2P_ENOMEM = -2,         /* device allocation failed */
    R2P_EHIP = -3,           /* HIP runtime error */
    R2P_ENAN = -4,           /* non-finite value met */
    R2P_ESTATE = -5,         /* call out of order (e.g. solve before setup) */
    R2P_ESINGULAR = -6       /* singular pivot block in a factorisation */
};

/* Well kinds and controls: the constraints of Eq 11-14. */
enum { R2P_INJECTOR = 0, R2P_PRODUCER = 1 };
enum { R2P_BHP = 0, R2P_WRATE = 1, R2P_ORATE = 2, R2P_LRATE = 3 };

typedef struct r2p_model r2p_model;
typedef struct r2p_jacobian r2p_jacobian;
typedef struct r2p_cpr r2p_cpr;

/* Model description ("Two-phase oil-water flow model", Eq 1-14).
 * Every array is host memory and is copied on create.
 *   kx/ky/kz_host[n]  permeability (mD, > 0); phi_host[n] porosity in (0,1).
 *   consts[12] = {beta_c (Darcy factor, 0.001127), alpha_c (ft^3/bbl),
 *                 rho_o, rho_w (reference densities, lbm/ft^3),
 *                 p_ref (reference pressure, psi), z_ref (its depth, ft),
 *                 c_o, c_w, c_r (compressibilities, 1/psi),
 *                 mu_o, mu_w (viscosities, cP), grav (1 on, 0 off)}.
 *   Wells: w_ptr_host[nw+1] offsets into w_cell_host (perforated cells, the
 *   first is the reference depth z_b); kind, control and target (STB/day for
 *   rates, psi for BHP; rate targets are magnitudes, injection positive);
 *   radius (ft) and skin.  A cell may be perforated by at most one well. */
typedef struct {
    int nx, ny, nz;
    double dx, dy, dz;    /* cell sizes, ft */
    double top;           /* depth of the top-layer cell centres, ft */
    const double *kx_host, *ky_host, *kz_host, *phi_host;
    double consts[12];
    int nw;
    const int *w_ptr_host, *w_cell_host, *w_kind_host, *w_ctrl_host;
    const double *w_target_host, *w_rw_host, *w_skin_host;
    int device;           /* HIP device ordinal */
} r2p_model_desc;

/* Options of the CPR preconditioner ("Matrix decoupling strategy",
 * "Local potential reordering technique", "Multi-stage preconditioner"). */
enum { R2P_DEC_NONE = 0, R2P_DEC_QI = 1, R2P_DEC_ABF = 2 };
enum { R2P_ORDER_NATURAL = 0, R2P_ORDER_POTENTIAL = 1 };
enum { R2P_CPR_TWO_STAGE = 0, R2P_CPR_FPF = 1 };
enum { R2P_FP64 = 0, R2P_FP32 = 1 };
typedef struct {
    int decouple;      /* R2P_DEC_*: D^-1 of Eq 29 (Quasi-IMPES or ABF) */
    int order;         /* R2P_ORDER_*: local order of each RAS subdomain (Eq 30-32) */
    int form;          /* R2P_CPR_*: two-stage, or Algorithm 2 (FPF) */
    int px, py;        /* RAS subdomains: px x py tiles of the x-y plane, full z columns (px*py <= 256,
                          px <= nx, py <= ny; a row may lie in at most 16 overlapped tiles) */
    int overlap;       /* RAS overlap in block-graph layers (>= 0) */
    double theta;      /* AMG strength threshold (0.25) */
    int max_coarse;    /* AMG: stop coarsening at this many rows (<= 2048) */
    int max_levels;    /* AMG: at most this many levels (<= 24) */
    int match_rounds;  /* AMG: handshake rounds per pairwise matching (4) */
    int agg_passes;    /* AMG: aggregation passes per level (1 or 2; 2 gives aggregates of ~4) */
    int precision;     /* R2P_FP64, or R2P_FP32: AMG and ILU stored and applied in FP32 */
    int kcycle;        /* AMG: the coarse correction of the kcycle finest levels is two
                          generalised-conjugate-residual steps, each preconditioned by a
                          cycle one level down (K-cycle); 0 gives the V-cycle.  A K-cycle
                          makes the preconditioner vary with its input: use it with the
                          flexible GMRES, not with BiCGSTAB (1) */
    int amg_cycles;    /* AMG: cycles per pressure stage (1..8), each on the residual of the
                          last: x_p = C(r_p), then x_p = x_p + C(r_p - A_pp x_p) (2) */
} r2p_cpr_opts;

enum { R2P_KRYLOV_FGMRES = 0, R2P_KRYLOV_BICGSTAB = 1 };
typedef struct {
    int restart;       /* FGMRES restart length m (1..64) */
    int maxit;         /* iteration limit */
    double rtol;       /* relative residual target on the decoupled system */
    int method;        /* R2P_KRYLOV_FGMRES, or R2P_KRYLOV_BICGSTAB (right-preconditioned,
                          zero start; one iteration = two CPR applications) */
} r2p_solve_opts;

typedef struct {
    int iterations;
    int status;        /* return code of the solve */
    double relres;     /* true ||D^-1(b - A y)|| / ||D^-1 b|| at exit */
    double ms_total;   /* host wall time of the call */
    int reorth;        /* second Gram-Schmidt passes (delayed by one iteration for restarts
                          up to 32, else selective) */
} r2p_solve_info;

enum { R2P_FORCING_FIXED = 0, R2P_FORCING_EW = 1 };
typedef struct {
    int max_newton;    /* Newton iteration limit (20) */
    double tol;        /* scaled residual tolerance (1e-8) */
    int forcing;       /* R2P_FORCING_FIXED: each solve to lin.rtol; R2P_FORCING_EW: Eq 26, second choice */
    double ds_max;     /* largest saturation change per Newton iteration (0.2; <= 0 disables) */
    r2p_cpr_opts cpr;
    r2p_solve_opts lin;
    int guess_rule;    /* when x_guess is taken: R2P_GUESS_SCALED_INF (its scaled residual
                          max-norm is below that of x^n), R2P_GUESS_L2 (its residual
                          2-norm is), R2P_GUESS_TRY (always; if Newton does not converge
                          from it, the step starts again from x^n) */
} r2p_newton_opts;
enum { R2P_GUESS_SCALED_INF = 0, R2P_GUESS_L2 = 1, R2P_GUESS_TRY = 2 };

#define R2P_HIST 32
/* Host wall times (ms) summed over the step's Newton iterations, stage by
 * stage as the paper's timing table splits the linear solve (Table 5):
 *   ms_assemble   residual, Jacobian and the scaled-norm test;
 *   ms_setup      the whole CPR set-up (r2p_setup_cpr), made of
 *     ms_decouple   decoupling D^-1 A (QI or ABF, Eq 29),
 *     ms_order      local potential reordering (dependency levels, local
 *                   order, Eq 30-33),
 *     ms_ras_setup  block ILU(0) of every subdomain,
 *     ms_amg_setup  the AMG hierarchy; it runs on its own host thread and
 *                   stream beside ms_order + ms_ras_setup, so ms_setup is
 *                   about ms_decouple + max(ms_order + ms_ras_setup,
 *                   ms_amg_setup);
 *   ms_solve      the Krylov solves (r2p_solve);
 *   ms_update     the Newton update (and the linear residual norm of EW);
 *   ms_total      the whole call: ms_assemble + ms_setup + ms_solve +
 *                 ms_update plus the warm-start test and copies. */
typedef struct {
    int status;              /* 0 converged, 1 not converged (x unchanged) */
    int newton_its;
    int linear_its;
    int used_guess;          /* 1 if x_guess was taken as the first iterate */
    double res_hist[R2P_HIST];   /* scaled residual norm per Newton iteration */
    double ms_assemble, ms_setup, ms_solve, ms_total;
    double ms_decouple, ms_order, ms_ras_setup, ms_amg_setup, ms_update;
    int setup_status;        /* status of the last CPR set-up: 0, or the failure of the
                                method that ended the step (R2P_NOT_CONVERGED for a stalled
                                AMG coarsening, R2P_ESINGULAR for a singular pivot) */
} r2p_newton_info;

/* ----------------------------------------------------------------- model */

/* Copy the model to the device and derive geometry (harmonic two-point
 * transmissibilities), Peaceman well indices and well reference depths.
 * Errors: R2P_EINVAL (bad sizes, k <= 0, phi outside (0,1), perforation out
 * of range or a cell perforated twice), R2P_ENOMEM, R2P_EHIP. */
int r2p_model_create(const r2p_model_desc *desc, r2p_model **out);
int r2p_model_destroy(r2p_model *m);
/* n cells, nw wells, nperf perforations; N = 2*(n+nw). */
int r2p_model_sizes(const r2p_model *m, int *n_host, int *nw_host, int *nperf_host);

/* x[N] <- oil-hydrostatic state through (p_ref, z_ref) with s_w = 0; BHP
 * wells at their target, rate wells at their top perforation's pressure. */
int r2p_initial_state(r2p_model *m, double *x, void *stream);

/* --------------------------------------------------------------- Jacobian */

/* Library-owned Jacobian storage for one model (reused across calls). */
int r2p_jacobian_create(r2p_model *m, r2p_jacobian **out);
int r2p_jacobian_destroy(r2p_jacobian *J);

/* Residual and Jacobian of the discrete system F(x) = 0 (Eq 15-23): J <-
 * dF/dx at x, b[N] <- -F(x), for the backward-Euler step x_old -> x of
 * length dt days.  Also records the oil potential of every cell (Eq 5) for
 * the reordering.  Asynchronous on `stream`.  x, x_old, b: device, length N.
 * Errors: R2P_EINVAL (dt <= 0, NULL). */
int r2p_assemble_jacobian(r2p_model *m, const double *x, const double *x_old, double dt,
                          r2p_jacobian *J, double *b, void *stream);

/* Scaled infinity norm of -b (the Newton stopping test): max over cells of
 * |F_a| dt / PV (PV = V phi / alpha_c) and over wells of |F_w|/|target|.
 * Synchronises `stream`.  NaN in b gives R2P_ENAN. */
int r2p_residual_norm(r2p_model *m, const double *b, double dt, double *norm_host, void *stream);

/* The same scaled norm for callers that cannot allocate device or pinned
 * memory (code under HIP graph capture, tight serving loops): asynchronous
 * on `stream`, it writes the norm (NaN if a residual entry is not finite)
 * into norm_dev, a device double owned by the caller, and allocates nothing.
 * Its per-workgroup partial maxima live in a library scratch array of
 * 4 MiB per GPU, held until the process ends: n + nw may be at most 2^26
 * (R2P_EINVAL beyond).  Calls that overlap on one GPU (other streams or
 * threads) share that array and race; the result equals r2p_residual_norm
 * bit for bit. */
int r2p_residual_norm_noalloc(r2p_model *m, const double *b, double dt, double *norm_dev,
                              void *stream);

/* y[N] <- J x[N] with J as currently stored (decoupled once set up). */
int r2p_spmv(r2p_jacobian *J, const double *x, double *y, void *stream);

/* Copy J to host block-CSR (2x2 blocks, row-major, columns ascending, cell
 * rows then well rows).  With rp_host == NULL only *nnzb_host is set.
 * Synchronises `stream`. */
int r2p_jacobian_export(r2p_jacobian *J, int *nnzb_host, int *rp_host, int *col_host,
                        double *val_host, void *stream);

/* -------------------------------------------------------------------- CPR */

int r2p_cpr_create(r2p_cpr **out);
int r2p_cpr_destroy(r2p_cpr *P);

/* Build the CPR preconditioner for an assembled J: decouple J in place
 * (Eq 29; the row operators are kept to transform right-hand sides), then
 * set up block ILU(0) on every overlapped subdomain in its local order (RAS
 * stage) and the aggregation AMG hierarchy of the pressure block A_pp
 * (restriction Pi_r of Eq 34).  Synchronises `stream` (level counts and
 * coarse sizes are read back).  J must have been assembled since its last
 * setup.  Returns 0; R2P_NOT_CONVERGED (a soft failure of the method) when
 * the AMG coarsening stalls with a coarsest level above the dense limit of
 * 4096 rows; or an error: R2P_ESTATE, R2P_EINVAL, R2P_ESINGULAR (singular
 * pivot block), R2P_ENOMEM.  The handle is not usable for solves after a
 * non-zero return until it is set up again. */
int r2p_setup_cpr(r2p_jacobian *J, const r2p_cpr_opts *opts, r2p_cpr *P, void *stream);

/* z[N] <- M^-1 f[N] for the decoupled system (two-stage form or Algorithm 2). */
int r2p_cpr_apply(r2p_cpr *P, const double *f, double *z, void *stream);

/* Stage solvers on their own, for inspection:
 *   x_p[n] <- one AMG V-cycle on A_pp for right-hand side f_p[n];
 *   y[N]   <- RAS with block ILU(0) subdomain solves (restricted scatter). */
int r2p_amg_vcycle(r2p_cpr *P, const double *f_p, double *x_p, void *stream);
int r2p_ras_apply(r2p_cpr *P, const double *r, double *y, void *stream);

/* Inspection of the AMG hierarchy (host copies; synchronises `stream`).
 * r2p_amg_info: number of levels and rows/nonzeros of level l.
 * r2p_amg_export_level: CSR of level l (columns ascending), its l1 row sums,
 * and agg[i] = row of level l+1 holding row i (NULL allowed; unset on the
 * last level). */
int r2p_amg_info(r2p_cpr *P, int level, int *nlev_host, int *n_host, int *nnz_host);
int r2p_amg_export_level(r2p_cpr *P, int level, int *rp_host, int *col_host, double *val_host,
                         double *l1_host, int *agg_host, void *stream);

/* Inspection of the RAS factors (host copies; synchronises `stream`).
 * r2p_ras_info: subdomain count, and for subdomain s its local rows,
 * factor blocks (off-diagonal L and U blocks) and level count.
 * r2p_ras_export: for subdomain s, glob[m] = global block row of each local
 * row (level order), level[m], owned[m], dinv[m][4] = inverse of U's
 * diagonal block; and for each off-diagonal factor block e:
 * erow[e], ecol[e] global block row/column and eval[e][4] (L for columns
 * before the row in the local order, else U). */
int r2p_ras_info(r2p_cpr *P, int s, int *nsub_host, int *m_host, int *nblk_host,
                 int *nlevels_host);
int r2p_ras_export(r2p_cpr *P, int s, int *glob_host, int *level_host, unsigned char *owned_host,
                   double *dinv_host, int *erow_host, int *ecol_host, double *eval_host,
                   void *stream);

/* ------------------------------------------------------------------ solve */

/* Solve A y = b for the Jacobian J (original, not decoupled, right-hand
 * side; D^-1 is applied inside: D^-1 A y = D^-1 b, Eq 29) by right
 * preconditioned flexible GMRES(restart) from y = 0 with the CPR
 * preconditioner P.  Classical Gram-Schmidt run twice, the second pass
 * delayed by one iteration (restart <= 32; selective second pass above);
 * convergence on the true residual of the decoupled system.
 * o->method = R2P_KRYLOV_BICGSTAB instead runs right-preconditioned
 * BiCGSTAB (the second Krylov solver of the numerical experiments, two CPR
 * applications per iteration) from y = 0 with shadow residual D^-1 b;
 * on convergence of the recursive residual the true one is checked and the
 * method restarts from it if it is above the target.
 * Synchronous.  Returns 0, R2P_NOT_CONVERGED (y holds the last iterate) or
 * R2P_BREAKDOWN, or an error. */
int r2p_solve(r2p_jacobian *J, r2p_cpr *P, const double *b, double *y,
              const r2p_solve_opts *opts, r2p_solve_info *info, void *stream);

/* One implicit time step x^n -> x^{n+1} by Newton's method ("Nonlinear
 * methods", Algorithm 1): assemble, test the scaled residual, set up CPR,
 * solve, update x += y (saturation change limited to ds_max, then clipped
 * to [0,1]).  Standard Newton solves every system to lin.rtol; with
 * R2P_FORCING_EW the tolerance follows the second forcing term of Eq 26,
 * clipped to [0.01, 0.1].  x_guess (device, may be NULL): a first iterate
 * to try, taken according to opts->guess_rule (by default only if its
 * scaled residual max-norm is below that of x^n); info->newton_its and
 * linear_its count every attempt, res_hist the last one.
 * x: device, in x^n, out x^{n+1}.  Synchronous.  Returns 0, or
 * R2P_NOT_CONVERGED with x unchanged (the caller shortens dt). */
int r2p_newton_step(r2p_model *m, double *x, double dt, const double *x_guess,
                    const r2p_newton_opts *opts, r2p_newton_info *info, void *stream);

/* Default options: QI, potential order, two-stage, 4x4 subdomains, overlap
 * 1, theta 0.25, coarse 500, 20 levels, 4 rounds, 2 passes, FP64; FGMRES(30) to 1e-8
 * with 300 iterations; Newton 20 iterations to 1e-8, ds_max 0.2. */
void r2p_default_newton_opts(r2p_newton_opts *o);

/* -------------------------------------------------- learned warm start
 * A 3D convolutional network that predicts the increment (dp / 100 psi,
 * ds_w / 0.1) of a time step from the state at its start; its prediction is the
 * first Newton iterate x_guess of r2p_newton_step, taken only when it lowers
 * the residual (the paper's Algorithm 1 with a different starting point).
 * Layers: conv 6 -> 32 + ReLU, `blocks` residual blocks
 * h <- h + conv(relu(conv(h))), conv 32 -> 2; 3x3x3 taps, zero padding.
 * Tensors are channels-last [crop][z][y][x][32] bfloat16 (uint16_t bit
 * patterns, round to nearest even) unless stated; feature and output
 * channels beyond 6 / 2 are zero.  Products accumulate in FP32; the master
 * weights are FP32, trained by Adam (beta 0.9 / 0.999, eps 1e-8) on the
 * mean squared error.  The compact parameter vector holds, per layer in the
 * order in, a_0, b_0, ..., a_{K-1}, b_{K-1}, out, W[27][cout][cin] then
 * b[cout]; tap t = 9 (dz+1) + 3 (dy+1) + (dx+1).  Every entry point is
 * asynchronous on `stream` unless stated. */
typedef struct r2p_cnn r2p_cnn;
int r2p_cnn_param_count(int blocks, long *n_host);
/* Weights start at zero: set them with r2p_cnn_set_params.  Synchronous. */
int r2p_cnn_create(int blocks, r2p_cnn **out);
int r2p_cnn_destroy(r2p_cnn *cnn);
/* Host FP32 compact vectors (r2p_cnn_param_count entries).  Synchronous;
 * setting parameters also resets the Adam state. */
int r2p_cnn_set_params(r2p_cnn *cnn, const float *theta_host);
int r2p_cnn_get_params(r2p_cnn *cnn, float *theta_host);
int r2p_cnn_get_grads(r2p_cnn *cnn, float *grad_host);
/* feat: device bf16 [nb][nz][ny][nx][32]; out: device FP32 [nb*nz*ny*nx][2]. */
int r2p_cnn_forward(r2p_cnn *cnn, const uint16_t *feat, int nb, int nz, int ny, int nx,
                    float *out, void *stream);
/* Forward, mean squared error against target (device FP32 [V][2]) and the
 * gradient of every parameter (kept in the handle); loss_host (may be NULL)
 * receives the loss, which makes the call synchronous. */
int r2p_cnn_backward(r2p_cnn *cnn, const uint16_t *feat, const float *target, int nb, int nz,
                     int ny, int nx, double *loss_host, void *stream);
/* One Adam step with learning rate lr on the gradients of the last backward. */
int r2p_cnn_sgd_step(r2p_cnn *cnn, float lr, void *stream);
/* One 32 -> 32 layer on caller tensors (device): out = epilogue(bias +
 * sum_t sum_i x[v + s off_t][i] w[t][o][i]) with s = -1 when flip (the
 * input-gradient form, w then holding the per-tap transposed weights);
 * epilogue: + addend, kept where mask > 0, ReLU when relu.  bias, addend,
 * mask may be NULL; out (bf16) and/or outf (FP32 [V][32]).  x, w, out 16-byte
 * aligned. */
int r2p_cnn_conv(const uint16_t *x, int nb, int nz, int ny, int nx, const uint16_t *w,
                 const float *bias, const uint16_t *addend, const uint16_t *mask, int relu,
                 int flip, uint16_t *out, float *outf, void *stream);
/* Weight and bias gradients of one 32 -> 32 layer: dw[t][o][i] =
 * sum_v gy[v][o] x[v + off_t][i], db[o] = sum_v gy[v][o] (device FP32).
 * Synchronous. */
int r2p_cnn_conv_dw(const uint16_t *gy, const uint16_t *x, int nb, int nz, int ny, int nx,
                    float *dw, float *db, void *stream);
/* Network input of a state x (device, the layout of r2p_initial_state) at the
 * start of a step of length dt: per cell (p - 4800)/1000, s_w,
 * (ln kx - 4.6)/2, (phi - 0.2)/0.1, a signed well source log(1 + V) with V
 * the pore-volume fraction a perforation's well can move in dt (+ injector,
 * - producer), ln dt; feat: device bf16 [n][32]. */
int r2p_cnn_features(r2p_model *m, const double *x, double dt, uint16_t *feat, void *stream);
/* Training target of a step: ((p_new - p_old)/100, (s_new - s_old)/0.1) per
 * cell, device FP32 [n][2]. */
int r2p_cnn_targets(r2p_model *m, const double *x_old, const double *x_new, float *target,
                    void *stream);
/* x_guess = x + prediction (p += 100 out_0, s_w += 0.1 out_1 clipped to
 * [0,1]; a rate well's p_b moves by its perforations' mean dp, a BHP well's
 * stays). */
int r2p_cnn_warm_start(r2p_model *m, r2p_cnn *cnn, const double *x, double dt, double *x_guess,
                       void *stream);

const char *r2p_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
