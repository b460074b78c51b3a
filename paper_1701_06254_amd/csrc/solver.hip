// CPR preconditioner application, flexible GMRES and Newton's method.
//
// Paper sections: "Multi-stage preconditioner" (Eq 34-35 and Algorithm 2;
// the two-stage form is Algorithm 2 entered at its third step with x = 0),
// restarted GMRES as the Krylov solver ("Numerical experiments", Examples
// 4-5), and "Nonlinear methods" (Algorithm 1, forcing terms of Eq 26).
//
// Device design.  The Arnoldi process is classical Gram-Schmidt run twice,
// with the second pass delayed by one iteration (DCGS2: Bielich, Langou,
// Thomas, Swirydowicz, Yamazaki and Boman, "Low-synch Gram-Schmidt with
// delayed reorthogonalization for Krylov solvers", Parallel Computing 2022).
// At iteration j the basis vector v_j has had one projection only.  One pass
// over the basis computes V^T w, w.w, V^T v_j and v_j.v_j together (fused
// multi-dot, fixed-order two-stage reduction, one read-back); the host then
// finishes v_j's second projection (its coefficients, its norm by
// Pythagoras, and the correction this makes to Hessenberg column j - 1) and
// w's first one; a second pass applies both, v_j <- (v_j - V s) / n_j and
// v_{j+1} <- (w - V h) / ||w - V h||, reading each basis vector once.  The
// flexible method keeps z_j = M v_j as computed: A Z = V H still holds with
// the corrected basis.  For restarts above 32 (where the fused pass would
// need too many registers) the second projection is done in the same
// iteration, when the first removes more than half of ||w||^2
// (Daniel-Gragg-Kaufman-Stewart criterion).  The (m+1) x m Hessenberg matrix
// and its Givens rotations live on the host.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <thread>

#include "r2p_impl.h"

int r2p_decouple_jacobian(r2p_jacobian *J, int kind, hipStream_t s);
int r2p_newton_update(r2p_model *m, const double *y, double *x, double ds_max, hipStream_t s);

constexpr int BS = 256;
constexpr int MAXV = 65;                // basis vectors + 1 (w.w)
constexpr int DCGS_MAX = 32;            // restarts up to this use the delayed second pass
constexpr int MAXG = 2 * DCGS_MAX + 1;  // values of the fused pass: V^T w, w.w, V^T v_j
constexpr int MDOT_BLOCKS = 1024;       // workgroups of the multi-dot (grid-stride over rows)

// ----------------------------------------------------------- multi-dot
// h[k] = V_k . w (k < nv) and h[nv] = w . w, in two launches.  k_mdot: each
// thread keeps one accumulator per basis vector (NV >= nv, a multiple of 4,
// unrolled) and walks rows with a grid stride, two rows per visit, so a
// visit issues the loads of every vector together; the reductions happen
// once, at the end: a fixed butterfly per wavefront, a fixed sum over the
// wavefronts, one partial per workgroup and k (k-major).  k_mdot_sum (one
// workgroup per k) adds the partials of k, each thread over a fixed stride
// of workgroups, then the same butterfly and wavefront sum, so the result
// does not depend on scheduling; it also writes the values straight into
// the pinned host buffer the solver reads after the stream synchronises.
// (A last-workgroup ticket in one launch would need a device-scope fence in
// every workgroup, which on this GPU writes back and invalidates the L2.)
//
// With UPD the launch first applies a Gram-Schmidt pass, w <- w - V h (h
// from the previous multi-dot), row by row in the same order as k_mupdate,
// and takes the products from the updated rows: the reorthogonalising pass
// and the next projection share one read of the basis.
template <int NV, bool UPD>
__global__ __launch_bounds__(BS) void k_mdot(const double *V, long ld, int nv, const double *hin,
                                             double *w, long N, double *part) {
    __shared__ double red[BS / 64][MAXV];
    __shared__ double hs[UPD ? MAXV : 1];
    if (UPD) {
        for (int k = threadIdx.x; k < nv; k += BS) hs[k] = hin[k];
        __syncthreads();
    }
    double acc[NV + 1];
#pragma unroll
    for (int k = 0; k <= NV; k++) acc[k] = 0.0;
    long stride = (long)gridDim.x * 2 * BS;
    for (long i0 = (long)blockIdx.x * 2 * BS + threadIdx.x; i0 < N; i0 += stride) {
        long i1 = i0 + BS;
        bool two = i1 < N;
        double w0 = w[i0], w1 = two ? w[i1] : 0.0;
        // vectors k >= nv re-read the last one (or w): no branch between the
        // loads, so they are all in flight together; those sums are dropped
        const double *vl = nv > 0 ? V + (long)(nv - 1) * ld : w;
        double a[NV], b[NV];
#pragma unroll
        for (int k = 0; k < NV; k++) {
            const double *vk = k < nv ? V + (long)k * ld : vl;
            a[k] = vk[i0];
            b[k] = two ? vk[i1] : 0.0;
        }
        if (UPD) {
#pragma unroll
            for (int k = 0; k < NV; k++) {
                if (k < nv) {
                    w0 -= hs[k] * a[k];
                    w1 -= hs[k] * b[k];
                }
            }
            w[i0] = w0;
            if (two) w[i1] = w1;
            else w1 = 0.0;
        }
#pragma unroll
        for (int k = 0; k < NV; k++) acc[k] += a[k] * w0 + b[k] * w1;
        acc[NV] += w0 * w0 + w1 * w1;
    }
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int nb = gridDim.x;
#pragma unroll
    for (int k = 0; k <= NV; k++) {
        if (k < nv || k == NV) {
            double v = acc[k];
            for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
            if (lane == 0) red[wid][k < nv ? k : nv] = v;
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k <= nv; k += BS) {
        double t = 0.0;
        for (int q = 0; q < BS / 64; q++) t += red[q][k];
        part[(long)k * nb + blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(BS) void k_mdot_sum(int nb, const double *part, double *h,
                                                 double *hout) {
    // one workgroup per value k; its sum in a fixed order: each thread over
    // a fixed stride of the partials, a butterfly per wavefront, then the
    // wavefronts in order
    __shared__ double red[BS / 64];
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, k = blockIdx.x;
    const double *pk = part + (long)k * nb;
    double v = 0.0;
    int b = threadIdx.x;
    // four strides requested together, added in the same order
    for (; b + 3 * BS < nb; b += 4 * BS) {
        double a[4];
#pragma unroll
        for (int u = 0; u < 4; u++) a[u] = pk[b + u * BS];
#pragma unroll
        for (int u = 0; u < 4; u++) v += a[u];
    }
    for (; b < nb; b += BS) v += pk[b];
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
    if (lane == 0) red[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < BS / 64; q++) t += red[q];
        h[k] = t;
        if (hout) hout[k] = t;
    }
}

__global__ __launch_bounds__(BS) void k_mupdate(const double *V, long ld, int nv, const double *h,
                                                const double *w, long N, double scale,
                                                double *out) {
    __shared__ double hs[MAXV];
    for (int k = threadIdx.x; k < nv; k += BS) hs[k] = h[k];
    __syncthreads();
    long i = (long)blockIdx.x * BS + threadIdx.x;
    if (i >= N) return;
    double t = w[i];
    for (int k = 0; k < nv; k++) t -= hs[k] * V[(long)k * ld + i];
    out[i] = t * scale;
}

// The fused pass of the delayed second projection, nv = j + 1 basis vectors
// (the last, v_j, projected once so far): values k < nv are V_k . w, nv is
// w . w, nv + 1 + k (k < nv) are V_k . v_j; partials as in k_mdot.
template <int NV>
__global__ __launch_bounds__(BS) void k_mdot2(const double *V, long ld, int nv, const double *w,
                                              long N, double *part) {
    __shared__ double red[BS / 64][2 * NV + 1];
    double acc[NV + 1], acg[NV];
#pragma unroll
    for (int k = 0; k <= NV; k++) acc[k] = 0.0;
#pragma unroll
    for (int k = 0; k < NV; k++) acg[k] = 0.0;
    long stride = (long)gridDim.x * 2 * BS;
    const double *vl = V + (long)(nv - 1) * ld;
    for (long i0 = (long)blockIdx.x * 2 * BS + threadIdx.x; i0 < N; i0 += stride) {
        long i1 = i0 + BS;
        bool two = i1 < N;
        double w0 = w[i0], w1 = two ? w[i1] : 0.0;
        double a[NV], b[NV];
#pragma unroll
        for (int k = 0; k < NV; k++) {
            const double *vk = k < nv ? V + (long)k * ld : vl;
            a[k] = vk[i0];
            b[k] = two ? vk[i1] : 0.0;
        }
        // v_j's values, picked from the loaded ones (no indexed registers)
        double q0 = 0.0, q1 = 0.0;
#pragma unroll
        for (int k = 0; k < NV; k++) {
            q0 = k == nv - 1 ? a[k] : q0;
            q1 = k == nv - 1 ? b[k] : q1;
        }
#pragma unroll
        for (int k = 0; k < NV; k++) {
            acc[k] += a[k] * w0 + b[k] * w1;
            acg[k] += a[k] * q0 + b[k] * q1;
        }
        acc[NV] += w0 * w0 + w1 * w1;
    }
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int nb = gridDim.x;
#pragma unroll
    for (int k = 0; k <= NV; k++) {
        if (k < nv || k == NV) {
            double v = acc[k];
            for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
            if (lane == 0) red[wid][k < nv ? k : nv] = v;
        }
    }
#pragma unroll
    for (int k = 0; k < NV; k++) {
        if (k < nv) {
            double v = acg[k];
            for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
            if (lane == 0) red[wid][nv + 1 + k] = v;
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k <= 2 * nv; k += BS) {
        double t = 0.0;
        for (int q = 0; q < BS / 64; q++) t += red[q][k];
        part[(long)k * nb + blockIdx.x] = t;
    }
}

// The second pass of iteration j: v_j <- (v_j - sum_k s_k V_k) / n_j in
// place, then out <- (w - sum_k h_k V_k - h_j v_j) / ||.|| (k < j), each
// basis vector read once.
struct Coef2 {
    double s[DCGS_MAX], h[DCGS_MAX];
    double hj, inv_nj, inv_hn;
};
__global__ __launch_bounds__(BS) void k_mupdate2(double *V, long ld, int j, Coef2 c,
                                                 const double *w, long N, double *out) {
    long i = (long)blockIdx.x * BS + threadIdx.x;
    if (i >= N) return;
    double vj = V[(long)j * ld + i], t = w[i];
    for (int k = 0; k < j; k++) {
        double vk = V[(long)k * ld + i];
        vj -= c.s[k] * vk;
        t -= c.h[k] * vk;
    }
    vj *= c.inv_nj;
    V[(long)j * ld + i] = vj;
    t -= c.hj * vj;
    out[i] = t * c.inv_hn;
}

struct Coef {
    double c[64];
};

// x += sum_k y_k Z_k
__global__ __launch_bounds__(BS) void k_maxpy(const double *Z, long ld, int nv, Coef y, long N,
                                              double *x) {
    long i = (long)blockIdx.x * BS + threadIdx.x;
    if (i >= N) return;
    double t = x[i];
    for (int k = 0; k < nv; k++) t += y.c[k] * Z[(long)k * ld + i];
    x[i] = t;
}

// out = x + a y (+ b z): the BiCGSTAB updates s = r - alpha v,
// x += alpha p^ + omega s^, r = s - omega t (out may alias x).
__global__ __launch_bounds__(BS) void k_axpbypz(long N, const double *x, double a, const double *y,
                                                double b, const double *z, double *out) {
    long i = (long)blockIdx.x * BS + threadIdx.x;
    if (i >= N) return;
    double v = x[i] + a * y[i];
    if (z) v = x[i] + (a * y[i] + b * z[i]);
    out[i] = v;
}

// p = r + beta (p - omega v)
__global__ __launch_bounds__(BS) void k_bicg_p(long N, const double *r, const double *v, double beta,
                                               double omega, double *p) {
    long i = (long)blockIdx.x * BS + threadIdx.x;
    if (i >= N) return;
    p[i] = r[i] + beta * (p[i] - omega * v[i]);
}

// r_orig = D (r_dec) per cell row: the residual of the undecoupled system.
__global__ void k_undecouple(int n, long N, const double4 *dec, const double *rd, double *r) {
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) {
        double4 M = dec[i];
        double det = M.x * M.w - M.y * M.z;
        double a = rd[2 * i], b = rd[2 * i + 1];
        r[2 * i] = (M.w * a - M.y * b) / det;
        r[2 * i + 1] = (-M.z * a + M.x * b) / det;
    } else if (2 * i < N) {
        r[2 * i] = rd[2 * i];
        r[2 * i + 1] = rd[2 * i + 1];
    }
}

struct Krylov {
    DBuf<double> V, Z, part, h, r, bd, w;
    HostPinned pin;
    double *pin_dev = nullptr;        // device address of pin
    long N = 0;
    int m = 0;
};

static Krylov &krylov_for(r2p_cpr *P);

// The pinned read-back buffer and its device address.
static int pin_ensure(Krylov &K, size_t bytes) {
    R2P_TRY(K.pin.ensure(bytes));
    void *d = nullptr;
    R2P_HIP(hipHostGetDevicePointer(&d, K.pin.p, 0));
    K.pin_dev = (double *)d;
    return 0;
}

// h = V^T w and w.w into K.h (and hhost); with upd (= K.h of the previous
// projection) w first loses V upd in the same launch.
static int mdot(Krylov &K, const double *V, int nv, double *w, long N, hipStream_t s,
                double *hhost, const double *upd = nullptr) {
    int nb = std::max(1, std::min(MDOT_BLOCKS, r2p_blocks(N, 2 * BS)));
    R2P_TRY(K.part.ensure((size_t)nb * MAXV));
#define R2P_MDOT(NVB)                                                               \
    do {                                                                            \
        if (upd) k_mdot<NVB, true><<<nb, BS, 0, s>>>(V, N, nv, upd, w, N, K.part.p); \
        else k_mdot<NVB, false><<<nb, BS, 0, s>>>(V, N, nv, nullptr, w, N, K.part.p); \
    } while (0)
    if (nv <= 4) R2P_MDOT(4);
    else if (nv <= 8) R2P_MDOT(8);
    else if (nv <= 12) R2P_MDOT(12);
    else if (nv <= 16) R2P_MDOT(16);
    else if (nv <= 20) R2P_MDOT(20);
    else if (nv <= 24) R2P_MDOT(24);
    else if (nv <= 28) R2P_MDOT(28);
    else if (nv <= 32) R2P_MDOT(32);
    else if (nv <= 48) R2P_MDOT(48);
    else R2P_MDOT(64);
#undef R2P_MDOT
    R2P_LAUNCH();
    k_mdot_sum<<<nv + 1, BS, 0, s>>>(nb, K.part.p, K.h.p, hhost ? K.pin_dev : nullptr);
    R2P_LAUNCH();
    if (hhost) {
        R2P_HIP(hipStreamSynchronize(s));
        memcpy(hhost, K.pin.p, sizeof(double) * (nv + 1));
    }
    return 0;
}

// The fused pass of the delayed second projection: out[0..nv) = V^T w,
// out[nv] = w.w, out[nv + 1 + k] = V_k . V_{nv-1} (k < nv); one read-back.
static int mdot2(Krylov &K, const double *V, int nv, const double *w, long N, hipStream_t s,
                 double *out) {
    int nb = std::max(1, std::min(MDOT_BLOCKS, r2p_blocks(N, 2 * BS)));
    R2P_TRY(K.part.ensure((size_t)nb * MAXG));
    if (nv <= 4) k_mdot2<4><<<nb, BS, 0, s>>>(V, N, nv, w, N, K.part.p);
    else if (nv <= 8) k_mdot2<8><<<nb, BS, 0, s>>>(V, N, nv, w, N, K.part.p);
    else if (nv <= 12) k_mdot2<12><<<nb, BS, 0, s>>>(V, N, nv, w, N, K.part.p);
    else if (nv <= 16) k_mdot2<16><<<nb, BS, 0, s>>>(V, N, nv, w, N, K.part.p);
    else if (nv <= 20) k_mdot2<20><<<nb, BS, 0, s>>>(V, N, nv, w, N, K.part.p);
    else if (nv <= 24) k_mdot2<24><<<nb, BS, 0, s>>>(V, N, nv, w, N, K.part.p);
    else if (nv <= 28) k_mdot2<28><<<nb, BS, 0, s>>>(V, N, nv, w, N, K.part.p);
    else k_mdot2<32><<<nb, BS, 0, s>>>(V, N, nv, w, N, K.part.p);
    R2P_LAUNCH();
    k_mdot_sum<<<2 * nv + 1, BS, 0, s>>>(nb, K.part.p, K.h.p, K.pin_dev);
    R2P_LAUNCH();
    R2P_HIP(hipStreamSynchronize(s));
    memcpy(out, K.pin.p, sizeof(double) * (2 * nv + 1));
    return 0;
}

// ------------------------------------------------------------------ CPR
int r2p_cpr_apply_impl(r2p_cpr *P, const double *f, double *z, hipStream_t s) {
    r2p_jacobian *J = P->J;
    if (P->o.form == R2P_CPR_FPF) {
        // Algorithm 2: x = R^-1 f; r = f - A x; x += Pi_p M^-1 Pi_r r;
        // r = f - A x; x += R^-1 r
        R2P_TRY(r2p_ras_solve(P, f, z, nullptr, 0, s));
        R2P_TRY(r2p_spmv_impl(J, z, P->t_r.p, f, s));
        R2P_TRY(r2p_amg_apply(P, P->t_r.p, 2, P->t_xp.p, s));
        R2P_TRY(r2p_pcol_residual(J, P->t_r.p, P->t_xp.p, P->t_y.p, s));
        R2P_TRY(r2p_ras_solve(P, P->t_y.p, z, P->t_xp.p, 1, s));
    } else {
        // x = Pi_p M^-1 Pi_r f; r = f - A x; x += R^-1 r
        R2P_TRY(r2p_amg_apply(P, f, 2, P->t_xp.p, s));
        R2P_TRY(r2p_pcol_residual(J, f, P->t_xp.p, P->t_r.p, s));
        R2P_TRY(r2p_ras_solve(P, P->t_r.p, z, P->t_xp.p, 0, s));
    }
    return 0;
}

extern "C" int r2p_cpr_create(r2p_cpr **out) {
    if (!out) { r2p_set_error("NULL argument"); return R2P_EINVAL; }
    *out = new r2p_cpr();
    return 0;
}

extern "C" int r2p_cpr_destroy(r2p_cpr *P) {
    delete P;
    return 0;
}

r2p_cpr::~r2p_cpr() {
    delete kry;
    for (hipEvent_t &e : aev)
        if (e) (void)hipEventDestroy(e);
    if (as) (void)hipStreamDestroy(as);
}

// The second stream and its two events, made on the first set-up.
static int ensure_amg_stream(r2p_cpr *P) {
    if (!P->as) R2P_HIP(hipStreamCreateWithFlags(&P->as, hipStreamNonBlocking));
    for (hipEvent_t &e : P->aev)
        if (!e) R2P_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return 0;
}

// The RAS and AMG set-ups read the decoupled Jacobian and write disjoint
// parts of the handle; each waits on the host for its own scan totals.
// The AMG set-up runs on a worker thread and its own stream (after the
// decoupling on s), the RAS set-up on s in this thread, so that the one's
// host waits and narrow kernels (one workgroup per subdomain) overlap the
// other's work.  Both are joined before return, and s then waits for the
// AMG stream.
static int setup_both(r2p_cpr *P, hipStream_t s) {
    R2P_TRY(ensure_amg_stream(P));
    int dev = 0;
    R2P_HIP(hipGetDevice(&dev));
    R2P_HIP(hipEventRecord(P->aev[0], s));
    R2P_HIP(hipStreamWaitEvent(P->as, P->aev[0], 0));
    int rc_amg = 0;
    std::string err_amg;
    auto amg = [&] {
        if (hipSetDevice(dev) != hipSuccess) {
            rc_amg = R2P_EHIP;
            err_amg = "hipSetDevice failed on the AMG set-up thread";
            return;
        }
        double ta = r2p_now_ms();
        rc_amg = r2p_amg_setup(P, P->as);
        P->ms_amg = r2p_now_ms() - ta;
        if (rc_amg) err_amg = r2p_last_error();
    };
    std::thread t;
    bool threaded = true;
    try {
        t = std::thread(amg);
    } catch (...) {
        threaded = false;
    }
    int rc = r2p_ras_setup(P, s);
    if (threaded) t.join();
    else if (!rc) amg();
    if (!rc && rc_amg) {
        r2p_set_error("%s", err_amg.c_str());
        rc = rc_amg;
    }
    if (rc) {
        (void)hipStreamSynchronize(P->as);
        return rc;
    }
    R2P_HIP(hipEventRecord(P->aev[1], P->as));
    R2P_HIP(hipStreamWaitEvent(s, P->aev[1], 0));
    return 0;
}

static int check_opts(const r2p_cpr_opts *o) {
    if (o->decouple < 0 || o->decouple > 2 || o->order < 0 || o->order > 1 || o->form < 0 ||
        o->form > 1 || o->px < 1 || o->py < 1 || o->px * o->py > 256 || o->overlap < 0 ||
        o->overlap > 8 || !(o->theta >= 0) || o->max_coarse < 1 || o->max_coarse > 2048 ||
        o->max_levels < 1 || o->match_rounds < 1 || o->agg_passes < 1 || o->agg_passes > 4 ||
        o->precision < 0 || o->precision > 1 || o->kcycle < 0 || o->kcycle > 23 ||
        o->amg_cycles < 1 || o->amg_cycles > 8) {
        r2p_set_error("invalid CPR options");
        return R2P_EINVAL;
    }
    return 0;
}

extern "C" int r2p_setup_cpr(r2p_jacobian *J, const r2p_cpr_opts *o, r2p_cpr *P, void *stream) {
    if (!J || !o || !P) { r2p_set_error("NULL argument"); return R2P_EINVAL; }
    R2P_TRY(check_opts(o));
    if (J->state != 1) { r2p_set_error("Jacobian not assembled since its last set-up"); return R2P_ESTATE; }
    hipStream_t s = (hipStream_t)stream;
    // cached structures belong to one model (by serial: a model allocated
    // where a destroyed one was is another model)
    if (P->serial != J->m->serial || P->o.px != o->px || P->o.py != o->py ||
        P->o.overlap != o->overlap)
        P->rs.ns = 0;   // membership must be rebuilt
    if (P->serial != J->m->serial) P->app_n = -1;
    P->serial = J->m->serial;
    P->ready = 0;
    P->J = J;
    P->o = *o;
    const Phys &ph = J->m->ph;
    long N = 2L * (ph.n + ph.nw);
    R2P_TRY(P->t_r.ensure(N));
    R2P_TRY(P->t_y.ensure(N));
    R2P_TRY(P->t_xp.ensure(ph.n));
    if (o->amg_cycles > 1) R2P_TRY(P->t_ares.ensure(ph.n));
    P->ms_dec = P->ms_order = P->ms_ras = P->ms_amg = 0.0;
    double t0 = r2p_now_ms();
    R2P_TRY(r2p_decouple_jacobian(J, o->decouple, s));
    R2P_HIP(hipStreamSynchronize(s));
    P->ms_dec = r2p_now_ms() - t0;
    int rc = setup_both(P, s);
    if (rc) return rc;          // errors, and the soft failure of a stalled coarsening
    P->ready = 1;
    return 0;
}

extern "C" int r2p_cpr_apply(r2p_cpr *P, const double *f, double *z, void *stream) {
    if (!P || !f || !z) { r2p_set_error("NULL argument"); return R2P_EINVAL; }
    if (!P->ready) { r2p_set_error("CPR not set up"); return R2P_ESTATE; }
    return r2p_cpr_apply_impl(P, f, z, (hipStream_t)stream);
}

extern "C" int r2p_amg_vcycle(r2p_cpr *P, const double *f_p, double *x_p, void *stream) {
    if (!P || !f_p || !x_p) { r2p_set_error("NULL argument"); return R2P_EINVAL; }
    if (!P->ready) { r2p_set_error("CPR not set up"); return R2P_ESTATE; }
    return r2p_amg_cycle(P, f_p, 1, x_p, (hipStream_t)stream);
}

extern "C" int r2p_ras_apply(r2p_cpr *P, const double *r, double *y, void *stream) {
    if (!P || !r || !y) { r2p_set_error("NULL argument"); return R2P_EINVAL; }
    if (!P->ready) { r2p_set_error("CPR not set up"); return R2P_ESTATE; }
    return r2p_ras_solve(P, r, y, nullptr, 0, (hipStream_t)stream);
}

// ---------------------------------------------------------------- FGMRES
// The Krylov workspace belongs to the CPR handle (the Newton step's handle
// belongs to its model) and is freed with it.
static Krylov &krylov_for(r2p_cpr *P) {
    if (!P->kry) P->kry = new Krylov();
    return *P->kry;
}

// Right-preconditioned BiCGSTAB on the decoupled system (the paper's other
// Krylov solver), from zero, shadow residual r^ = b.  Converged when the
// recursive residual reaches rtol ||b||; the true residual is then checked
// and, if it is above the target, the recurrences restart from it.  Dots
// are the fused multi-dot (fixed-order reduction), read back per use.
static int solve_bicgstab(r2p_jacobian *J, r2p_cpr *P, Krylov &K, double bnorm, double *y,
                          const r2p_solve_opts *o, r2p_solve_info &inf, int &status,
                          hipStream_t s) {
    const Phys &ph = J->m->ph;
    long N = 2L * (ph.n + ph.nw);
    R2P_TRY(K.V.ensure((size_t)8 * N));
    double *r = K.V.p, *rh = r + N, *p = rh + N, *v = p + N, *pp = v + N, *sv = pp + N,
           *sp = sv + N, *t = sp + N;
    int nb = r2p_blocks(N, BS);
    R2P_HIP(hipMemcpyAsync(r, K.bd.p, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    R2P_HIP(hipMemcpyAsync(rh, K.bd.p, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    R2P_HIP(hipMemsetAsync(p, 0, sizeof(double) * N, s));
    R2P_HIP(hipMemsetAsync(v, 0, sizeof(double) * N, s));
    double rho_prev = 1.0, alpha = 1.0, omega = 1.0;
    bool fresh = true;
    int it = 0;
    status = R2P_NOT_CONVERGED;
    while (it < o->maxit) {
        double h[2];
        R2P_TRY(mdot(K, rh, 1, r, N, s, h));
        double rho = h[0];
        if (rho == 0.0 || rho != rho) { status = R2P_BREAKDOWN; break; }
        if (fresh) {
            R2P_HIP(hipMemcpyAsync(p, r, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
        } else {
            double beta = (rho / rho_prev) * (alpha / omega);
            k_bicg_p<<<nb, BS, 0, s>>>(N, r, v, beta, omega, p);
            R2P_LAUNCH();
        }
        fresh = false;
        R2P_TRY(r2p_cpr_apply_impl(P, p, pp, s));
        R2P_TRY(r2p_spmv_impl(J, pp, v, nullptr, s));
        R2P_TRY(mdot(K, rh, 1, v, N, s, h));
        if (h[0] == 0.0 || h[0] != h[0]) { status = R2P_BREAKDOWN; break; }
        alpha = rho / h[0];
        k_axpbypz<<<nb, BS, 0, s>>>(N, r, -alpha, v, 0.0, nullptr, sv);
        R2P_LAUNCH();
        it++;
        R2P_TRY(mdot(K, nullptr, 0, sv, N, s, h));
        bool conv = false;
        if (sqrt(h[0]) <= o->rtol * bnorm) {
            k_axpbypz<<<nb, BS, 0, s>>>(N, y, alpha, pp, 0.0, nullptr, y);
            R2P_LAUNCH();
            conv = true;
        } else {
            R2P_TRY(r2p_cpr_apply_impl(P, sv, sp, s));
            R2P_TRY(r2p_spmv_impl(J, sp, t, nullptr, s));
            R2P_TRY(mdot(K, sv, 1, t, N, s, h));          // h[0] = t.s, h[1] = t.t
            omega = h[1] > 0.0 ? h[0] / h[1] : 0.0;
            k_axpbypz<<<nb, BS, 0, s>>>(N, y, alpha, pp, omega, sp, y);
            R2P_LAUNCH();
            k_axpbypz<<<nb, BS, 0, s>>>(N, sv, -omega, t, 0.0, nullptr, r);
            R2P_LAUNCH();
            rho_prev = rho;
            R2P_TRY(mdot(K, nullptr, 0, r, N, s, h));
            if (sqrt(h[0]) <= o->rtol * bnorm) conv = true;
            else if (omega == 0.0) { status = R2P_BREAKDOWN; break; }
        }
        if (conv) {
            R2P_TRY(r2p_spmv_impl(J, y, r, K.bd.p, s));  // true residual bd - A y
            R2P_TRY(mdot(K, nullptr, 0, r, N, s, h));
            inf.relres = sqrt(h[0]) / bnorm;
            if (sqrt(h[0]) <= o->rtol * bnorm) { status = 0; break; }
            R2P_HIP(hipMemcpyAsync(rh, r, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
            rho_prev = alpha = omega = 1.0;
            fresh = true;
        }
    }
    if (status != 0) {
        double h[2];
        R2P_TRY(r2p_spmv_impl(J, y, r, K.bd.p, s));
        R2P_TRY(mdot(K, nullptr, 0, r, N, s, h));
        inf.relres = sqrt(h[0]) / bnorm;
    }
    inf.iterations = it;
    return 0;
}

extern "C" int r2p_solve(r2p_jacobian *J, r2p_cpr *P, const double *b, double *y,
                         const r2p_solve_opts *o, r2p_solve_info *info, void *stream) {
    auto t0 = std::chrono::steady_clock::now();
    if (!J || !P || !b || !y || !o) { r2p_set_error("NULL argument"); return R2P_EINVAL; }
    if (!P->ready || P->J != J || J->state != 2) { r2p_set_error("CPR not set up for this Jacobian"); return R2P_ESTATE; }
    if (o->restart < 1 || o->restart > 64 || o->maxit < 1 || !(o->rtol > 0) ||
        (o->method != R2P_KRYLOV_FGMRES && o->method != R2P_KRYLOV_BICGSTAB)) {
        r2p_set_error("invalid solve options");
        return R2P_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    const Phys &ph = J->m->ph;
    long N = 2L * (ph.n + ph.nw);
    int m = o->restart;
    Krylov &K = krylov_for(P);
    R2P_TRY(K.V.ensure((size_t)(m + 1) * N));
    R2P_TRY(K.Z.ensure((size_t)m * N));
    R2P_TRY(K.r.ensure(N));
    R2P_TRY(K.bd.ensure(N));
    R2P_TRY(K.h.ensure(MAXG > MAXV ? MAXG : MAXV));
    R2P_TRY(pin_ensure(K, sizeof(double) * (MAXG > MAXV ? MAXG : MAXV) * 2));
    R2P_TRY(r2p_decouple_rhs(J, b, K.bd.p, s));
    double hb[MAXV];
    R2P_TRY(mdot(K, nullptr, 0, K.bd.p, N, s, hb));
    double bnorm = sqrt(hb[0]);
    R2P_HIP(hipMemsetAsync(y, 0, sizeof(double) * N, s));
    r2p_solve_info inf{};
    int status = R2P_NOT_CONVERGED;
    if (!(bnorm == bnorm) || std::isinf(bnorm)) { r2p_set_error("non-finite right-hand side"); return R2P_ENAN; }
    if (bnorm == 0.0) {
        status = 0;
        inf.relres = 0.0;
    } else if (o->method == R2P_KRYLOV_BICGSTAB) {
        R2P_TRY(solve_bicgstab(J, P, K, bnorm, y, o, inf, status, s));
    } else {
        // Hr: the Hessenberg matrix as computed (the delayed second pass
        // corrects its previous column); H: Hr after the Givens rotations,
        // recomputed over columns 0..j at every iteration (g: the rotated
        // right-hand side beta e_1)
        std::vector<double> Hr((size_t)(m + 1) * m, 0.0), H((size_t)(m + 1) * m, 0.0);
        std::vector<double> cs(m), sn(m), g(m + 1), yv(m);
        R2P_HIP(hipMemcpyAsync(K.r.p, K.bd.p, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
        double beta = bnorm;
        int total = 0;
        int nblk = r2p_blocks(N, BS);
        const bool delayed = m <= DCGS_MAX;
        auto rotate = [&](int jj) -> bool {
            std::fill(g.begin(), g.end(), 0.0);
            g[0] = beta;
            for (int c = 0; c <= jj; c++) {
                for (int i = 0; i <= c + 1; i++) H[(size_t)i * m + c] = Hr[(size_t)i * m + c];
                for (int i = 0; i < c; i++) {
                    double a = H[(size_t)i * m + c], b = H[(size_t)(i + 1) * m + c];
                    H[(size_t)i * m + c] = cs[i] * a + sn[i] * b;
                    H[(size_t)(i + 1) * m + c] = -sn[i] * a + cs[i] * b;
                }
                double a = H[(size_t)c * m + c], b = H[(size_t)(c + 1) * m + c];
                double den = sqrt(a * a + b * b);
                if (den == 0.0 || den != den) return false;
                cs[c] = a / den;
                sn[c] = b / den;
                H[(size_t)c * m + c] = den;
                H[(size_t)(c + 1) * m + c] = 0.0;
                g[c + 1] = -sn[c] * g[c];
                g[c] = cs[c] * g[c];
            }
            return true;
        };
        while (total < o->maxit) {
            k_mupdate<<<nblk, BS, 0, s>>>(nullptr, N, 0, K.h.p, K.r.p, N, 1.0 / beta, K.V.p);
            R2P_LAUNCH();
            int k = 0;
            bool stop = false;
            for (int j = 0; j < m && total < o->maxit; j++) {
                double *vj = K.V.p + (size_t)j * N, *zj = K.Z.p + (size_t)j * N;
                double *w = K.V.p + (size_t)(j + 1) * N;
                R2P_TRY(r2p_cpr_apply_impl(P, vj, zj, s));
                R2P_TRY(r2p_spmv_impl(J, zj, w, nullptr, s));
                double hh[MAXV], hn;
                if (delayed) {
                    // t = V^T w, w.w, q = V^T v_j in one pass
                    double gv[MAXG];
                    R2P_TRY(mdot2(K, K.V.p, j + 1, w, N, s, gv));
                    const double *t = gv, *q = gv + j + 2;
                    double ww = gv[j + 1];
                    Coef2 c{};
                    double nj = 1.0, hj = t[j];
                    if (j > 0) {
                        // v_j's second projection: s = q[0..j), n_j^2 = v_j.v_j - |s|^2
                        double ss = 0.0, st = 0.0;
                        for (int i = 0; i < j; i++) { ss += q[i] * q[i]; st += q[i] * t[i]; }
                        double nj2 = q[j] - ss;
                        if (!(nj2 > 0.0)) { status = R2P_BREAKDOWN; stop = true; total++; break; }
                        nj = sqrt(nj2);
                        // A z_{j-1} = V h_{j-1} + h_{j,j-1} v_j before the correction
                        double hsub = Hr[(size_t)j * m + j - 1];
                        for (int i = 0; i < j; i++) Hr[(size_t)i * m + j - 1] += hsub * q[i];
                        Hr[(size_t)j * m + j - 1] = hsub * nj;
                        hj = (t[j] - st) / nj;
                        for (int i = 0; i < j; i++) c.s[i] = q[i];
                        inf.reorth++;
                    }
                    double hs = hj * hj;
                    for (int i = 0; i < j; i++) { hh[i] = t[i]; hs += t[i] * t[i]; c.h[i] = t[i]; }
                    hh[j] = hj;
                    double wn2 = ww - hs;
                    hn = wn2 > 0.0 ? sqrt(wn2) : 0.0;
                    c.hj = hj;
                    c.inv_nj = 1.0 / nj;
                    c.inv_hn = hn > 0.0 ? 1.0 / hn : 0.0;
                    k_mupdate2<<<nblk, BS, 0, s>>>(K.V.p, N, j, c, w, N, w);
                    R2P_LAUNCH();
                } else {
                    R2P_TRY(mdot(K, K.V.p, j + 1, w, N, s, hh));
                    double ww = hh[j + 1], hs = 0.0;
                    for (int i = 0; i <= j; i++) hs += hh[i] * hh[i];
                    double wn2 = ww - hs;
                    if (wn2 > 0.49 * ww) {
                        hn = sqrt(wn2);
                        k_mupdate<<<nblk, BS, 0, s>>>(K.V.p, N, j + 1, K.h.p, w, N, 1.0 / hn, w);
                        R2P_LAUNCH();
                    } else {
                        // second Gram-Schmidt pass
                        inf.reorth++;
                        double h2[MAXV];
                        R2P_TRY(mdot(K, K.V.p, j + 1, w, N, s, h2, K.h.p));
                        double hs2 = 0.0;
                        for (int i = 0; i <= j; i++) { hh[i] += h2[i]; hs2 += h2[i] * h2[i]; }
                        double wn = h2[j + 1] - hs2;
                        hn = wn > 0.0 ? sqrt(wn) : 0.0;
                        if (hn > 0.0) {
                            k_mupdate<<<nblk, BS, 0, s>>>(K.V.p, N, j + 1, K.h.p, w, N, 1.0 / hn, w);
                            R2P_LAUNCH();
                        }
                    }
                }
                for (int i = 0; i <= j; i++) Hr[(size_t)i * m + j] = hh[i];
                Hr[(size_t)(j + 1) * m + j] = hn;
                total++;
                if (!rotate(j)) { status = R2P_BREAKDOWN; stop = true; break; }
                k = j + 1;
                if (fabs(g[j + 1]) <= o->rtol * bnorm || hn == 0.0) break;
            }
            if (k > 0) {
                for (int i = k - 1; i >= 0; i--) {
                    double sum = g[i];
                    for (int t = i + 1; t < k; t++) sum -= H[(size_t)i * m + t] * yv[t];
                    yv[i] = sum / H[(size_t)i * m + i];
                }
                Coef cf;
                for (int i = 0; i < k; i++) cf.c[i] = yv[i];
                k_maxpy<<<nblk, BS, 0, s>>>(K.Z.p, N, k, cf, N, y);
                R2P_LAUNCH();
            }
            R2P_TRY(r2p_spmv_impl(J, y, K.r.p, K.bd.p, s));
            double rr[2];
            R2P_TRY(mdot(K, nullptr, 0, K.r.p, N, s, rr));
            beta = sqrt(rr[0]);
            inf.relres = beta / bnorm;
            if (beta <= o->rtol * bnorm) { status = 0; break; }
            if (stop || beta == 0.0 || beta != beta) break;
        }
        inf.iterations = total;
    }
    inf.status = status;
    inf.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
    return status;
}

// ---------------------------------------------------------------- Newton
extern "C" void r2p_default_newton_opts(r2p_newton_opts *o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->max_newton = 20;
    o->tol = 1e-8;
    o->forcing = R2P_FORCING_FIXED;
    o->ds_max = 0.2;
    o->cpr.decouple = R2P_DEC_QI;
    o->cpr.order = R2P_ORDER_POTENTIAL;
    o->cpr.form = R2P_CPR_TWO_STAGE;
    o->cpr.px = 4;
    o->cpr.py = 4;
    o->cpr.overlap = 1;
    o->cpr.theta = 0.25;
    o->cpr.max_coarse = 500;
    o->cpr.max_levels = 20;
    o->cpr.match_rounds = 4;
    o->cpr.agg_passes = 2;
    o->cpr.precision = R2P_FP64;
    o->cpr.kcycle = 1;
    o->cpr.amg_cycles = 2;
    o->lin.restart = 30;
    o->lin.maxit = 300;
    o->lin.rtol = 1e-8;
    o->lin.method = R2P_KRYLOV_FGMRES;
    o->guess_rule = R2P_GUESS_SCALED_INF;
}

struct NewtonWork {
    r2p_model *m = nullptr;
    r2p_jacobian *J = nullptr;
    r2p_cpr *P = nullptr;
    DBuf<double> xold, xk, b, y, t;
    ~NewtonWork() {
        if (J) r2p_jacobian_destroy(J);
        if (P) r2p_cpr_destroy(P);
    }
};

void r2p_newton_work_free(NewtonWork *W) { delete W; }

double r2p_now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
static double now_ms() { return r2p_now_ms(); }

// Newton iterations of Algorithm 1 from the iterate in W->xk (old state in
// W->xold); status 0 when the scaled residual test passes.  Iteration counts
// and timings accumulate in inf.
static int newton_loop(NewtonWork *W, Krylov &K, r2p_model *m, double dt,
                       const r2p_newton_opts *o, long N, hipStream_t s, r2p_newton_info &inf,
                       int &status) {
    void *stream = (void *)s;
    status = R2P_NOT_CONVERGED;
    double eta = 0.1, prev_fn = 0.0, prev_rn = 0.0;
    for (int it = 0; it <= o->max_newton; it++) {
        double ta = now_ms();
        R2P_TRY(r2p_assemble_jacobian(m, W->xk.p, W->xold.p, dt, W->J, W->b.p, stream));
        double sn = 0.0;
        int rc = r2p_residual_norm(m, W->b.p, dt, &sn, stream);
        inf.ms_assemble += now_ms() - ta;
        inf.res_hist[it] = sn;
        if (rc == R2P_ENAN) break;
        R2P_TRY(rc);
        if (sn <= o->tol) { status = 0; break; }
        if (it == o->max_newton) break;
        double hb[2];
        R2P_TRY(mdot(K, nullptr, 0, W->b.p, N, s, hb));
        double fn = sqrt(hb[0]);
        if (o->forcing == R2P_FORCING_EW && it > 0) {
            eta = fabs(fn - prev_rn) / prev_fn;
            eta = eta < 0.01 ? 0.01 : (eta > 0.1 ? 0.1 : eta);
        }
        double ts = now_ms();
        rc = r2p_setup_cpr(W->J, &o->cpr, W->P, stream);
        inf.ms_setup += now_ms() - ts;
        inf.ms_decouple += W->P->ms_dec;
        inf.ms_order += W->P->ms_order;
        inf.ms_ras_setup += W->P->ms_ras;
        inf.ms_amg_setup += W->P->ms_amg;
        inf.setup_status = rc;
        // a failure of the method (stalled coarsening, a singular pivot) ends
        // the step as not converged, so that the caller shortens it
        if (rc > 0 || rc == R2P_ESINGULAR) break;
        if (rc) return rc;
        r2p_solve_opts lo = o->lin;
        if (o->forcing == R2P_FORCING_EW) lo.rtol = eta;
        r2p_solve_info si{};
        double tl = now_ms();
        rc = r2p_solve(W->J, W->P, W->b.p, W->y.p, &lo, &si, stream);
        inf.ms_solve += now_ms() - tl;
        inf.linear_its += si.iterations;
        if (rc < 0) return rc;
        if (rc != 0 && o->forcing == R2P_FORCING_FIXED) break;
        double tu = now_ms();
        if (o->forcing == R2P_FORCING_EW) {
            // ||b - J y|| of the undecoupled system (Eq 27)
            R2P_TRY(r2p_spmv_impl(W->J, W->y.p, W->t.p, K.bd.p, s));
            k_undecouple<<<r2p_blocks(m->ph.n + m->ph.nw, BS), BS, 0, s>>>(m->ph.n, N, W->J->dec.p, W->t.p, W->t.p);
            R2P_LAUNCH();
            double hr[2];
            R2P_TRY(mdot(K, nullptr, 0, W->t.p, N, s, hr));
            prev_rn = sqrt(hr[0]);
            prev_fn = fn;
        }
        R2P_TRY(r2p_newton_update(m, W->y.p, W->xk.p, o->ds_max, s));
        R2P_HIP(hipStreamSynchronize(s));
        inf.ms_update += now_ms() - tu;
        inf.newton_its++;
    }
    return 0;
}

extern "C" int r2p_newton_step(r2p_model *m, double *x, double dt, const double *x_guess,
                               const r2p_newton_opts *o, r2p_newton_info *info, void *stream) {
    double T0 = now_ms();
    if (!m || !x || !o) { r2p_set_error("NULL argument"); return R2P_EINVAL; }
    if (!(dt > 0) || o->max_newton < 1 || o->max_newton >= R2P_HIST || !(o->tol > 0) ||
        o->guess_rule < 0 || o->guess_rule > 2) {
        r2p_set_error("invalid Newton options");
        return R2P_EINVAL;
    }
    R2P_TRY(check_opts(&o->cpr));
    hipStream_t s = (hipStream_t)stream;
    // the workspace (Jacobian, CPR, vectors) belongs to the model
    if (!m->newton) {
        NewtonWork *W0 = new NewtonWork();
        W0->m = m;
        int rc = r2p_jacobian_create(m, &W0->J);
        if (!rc) rc = r2p_cpr_create(&W0->P);
        if (rc) { delete W0; return rc; }
        m->newton = W0;
    }
    NewtonWork *W = m->newton;
    long N = 2L * (m->ph.n + m->ph.nw);
    R2P_TRY(W->xold.ensure(N));
    R2P_TRY(W->xk.ensure(N));
    R2P_TRY(W->b.ensure(N));
    R2P_TRY(W->y.ensure(N));
    R2P_TRY(W->t.ensure(N));
    r2p_newton_info inf{};
    R2P_HIP(hipMemcpyAsync(W->xold.p, x, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    R2P_HIP(hipMemcpyAsync(W->xk.p, x, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    Krylov &K = krylov_for(W->P);
    R2P_TRY(K.h.ensure(MAXV));
    R2P_TRY(pin_ensure(K, sizeof(double) * (MAXG > MAXV ? MAXG : MAXV) * 2));
    if (x_guess) {
        double ng = 0.0, n0 = 0.0, hb[2];
        int rc = 0;
        bool take = o->guess_rule == R2P_GUESS_TRY;
        if (!take) {
            R2P_TRY(r2p_assemble_jacobian(m, x_guess, W->xold.p, dt, W->J, W->b.p, stream));
            if (o->guess_rule == R2P_GUESS_L2) {
                R2P_TRY(mdot(K, nullptr, 0, W->b.p, N, s, hb));
                ng = hb[0];
                rc = ng == ng ? 0 : R2P_ENAN;
            } else {
                rc = r2p_residual_norm(m, W->b.p, dt, &ng, stream);
            }
            R2P_TRY(r2p_assemble_jacobian(m, x, W->xold.p, dt, W->J, W->b.p, stream));
            if (o->guess_rule == R2P_GUESS_L2) {
                R2P_TRY(mdot(K, nullptr, 0, W->b.p, N, s, hb));
                n0 = hb[0];
            } else {
                R2P_TRY(r2p_residual_norm(m, W->b.p, dt, &n0, stream));
            }
            take = rc == 0 && ng < n0;
        }
        if (take) {
            R2P_HIP(hipMemcpyAsync(W->xk.p, x_guess, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
            inf.used_guess = 1;
        }
    }
    int status = R2P_NOT_CONVERGED;
    R2P_TRY(newton_loop(W, K, m, dt, o, N, s, inf, status));
    if (status != 0 && inf.used_guess) {
        // the learned start did not converge: start again from x^n
        R2P_HIP(hipMemcpyAsync(W->xk.p, x, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
        inf.used_guess = 0;
        R2P_TRY(newton_loop(W, K, m, dt, o, N, s, inf, status));
    }
    if (status == 0)
        R2P_HIP(hipMemcpyAsync(x, W->xk.p, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    R2P_HIP(hipStreamSynchronize(s));
    inf.status = status;
    inf.ms_total = now_ms() - T0;
    if (info) *info = inf;
    return status;
}
