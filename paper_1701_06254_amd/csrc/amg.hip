// Aggregation AMG on the pressure block A_pp (the M(A_pp)^-1 stage of the
// "Multi-stage preconditioner", Algorithm 2, with restriction Pi_r of Eq 34).
//
// The paper names AMG without fixing a variant.  Reading used here:
// strength -a_ij >= theta * max_{k!=i}(-a_ik) with -a_ij > 0; pairwise
// matching by handshakes (each unmatched row proposes its strongest
// unmatched strong neighbour, ties to the smaller index; mutual proposals
// pair up; `match_rounds` rounds); rows still unmatched join the pair of
// their strongest strong neighbour that is in a pair, else stay singletons;
// aggregates numbered by their leader (smaller row of the pair or the singleton); `agg_passes` passes per
// level, each on the Galerkin product of the previous one; piecewise-constant
// prolongation and Galerkin coarse matrices summed in ascending fine row and
// stored column order; l1-Jacobi smoothing (d_i = sum_j |a_ij|), one sweep
// before and after the coarse correction; V-cycle; the coarsest level is
// solved with its explicit inverse, computed once per set-up by dense LU
// with partial pivoting in FP64.
//
// Every set-up decision (strength, matching, joins, numbering) is integer
// work on values summed in a fixed order, so the hierarchy is reproducible.
// Compiled without floating-point contraction.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "r2p_impl.h"

constexpr int BS = 256;
constexpr int G = 4;                // lanes per row of the coarse-level row kernels
constexpr int KO_BLOCKS = 1024;     // grid of the K-cycle orthogonalisation pass

// ------------------------------------------------------- level 0 = A_pp
__global__ void k_app_count(Phys P, int *cnt) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= P.n) return;
    int nxy = P.nx * P.ny;
    int i = c % P.nx, j = (c / P.nx) % P.ny, k = c / nxy;
    cnt[c] = 1 + (i > 0) + (i + 1 < P.nx) + (j > 0) + (j + 1 < P.ny) + (k > 0) + (k + 1 < P.nz);
}

__global__ void k_app_cols(Phys P, const int *rp, int *col, int *slot) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= P.n) return;
    int nxy = P.nx * P.ny;
    int i = c % P.nx, j = (c / P.nx) % P.ny, k = c / nxy;
    int z = rp[c];
    const int order[7] = {5, 3, 1, 0, 2, 4, 6};
    bool ex[7] = {true, i > 0, i + 1 < P.nx, j > 0, j + 1 < P.ny, k > 0, k + 1 < P.nz};
    for (int oi = 0; oi < 7; oi++) {
        int sl = order[oi];
        if (!ex[sl]) continue;
        col[z] = c + slot_offset(sl, P.nx, nxy);
        slot[z] = sl;
        z++;
    }
}

__global__ void k_app_vals(int n, const int *rp, const int *slot, const double2 *vp, double *val) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    for (int z = rp[c]; z < rp[c + 1]; z++) val[z] = vp[(long)slot[z] * n + c].x;
}

// The same level-0 operator in the 7-slot stencil layout of the Jacobian
// (absent neighbours hold 0), for the coalesced level-0 cycle kernels.
__global__ void k_app_v7(int n, const double2 *vp, double *v7) {
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t < 7L * n) v7[t] = vp[t].x;
}

// Rows of a CSR-like structure longer than a threshold: next-level rows with
// more than BIG members (restricted by a wavefront), and matrix rows with
// more than HEAVY entries (smoothed by a wavefront).  Aggregates that
// absorbed many unmatched rows make a few coarse rows hundreds of entries
// long; one thread per row would serialise the whole launch on them.
constexpr int BIG = 16;
constexpr int HEAVY = 32;
__global__ void k_long_flag(int n, const int *ptr, int thr, int *flag) {
    int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I < n) flag[I] = ptr[I + 1] - ptr[I] > thr;
    if (I == n) flag[I] = 0;
}

__global__ void k_long_list(int n, const int *ptr, int thr, const int *scan, int *list) {
    int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I < n && ptr[I + 1] - ptr[I] > thr) list[scan[I]] = I;
}

// ------------------------------------------------------------- matching
// The row scans below give a group of GS lanes to each row: lanes stride over
// the row's entries (ascending within a lane), then a butterfly combines the
// lanes.  The reductions are exact (a maximum, or the strongest column with
// ties to the smaller column, which is what a scan in ascending column order
// keeps), so the result equals the sequential one bit for bit.
constexpr int GS = 8;

__device__ __forceinline__ void row_group(int n, int &i, int &g) {
    i = blockIdx.x * (blockDim.x / GS) + (int)threadIdx.x / GS;
    g = threadIdx.x % GS;
    (void)n;
}

// (s, j) replaced by (s2, j2) when that is stronger, or as strong with a
// smaller column (j = -1: none).
__device__ __forceinline__ void take_stronger(double &s, int &j, double s2, int j2) {
    if (j2 >= 0 && (j < 0 || s2 > s || (s2 == s && j2 < j))) { s = s2; j = j2; }
}

// a_ji by binary search of row j (columns ascend), 0 when j stores no i.
__device__ __forceinline__ double entry_of(const int *rp, const int *col, const double *val, int j,
                                           int i) {
    int lo = rp[j], hi = rp[j + 1];
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        int c = col[mid];
        if (c == i) return val[mid];
        if (c < i) lo = mid + 1;
        else hi = mid;
    }
    return 0.0;
}

// Coupling weights w[z] = -(a_ij + a_ji)/2 of every stored off-diagonal
// entry z = (i, j) (0 on the diagonal), the same number from either row,
// and M_i = max(0, max_j w_ij).
__global__ void k_weights(int n, const int *rp, const int *col, const double *val, double *w,
                          double *M, int *match) {
    int i, g;
    row_group(n, i, g);
    if (i >= n) return;                        // whole groups leave together
    double mx = 0.0;
    for (int z = rp[i] + g; z < rp[i + 1]; z += GS) {
        int j = col[z];
        double wz = 0.0;
        if (j != i) wz = -(val[z] + entry_of(rp, col, val, j, i)) / 2.0;
        w[z] = wz;
        if (wz > mx) mx = wz;
    }
    for (int d = 1; d < GS; d <<= 1) mx = fmax(mx, __shfl_xor(mx, d, 64));
    if (g == 0) {
        M[i] = mx;
        match[i] = -1;
    }
}

// The symmetric strength relation: w_ij > 0 and w_ij reaches theta of the
// largest weight of row i or of row j.
__device__ __forceinline__ bool strong_pair(double wij, double Mi, double Mj, double theta) {
    return wij > 0.0 && (wij >= theta * Mi || wij >= theta * Mj);
}

// Strongest strong neighbour j of an unmatched row i with match[j] < 0
// (propose) or >= 0 (join), ties to the smaller column; -1 if none.
template <bool JOIN>
__device__ __forceinline__ void strongest(int n, const int *rp, const int *col, const double *w,
                                          const double *M, double theta, const int *match,
                                          int *out) {
    int i, g;
    row_group(n, i, g);
    if (i >= n) return;
    double best = 0.0;
    int best_j = -1;
    if (match[i] < 0) {
        double Mi = M[i];
        for (int z = rp[i] + g; z < rp[i + 1]; z += GS) {
            int j = col[z];
            double s = w[z];
            bool free_j = match[j] < 0;
            if (j == i || free_j == JOIN || !strong_pair(s, Mi, M[j], theta)) continue;
            if (s > best) { best = s; best_j = j; }
        }
    }
    for (int d = 1; d < GS; d <<= 1) {
        double s2 = __shfl_xor(best, d, 64);
        int j2 = __shfl_xor(best_j, d, 64);
        take_stronger(best, best_j, s2, j2);
    }
    if (g == 0) out[i] = best_j;
}

__global__ void k_propose(int n, const int *rp, const int *col, const double *w, const double *M,
                          double theta, const int *match, int *prop) {
    strongest<false>(n, rp, col, w, M, theta, match, prop);
}

__global__ void k_accept(int n, const int *prop, int *match) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int j = prop[i];
    if (match[i] < 0 && j >= 0 && prop[j] == i) match[i] = j;
}

// Unmatched rows: strongest strong neighbour that is in a pair (or -1).
__global__ void k_join(int n, const int *rp, const int *col, const double *w, const double *M,
                       double theta, const int *match, int *jt) {
    strongest<true>(n, rp, col, w, M, theta, match, jt);
}

__global__ void k_leader_flag(int n, const int *match, const int *jt, int *flag) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int j = match[i];
    flag[i] = (j >= 0 && i < j) || (j < 0 && jt[i] < 0);
}

__global__ void k_number(int n, const int *match, const int *jt, const int *cid, int *agg) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int j = match[i];
    int lead;
    if (j >= 0) lead = i < j ? i : j;
    else if (jt[i] < 0) lead = i;
    else {
        int k = jt[i];
        int mk = match[k];
        lead = k < mk ? k : mk;
    }
    agg[i] = cid[lead];
}

// Composition of a pass with the aggregation so far: agg[i] <- a[agg[i]].
__global__ void k_compose(int n, const int *a, int *agg) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) agg[i] = a[agg[i]];
}

__global__ void k_iota(int n, int *a) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = i;
}

// Member lists (CSR) of the aggregates, ascending within each list: the
// rows are stably sorted by aggregate, then every list start is marked.
__global__ void k_member_keys(int n, const int *agg, unsigned *key, unsigned *val) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) { key[i] = (unsigned)agg[i]; val[i] = (unsigned)i; }
}

__global__ void k_member_ptr(int n, int nc, const unsigned *key, int *mptr) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n && (k == 0 || key[k] != key[k - 1])) mptr[key[k]] = k;
    if (k == 0) mptr[nc] = n;
}

// ------------------------------------------------------------- Galerkin
// A_c = P^T A P by expand-sort-compress: every stored entry a_ij becomes the
// term (agg(i), agg(j), a_ij); the terms are stably sorted by coarse column
// and then by coarse row, so equal (I, J) terms stay in ascending (row,
// stored column) order and are summed in that order.
__global__ void k_gal_expand(int n, const int *rp, const int *agg, unsigned *keyI,
                             const int *col, unsigned *keyJ, unsigned *idx) {
    int i, g;
    row_group(n, i, g);
    if (i >= n) return;
    unsigned I = (unsigned)agg[i];
    for (int z = rp[i] + g; z < rp[i + 1]; z += GS) {
        keyI[z] = I;
        keyJ[z] = (unsigned)agg[col[z]];
        idx[z] = (unsigned)z;
    }
}

__global__ void k_gather_u(int m, const unsigned *idx, const unsigned *src, unsigned *dst) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) dst[k] = src[idx[k]];
}

// keyI, keyJ: the terms' coarse rows and columns in sorted order.
__global__ void k_gal_flags(int m, const unsigned *keyI, const unsigned *keyJ, int *flag) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    bool f = k == 0;
    if (!f) f = keyI[k] != keyI[k - 1] || keyJ[k] != keyJ[k - 1];
    flag[k] = f;
}

// The first term of every run of equal (I, J) records where its run starts;
// the run of output entry u is then [start[u], start[u + 1]).
__global__ void k_gal_runs(int m, int nc, const unsigned *keyI, const unsigned *keyJ,
                           const int *uidx, int *start, int *rpc, int nnzc) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0) { rpc[nc] = nnzc; start[nnzc] = m; }
    if (k >= m) return;
    bool first = k == 0 || keyI[k] != keyI[k - 1] || keyJ[k] != keyJ[k - 1];
    if (!first) return;
    start[uidx[k]] = k;
    if (k == 0 || keyI[k - 1] != keyI[k]) rpc[keyI[k]] = uidx[k];
}

// One thread per coarse entry: its terms summed in sorted order (ascending
// fine row, then stored column), four terms' loads in flight at a time.
__global__ void k_gal_sum(int nnzc, const int *start, const unsigned *idx, const unsigned *keyJ,
                          const double *val, int *colc, double *valc) {
    int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= nnzc) return;
    int a = start[u], b = start[u + 1];
    double s = 0.0;
    int t = a;
    for (; t + 4 <= b; t += 4) {
        unsigned i0 = idx[t], i1 = idx[t + 1], i2 = idx[t + 2], i3 = idx[t + 3];
        double v0 = val[i0], v1 = val[i1], v2 = val[i2], v3 = val[i3];
        s += v0;
        s += v1;
        s += v2;
        s += v3;
    }
    for (; t < b; t++) s += val[idx[t]];
    colc[u] = (int)keyJ[a];
    valc[u] = s;
}

__global__ void k_l1(int n, const int *rp, const double *val, double *l1) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int z = rp[i]; z < rp[i + 1]; z++) s += fabs(val[z]);
    l1[i] = s;
}

template <class T>
__global__ void k_castv(long n, const double *a, T *b) {
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) b[i] = (T)a[i];
}

// ------------------------------------------------------------- coarsest
__global__ void k_to_dense(int n, const int *rp, const int *col, const double *val, double *a) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int j = 0; j < n; j++) a[(long)i * n + j] = 0.0;
    for (int z = rp[i]; z < rp[i + 1]; z++) a[(long)i * n + col[z]] += val[z];
}

// LU with partial pivoting (largest magnitude, ties to the smaller row) by
// one workgroup, in place (unit L below the diagonal, U on and above).
__global__ __launch_bounds__(1024) void k_dense_lu(int n, double *a, int *piv, int *status) {
    __shared__ double sv[1024];
    __shared__ int si[1024];
    int tid = threadIdx.x, nt = blockDim.x;
    for (int k = 0; k < n; k++) {
        double best = -1.0;
        int bi = n;
        for (int i = k + tid; i < n; i += nt) {
            double v = fabs(a[(long)i * n + k]);
            if (v > best || (v == best && i < bi)) { best = v; bi = i; }
        }
        sv[tid] = best;
        si[tid] = bi;
        __syncthreads();
        for (int w = nt / 2; w > 0; w >>= 1) {
            if (tid < w) {
                double v = sv[tid + w];
                int ii = si[tid + w];
                if (v > sv[tid] || (v == sv[tid] && ii < si[tid])) { sv[tid] = v; si[tid] = ii; }
            }
            __syncthreads();
        }
        int p = si[0];
        double pv = sv[0];
        __syncthreads();
        if (tid == 0) piv[k] = p;
        if (pv == 0.0 || pv != pv) {
            if (tid == 0) *status = 1;
            return;
        }
        if (p != k)
            for (int j = tid; j < n; j += nt) {
                double t = a[(long)k * n + j];
                a[(long)k * n + j] = a[(long)p * n + j];
                a[(long)p * n + j] = t;
            }
        __syncthreads();
        double inv = 1.0 / a[(long)k * n + k];
        for (int i = k + 1 + tid; i < n; i += nt) a[(long)i * n + k] = a[(long)i * n + k] * inv;
        __syncthreads();
        long rem = (long)(n - k - 1) * (n - k - 1);
        for (long t = tid; t < rem; t += nt) {
            int i = k + 1 + (int)(t / (n - k - 1)), j = k + 1 + (int)(t % (n - k - 1));
            double l = a[(long)i * n + k];
            if (l != 0.0) a[(long)i * n + j] -= l * a[(long)k * n + j];
        }
        __syncthreads();
    }
}

// Column c of the inverse from the LU factors, one wavefront per column:
// x = P e_c, then the unit-lower and upper triangular solves, each row's
// inner product split over the lanes (row i of the factors is read by every
// column's wavefront, so it is served from L2) and summed by a fixed
// butterfly.  Written column-major, invT[c*n + i] = (A^-1)_ic, so the
// coarse solve reads it coalesced.
__global__ __launch_bounds__(64) void k_dense_inv_col(int n, const double *a, const int *piv,
                                                      const int *status, double *invT) {
    extern __shared__ double xs[];
    if (*status) return;             // singular: the factors are incomplete
    int c = blockIdx.x, lane = threadIdx.x;
    for (int i = lane; i < n; i += 64) xs[i] = i == c ? 1.0 : 0.0;
    __syncthreads();
    if (lane == 0)
        for (int k = 0; k < n; k++) {
            int p = piv[k];
            if (p != k && p >= 0 && p < n) {
                double t = xs[k];
                xs[k] = xs[p];
                xs[p] = t;
            }
        }
    __syncthreads();
    for (int i = 1; i < n; i++) {
        double s = 0.0;
        for (int j = lane; j < i; j += 64) s += a[(long)i * n + j] * xs[j];
        for (int d = 32; d > 0; d >>= 1) s += __shfl_xor(s, d, 64);
        __syncthreads();
        if (lane == 0) xs[i] -= s;
        __syncthreads();
    }
    for (int i = n - 1; i >= 0; i--) {
        double s = 0.0;
        for (int j = i + 1 + lane; j < n; j += 64) s += a[(long)i * n + j] * xs[j];
        for (int d = 32; d > 0; d >>= 1) s += __shfl_xor(s, d, 64);
        __syncthreads();
        if (lane == 0) xs[i] = (xs[i] - s) / a[(long)i * n + i];
        __syncthreads();
    }
    for (int i = lane; i < n; i += 64) invT[(long)c * n + i] = xs[i];
}

// --------------------------------------------------------------- set-up
// Everything runs in order on one stream; the host waits only where it
// needs a count (the scans that return totals) and for the final status.
// Member lists (CSR, ascending) of the nc aggregates of agg[0..n).
static int build_members(r2p_cpr *P, int n, const int *agg, int nc, DBuf<int> &mptr,
                         DBuf<int> &mem, hipStream_t s) {
    SetupWork &W = P->aws;
    DBuf<unsigned> &key = W.u[0], &kt = W.u[1], &vt = W.u[2];
    DBuf<int> &hist = W.i[0];
    R2P_TRY(mptr.ensure(nc + 1));
    R2P_TRY(mem.ensure(n));
    R2P_TRY(key.ensure(n));
    R2P_TRY(kt.ensure(n));
    R2P_TRY(vt.ensure(n));
    unsigned *val = (unsigned *)mem.p;
    k_member_keys<<<r2p_blocks(n, BS), BS, 0, s>>>(n, agg, key.p, val);
    R2P_LAUNCH();
    R2P_TRY(r2p_sort_pairs(key.p, val, kt.p, vt.p, n, r2p_bits_for(nc), hist, P->aiscratch,
                           P->apin, s));
    k_member_ptr<<<r2p_blocks(n, BS), BS, 0, s>>>(n, nc, key.p, mptr.p);
    R2P_LAUNCH();
    return 0;
}

static int galerkin(r2p_cpr *P, int n, int nnz, const int *rp, const int *col, const double *val,
                    const int *agg, int nc, DBuf<int> &rpc, DBuf<int> &colc, DBuf<double> &valc,
                    int *nnzc, hipStream_t s) {
    SetupWork &W = P->aws;
    DBuf<unsigned> &keyI = W.u[0], &keyJz = W.u[1], &keyIs = W.u[2], &idx = W.u[3], &kt = W.u[4],
                   &vt = W.u[5];
    DBuf<int> &flag = W.i[0], &hist = W.i[1];
    R2P_TRY(keyI.ensure(nnz));
    R2P_TRY(keyJz.ensure(nnz));
    R2P_TRY(keyIs.ensure(nnz));
    R2P_TRY(idx.ensure(nnz));
    R2P_TRY(kt.ensure(nnz));
    R2P_TRY(vt.ensure(nnz));
    R2P_TRY(flag.ensure(nnz + 1));
    k_gal_expand<<<r2p_blocks(n, BS / GS), BS, 0, s>>>(n, rp, agg, keyI.p, col, keyJz.p, idx.p);
    R2P_LAUNCH();
    int bits = r2p_bits_for(nc);
    // stable by coarse column, then stable by coarse row
    R2P_HIP(hipMemcpyAsync(kt.p, keyJz.p, sizeof(unsigned) * nnz, hipMemcpyDeviceToDevice, s));
    R2P_HIP(hipMemcpyAsync(keyIs.p, kt.p, sizeof(unsigned) * nnz, hipMemcpyDeviceToDevice, s));
    R2P_TRY(r2p_sort_pairs(keyIs.p, idx.p, kt.p, vt.p, nnz, bits, hist, P->aiscratch, P->apin, s));
    k_gather_u<<<r2p_blocks(nnz, BS), BS, 0, s>>>(nnz, idx.p, keyI.p, keyIs.p);
    R2P_LAUNCH();
    R2P_TRY(r2p_sort_pairs(keyIs.p, idx.p, kt.p, vt.p, nnz, bits, hist, P->aiscratch, P->apin, s));
    // the coarse columns in sorted order, gathered once (kt is free again)
    k_gather_u<<<r2p_blocks(nnz, BS), BS, 0, s>>>(nnz, idx.p, keyJz.p, kt.p);
    R2P_LAUNCH();
    k_gal_flags<<<r2p_blocks(nnz, BS), BS, 0, s>>>(nnz, keyIs.p, kt.p, flag.p);
    R2P_LAUNCH();
    R2P_HIP(hipMemsetAsync(flag.p + nnz, 0, sizeof(int), s));
    int nnz_c = 0;
    R2P_TRY(r2p_scan_int(flag.p, flag.p, nnz + 1, &nnz_c, P->aiscratch, P->apin, s));
    R2P_TRY(rpc.ensure(nc + 1));
    R2P_TRY(colc.ensure(nnz_c));
    R2P_TRY(valc.ensure(nnz_c));
    DBuf<int> &start = W.i[2];
    R2P_TRY(start.ensure(nnz_c + 1));
    k_gal_runs<<<r2p_blocks(nnz, BS), BS, 0, s>>>(nnz, nc, keyIs.p, kt.p, flag.p, start.p, rpc.p,
                                                 nnz_c);
    R2P_LAUNCH();
    k_gal_sum<<<r2p_blocks(nnz_c, BS), BS, 0, s>>>(nnz_c, start.p, idx.p, kt.p, val, colc.p,
                                                   valc.p);
    R2P_LAUNCH();
    *nnzc = nnz_c;
    return 0;
}

// One aggregation pass: agg (row -> aggregate) and the aggregate count.
static int aggregate_pass(r2p_cpr *P, int n, int nnz, const int *rp, const int *col,
                          const double *val, DBuf<int> &agg, int *nc, hipStream_t s) {
    SetupWork &W = P->aws;
    DBuf<double> &M = W.d[0], &wgt = W.d[1];
    DBuf<int> &match = W.i[0], &prop = W.i[1], &flag = W.i[2], &jt = W.i[3];
    R2P_TRY(M.ensure(n));
    R2P_TRY(wgt.ensure(nnz));
    R2P_TRY(match.ensure(n));
    R2P_TRY(prop.ensure(n));
    R2P_TRY(jt.ensure(n));
    R2P_TRY(flag.ensure(n + 1));
    int nb = r2p_blocks(n, BS), ng = r2p_blocks(n, BS / GS);
    double th = P->o.theta;
    k_weights<<<ng, BS, 0, s>>>(n, rp, col, val, wgt.p, M.p, match.p);
    R2P_LAUNCH();
    for (int r = 0; r < P->o.match_rounds; r++) {
        k_propose<<<ng, BS, 0, s>>>(n, rp, col, wgt.p, M.p, th, match.p, prop.p);
        R2P_LAUNCH();
        k_accept<<<nb, BS, 0, s>>>(n, prop.p, match.p);
        R2P_LAUNCH();
    }
    k_join<<<ng, BS, 0, s>>>(n, rp, col, wgt.p, M.p, th, match.p, jt.p);
    R2P_LAUNCH();
    k_leader_flag<<<nb, BS, 0, s>>>(n, match.p, jt.p, flag.p);
    R2P_LAUNCH();
    R2P_HIP(hipMemsetAsync(flag.p + n, 0, sizeof(int), s));
    int cnt = 0;
    R2P_TRY(r2p_scan_int(flag.p, flag.p, n + 1, &cnt, P->aiscratch, P->apin, s));
    R2P_TRY(agg.ensure(n));
    k_number<<<nb, BS, 0, s>>>(n, match.p, jt.p, flag.p, agg.p);
    R2P_LAUNCH();
    *nc = cnt;
    return 0;
}

// List (ascending) of the rows i < n with ptr[i+1] - ptr[i] > thr.
static int long_rows(r2p_cpr *P, int n, const int *ptr, int thr, DBuf<int> &list, int *count,
                     hipStream_t s) {
    DBuf<int> &flag = P->aws.i[0];
    R2P_TRY(flag.ensure(n + 1));
    k_long_flag<<<r2p_blocks(n + 1, BS), BS, 0, s>>>(n, ptr, thr, flag.p);
    R2P_LAUNCH();
    int cnt = 0;
    R2P_TRY(r2p_scan_int(flag.p, flag.p, n + 1, &cnt, P->aiscratch, P->apin, s));
    R2P_TRY(list.ensure(cnt));
    k_long_list<<<r2p_blocks(n, BS), BS, 0, s>>>(n, ptr, thr, flag.p, list.p);
    R2P_LAUNCH();
    *count = cnt;
    return 0;
}

int r2p_amg_setup(r2p_cpr *P, hipStream_t s) {
    r2p_jacobian *J = P->J;
    const Phys &ph = J->m->ph;
    int n = ph.n;
    AmgLevel &L0 = P->lv[0];
    // level 0 structure (static per model)
    if (P->app_n != n) {
        R2P_TRY(L0.rp.ensure(n + 1));
        k_app_count<<<r2p_blocks(n, BS), BS, 0, s>>>(ph, L0.rp.p);
        R2P_LAUNCH();
        R2P_HIP(hipMemsetAsync(L0.rp.p + n, 0, sizeof(int), s));
        int nnz = 0;
        R2P_TRY(r2p_scan_int(L0.rp.p, L0.rp.p, n + 1, &nnz, P->aiscratch, P->apin, s));
        R2P_TRY(L0.col.ensure(nnz));
        R2P_TRY(P->iscratch2.ensure(nnz));
        k_app_cols<<<r2p_blocks(n, BS), BS, 0, s>>>(ph, L0.rp.p, L0.col.p, P->iscratch2.p);
        R2P_LAUNCH();
        L0.n = n;
        L0.nnz = nnz;
        P->app_n = n;
    }
    R2P_TRY(L0.val.ensure(L0.nnz));
    k_app_vals<<<r2p_blocks(n, BS), BS, 0, s>>>(n, L0.rp.p, P->iscratch2.p, J->vp.p, L0.val.p);
    R2P_LAUNCH();
    R2P_TRY(L0.v7.ensure(7L * n));
    k_app_v7<<<r2p_blocks(7L * n, BS), BS, 0, s>>>(n, J->vp.p, L0.v7.p);
    R2P_LAUNCH();
    if (P->o.precision == R2P_FP32) {
        R2P_TRY(L0.v7f.ensure(7L * n));
        k_castv<float><<<r2p_blocks(7L * n, BS), BS, 0, s>>>(7L * n, L0.v7.p, L0.v7f.p);
        R2P_LAUNCH();
    }
    int maxlev = std::min(std::max(P->o.max_levels, 1), 24);
    int passes = std::max(P->o.agg_passes, 1);
    int l = 0;
    while (P->lv[l].n > P->o.max_coarse && l + 1 < maxlev) {
        AmgLevel &A = P->lv[l];
        AmgLevel &C = P->lv[l + 1];
        R2P_TRY(A.agg.ensure(A.n));
        k_iota<<<r2p_blocks(A.n, BS), BS, 0, s>>>(A.n, A.agg.p);
        R2P_LAUNCH();
        // successive passes, each on the Galerkin product of the previous one
        DBuf<int> *crp = P->aws.crp, *ccol = P->aws.ccol;
        DBuf<double> *cval = P->aws.cval;
        const int *rp = A.rp.p, *col = A.col.p;
        const double *val = A.val.p;
        int cn = A.n, nc = A.n, nnzc = 0, cnnz = A.nnz;
        for (int p = 0; p < passes; p++) {
            DBuf<int> &a = P->aws.agg;
            R2P_TRY(aggregate_pass(P, cn, cnnz, rp, col, val, a, &nc, s));
            bool last = p == passes - 1;
            DBuf<int> &orp = last ? C.rp : crp[p & 1];
            DBuf<int> &ocol = last ? C.col : ccol[p & 1];
            DBuf<double> &oval = last ? C.val : cval[p & 1];
            R2P_TRY(galerkin(P, cn, cnnz, rp, col, val, a.p, nc, orp, ocol, oval, &nnzc, s));
            cnnz = nnzc;
            k_compose<<<r2p_blocks(A.n, BS), BS, 0, s>>>(A.n, a.p, A.agg.p);
            R2P_LAUNCH();
            rp = orp.p; col = ocol.p; val = oval.p;
            cn = nc;
        }
        if (nc >= A.n) break;   // no coarsening progress
        C.n = nc;
        C.nnz = nnzc;
        R2P_TRY(build_members(P, A.n, A.agg.p, nc, A.mptr, A.mem, s));
        R2P_TRY(long_rows(P, nc, A.mptr.p, BIG, A.big, &A.nbig, s));
        R2P_TRY(long_rows(P, nc, C.rp.p, HEAVY, C.heavy, &C.nheavy, s));
        l++;
    }
    P->nlev = l + 1;
    bool f32 = P->o.precision == R2P_FP32;
    for (int k = 0; k < P->nlev; k++) {
        AmgLevel &A = P->lv[k];
        R2P_TRY(A.l1.ensure(A.n));
        k_l1<<<r2p_blocks(A.n, BS), BS, 0, s>>>(A.n, A.rp.p, A.val.p, A.l1.p);
        R2P_LAUNCH();
        if (f32) {
            R2P_TRY(A.f32.val.ensure(A.nnz));
            R2P_TRY(A.f32.l1.ensure(A.n));
            R2P_TRY(A.bf.ensure(A.n));
            R2P_TRY(A.xf.ensure(A.n));
            R2P_TRY(A.xof.ensure(A.n));
            k_castv<float><<<r2p_blocks(A.nnz, BS), BS, 0, s>>>(A.nnz, A.val.p, A.f32.val.p);
            R2P_LAUNCH();
            k_castv<float><<<r2p_blocks(A.n, BS), BS, 0, s>>>(A.n, A.l1.p, A.f32.l1.p);
            R2P_LAUNCH();
        }
        R2P_TRY(A.b.ensure(A.n));
        R2P_TRY(A.x.ensure(A.n));
        R2P_TRY(A.xo.ensure(A.n));
        // K-cycle work vectors on the levels whose systems the K-cycle solves
        if (k >= 1 && k <= P->o.kcycle && k < P->nlev - 1) {
            if (f32) R2P_TRY(A.kvf.ensure(4L * A.n));
            else R2P_TRY(A.kv.ensure(4L * A.n));
            // partial pairs of the K-cycle products on this level (and of the
            // orthogonalisation pass, KO_BLOCKS at most)
            long nbk = r2p_blocks(A.n, BS / G) + r2p_blocks(A.nheavy, BS / 64);
            R2P_TRY(P->kpart.ensure(2 * std::max(nbk, (long)KO_BLOCKS)));
        }
    }
    R2P_TRY(P->kscal.ensure(4 * 24));
    // coarsest level: dense LU and inverse (FP64)
    AmgLevel &C = P->lv[P->nlev - 1];
    int nc = C.n;
    if (nc > 4096) {
        // coarsening stalled: a soft failure of the method (no dense solve of that size)
        r2p_set_error("AMG coarsening stalled: coarsest level of %d rows", nc);
        return R2P_NOT_CONVERGED;
    }
    P->ncoarse = nc;
    R2P_TRY(P->lu.ensure((size_t)nc * nc));
    R2P_TRY(P->cinv.ensure((size_t)nc * nc));
    R2P_TRY(P->piv.ensure(nc));
    R2P_TRY(P->astatus.ensure(1));
    R2P_TRY(P->apin.ensure(64));
    R2P_HIP(hipMemsetAsync(P->astatus.p, 0, sizeof(int), s));
    k_to_dense<<<r2p_blocks(nc, BS), BS, 0, s>>>(nc, C.rp.p, C.col.p, C.val.p, P->lu.p);
    R2P_LAUNCH();
    k_dense_lu<<<1, 1024, 0, s>>>(nc, P->lu.p, P->piv.p, P->astatus.p);
    R2P_LAUNCH();
    k_dense_inv_col<<<nc, 64, sizeof(double) * nc, s>>>(nc, P->lu.p, P->piv.p, P->astatus.p,
                                                          P->cinv.p);
    R2P_LAUNCH();
    int *h = (int *)P->apin.p;
    R2P_HIP(hipMemcpyAsync(h, P->astatus.p, sizeof(int), hipMemcpyDeviceToHost, s));
    R2P_HIP(hipStreamSynchronize(s));
    if (*h) { r2p_set_error("coarsest AMG matrix is singular"); return R2P_ESINGULAR; }
    return 0;
}

// --------------------------------------------------------------- V-cycle
// Levels below the finest are CSR.  A group of G lanes takes one row (lanes
// stride over its entries two at a time, both requested before either is
// used, then a fixed butterfly), so a wavefront reads the entries of 64 / G
// consecutive rows contiguously; with about 8 entries per row every lane
// issues its loads at once.  Rows longer than HEAVY get a wavefront each in
// trailing workgroups, four entries per lane in flight.  The iterate every
// row reads is formed beforehand: the pre-smoothed x = b / d by the
// restriction that produces b, and the prolonged x + P xc by a pass over the
// fine rows, so each entry costs one gather.

template <class T>
struct CsrArgs {
    int n, nbs;                  // rows; workgroups of the G-lanes-per-row part
    const int *heavy;            // rows longer than HEAVY, one wavefront each
    int nheavy;
    const int *rp, *col;
    const T *val, *l1;
    const T *b;                  // right-hand side of this level
    const T *x;                  // iterate: pre-smoothed (down), prolonged (up)
    T *xo;                       // down: residual b - A x; up: x + (b - A x) / d
};

// MODE: CSR_DOWN xo = b - A x; CSR_UP xo = x + (b - A x) / d; CSR_PRODUCT xo = A x.
enum { CSR_DOWN = 0, CSR_UP = 1, CSR_PRODUCT = 2 };
template <class T, int MODE>
__global__ __launch_bounds__(256) void k_csr_level(CsrArgs<T> A) {
    int i, lane0;
    T acc = (T)0;
    if ((int)blockIdx.x < A.nbs) {
        i = xcd_block(blockIdx.x, A.nbs) * (blockDim.x / G) + (int)threadIdx.x / G;
        lane0 = threadIdx.x % G;
        if (i >= A.n) return;                 // whole groups leave together
        int z0 = A.rp[i], z1 = A.rp[i + 1];
        if (z1 - z0 > HEAVY) return;
        for (int z = z0 + lane0; z < z1; z += 2 * G) {
            int zb = z + G < z1 ? z + G : z;
            int ca = A.col[z], cb = A.col[zb];
            T va = A.val[z], vb = A.val[zb];
            T xa = A.x[ca], xb = A.x[cb];
            acc += va * xa + (z + G < z1 ? vb * xb : (T)0);
        }
#pragma unroll
        for (int d = 1; d < G; d <<= 1) acc += __shfl_xor(acc, d, 64);
    } else {
        int w = ((int)blockIdx.x - A.nbs) * (blockDim.x >> 6) + (threadIdx.x >> 6);
        if (w >= A.nheavy) return;
        lane0 = threadIdx.x & 63;
        i = A.heavy[w];
        int z0 = A.rp[i], z1 = A.rp[i + 1];
        for (int z = z0 + lane0; z < z1; z += 256) {
            T t[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                int zz = z + 64 * u < z1 ? z + 64 * u : z;
                T v = A.val[zz] * A.x[A.col[zz]];
                t[u] = z + 64 * u < z1 ? v : (T)0;
            }
            acc += (t[0] + t[1]) + (t[2] + t[3]);
        }
        for (int d = 1; d < 64; d <<= 1) acc += __shfl_xor(acc, d, 64);
    }
    if (lane0 == 0)
        A.xo[i] = MODE == CSR_UP ? A.x[i] + (A.b[i] - acc) / A.l1[i]
                                 : (MODE == CSR_DOWN ? A.b[i] - acc : acc);
}

// Restriction P^T r: a group of GR lanes per coarse row (lanes stride over
// the members two at a time, then a fixed butterfly; aggregates average 2-4
// members);
// aggregates with more than BIG members (up to about a thousand on the
// coarse levels) get a wavefront each in trailing workgroups, four members
// per lane in flight.  When the coarse level is smoothed (xc given), its
// pre-smoothed iterate b / d is formed here.
constexpr int GR = 2;
template <class T>
__global__ __launch_bounds__(256) void k_restrict(int nc, int nbs, const int *mptr, const int *mem,
                                                  const int *big, int nbig, const T *r, T *bc,
                                                  const T *l1c, T *xc) {
    int I, lane0;
    T acc = (T)0;
    if ((int)blockIdx.x < nbs) {
        I = blockIdx.x * (blockDim.x / GR) + (int)threadIdx.x / GR;
        lane0 = threadIdx.x % GR;
        if (I >= nc) return;
        int a = mptr[I], b = mptr[I + 1];
        if (b - a > BIG) return;
        // two members per lane in flight
        for (int t = a + lane0; t < b; t += 2 * GR) {
            int tb = t + GR < b ? t + GR : t;
            int ma = mem[t], mb = mem[tb];
            T ra = r[ma], rb = r[mb];
            acc += ra + (t + GR < b ? rb : (T)0);
        }
#pragma unroll
        for (int d = 1; d < GR; d <<= 1) acc += __shfl_xor(acc, d, 64);
    } else {
        int w = ((int)blockIdx.x - nbs) * (blockDim.x >> 6) + (threadIdx.x >> 6);
        if (w >= nbig) return;
        lane0 = threadIdx.x & 63;
        I = big[w];
        int a = mptr[I], b = mptr[I + 1];
        for (int t = a + lane0; t < b; t += 256) {
            T v[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                T rv = r[mem[t + 64 * u < b ? t + 64 * u : t]];
                v[u] = t + 64 * u < b ? rv : (T)0;
            }
            acc += (v[0] + v[1]) + (v[2] + v[3]);
        }
        for (int d = 1; d < 64; d <<= 1) acc += __shfl_xor(acc, d, 64);
    }
    if (lane0 == 0) {
        bc[I] = acc;
        if (xc) xc[I] = acc / l1c[I];
    }
}

// Prolongation of the coarse correction onto a fine level's iterate:
// x_j += xc[agg_j], one thread per fine row.
template <class T>
__global__ void k_prolong(int n, const int *agg, const T *xc, T *x) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) x[j] = x[j] + xc[agg[j]];
}

// Level 0 in the 7-slot layout: columns are implied by the grid (clamped at
// the boundary, where the coefficient is 0) and summed in ascending order.
template <class T>
struct Level0 {
    int n, nx, nxy;
    const T *v7, *l1;
    const double *f;
    int fstride;
};

template <class T>
__global__ void k_down0(Level0<T> A, T *x, T *r) {
    int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    const int order[7] = {5, 3, 1, 0, 2, 4, 6};
    T bi = (T)A.f[(long)A.fstride * i];
    x[i] = bi / A.l1[i];
    T s = bi;
#pragma unroll
    for (int oi = 0; oi < 7; oi++) {
        int sl = order[oi];
        int j = i + slot_offset(sl, A.nx, A.nxy);
        j = j < 0 ? 0 : (j >= A.n ? A.n - 1 : j);
        s -= ld_stream(&A.v7[(long)sl * A.n + i]) * ((T)A.f[(long)A.fstride * j] / A.l1[j]);
    }
    r[i] = s;
}

// Post-smoothing of level 0 on the prolonged iterate x (= x + P xc).
// With ACC the result is added to xo (xo = xo + result, as a separate
// addition would) instead of replacing it.
template <class T, bool ACC>
__global__ void k_up0(Level0<T> A, const T *x, double *xo) {
    int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    const int order[7] = {5, 3, 1, 0, 2, 4, 6};
    T s = (T)A.f[(long)A.fstride * i];
#pragma unroll
    for (int oi = 0; oi < 7; oi++) {
        int sl = order[oi];
        int j = i + slot_offset(sl, A.nx, A.nxy);
        j = j < 0 ? 0 : (j >= A.n ? A.n - 1 : j);
        s -= ld_stream(&A.v7[(long)sl * A.n + i]) * x[j];
    }
    double v = (double)(x[i] + s / A.l1[i]);
    xo[i] = ACC ? xo[i] + v : v;
}

// Coarsest solve x = A_c^-1 b with the stored inverse (column-major, so a
// column read by 64 lanes is contiguous).  A workgroup of CS_WAVES
// wavefronts covers 64 rows; wavefront w sums its quarter of the columns,
// then the quarters are added in wavefront order.
constexpr int CS_WAVES = 4;
template <class T>
__global__ __launch_bounds__(64 * CS_WAVES) void k_coarse_solve(int n, const double *invT,
                                                                const T *b, const double *f,
                                                                int fstride, T *x, double *xd) {
    __shared__ double part[CS_WAVES][64];
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int i = blockIdx.x * 64 + lane;
    int q = (n + CS_WAVES - 1) / CS_WAVES;
    int c0 = w * q, c1 = min(n, c0 + q);
    int ii = i < n ? i : n - 1;
    double s = 0.0;
#pragma unroll 8
    for (int c = c0; c < c1; c++) {
        double bc = f ? f[(long)fstride * c] : (double)b[c];
        s += invT[(long)c * n + ii] * bc;
    }
    part[w][lane] = s;
    __syncthreads();
    if (w != 0 || i >= n) return;
    double t = part[0][lane];
    for (int k = 1; k < CS_WAVES; k++) t += part[k][lane];
    if (xd) xd[i] = t;
    else x[i] = (T)t;
}

// ------------------------------------------------------------- K-cycle
// Two generalised-conjugate-residual steps on a coarse level c (the
// corrections of the `kcycle` finest levels): p1 = C(b), q1 = A p1,
// a1 = (q1.b)/(q1.q1), r = b - a1 q1; p2 = C(r), q2 = A p2,
// beta = (q1.q2)/(q1.q1), p2 -= beta p1, q2 -= beta q1, a2 = (q2.r)/(q2.q2);
// the correction a1 p1 + a2 p2 is added by the prolongation.  The scalars
// stay on the device: the kernels that produce q1, q2 and the orthogonalised
// q2 also write per-workgroup partial sums of the dot products they feed,
// and one small workgroup adds the partials in workgroup order and forms
// the scalar, so nothing is read back and the sums do not depend on
// scheduling.

// Workgroup sum of (s0, s1) into part[blockIdx.x], part[gridDim.x + blockIdx.x].
__device__ __forceinline__ void block_partials(double s0, double s1, double *part) {
    __shared__ double red[2][BS / 64];
    for (int d = 32; d > 0; d >>= 1) {
        s0 += __shfl_xor(s0, d, 64);
        s1 += __shfl_xor(s1, d, 64);
    }
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) { red[0][wv] = s0; red[1][wv] = s1; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t0 = 0.0, t1 = 0.0;
        for (int q = 0; q < BS / 64; q++) { t0 += red[0][q]; t1 += red[1][q]; }
        part[blockIdx.x] = t0;
        part[gridDim.x + blockIdx.x] = t1;
    }
}

// q = A p on a CSR level with the launch shape of k_csr_level (rows by
// groups of G lanes, rows longer than HEAVY by a wavefront in trailing
// workgroups), with per-workgroup partial dot products of q:
// DOT 0: (q.q, q.b); DOT 1: (q1.q, 0).
template <class T, int DOT>
__global__ __launch_bounds__(BS) void k_kspmv(CsrArgs<T> A, const T *q1, double *part) {
    double s0 = 0.0, s1 = 0.0;
    if ((int)blockIdx.x < A.nbs) {
        int i = xcd_block(blockIdx.x, A.nbs) * (BS / G) + (int)threadIdx.x / G;
        int lane0 = threadIdx.x % G;
        bool valid = i < A.n;
        int z0 = valid ? A.rp[i] : 0, z1 = valid ? A.rp[i + 1] : 0;
        bool heavy = z1 - z0 > HEAVY;
        T acc = (T)0;
        if (!heavy) {
            for (int z = z0 + lane0; z < z1; z += 2 * G) {
                int zb = z + G < z1 ? z + G : z;
                int ca = A.col[z], cb = A.col[zb];
                T va = A.val[z], vb = A.val[zb];
                T xa = A.x[ca], xb = A.x[cb];
                acc += va * xa + (z + G < z1 ? vb * xb : (T)0);
            }
        }
#pragma unroll
        for (int d = 1; d < G; d <<= 1) acc += __shfl_xor(acc, d, 64);
        if (lane0 == 0 && valid && !heavy) {
            A.xo[i] = acc;
            double q = (double)acc;
            if (DOT == 0) { s0 = q * q; s1 = q * (double)A.b[i]; }
            else s0 = (double)q1[i] * q;
        }
    } else {
        int w = ((int)blockIdx.x - A.nbs) * (BS / 64) + (int)(threadIdx.x >> 6);
        int lane = threadIdx.x & 63;
        if (w < A.nheavy) {
            int i = A.heavy[w];
            int z0 = A.rp[i], z1 = A.rp[i + 1];
            T acc = (T)0;
            for (int z = z0 + lane; z < z1; z += 256) {
                T t[4];
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    int zz = z + 64 * u < z1 ? z + 64 * u : z;
                    T v = A.val[zz] * A.x[A.col[zz]];
                    t[u] = z + 64 * u < z1 ? v : (T)0;
                }
                acc += (t[0] + t[1]) + (t[2] + t[3]);
            }
            for (int d = 1; d < 64; d <<= 1) acc += __shfl_xor(acc, d, 64);
            if (lane == 0) {
                A.xo[i] = acc;
                double q = (double)acc;
                if (DOT == 0) { s0 = q * q; s1 = q * (double)A.b[i]; }
                else s0 = (double)q1[i] * q;
            }
        }
    }
    block_partials(s0, s1, part);
}

// ks = {q1.q1, a1, beta, a2} from nb partial pairs: step 0 from
// (q1.q1, q1.b); 1 from q1.q2; 2 from (q2.q2, q2.r).  A zero denominator
// gives a zero step.
__global__ __launch_bounds__(1024) void k_kfin(int nb, const double *part, int step, double *ks) {
    __shared__ double red[2][1024 / 64];
    double s0 = 0.0, s1 = 0.0;
    // eight strides of partials requested together, then added in the same
    // order as one at a time (the result does not change)
    int st = blockDim.x, b = threadIdx.x;
    for (; b + 7 * st < nb; b += 8 * st) {
        double a0[8], a1[8];
#pragma unroll
        for (int u = 0; u < 8; u++) { a0[u] = part[b + u * st]; a1[u] = part[nb + b + u * st]; }
#pragma unroll
        for (int u = 0; u < 8; u++) { s0 += a0[u]; s1 += a1[u]; }
    }
    for (; b < nb; b += st) { s0 += part[b]; s1 += part[nb + b]; }
    for (int d = 32; d > 0; d >>= 1) {
        s0 += __shfl_xor(s0, d, 64);
        s1 += __shfl_xor(s1, d, 64);
    }
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) { red[0][wv] = s0; red[1][wv] = s1; }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double t0 = 0.0, t1 = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); q++) { t0 += red[0][q]; t1 += red[1][q]; }
    if (step == 0) {
        ks[0] = t0;
        ks[1] = t0 > 0.0 ? t1 / t0 : 0.0;
    } else if (step == 1) {
        ks[2] = ks[0] > 0.0 ? t0 / ks[0] : 0.0;
    } else {
        ks[3] = t0 > 0.0 ? t1 / t0 : 0.0;
    }
}

// r = b - a1 q1 (in place of b) and the next cycle's pre-smoothed iterate r / d.
template <class T>
__global__ void k_kres(int n, T *b, const T *q1, const double *ks, const T *l1, T *x) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    T r = (T)((double)b[i] - ks[1] * (double)q1[i]);
    b[i] = r;
    x[i] = r / l1[i];
}

// p2 -= beta p1, q2 -= beta q1, with partials of (q2.q2, q2.r) of the
// updated q2 (grid-stride over KO_BLOCKS workgroups).
template <class T>
__global__ __launch_bounds__(BS) void k_korth(int n, const T *p1, T *p2, const T *q1, T *q2,
                                              const T *r, const double *ks, double *part) {
    double beta = ks[2], s0 = 0.0, s1 = 0.0;
    for (int i = blockIdx.x * BS + threadIdx.x; i < n; i += gridDim.x * BS) {
        p2[i] = (T)((double)p2[i] - beta * (double)p1[i]);
        T q = (T)((double)q2[i] - beta * (double)q1[i]);
        q2[i] = q;
        s0 += (double)q * (double)q;
        s1 += (double)q * (double)r[i];
    }
    block_partials(s0, s1, part);
}

// Prolongation of the K-cycle correction: x_j += a1 p1[agg_j] + a2 p2[agg_j].
template <class T>
__global__ void k_prolong_k(int n, const int *agg, const T *p1, const T *p2, const double *ks,
                            T *x) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    int I = agg[j];
    T c = (T)(ks[1] * (double)p1[I] + ks[3] * (double)p2[I]);
    x[j] = x[j] + c;
}

// --------------------------------------------------------------- cycle
template <class T>
struct Cycle {
    r2p_cpr *P;
    hipStream_t s;
    int nl;
    bool acc = false;            // add the result to xp (hierarchies of two or more levels)
    static const T *vals(AmgLevel &A) {
        if constexpr (sizeof(T) == 4) return A.f32.val.p; else return (const T *)A.val.p;
    }
    static const T *l1s(AmgLevel &A) {
        if constexpr (sizeof(T) == 4) return A.f32.l1.p; else return (const T *)A.l1.p;
    }
    static T *vb(AmgLevel &A) {
        if constexpr (sizeof(T) == 4) return A.bf.p; else return (T *)A.b.p;
    }
    static T *vx(AmgLevel &A) {
        if constexpr (sizeof(T) == 4) return A.xf.p; else return (T *)A.x.p;
    }
    static T *vxo(AmgLevel &A) {
        if constexpr (sizeof(T) == 4) return A.xof.p; else return (T *)A.xo.p;
    }
    static T *kv(AmgLevel &A) {
        if constexpr (sizeof(T) == 4) return A.kvf.p; else return (T *)A.kv.p;
    }
    CsrArgs<T> csr(AmgLevel &A, const T *x, T *xo) {
        CsrArgs<T> a;
        a.n = A.n; a.nbs = r2p_blocks(A.n, BS / G);
        a.heavy = A.heavy.p; a.nheavy = A.nheavy;
        a.rp = A.rp.p; a.col = A.col.p; a.val = vals(A); a.l1 = l1s(A);
        a.b = vb(A);
        a.x = x; a.xo = xo;
        return a;
    }
    template <int MODE>
    int csr_launch(AmgLevel &A, const T *x, T *xo) {
        CsrArgs<T> D = csr(A, x, xo);
        k_csr_level<T, MODE><<<D.nbs + r2p_blocks(A.nheavy, BS / 64), BS, 0, s>>>(D);
        R2P_LAUNCH();
        return 0;
    }
    // Restriction of level l's residual (in its xo) to level l+1's right-hand
    // side, with l+1's pre-smoothed iterate when l+1 is smoothed.
    int restrict_to(int l) {
        AmgLevel &A = P->lv[l], &C = P->lv[l + 1];
        bool smooth = l + 1 < nl - 1;
        int nbs = r2p_blocks(C.n, BS / GR);
        k_restrict<T><<<nbs + r2p_blocks(A.nbig, BS / 64), BS, 0, s>>>(
            C.n, nbs, A.mptr.p, A.mem.p, A.big.p, A.nbig, vxo(A), vb(C),
            smooth ? l1s(C) : nullptr, smooth ? vx(C) : nullptr);
        R2P_LAUNCH();
        return 0;
    }
    // The coarse correction of level l, added to level l's iterate vx(l).
    int correct(int l) {
        AmgLevel &A = P->lv[l], &C = P->lv[l + 1];
        int c = l + 1;
        if (l < P->o.kcycle && c < nl - 1) {
            int n = C.n;
            T *p1 = kv(C), *p2 = p1 + n, *q1 = p2 + n, *q2 = q1 + n;
            double *ks = P->kscal.p + 4 * c, *part = P->kpart.p;
            int nbs = r2p_blocks(n, BS / G), nbk = nbs + r2p_blocks(C.nheavy, BS / 64);
            int nbo = std::max(1, std::min(KO_BLOCKS, r2p_blocks(n, BS)));
            R2P_TRY(coarse(c, p1));
            k_kspmv<T, 0><<<nbk, BS, 0, s>>>(csr(C, p1, q1), nullptr, part);
            R2P_LAUNCH();
            k_kfin<<<1, 1024, 0, s>>>(nbk, part, 0, ks);
            R2P_LAUNCH();
            k_kres<T><<<r2p_blocks(n, BS), BS, 0, s>>>(n, vb(C), q1, ks, l1s(C), vx(C));
            R2P_LAUNCH();
            R2P_TRY(coarse(c, p2));
            k_kspmv<T, 1><<<nbk, BS, 0, s>>>(csr(C, p2, q2), q1, part);
            R2P_LAUNCH();
            k_kfin<<<1, 1024, 0, s>>>(nbk, part, 1, ks);
            R2P_LAUNCH();
            k_korth<T><<<nbo, BS, 0, s>>>(n, p1, p2, q1, q2, vb(C), ks, part);
            R2P_LAUNCH();
            k_kfin<<<1, 1024, 0, s>>>(nbo, part, 2, ks);
            R2P_LAUNCH();
            k_prolong_k<T><<<r2p_blocks(A.n, BS), BS, 0, s>>>(A.n, A.agg.p, p1, p2, ks, vx(A));
            R2P_LAUNCH();
        } else {
            R2P_TRY(coarse(c, vxo(C)));
            k_prolong<T><<<r2p_blocks(A.n, BS), BS, 0, s>>>(A.n, A.agg.p, vxo(C), vx(A));
            R2P_LAUNCH();
        }
        return 0;
    }
    // One cycle on a coarse (CSR) level c >= 1 whose right-hand side is in
    // vb(c) and, unless c is the coarsest, pre-smoothed iterate in vx(c);
    // the result goes to out.
    int coarse(int c, T *out) {
        AmgLevel &A = P->lv[c];
        if (c == nl - 1) {
            k_coarse_solve<T><<<r2p_blocks(A.n, 64), 64 * CS_WAVES, 0, s>>>(
                A.n, P->cinv.p, vb(A), nullptr, 1, out, nullptr);
            R2P_LAUNCH();
            return 0;
        }
        // the level's xo holds its residual until the correction is added
        R2P_TRY(csr_launch<CSR_DOWN>(A, vx(A), vxo(A)));
        R2P_TRY(restrict_to(c));
        R2P_TRY(correct(c));
        return csr_launch<CSR_UP>(A, vx(A), out);
    }
    // The cycle from level 0 (7-slot stencil) with right-hand side f (stride
    // fstride), result in xp.
    int run(const double *f, int fstride, double *xp) {
        if (nl == 1) {
            AmgLevel &C = P->lv[0];
            k_coarse_solve<T><<<r2p_blocks(C.n, 64), 64 * CS_WAVES, 0, s>>>(
                C.n, P->cinv.p, vb(C), f, fstride, vx(C), xp);
            R2P_LAUNCH();
            return 0;
        }
        const Phys &ph = P->J->m->ph;
        Level0<T> Z;
        AmgLevel &A = P->lv[0];
        Z.n = A.n; Z.nx = ph.nx; Z.nxy = ph.nx * ph.ny;
        if constexpr (sizeof(T) == 4) Z.v7 = A.v7f.p; else Z.v7 = (const T *)A.v7.p;
        Z.l1 = l1s(A);
        Z.f = f;
        Z.fstride = fstride;
        k_down0<T><<<r2p_blocks(A.n, BS), BS, 0, s>>>(Z, vx(A), vxo(A));
        R2P_LAUNCH();
        R2P_TRY(restrict_to(0));
        R2P_TRY(correct(0));
        if (acc)
            k_up0<T, true><<<r2p_blocks(Z.n, BS), BS, 0, s>>>(Z, vx(A), xp);
        else
            k_up0<T, false><<<r2p_blocks(Z.n, BS), BS, 0, s>>>(Z, vx(A), xp);
        R2P_LAUNCH();
        return 0;
    }
};

int r2p_amg_cycle(r2p_cpr *P, const double *f, int fstride, double *xp, hipStream_t s) {
    if (P->o.precision == R2P_FP32) {
        Cycle<float> c{P, s, P->nlev};
        return c.run(f, fstride, xp);
    }
    Cycle<double> c{P, s, P->nlev};
    return c.run(f, fstride, xp);
}

// r = f - A_pp xp on level 0 (the 7-slot stencil, summed as in k_up0), FP64.
template <class T>
__global__ void k_res0(Level0<T> A, const double *xp, double *r) {
    int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    const int order[7] = {5, 3, 1, 0, 2, 4, 6};
    double s = A.f[(long)A.fstride * i];
#pragma unroll
    for (int oi = 0; oi < 7; oi++) {
        int sl = order[oi];
        int j = i + slot_offset(sl, A.nx, A.nxy);
        j = j < 0 ? 0 : (j >= A.n ? A.n - 1 : j);
        s -= (double)ld_stream(&A.v7[(long)sl * A.n + i]) * xp[j];
    }
    r[i] = s;
}

// The pressure stage: amg_cycles cycles on A_pp xp = f_p from xp = 0, each
// on the residual of the last (xp = C(f_p), then xp = xp + C(f_p - A_pp xp)).
template <class T>
static int amg_apply_t(r2p_cpr *P, const double *f, int fstride, double *xp, hipStream_t s) {
    R2P_TRY(r2p_amg_cycle(P, f, fstride, xp, s));
    if (P->o.amg_cycles < 2 || P->nlev < 2) return 0;
    AmgLevel &A = P->lv[0];
    const Phys &ph = P->J->m->ph;
    Level0<T> Z;
    Z.n = A.n; Z.nx = ph.nx; Z.nxy = ph.nx * ph.ny;
    if constexpr (sizeof(T) == 4) Z.v7 = A.v7f.p; else Z.v7 = (const T *)A.v7.p;
    Z.l1 = nullptr;
    Z.f = f;
    Z.fstride = fstride;
    for (int k = 1; k < P->o.amg_cycles; k++) {
        k_res0<T><<<r2p_blocks(A.n, BS), BS, 0, s>>>(Z, xp, P->t_ares.p);
        R2P_LAUNCH();
        // the cycle's last kernel adds its result to xp
        Cycle<T> c{P, s, P->nlev};
        c.acc = true;
        R2P_TRY(c.run(P->t_ares.p, 1, xp));
    }
    return 0;
}

int r2p_amg_apply(r2p_cpr *P, const double *f, int fstride, double *xp, hipStream_t s) {
    if (P->o.precision == R2P_FP32) return amg_apply_t<float>(P, f, fstride, xp, s);
    return amg_apply_t<double>(P, f, fstride, xp, s);
}

extern "C" int r2p_amg_info(r2p_cpr *P, int level, int *nlev, int *n, int *nnz) {
    if (!P || !P->ready) { r2p_set_error("CPR not set up"); return R2P_ESTATE; }
    if (nlev) *nlev = P->nlev;
    if (level >= 0 && level < P->nlev) {
        if (n) *n = P->lv[level].n;
        if (nnz) *nnz = P->lv[level].nnz;
    }
    return 0;
}

extern "C" int r2p_amg_export_level(r2p_cpr *P, int level, int *rp, int *col, double *val,
                                    double *l1, int *agg, void *stream) {
    if (!P || !P->ready) { r2p_set_error("CPR not set up"); return R2P_ESTATE; }
    if (level < 0 || level >= P->nlev) { r2p_set_error("bad level"); return R2P_EINVAL; }
    R2P_HIP(hipStreamSynchronize((hipStream_t)stream));
    AmgLevel &A = P->lv[level];
    if (rp) R2P_HIP(hipMemcpy(rp, A.rp.p, sizeof(int) * (A.n + 1), hipMemcpyDeviceToHost));
    if (col) R2P_HIP(hipMemcpy(col, A.col.p, sizeof(int) * A.nnz, hipMemcpyDeviceToHost));
    if (val) R2P_HIP(hipMemcpy(val, A.val.p, sizeof(double) * A.nnz, hipMemcpyDeviceToHost));
    if (l1) R2P_HIP(hipMemcpy(l1, A.l1.p, sizeof(double) * A.n, hipMemcpyDeviceToHost));
    if (agg && level < P->nlev - 1)
        R2P_HIP(hipMemcpy(agg, A.agg.p, sizeof(int) * A.n, hipMemcpyDeviceToHost));
    return 0;
}
