// Restricted additive Schwarz with block ILU(0) subdomain solves, on the
// local potential order of each subdomain.
//
// Paper sections: "Local potential reordering technique" (Eq 30-33) and the
// RAS stage R(A)^-1 of the "Multi-stage preconditioner" (Algorithm 2).
// Readings: subdomains are px x py tiles of the x-y plane with full columns;
// a well belongs to the tile of its first perforation; the overlapped set is
// every block row within `overlap` block-graph layers of the owned rows,
// couplings leaving it dropped; the local order sorts cells by descending
// oil potential (ties: ascending natural index) and puts wells last.
//
// Device design.  ILU(0) and its triangular solves depend only on which end
// of every coupling comes first in the local order, so each subdomain's rows
// are grouped into levels of its dependency graph (longest-path depth from
// the rows with no predecessor); rows of a level are independent.  Within a
// row, predecessors and successors are kept in local order, so every block
// update happens in the same sequence as a sequential ILU(0) in that order.
// One workgroup processes one subdomain level by level, with a workgroup
// barrier between levels (no cross-workgroup synchronisation).
//
// Compiled without floating-point contraction (reproducible block products).
#include <algorithm>
#include <cstring>

#include "r2p_impl.h"

constexpr int BS = 256;
constexpr int WG = 1024;   // threads of a subdomain workgroup

// Block sources: >= 0 slot block index (slot*n + row) into vp/vs;
// -(1+q) cw[q]; -(1+nperf+q) wc[q]; -(1+2*nperf+w) wd[w].
struct BlkSrc {
    const double2 *vp, *vs, *cw, *wc;
    const double *wd;
    int nperf;
};

__device__ __forceinline__ void load_block(const BlkSrc &B, int src, double *a) {
    if (src >= 0) {
        double2 p = B.vp[src], s = B.vs[src];
        a[0] = p.x; a[1] = s.x; a[2] = p.y; a[3] = s.y;
    } else {
        int t = -src - 1;
        if (t < B.nperf) {
            double2 c = B.cw[t];
            a[0] = c.x; a[1] = 0.0; a[2] = c.y; a[3] = 0.0;
        } else if (t < 2 * B.nperf) {
            double2 c = B.wc[t - B.nperf];
            a[0] = c.x; a[1] = c.y; a[2] = 0.0; a[3] = 0.0;
        } else {
            a[0] = B.wd[t - 2 * B.nperf]; a[1] = 0.0; a[2] = 0.0; a[3] = 1.0;
        }
    }
}

// ------------------------------------------------------------- membership
__global__ void k_owner_mask(Phys P, int px, int py, const int *w_ptr, const int *perf_cell,
                             unsigned long long *mask, int *owner) {
    long g = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (g >= P.n + P.nw) return;
    int c = g < P.n ? (int)g : perf_cell[w_ptr[g - P.n]];
    int i = c % P.nx, j = (c / P.nx) % P.ny;
    int a = (int)(((long)i * px) / P.nx), b = (int)(((long)j * py) / P.ny);
    int s = a + px * b;
    owner[g] = s;
    mask[g] = 1ull << s;
}

// One layer of breadth-first growth on the block graph (pull form).
__global__ void k_dilate(Phys P, const int *cell_perf, const int *perf_well, const int *w_ptr,
                         const int *perf_cell, const unsigned long long *in,
                         unsigned long long *out) {
    long g = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (g >= P.n + P.nw) return;
    unsigned long long m = in[g];
    if (g < P.n) {
        int c = (int)g, nxy = P.nx * P.ny;
        int i = c % P.nx, j = (c / P.nx) % P.ny, k = c / nxy;
        if (k > 0) m |= in[c - nxy];
        if (j > 0) m |= in[c - P.nx];
        if (i > 0) m |= in[c - 1];
        if (i + 1 < P.nx) m |= in[c + 1];
        if (j + 1 < P.ny) m |= in[c + P.nx];
        if (k + 1 < P.nz) m |= in[c + nxy];
        int q = cell_perf[c];
        if (q >= 0) m |= in[P.n + perf_well[q]];
    } else {
        int w = (int)(g - P.n);
        for (int q = w_ptr[w]; q < w_ptr[w + 1]; q++) m |= in[perf_cell[q]];
    }
    out[g] = m;
}

__global__ void k_member_flags(long R, int ns, const unsigned long long *mask, int *flags) {
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= (long)ns * R) return;
    int s = (int)(t / R);
    long g = t - (long)s * R;
    flags[t] = (int)((mask[g] >> s) & 1ull);
}

__global__ void k_member_scatter(long R, int ns, const unsigned long long *mask, const int *owner,
                                 int *loc /* in: exclusive scan; out: local index or -1 */,
                                 int *glob_nat, unsigned char *owned_nat, int *sub_of) {
    long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= (long)ns * R) return;
    int s = (int)(t / R);
    long g = t - (long)s * R;
    if ((mask[g] >> s) & 1ull) {
        int l = loc[t];
        glob_nat[l] = (int)g;
        owned_nat[l] = owner[g] == s;
        sub_of[l] = s;
    } else {
        loc[t] = -1;
    }
}

__global__ void k_sub_offsets(long R, int ns, const int *scan, int mtot, int *off) {
    int s = threadIdx.x;
    if (s < ns) off[s] = scan[(long)s * R];
    if (s == ns) off[ns] = mtot;
}

// Neighbours of global row g in ascending global order, with block sources.
// Returns the count; writes at most 64 entries (cells have <= 7).
__device__ int row_neighbours(const Phys &P, const int *cell_perf, const int *perf_well,
                              const int *w_ptr, const int *perf_cell, int g, int *nb, int *src,
                              int cap) {
    int cnt = 0;
    if (g < P.n) {
        int c = g, nxy = P.nx * P.ny;
        int i = c % P.nx, j = (c / P.nx) % P.ny, k = c / nxy;
        if (k > 0) { nb[cnt] = c - nxy; src[cnt] = 5 * P.n + c; cnt++; }
        if (j > 0) { nb[cnt] = c - P.nx; src[cnt] = 3 * P.n + c; cnt++; }
        if (i > 0) { nb[cnt] = c - 1; src[cnt] = 1 * P.n + c; cnt++; }
        if (i + 1 < P.nx) { nb[cnt] = c + 1; src[cnt] = 2 * P.n + c; cnt++; }
        if (j + 1 < P.ny) { nb[cnt] = c + P.nx; src[cnt] = 4 * P.n + c; cnt++; }
        if (k + 1 < P.nz) { nb[cnt] = c + nxy; src[cnt] = 6 * P.n + c; cnt++; }
        int q = cell_perf[c];
        if (q >= 0) { nb[cnt] = P.n + perf_well[q]; src[cnt] = -(1 + q); cnt++; }
    }
    return cnt;
}

__global__ void k_adj_count(Phys P, int mtot, long R, const int *glob_nat, const int *sub_of,
                            const int *loc, const int *cell_perf, const int *perf_well,
                            const int *w_ptr, const int *perf_cell, int *deg) {
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= mtot) return;
    int g = glob_nat[l];
    const int *ls = loc + (long)sub_of[l] * R;
    int cnt = 0;
    if (g < P.n) {
        int nb[8], src[8];
        int k = row_neighbours(P, cell_perf, perf_well, w_ptr, perf_cell, g, nb, src, 8);
        for (int t = 0; t < k; t++) cnt += ls[nb[t]] >= 0;
    } else {
        int w = g - P.n;
        for (int q = w_ptr[w]; q < w_ptr[w + 1]; q++) cnt += ls[perf_cell[q]] >= 0;
    }
    deg[l] = cnt;
}

__global__ void k_adj_fill(Phys P, int mtot, long R, const int *glob_nat, const int *sub_of,
                           const int *loc, const int *cell_perf, const int *perf_well,
                           const int *w_ptr, const int *perf_cell, const int *aptr, int *adj,
                           int *asrc, int *dsrc) {
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= mtot) return;
    int g = glob_nat[l];
    const int *ls = loc + (long)sub_of[l] * R;
    int e = aptr[l];
    if (g < P.n) {
        int nb[8], src[8];
        int k = row_neighbours(P, cell_perf, perf_well, w_ptr, perf_cell, g, nb, src, 8);
        for (int t = 0; t < k; t++) {
            int h = ls[nb[t]];
            if (h >= 0) { adj[e] = h; asrc[e] = src[t]; e++; }
        }
        dsrc[l] = g;
    } else {
        int w = g - P.n;
        for (int q = w_ptr[w]; q < w_ptr[w + 1]; q++) {
            int h = ls[perf_cell[q]];
            if (h >= 0) { adj[e] = h; asrc[e] = -(1 + P.nperf + q); e++; }
        }
        dsrc[l] = -(1 + 2 * P.nperf + w);
    }
}

static int ras_static(r2p_cpr *P, hipStream_t s) {
    r2p_model *m = P->J->m;
    const Phys &ph = m->ph;
    RasStatic &S = P->rs;
    int ns = P->o.px * P->o.py;
    if (S.ns == ns && S.px == P->o.px && S.py == P->o.py && S.overlap == P->o.overlap) return 0;
    long R = ph.n + ph.nw;
    DBuf<unsigned long long> mk0, mk1;
    DBuf<int> owner, loc;
    R2P_TRY(mk0.ensure(R));
    R2P_TRY(mk1.ensure(R));
    R2P_TRY(owner.ensure(R));
    R2P_TRY(loc.ensure((size_t)ns * R));
    k_owner_mask<<<r2p_blocks(R, BS), BS, 0, s>>>(ph, P->o.px, P->o.py, m->w_ptr.p, m->perf_cell.p,
                                                 mk0.p, owner.p);
    R2P_LAUNCH();
    unsigned long long *a = mk0.p, *b = mk1.p;
    for (int d = 0; d < P->o.overlap; d++) {
        k_dilate<<<r2p_blocks(R, BS), BS, 0, s>>>(ph, m->cell_perf.p, m->perf_well.p, m->w_ptr.p,
                                                 m->perf_cell.p, a, b);
        R2P_LAUNCH();
        std::swap(a, b);
    }
    long NR = (long)ns * R;
    if (NR >= (1L << 31)) { r2p_set_error("too many subdomain rows"); return R2P_EINVAL; }
    k_member_flags<<<r2p_blocks(NR, BS), BS, 0, s>>>(R, ns, a, loc.p);
    R2P_LAUNCH();
    int mtot = 0;
    R2P_TRY(r2p_scan_int(loc.p, loc.p, (int)NR, &mtot, P->iscratch, P->pin, s));
    S.mtot = mtot;
    R2P_TRY(S.glob_nat.ensure(mtot));
    R2P_TRY(S.owned_nat.ensure(mtot));
    R2P_TRY(S.sub_of.ensure(mtot));
    R2P_TRY(S.dsrc.ensure(mtot));
    R2P_TRY(S.aptr.ensure(mtot + 1));
    DBuf<int> off;
    R2P_TRY(off.ensure(ns + 1));
    k_sub_offsets<<<1, 128, 0, s>>>(R, ns, loc.p, mtot, off.p);
    R2P_LAUNCH();
    k_member_scatter<<<r2p_blocks(NR, BS), BS, 0, s>>>(R, ns, a, owner.p, loc.p, S.glob_nat.p,
                                                       S.owned_nat.p, S.sub_of.p);
    R2P_LAUNCH();
    S.h_off.assign(ns + 1, 0);
    R2P_HIP(hipMemcpyAsync(S.h_off.data(), off.p, sizeof(int) * (ns + 1), hipMemcpyDeviceToHost, s));
    k_adj_count<<<r2p_blocks(mtot, BS), BS, 0, s>>>(ph, mtot, R, S.glob_nat.p, S.sub_of.p, loc.p,
                                                   m->cell_perf.p, m->perf_well.p, m->w_ptr.p,
                                                   m->perf_cell.p, S.aptr.p);
    R2P_LAUNCH();
    int nadj = 0;
    R2P_TRY(r2p_scan_int(S.aptr.p, S.aptr.p, mtot + 1, &nadj, P->iscratch, P->pin, s));
    S.nadj = nadj;
    R2P_TRY(S.adj.ensure(nadj));
    R2P_TRY(S.asrc.ensure(nadj));
    k_adj_fill<<<r2p_blocks(mtot, BS), BS, 0, s>>>(ph, mtot, R, S.glob_nat.p, S.sub_of.p, loc.p,
                                                  m->cell_perf.p, m->perf_well.p, m->w_ptr.p,
                                                  m->perf_cell.p, S.aptr.p, S.adj.p, S.asrc.p,
                                                  S.dsrc.p);
    R2P_LAUNCH();
    R2P_HIP(hipStreamSynchronize(s));
    S.ns = ns; S.px = P->o.px; S.py = P->o.py; S.overlap = P->o.overlap;
    return 0;
}

// ---------------------------------------------------------------- order
// True when global row h precedes global row g in the local order.
__device__ __forceinline__ bool before(int h, int g, int n, int order, const double *phi) {
    bool hc = h < n, gc = g < n;
    if (hc != gc) return hc;            // cells before wells
    if (!hc || order == R2P_ORDER_NATURAL) return h < g;
    double a = phi[h], b = phi[g];
    return a > b || (a == b && h < g);
}

// Longest-path level, relaxed in place until nothing changes (levels only
// grow and are bounded, so the fixed point is the longest-path depth).
__global__ void k_levels(int mtot, int n, int order, const double *phi, const int *glob_nat,
                         const int *aptr, const int *adj, int *lev, int *changed) {
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= mtot) return;
    int g = glob_nat[l];
    int best = 0;
    for (int e = aptr[l]; e < aptr[l + 1]; e++) {
        int h = adj[e];
        if (before(glob_nat[h], g, n, order, phi)) {
            int v = __hip_atomic_load(&lev[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
            best = v > best ? v : best;
        }
    }
    int cur = lev[l];
    if (best > cur) {
        __hip_atomic_store(&lev[l], best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        *changed = 1;
    }
}

// Deepest level of every subdomain: rows of a subdomain are contiguous, so a
// workgroup meets at most a few subdomains; it reduces in LDS first.
__global__ void k_sub_maxlev(int mtot, int ns, const int *sub_of, const int *lev, int *mx) {
    __shared__ int smax[64];
    if (threadIdx.x < 64) smax[threadIdx.x] = 0;
    __syncthreads();
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < mtot) atomicMax(&smax[sub_of[l]], lev[l]);
    __syncthreads();
    if (threadIdx.x < ns && smax[threadIdx.x] > 0) atomicMax(&mx[threadIdx.x], smax[threadIdx.x]);
}

__global__ void k_level_count(int mtot, const int *sub_of, const int *lev, const int *lbase,
                              int *cnt) {
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= mtot) return;
    atomicAdd(&cnt[lbase[sub_of[l]] + lev[l]], 1);
}

// Position of every row: its level's start plus a slot taken with an atomic
// counter.  Rows of a level are independent and each row's arithmetic depends
// only on its own entries and its predecessors' values, so the order inside
// a level changes the memory layout but not one bit of any result.
__global__ void k_level_place(int mtot, const int *sub_of, const int *lev, const int *lbase,
                              const int *lstart, int *fill, int *pos) {
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= mtot) return;
    int key = lbase[sub_of[l]] + lev[l];
    pos[l] = lstart[key] + atomicAdd(&fill[key], 1);
}

__global__ void k_perm_scatter(int mtot, const int *pos, int *perm) {
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < mtot) perm[pos[l]] = l;
}

__global__ void k_perm_gather(int mtot, const int *perm, const int *glob_nat,
                              const unsigned char *owned_nat, const int *aptr, int *pos,
                              int *glob, unsigned char *owned, int *edeg) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= mtot) return;
    int l = perm[p];
    pos[l] = p;
    glob[p] = glob_nat[l];
    owned[p] = owned_nat[l];
    edeg[p] = aptr[l + 1] - aptr[l];
}

// Factor entries of row p: predecessors then successors, each in ascending
// local order (insertion sort on the global rows, done in the output arrays).
__global__ void k_entries(int mtot, int n, int order, const double *phi, const int *perm,
                          const int *glob_nat, const int *aptr, const int *adj, const int *asrc,
                          const int *pos, const int *eptr, int *ecol, int *esrc, int *nl,
                          int *eglob) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= mtot) return;
    int l = perm[p];
    int g = glob_nat[l];
    int e0 = eptr[p], e = e0;
    for (int t = aptr[l]; t < aptr[l + 1]; t++) {
        int h = glob_nat[adj[t]];
        if (before(h, g, n, order, phi)) { ecol[e] = pos[adj[t]]; esrc[e] = asrc[t]; eglob[e] = h; e++; }
    }
    int nlp = e - e0;
    for (int t = aptr[l]; t < aptr[l + 1]; t++) {
        int h = glob_nat[adj[t]];
        if (!before(h, g, n, order, phi)) { ecol[e] = pos[adj[t]]; esrc[e] = asrc[t]; eglob[e] = h; e++; }
    }
    nl[p] = nlp;
    // insertion sorts of [e0, e0+nlp) and [e0+nlp, e)
    for (int part = 0; part < 2; part++) {
        int a = part == 0 ? e0 : e0 + nlp, b = part == 0 ? e0 + nlp : e;
        for (int u = a + 1; u < b; u++) {
            int vg = eglob[u], vc = ecol[u], vs = esrc[u], k = u - 1;
            while (k >= a && before(vg, eglob[k], n, order, phi)) {
                eglob[k + 1] = eglob[k]; ecol[k + 1] = ecol[k]; esrc[k + 1] = esrc[k];
                k--;
            }
            eglob[k + 1] = vg; ecol[k + 1] = vc; esrc[k + 1] = vs;
        }
    }
}

// ---------------------------------------------------------- factorisation
struct FactArgs {
    BlkSrc B;
    const int *off;          // ns+1 (device)
    const int *lptr, *lbase, *nlev;
    const int *perm, *dsrc, *eptr, *nl, *ecol, *esrc;
    double *eval, *dinv;
    int *status;
};

// Block ILU(0), one workgroup per subdomain, level by level (IKJ form):
// for every predecessor q in local order: L_pq = A_pq U_qq^-1, then
// A_pj -= L_pq U_qj for each later entry j of row p that row q also holds.
__global__ __launch_bounds__(WG) void k_bilu0(FactArgs A) {
    int s = blockIdx.x;
    int nlev = A.nlev[s];
    const int *lp = A.lptr + A.lbase[s];
    for (int L = 0; L < nlev; L++) {
        for (int p = lp[L] + threadIdx.x; p < lp[L + 1]; p += blockDim.x) {
            int e0 = A.eptr[p], e1 = A.eptr[p + 1], el = e0 + A.nl[p];
            for (int e = e0; e < e1; e++) load_block(A.B, A.esrc[e], &A.eval[4 * (long)e]);
            double d[4];
            load_block(A.B, A.dsrc[A.perm[p]], d);
            for (int e = e0; e < el; e++) {
                int q = A.ecol[e];
                double *a = &A.eval[4 * (long)e];
                const double *dk = &A.dinv[4 * (long)q];
                double l0 = a[0] * dk[0] + a[1] * dk[2];
                double l1 = a[0] * dk[1] + a[1] * dk[3];
                double l2 = a[2] * dk[0] + a[3] * dk[2];
                double l3 = a[2] * dk[1] + a[3] * dk[3];
                a[0] = l0; a[1] = l1; a[2] = l2; a[3] = l3;
                int u0 = A.eptr[q] + A.nl[q], u1 = A.eptr[q + 1];
                // later entries of row p: remaining predecessors, the diagonal, successors
                for (int e2 = e + 1; e2 <= e1; e2++) {
                    // e2 == el stands for the diagonal (visited between L and U)
                    int cj;
                    double *t;
                    bool diag = false;
                    if (e2 < el) { cj = A.ecol[e2]; t = &A.eval[4 * (long)e2]; }
                    else if (e2 == el) { cj = p; t = d; diag = true; }
                    else { cj = A.ecol[e2 - 1]; t = &A.eval[4 * (long)(e2 - 1)]; }
                    (void)diag;
                    for (int y = u0; y < u1; y++) {
                        if (A.ecol[y] == cj) {
                            const double *u = &A.eval[4 * (long)y];
                            t[0] -= l0 * u[0] + l1 * u[2];
                            t[1] -= l0 * u[1] + l1 * u[3];
                            t[2] -= l2 * u[0] + l3 * u[2];
                            t[3] -= l2 * u[1] + l3 * u[3];
                            break;
                        }
                    }
                }
            }
            double det = d[0] * d[3] - d[1] * d[2];
            if (det == 0.0 || det != det) atomicOr(A.status, 1);
            double *di = &A.dinv[4 * (long)p];
            di[0] = d[3] / det; di[1] = -d[1] / det; di[2] = -d[2] / det; di[3] = d[0] / det;
        }
        __syncthreads();
    }
}

template <class T>
__global__ void k_cast(long n, const double *a, T *b) {
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) b[i] = (T)a[i];
}

// --------------------------------------------------------------- solve
template <class T>
struct SolveArgs {
    const int *lptr, *lbase, *nlev;
    const int *glob, *eptr, *nl, *ecol;
    const unsigned char *owned;
    const T *eval, *dinv;
    T *y;                      // local work vector, 2 per position
    const double *r;           // input, global
    double *out;               // output, global
    const double *xp;          // optional Pi_p addend (cells' pressure)
    int accumulate;
    int n;
};

// Forward then backward substitution of one subdomain per workgroup; the
// gather R_s^delta r is fused into the first sweep and the restricted
// scatter R_s^0^T into the second.
template <class T>
__global__ __launch_bounds__(WG) void k_ras_solve(SolveArgs<T> A) {
    int s = blockIdx.x;
    int nlev = A.nlev[s];
    const int *lp = A.lptr + A.lbase[s];
    for (int L = 0; L < nlev; L++) {
        for (int p = lp[L] + threadIdx.x; p < lp[L + 1]; p += blockDim.x) {
            int g = A.glob[p];
            T t0 = (T)A.r[2 * (long)g], t1 = (T)A.r[2 * (long)g + 1];
            int e0 = A.eptr[p], el = e0 + A.nl[p];
            for (int e = e0; e < el; e++) {
                int q = A.ecol[e];
                const T *l = &A.eval[4 * (long)e];
                T y0 = A.y[2 * (long)q], y1 = A.y[2 * (long)q + 1];
                t0 -= l[0] * y0 + l[1] * y1;
                t1 -= l[2] * y0 + l[3] * y1;
            }
            A.y[2 * (long)p] = t0;
            A.y[2 * (long)p + 1] = t1;
        }
        __syncthreads();
    }
    for (int L = nlev - 1; L >= 0; L--) {
        for (int p = lp[L] + threadIdx.x; p < lp[L + 1]; p += blockDim.x) {
            T t0 = A.y[2 * (long)p], t1 = A.y[2 * (long)p + 1];
            int e1 = A.eptr[p + 1], eu = A.eptr[p] + A.nl[p];
            for (int e = eu; e < e1; e++) {
                int q = A.ecol[e];
                const T *u = &A.eval[4 * (long)e];
                T y0 = A.y[2 * (long)q], y1 = A.y[2 * (long)q + 1];
                t0 -= u[0] * y0 + u[1] * y1;
                t1 -= u[2] * y0 + u[3] * y1;
            }
            const T *di = &A.dinv[4 * (long)p];
            T z0 = di[0] * t0 + di[1] * t1;
            T z1 = di[2] * t0 + di[3] * t1;
            A.y[2 * (long)p] = z0;
            A.y[2 * (long)p + 1] = z1;
            if (A.owned[p]) {
                long g = A.glob[p];
                double o0 = (double)z0, o1 = (double)z1;
                if (A.accumulate) {
                    // out = (out + Pi_p xp) + z, the order of Algorithm 2's updates
                    double v0 = A.out[2 * g];
                    if (A.xp && g < A.n) v0 += A.xp[g];
                    A.out[2 * g] = v0 + o0;
                    A.out[2 * g + 1] += o1;
                } else {
                    if (A.xp && g < A.n) o0 += A.xp[g];
                    A.out[2 * g] = o0;
                    A.out[2 * g + 1] = o1;
                }
            }
        }
        __syncthreads();
    }
}

// --------------------------------------------------------------- set-up
int r2p_ras_setup(r2p_cpr *P, hipStream_t s) {
    R2P_TRY(ras_static(P, s));
    r2p_jacobian *J = P->J;
    r2p_model *m = J->m;
    const Phys &ph = m->ph;
    RasStatic &S = P->rs;
    RasDyn &D = P->rd;
    int mtot = S.mtot, ns = S.ns, order = P->o.order;
    R2P_TRY(D.lev.ensure(mtot));
    R2P_TRY(D.pos.ensure(mtot));
    R2P_TRY(D.perm.ensure(mtot));
    R2P_TRY(D.glob.ensure(mtot));
    R2P_TRY(D.owned.ensure(mtot));
    R2P_TRY(D.eptr.ensure(mtot + 1));
    R2P_TRY(D.nl.ensure(mtot));
    R2P_TRY(D.ecol.ensure(S.nadj));
    R2P_TRY(D.esrc.ensure(S.nadj));
    R2P_TRY(D.counters.ensure(64 + 2 * ns));
    R2P_TRY(P->pin.ensure(1 << 16));
    // 1. levels
    R2P_HIP(hipMemsetAsync(D.lev.p, 0, sizeof(int) * mtot, s));
    int *changed = D.counters.p;
    int *hflag = (int *)P->pin.p;
    for (int it = 0; it < mtot + 2; it += 8) {
        R2P_HIP(hipMemsetAsync(changed, 0, sizeof(int), s));
        for (int k = 0; k < 8; k++) {
            k_levels<<<r2p_blocks(mtot, BS), BS, 0, s>>>(mtot, ph.n, order, J->phi_o.p,
                                                        S.glob_nat.p, S.aptr.p, S.adj.p, D.lev.p,
                                                        changed);
            R2P_LAUNCH();
        }
        R2P_HIP(hipMemcpyAsync(hflag, changed, sizeof(int), hipMemcpyDeviceToHost, s));
        R2P_HIP(hipStreamSynchronize(s));
        if (*hflag == 0) break;
    }
    // 2. level counts per subdomain
    int *dmax = D.counters.p + 64;
    R2P_HIP(hipMemsetAsync(dmax, 0, sizeof(int) * ns, s));
    k_sub_maxlev<<<r2p_blocks(mtot, BS), BS, 0, s>>>(mtot, ns, S.sub_of.p, D.lev.p, dmax);
    R2P_LAUNCH();
    std::vector<int> maxlev(ns);
    R2P_HIP(hipMemcpyAsync(hflag, dmax, sizeof(int) * ns, hipMemcpyDeviceToHost, s));
    R2P_HIP(hipStreamSynchronize(s));
    D.h_nlev.assign(ns, 0);
    D.h_lbase.assign(ns + 1, 0);
    for (int t = 0; t < ns; t++) {
        int cnt = S.h_off[t + 1] - S.h_off[t];
        D.h_nlev[t] = cnt > 0 ? hflag[t] + 1 : 0;
        D.h_lbase[t + 1] = D.h_lbase[t] + D.h_nlev[t] + 1;
    }
    int nseg = D.h_lbase[ns];
    R2P_TRY(D.lptr_dev.ensure(nseg + 1));
    R2P_TRY(D.sub_lbase.ensure(ns));
    R2P_TRY(D.sub_nlev.ensure(ns));
    DBuf<int> fill;
    R2P_TRY(fill.ensure(nseg + 1));
    R2P_HIP(hipMemcpyAsync(D.sub_lbase.p, D.h_lbase.data(), sizeof(int) * ns, hipMemcpyHostToDevice, s));
    R2P_HIP(hipMemcpyAsync(D.sub_nlev.p, D.h_nlev.data(), sizeof(int) * ns, hipMemcpyHostToDevice, s));
    R2P_HIP(hipMemsetAsync(D.lptr_dev.p, 0, sizeof(int) * (nseg + 1), s));
    k_level_count<<<r2p_blocks(mtot, BS), BS, 0, s>>>(mtot, S.sub_of.p, D.lev.p, D.sub_lbase.p,
                                                     D.lptr_dev.p);
    R2P_LAUNCH();
    R2P_TRY(r2p_scan_int(D.lptr_dev.p, D.lptr_dev.p, nseg + 1, nullptr, P->iscratch, P->pin, s));
    R2P_HIP(hipMemsetAsync(fill.p, 0, sizeof(int) * (nseg + 1), s));
    k_level_place<<<r2p_blocks(mtot, BS), BS, 0, s>>>(mtot, S.sub_of.p, D.lev.p, D.sub_lbase.p,
                                                     D.lptr_dev.p, fill.p, D.pos.p);
    R2P_LAUNCH();
    k_perm_scatter<<<r2p_blocks(mtot, BS), BS, 0, s>>>(mtot, D.pos.p, D.perm.p);
    R2P_LAUNCH();
    DBuf<int> edeg;
    R2P_TRY(edeg.ensure(mtot + 1));
    R2P_HIP(hipMemsetAsync(edeg.p + mtot, 0, sizeof(int), s));
    k_perm_gather<<<r2p_blocks(mtot, BS), BS, 0, s>>>(mtot, D.perm.p, S.glob_nat.p, S.owned_nat.p,
                                                     S.aptr.p, D.pos.p, D.glob.p, D.owned.p,
                                                     edeg.p);
    R2P_LAUNCH();
    int nent = 0;
    R2P_TRY(r2p_scan_int(edeg.p, D.eptr.p, mtot + 1, &nent, P->iscratch, P->pin, s));
    DBuf<int> eglob;
    R2P_TRY(eglob.ensure(S.nadj));
    k_entries<<<r2p_blocks(mtot, BS), BS, 0, s>>>(mtot, ph.n, order, J->phi_o.p, D.perm.p,
                                                 S.glob_nat.p, S.aptr.p, S.adj.p, S.asrc.p, D.pos.p,
                                                 D.eptr.p, D.ecol.p, D.esrc.p, D.nl.p, eglob.p);
    R2P_LAUNCH();
    // 3. numeric factorisation in FP64
    R2P_TRY(D.f64.eval.ensure(4L * S.nadj));
    R2P_TRY(D.f64.dinv.ensure(4L * mtot));
    R2P_TRY(P->status.ensure(4));
    R2P_HIP(hipMemsetAsync(P->status.p, 0, sizeof(int), s));
    FactArgs F;
    F.B.vp = J->vp.p; F.B.vs = J->vs.p; F.B.cw = J->cw.p; F.B.wc = J->wc.p; F.B.wd = J->wd.p;
    F.B.nperf = ph.nperf;
    F.off = nullptr;
    F.lptr = D.lptr_dev.p; F.lbase = D.sub_lbase.p; F.nlev = D.sub_nlev.p;
    F.perm = D.perm.p; F.dsrc = S.dsrc.p; F.eptr = D.eptr.p; F.nl = D.nl.p; F.ecol = D.ecol.p;
    F.esrc = D.esrc.p; F.eval = D.f64.eval.p; F.dinv = D.f64.dinv.p; F.status = P->status.p;
    k_bilu0<<<ns, WG, 0, s>>>(F);
    R2P_LAUNCH();
    if (P->o.precision == R2P_FP32) {
        R2P_TRY(D.f32.eval.ensure(4L * S.nadj));
        R2P_TRY(D.f32.dinv.ensure(4L * mtot));
        k_cast<float><<<r2p_blocks(4L * S.nadj, BS), BS, 0, s>>>(4L * S.nadj, D.f64.eval.p, D.f32.eval.p);
        R2P_LAUNCH();
        k_cast<float><<<r2p_blocks(4L * mtot, BS), BS, 0, s>>>(4L * mtot, D.f64.dinv.p, D.f32.dinv.p);
        R2P_LAUNCH();
        R2P_TRY(P->t_rasf.ensure(2L * mtot));
    } else {
        R2P_TRY(P->t_ras.ensure(2L * mtot));
    }
    R2P_HIP(hipMemcpyAsync(hflag, P->status.p, sizeof(int), hipMemcpyDeviceToHost, s));
    R2P_HIP(hipStreamSynchronize(s));
    if (*hflag) { r2p_set_error("singular diagonal block in block ILU(0)"); return R2P_ESINGULAR; }
    D.maxlev = 0;
    for (int t = 0; t < ns; t++) D.maxlev = std::max(D.maxlev, D.h_nlev[t]);
    return 0;
}

int r2p_ras_solve(r2p_cpr *P, const double *r, double *out, const double *xp, int accumulate,
                  hipStream_t s) {
    RasDyn &D = P->rd;
    const int ns = P->rs.ns;
    if (P->o.precision == R2P_FP32) {
        SolveArgs<float> A;
        A.lptr = D.lptr_dev.p; A.lbase = D.sub_lbase.p; A.nlev = D.sub_nlev.p;
        A.glob = D.glob.p; A.eptr = D.eptr.p; A.nl = D.nl.p; A.ecol = D.ecol.p; A.owned = D.owned.p;
        A.eval = D.f32.eval.p; A.dinv = D.f32.dinv.p; A.y = P->t_rasf.p;
        A.r = r; A.out = out; A.xp = xp; A.accumulate = accumulate; A.n = P->J->m->ph.n;
        k_ras_solve<float><<<ns, WG, 0, s>>>(A);
    } else {
        SolveArgs<double> A;
        A.lptr = D.lptr_dev.p; A.lbase = D.sub_lbase.p; A.nlev = D.sub_nlev.p;
        A.glob = D.glob.p; A.eptr = D.eptr.p; A.nl = D.nl.p; A.ecol = D.ecol.p; A.owned = D.owned.p;
        A.eval = D.f64.eval.p; A.dinv = D.f64.dinv.p; A.y = P->t_ras.p;
        A.r = r; A.out = out; A.xp = xp; A.accumulate = accumulate; A.n = P->J->m->ph.n;
        k_ras_solve<double><<<ns, WG, 0, s>>>(A);
    }
    R2P_LAUNCH();
    return 0;
}

// --------------------------------------------------------------- export
extern "C" int r2p_ras_info(r2p_cpr *P, int sub, int *nsub, int *m, int *nblk, int *nlevels) {
    if (!P || !P->ready) { r2p_set_error("CPR not set up"); return R2P_ESTATE; }
    if (nsub) *nsub = P->rs.ns;
    if (sub < 0 || sub >= P->rs.ns) return 0;
    int a = P->rs.h_off[sub], b = P->rs.h_off[sub + 1];
    if (m) *m = b - a;
    if (nlevels) *nlevels = P->rd.h_nlev[sub];
    if (nblk) {
        int e[2];
        R2P_HIP(hipMemcpy(&e[0], P->rd.eptr.p + a, sizeof(int), hipMemcpyDeviceToHost));
        R2P_HIP(hipMemcpy(&e[1], P->rd.eptr.p + b, sizeof(int), hipMemcpyDeviceToHost));
        *nblk = e[1] - e[0];
    }
    return 0;
}

extern "C" int r2p_ras_export(r2p_cpr *P, int sub, int *glob, int *level, unsigned char *owned,
                              double *dinv, int *erow, int *ecol, double *eval, void *stream) {
    if (!P || !P->ready) { r2p_set_error("CPR not set up"); return R2P_ESTATE; }
    if (sub < 0 || sub >= P->rs.ns) { r2p_set_error("bad subdomain"); return R2P_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    R2P_HIP(hipStreamSynchronize(s));
    int a = P->rs.h_off[sub], b = P->rs.h_off[sub + 1], m = b - a;
    std::vector<int> g(m), pm(m), lv(P->rs.mtot), ep(m + 1), nl(m);
    std::vector<unsigned char> ow(m);
    R2P_HIP(hipMemcpy(g.data(), P->rd.glob.p + a, sizeof(int) * m, hipMemcpyDeviceToHost));
    R2P_HIP(hipMemcpy(pm.data(), P->rd.perm.p + a, sizeof(int) * m, hipMemcpyDeviceToHost));
    R2P_HIP(hipMemcpy(lv.data(), P->rd.lev.p, sizeof(int) * P->rs.mtot, hipMemcpyDeviceToHost));
    R2P_HIP(hipMemcpy(ep.data(), P->rd.eptr.p + a, sizeof(int) * (m + 1), hipMemcpyDeviceToHost));
    R2P_HIP(hipMemcpy(nl.data(), P->rd.nl.p + a, sizeof(int) * m, hipMemcpyDeviceToHost));
    R2P_HIP(hipMemcpy(ow.data(), P->rd.owned.p + a, m, hipMemcpyDeviceToHost));
    int ne = ep[m] - ep[0];
    std::vector<int> ec(ne);
    std::vector<double> ev(4L * ne), dv(4L * m);
    R2P_HIP(hipMemcpy(ec.data(), P->rd.ecol.p + ep[0], sizeof(int) * ne, hipMemcpyDeviceToHost));
    R2P_HIP(hipMemcpy(ev.data(), P->rd.f64.eval.p + 4L * ep[0], sizeof(double) * 4 * ne, hipMemcpyDeviceToHost));
    R2P_HIP(hipMemcpy(dv.data(), P->rd.f64.dinv.p + 4L * a, sizeof(double) * 4 * m, hipMemcpyDeviceToHost));
    std::vector<int> gpos(P->rs.mtot, -1);
    for (int p = 0; p < m; p++) {
        if (glob) glob[p] = g[p];
        if (level) level[p] = lv[pm[p]];
        if (owned) owned[p] = ow[p];
        if (dinv) memcpy(dinv + 4L * p, dv.data() + 4L * p, 4 * sizeof(double));
        for (int e = ep[p]; e < ep[p + 1]; e++) {
            int k = e - ep[0];
            if (erow) erow[k] = g[p];
            if (ecol) ecol[k] = g[ec[k] - a];
            if (eval) memcpy(eval + 4L * k, ev.data() + 4L * k, 4 * sizeof(double));
        }
    }
    return 0;
}
