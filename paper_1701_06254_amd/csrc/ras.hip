// Restricted additive Schwarz subdomains (the RAS stage R(A)^-1 of
// Algorithm 2 in the "Multi-stage preconditioner" section).
//
// Readings: subdomains are px x py tiles of the x-y plane with full columns;
// a well belongs to the tile of its first perforation; the overlapped set is
// every block row within `overlap` block-graph layers of the owned rows,
// couplings leaving it dropped.  This file builds that membership and each
// subdomain's local adjacency (with the source of every coupling block); it
// depends on the model and the subdomain options only, so it is built once
// and cached.  Ordering, factorisation and solves live in ras_solve.hip.
#include <algorithm>
#include <cstring>

#include "r2p_impl.h"

constexpr int BS = 256;

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

// Neighbours of cell row c in ascending global order, with block sources.
__device__ int cell_neighbours(const Phys &P, const int *cell_perf, const int *perf_well, int c,
                               int *nb, int *src) {
    int cnt = 0;
    int nxy = P.nx * P.ny;
    int i = c % P.nx, j = (c / P.nx) % P.ny, k = c / nxy;
    if (k > 0) { nb[cnt] = c - nxy; src[cnt] = 5 * P.n + c; cnt++; }
    if (j > 0) { nb[cnt] = c - P.nx; src[cnt] = 3 * P.n + c; cnt++; }
    if (i > 0) { nb[cnt] = c - 1; src[cnt] = 1 * P.n + c; cnt++; }
    if (i + 1 < P.nx) { nb[cnt] = c + 1; src[cnt] = 2 * P.n + c; cnt++; }
    if (j + 1 < P.ny) { nb[cnt] = c + P.nx; src[cnt] = 4 * P.n + c; cnt++; }
    if (k + 1 < P.nz) { nb[cnt] = c + nxy; src[cnt] = 6 * P.n + c; cnt++; }
    int q = cell_perf[c];
    if (q >= 0) { nb[cnt] = P.n + perf_well[q]; src[cnt] = -(1 + q); cnt++; }
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
        int k = cell_neighbours(P, cell_perf, perf_well, g, nb, src);
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
        int k = cell_neighbours(P, cell_perf, perf_well, g, nb, src);
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

int r2p_ras_static(r2p_cpr *P, hipStream_t s) {
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
    R2P_HIP(hipMemsetAsync(S.aptr.p + mtot, 0, sizeof(int), s));
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
