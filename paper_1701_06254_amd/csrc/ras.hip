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
// A row's subdomains are the set bits of an MW-word mask (subdomain s is bit
// s mod 64 of word s / 64).  Row g's memberships, in ascending subdomain
// order, have local rows slot[g][0 ..] (local rows are numbered over all
// subdomains, each subdomain's rows contiguous and in natural order).
constexpr int MSLOT = 16;  // subdomains one row may belong to

__global__ void k_owner_mask(Phys P, int px, int py, int mw, const int *w_ptr,
                             const int *perf_cell, unsigned long long *mask, int *owner) {
    long g = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (g >= P.n + P.nw) return;
    int c = g < P.n ? (int)g : perf_cell[w_ptr[g - P.n]];
    int i = c % P.nx, j = (c / P.nx) % P.ny;
    int a = (int)(((long)i * px) / P.nx), b = (int)(((long)j * py) / P.ny);
    int s = a + px * b;
    owner[g] = s;
    for (int k = 0; k < mw; k++) mask[g * mw + k] = (s >> 6) == k ? 1ull << (s & 63) : 0ull;
}

// One layer of breadth-first growth on the block graph (pull form).
__global__ void k_dilate(Phys P, int mw, const int *cell_perf, const int *perf_well,
                         const int *w_ptr, const int *perf_cell, const unsigned long long *in,
                         unsigned long long *out) {
    long g = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (g >= P.n + P.nw) return;
    int nb[7], cnt = 0;
    if (g < P.n) {
        int c = (int)g, nxy = P.nx * P.ny;
        int i = c % P.nx, j = (c / P.nx) % P.ny, k = c / nxy;
        if (k > 0) nb[cnt++] = c - nxy;
        if (j > 0) nb[cnt++] = c - P.nx;
        if (i > 0) nb[cnt++] = c - 1;
        if (i + 1 < P.nx) nb[cnt++] = c + 1;
        if (j + 1 < P.ny) nb[cnt++] = c + P.nx;
        if (k + 1 < P.nz) nb[cnt++] = c + nxy;
        int q = cell_perf[c];
        if (q >= 0) nb[cnt++] = P.n + perf_well[q];
    }
    for (int k = 0; k < mw; k++) {
        unsigned long long m = in[g * mw + k];
        if (g < P.n) {
            for (int t = 0; t < cnt; t++) m |= in[(long)nb[t] * mw + k];
        } else {
            int w = (int)(g - P.n);
            for (int q = w_ptr[w]; q < w_ptr[w + 1]; q++) m |= in[(long)perf_cell[q] * mw + k];
        }
        out[g * mw + k] = m;
    }
}

__global__ void k_member_count(long R, int mw, const unsigned long long *mask, int *cnt) {
    long g = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (g > R) return;
    int c = 0;
    if (g < R)
        for (int k = 0; k < mw; k++) c += __popcll(mask[g * mw + k]);
    cnt[g] = c;
}

// (subdomain, row) pairs in row order; a stable sort by subdomain then
// lists each subdomain's rows in natural order.
__global__ void k_member_pairs(long R, int mw, const unsigned long long *mask, const int *start,
                               unsigned *key, unsigned *val) {
    long g = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (g >= R) return;
    int e = start[g];
    for (int k = 0; k < mw; k++) {
        unsigned long long m = mask[g * mw + k];
        while (m) {
            int b = __ffsll((long long)m) - 1;
            key[e] = 64 * k + b;
            val[e] = (unsigned)g;
            e++;
            m &= m - 1;
        }
    }
}

// Rank of subdomain s among row g's subdomains (s must be one of them).
__device__ __forceinline__ int member_rank(const unsigned long long *mask, int mw, long g, int s) {
    int r = 0;
    for (int k = 0; k < (s >> 6); k++) r += __popcll(mask[g * mw + k]);
    unsigned long long below = (s & 63) ? mask[g * mw + (s >> 6)] & ((1ull << (s & 63)) - 1) : 0ull;
    return r + __popcll(below);
}

__global__ void k_member_fill(int mtot, int ns, int mw, const unsigned *key, const unsigned *val,
                              const unsigned long long *mask, const int *owner, int *glob_nat,
                              unsigned char *owned_nat, int *sub_of, int *slot, int *off,
                              int *err) {
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= mtot) return;
    int s = (int)key[l];
    long g = val[l];
    glob_nat[l] = (int)g;
    owned_nat[l] = owner[g] == s;
    sub_of[l] = s;
    if (l == 0 || (int)key[l - 1] != s) off[s] = l;
    if (l == mtot - 1) off[ns] = mtot;
    int r = member_rank(mask, mw, g, s);
    if (r < MSLOT) slot[g * MSLOT + r] = l;
    else atomicOr(err, 1);
}

// Local row of global row g in subdomain s, or -1.
__device__ __forceinline__ int local_row(const unsigned long long *mask, int mw, const int *slot,
                                         long g, int s) {
    if (!((mask[g * mw + (s >> 6)] >> (s & 63)) & 1ull)) return -1;
    return slot[g * MSLOT + member_rank(mask, mw, g, s)];
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

__global__ void k_adj_count(Phys P, int mtot, int mw, const int *glob_nat, const int *sub_of,
                            const unsigned long long *mask, const int *slot, const int *cell_perf,
                            const int *perf_well, const int *w_ptr, const int *perf_cell,
                            int *deg) {
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= mtot) return;
    int g = glob_nat[l], sd = sub_of[l];
    int cnt = 0;
    if (g < P.n) {
        int nb[8], src[8];
        int k = cell_neighbours(P, cell_perf, perf_well, g, nb, src);
        for (int t = 0; t < k; t++) cnt += local_row(mask, mw, slot, nb[t], sd) >= 0;
    } else {
        int w = g - P.n;
        for (int q = w_ptr[w]; q < w_ptr[w + 1]; q++)
            cnt += local_row(mask, mw, slot, perf_cell[q], sd) >= 0;
    }
    deg[l] = cnt;
}

__global__ void k_adj_fill(Phys P, int mtot, int mw, const int *glob_nat, const int *sub_of,
                           const unsigned long long *mask, const int *slot, const int *cell_perf,
                           const int *perf_well, const int *w_ptr, const int *perf_cell,
                           const int *aptr, int *adj, int *asrc, int *dsrc) {
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= mtot) return;
    int g = glob_nat[l], sd = sub_of[l];
    int e = aptr[l];
    if (g < P.n) {
        int nb[8], src[8];
        int k = cell_neighbours(P, cell_perf, perf_well, g, nb, src);
        for (int t = 0; t < k; t++) {
            int h = local_row(mask, mw, slot, nb[t], sd);
            if (h >= 0) { adj[e] = h; asrc[e] = src[t]; e++; }
        }
        dsrc[l] = g;
    } else {
        int w = g - P.n;
        for (int q = w_ptr[w]; q < w_ptr[w + 1]; q++) {
            int h = local_row(mask, mw, slot, perf_cell[q], sd);
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
    if (P->o.px > ph.nx || P->o.py > ph.ny) {
        r2p_set_error("more subdomain tiles (%d x %d) than grid columns (%d x %d)", P->o.px,
                      P->o.py, ph.nx, ph.ny);
        return R2P_EINVAL;
    }
    long R = ph.n + ph.nw;
    int mw = (ns + 63) / 64;
    DBuf<unsigned long long> mk0, mk1;
    DBuf<int> owner, start, slot, err, hist;
    DBuf<unsigned> key, val, kt, vt;
    R2P_TRY(mk0.ensure((size_t)R * mw));
    R2P_TRY(mk1.ensure((size_t)R * mw));
    R2P_TRY(owner.ensure(R));
    k_owner_mask<<<r2p_blocks(R, BS), BS, 0, s>>>(ph, P->o.px, P->o.py, mw, m->w_ptr.p,
                                                 m->perf_cell.p, mk0.p, owner.p);
    R2P_LAUNCH();
    unsigned long long *a = mk0.p, *b = mk1.p;
    for (int d = 0; d < P->o.overlap; d++) {
        k_dilate<<<r2p_blocks(R, BS), BS, 0, s>>>(ph, mw, m->cell_perf.p, m->perf_well.p,
                                                 m->w_ptr.p, m->perf_cell.p, a, b);
        R2P_LAUNCH();
        std::swap(a, b);
    }
    // memberships: count, scan, (subdomain, row) pairs, stable sort by subdomain
    R2P_TRY(start.ensure(R + 1));
    k_member_count<<<r2p_blocks(R + 1, BS), BS, 0, s>>>(R, mw, a, start.p);
    R2P_LAUNCH();
    int mtot = 0;
    R2P_TRY(r2p_scan_int(start.p, start.p, (int)(R + 1), &mtot, P->iscratch, P->pin, s));
    S.mtot = mtot;
    R2P_TRY(key.ensure(mtot));
    R2P_TRY(val.ensure(mtot));
    R2P_TRY(kt.ensure(mtot));
    R2P_TRY(vt.ensure(mtot));
    k_member_pairs<<<r2p_blocks(R, BS), BS, 0, s>>>(R, mw, a, start.p, key.p, val.p);
    R2P_LAUNCH();
    R2P_TRY(r2p_sort_pairs(key.p, val.p, kt.p, vt.p, mtot, r2p_bits_for(ns), hist, P->iscratch,
                           P->pin, s));
    R2P_TRY(S.glob_nat.ensure(mtot));
    R2P_TRY(S.owned_nat.ensure(mtot));
    R2P_TRY(S.sub_of.ensure(mtot));
    R2P_TRY(S.dsrc.ensure(mtot));
    R2P_TRY(S.aptr.ensure(mtot + 1));
    R2P_TRY(slot.ensure((size_t)R * MSLOT));
    R2P_TRY(err.ensure(1));
    DBuf<int> off;
    R2P_TRY(off.ensure(ns + 1));
    R2P_HIP(hipMemsetAsync(err.p, 0, sizeof(int), s));
    // every tile owns at least one column of cells, so every offset is set
    k_member_fill<<<r2p_blocks(mtot, BS), BS, 0, s>>>(mtot, ns, mw, key.p, val.p, a, owner.p,
                                                     S.glob_nat.p, S.owned_nat.p, S.sub_of.p,
                                                     slot.p, off.p, err.p);
    R2P_LAUNCH();
    S.h_off.assign(ns + 1, 0);
    int herr = 0;
    R2P_HIP(hipMemcpyAsync(S.h_off.data(), off.p, sizeof(int) * (ns + 1), hipMemcpyDeviceToHost, s));
    R2P_HIP(hipMemcpyAsync(&herr, err.p, sizeof(int), hipMemcpyDeviceToHost, s));
    R2P_HIP(hipStreamSynchronize(s));
    if (herr) {
        r2p_set_error("a row belongs to more than %d overlapped subdomains (tiles too small for "
                      "the overlap)", MSLOT);
        return R2P_EINVAL;
    }
    k_adj_count<<<r2p_blocks(mtot, BS), BS, 0, s>>>(ph, mtot, mw, S.glob_nat.p, S.sub_of.p, a,
                                                   slot.p, m->cell_perf.p, m->perf_well.p,
                                                   m->w_ptr.p, m->perf_cell.p, S.aptr.p);
    R2P_LAUNCH();
    R2P_HIP(hipMemsetAsync(S.aptr.p + mtot, 0, sizeof(int), s));
    int nadj = 0;
    R2P_TRY(r2p_scan_int(S.aptr.p, S.aptr.p, mtot + 1, &nadj, P->iscratch, P->pin, s));
    S.nadj = nadj;
    R2P_TRY(S.adj.ensure(nadj));
    R2P_TRY(S.asrc.ensure(nadj));
    k_adj_fill<<<r2p_blocks(mtot, BS), BS, 0, s>>>(ph, mtot, mw, S.glob_nat.p, S.sub_of.p, a,
                                                  slot.p, m->cell_perf.p, m->perf_well.p,
                                                  m->w_ptr.p, m->perf_cell.p, S.aptr.p, S.adj.p,
                                                  S.asrc.p, S.dsrc.p);
    R2P_LAUNCH();
    R2P_HIP(hipStreamSynchronize(s));
    S.ns = ns; S.px = P->o.px; S.py = P->o.py; S.overlap = P->o.overlap;
    return 0;
}
