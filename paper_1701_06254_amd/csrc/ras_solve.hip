// Block ILU(0) set-up and application for the RAS stage, on the local order
// of every subdomain ("Local potential reordering technique", Eq 30-33; RAS
// stage R(A)^-1 of Algorithm 2).
//
// Device design.  ILU(0) and its triangular solves depend only on which end
// of every coupling comes first in the local order, so the rows of each
// subdomain are grouped into levels of the dependency graph (longest-path
// depth); rows of a level are independent.  Inside a row, predecessors and
// successors stay in local order, so every block update happens in the same
// sequence as a sequential ILU(0) in that order and the factors match it.
//
// One workgroup (8 wavefronts) processes one subdomain level by level, a
// workgroup barrier between levels; a wavefront takes a slice of 32 rows of
// a level, two lanes per row (each lane takes every other block of the row;
// a lane holds two blocks in registers, which covers the L or U part of all
// but a few rows: the rows of a slice with more than four blocks, well rows
// and a few others, read the rest from memory), and the wavefronts take the
// slices of the subdomain in turn.  Levels are a
// latency chain, so nothing a step waits for is requested in that step:
// the static data of a slice (columns, factor blocks, right-hand side) are
// requested three and four steps ahead; the y values its rows need that
// were finished two steps earlier are requested then; the rest were
// finished in the last few levels and are read from an LDS ring that holds
// the results of the most recent rows.  Which of these applies to an entry
// follows from the fixed schedule, so the set-up marks it in the entry's
// column.  One CU streams a subdomain's factors
// at the rate its outstanding L2 misses allow, so helper workgroups of the
// same launch, placed on the subdomain's XCD, read the static data of the
// slices some levels ahead of the sweep into that XCD's L2; the sweep then
// finds them in L2 rather than in HBM.  The gather of the right-hand side
// into local order and the restricted scatter of the result run as separate
// full-device kernels.
//
// Compiled without floating-point contraction (reproducible block products).
#include <algorithm>
#include <cstring>

#include "r2p_impl.h"

constexpr int BS = 256;
constexpr int WG = 1024;               // threads of a subdomain workgroup
constexpr int NWAVE = WG / 64;
// Sweep workgroup: 8 wavefronts of up to 256 VGPRs (FP64), 12 of up to 168
// (FP32, whose buffers fit in that); the wavefronts take a subdomain's slices
// in turn.
template <class T>
struct Sweep {
    static constexpr int wg = sizeof(T) == 4 ? 768 : 512;
    static constexpr int ncw = wg / 64;
};
constexpr int LK = 4;                  // sweep: slot pairs per round of a long (well) row
constexpr int MAXK = 2;                // entries per lane held in registers (two lanes per row)
constexpr int RAS_PAD = MAXK * RAS_SLICE;   // padding after the entry arrays: every task reads MAXK slot pairs
constexpr int MAXLEV = 4096;           // levels per subdomain (set-up limit)
constexpr int PROG_STRIDE = 64;        // ints between two sweeps' progress counters
// A factor entry's column (local position, < 2^28) carries in its top bits
// where the sweep finds that column's y value (set after the factorisation):
constexpr int COL_BITS = 28;
constexpr int COL_MASK = (1 << COL_BITS) - 1;
constexpr int F_RING = 0;              // the LDS ring (finished in the last levels)
constexpr int F_PRE = 1;               // loaded from y two steps before the task runs
constexpr int F_SLOW = 2;              // loaded from y when the task runs (rare)
// padding entries are -1: their top bits read as 15

// True when global row h precedes global row g in the local order.
__device__ __forceinline__ bool before(int h, int g, int n, int order, const double *phi) {
    bool hc = h < n, gc = g < n;
    if (hc != gc) return hc;            // cells before wells
    if (!hc || order == R2P_ORDER_NATURAL) return h < g;
    double a = phi[h], b = phi[g];
    return a > b || (a == b && h < g);
}

// ------------------------------------------------------------------ levels
// Longest-path level of every local row, one workgroup per subdomain, by
// Kahn's algorithm in rounds: round t holds exactly the rows whose last
// predecessor was in round t-1, so a row's round is 1 + the deepest round of
// its predecessors (0 for rows without one).  Each row enters the
// subdomain's queue once; the order inside a round depends on scheduling,
// the rounds do not.  The direction of every coupling comes precomputed
// (apred).  When the subdomain has at most LEV_LDS_ROWS rows and no
// in-degree above 255, the in-degrees live in LDS as packed bytes (a 32-bit
// LDS atomic subtracts 1 from one byte; a counter >= 1 never borrows);
// otherwise in global memory.
constexpr int LEV_LDS_WORDS = 38912;              // 152 KiB of packed counters
constexpr int LEV_LDS_ROWS = 4 * LEV_LDS_WORDS;
__global__ __launch_bounds__(WG) void k_levels(const int *suboff, const int *aptr, const int *adj,
                                               const unsigned char *apred, const int *npred,
                                               int *indeg, int *queue, int *lev, int *nlev) {
    __shared__ unsigned cnt[LEV_LDS_WORDS];
    __shared__ int tail, maxd;
    int sub = blockIdx.x;
    int a = suboff[sub], b = suboff[sub + 1];
    if (threadIdx.x == 0) { tail = a; maxd = 0; }
    __syncthreads();
    int md = 0;
    for (int l = a + (int)threadIdx.x; l < b; l += WG) md = max(md, npred[l]);
    atomicMax(&maxd, md);
    __syncthreads();
    const bool in_lds = b - a <= LEV_LDS_ROWS && maxd <= 255;
    if (in_lds) {
        for (int w = threadIdx.x; w < (b - a + 3) / 4; w += WG) {
            unsigned v = 0;
            for (int k = 0; k < 4; k++) {
                int l = a + 4 * w + k;
                if (l < b) v |= (unsigned)npred[l] << (8 * k);
            }
            cnt[w] = v;
        }
    }
    for (int l = a + (int)threadIdx.x; l < b; l += WG) {
        int d = npred[l];
        if (!in_lds) indeg[l] = d;
        if (d == 0) queue[atomicAdd(&tail, 1)] = l;
    }
    __syncthreads();
    int qs = a, qe = tail, t = 0;
    __syncthreads();
    while (qs < qe) {
        for (int q = qs + (int)threadIdx.x; q < qe; q += WG) {
            int l = queue[q];
            lev[l] = t;
            int e0 = aptr[l], e1 = aptr[l + 1];
            // the first AE couplings' loads and decrements are in flight
            // together; a longer row does the rest in turn
            constexpr int AE = 8;
            int hh[AE];
            bool succ[AE];
#pragma unroll
            for (int k = 0; k < AE; k++) {
                bool in = e0 + k < e1;
                hh[k] = in ? adj[e0 + k] : l;
                succ[k] = in && !apred[e0 + k];
            }
            int last[AE];
#pragma unroll
            for (int k = 0; k < AE; k++) {
                last[k] = 0;
                if (succ[k]) {
                    if (in_lds) {
                        int r = hh[k] - a, sh = 8 * (r & 3);
                        last[k] = ((atomicSub(&cnt[r >> 2], 1u << sh) >> sh) & 255u) == 1u;
                    } else {
                        last[k] = atomicSub(&indeg[hh[k]], 1) == 1;
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < AE; k++)
                if (last[k]) queue[atomicAdd(&tail, 1)] = hh[k];
            for (int e = e0 + AE; e < e1; e++) {
                if (apred[e]) continue;
                int h = adj[e];
                bool done;
                if (in_lds) {
                    int r = h - a, sh = 8 * (r & 3);
                    done = ((atomicSub(&cnt[r >> 2], 1u << sh) >> sh) & 255u) == 1u;
                } else {
                    done = atomicSub(&indeg[h], 1) == 1;
                }
                if (done) queue[atomicAdd(&tail, 1)] = h;
            }
        }
        __syncthreads();
        qs = qe;
        qe = tail;
        t++;
        __syncthreads();
    }
    if (threadIdx.x == 0) nlev[sub] = t;
}

__global__ void k_pred_count(int mtot, int n, int order, const double *phi, const int *glob_nat,
                             const int *aptr, const int *adj, unsigned char *apred, int *nl,
                             int *nu) {
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= mtot) return;
    int g = glob_nat[l], a = 0;
    for (int e = aptr[l]; e < aptr[l + 1]; e++) {
        bool p = before(glob_nat[adj[e]], g, n, order, phi);
        apred[e] = p;
        a += p;
    }
    nl[l] = a;
    nu[l] = aptr[l + 1] - aptr[l] - a;
}

__global__ void k_level_count(int mtot, const int *sub_of, const int *lev, const int *lbase,
                              int *cnt) {
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= mtot) return;
    atomicAdd(&cnt[lbase[sub_of[l]] + lev[l]], 1);
}

// Sort key of a row: its level segment, then descending predecessor count
// (so the widest rows of a level share slices); the sort is stable, rows with
// equal keys stay in natural local order.
__global__ void k_order_keys(int mtot, const int *sub_of, const int *lev, const int *lbase,
                             const int *nl, unsigned *key, unsigned *val) {
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= mtot) return;
    unsigned seg = (unsigned)(lbase[sub_of[l]] + lev[l]);
    unsigned w = 7u - (unsigned)min(nl[l], 7);
    key[l] = (seg << 3) | w;
    val[l] = (unsigned)l;
}

__global__ void k_perm_gather(int mtot, const unsigned *perm, const int *glob_nat,
                              const unsigned char *owned_nat, const int *nlnat, const int *nunat,
                              const int *dsrc_nat, int *pos, int *permi, int *glob,
                              unsigned char *owned, int *nl, int *nu, int *dsrc) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= mtot) return;
    int l = (int)perm[p];
    permi[p] = l;
    pos[l] = p;
    glob[p] = glob_nat[l];
    owned[p] = owned_nat[l];
    nl[p] = nlnat[l];
    nu[p] = nunat[l];
    dsrc[p] = dsrc_nat[l];
}

__global__ void k_slice_count(int nseg, const int *lptr, int *nsl) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < nseg) nsl[g] = (lptr[g + 1] - lptr[g] + RAS_ROWS - 1) / RAS_ROWS;
    if (g == nseg) nsl[g] = 0;
}

// One thread per slice: rows, widths, and the slice of every position.
__global__ void k_slice_fill(int nseg, const int *lptr, const int *soff, int nslice,
                             const int *nl, const int *nu, int *st, int *cn, int *wl, int *wu,
                             int *sl_of) {
    int g = blockIdx.x;             // one workgroup per level segment
    if (g >= nseg) return;
    int a = soff[g], b = soff[g + 1];
    for (int sl = a + (int)threadIdx.x; sl < b; sl += blockDim.x) {
        int start = lptr[g] + (sl - a) * RAS_ROWS;
        int cnt = min(RAS_ROWS, lptr[g + 1] - start);
        int ml = 0, mu = 0;
        for (int t = 0; t < cnt; t++) {
            ml = max(ml, nl[start + t]);
            mu = max(mu, nu[start + t]);
            sl_of[start + t] = sl;
        }
        st[sl] = start;
        cn[sl] = cnt;
        wl[sl] = ml;
        wu[sl] = mu;
    }
}

__global__ void k_slice_size(int nslice, const int *w, int *sz) {
    int sl = blockIdx.x * blockDim.x + threadIdx.x;
    if (sl < nslice) sz[sl] = (w[sl] + 1) / 2 * RAS_SLICE;
    if (sl == nslice) sz[sl] = 0;
}

// Entries of position p in its slice: predecessors and successors, each in
// ascending local order (insertion sort over the strided slots).
__device__ __forceinline__ void fill_row_long(int p, int n, int order, const double *phi, const int *permi,
                              const int *glob_nat, const int *aptr, const int *adj,
                               const int *asrc, const int *pos, const int *glob, const int *sl_of,
                              const int *sl_st, const int *sl_bl, const int *sl_bu, int *lcol,
                              int *lsrc, int *ucol, int *usrc) {
    int l = permi[p], g = glob_nat[l];
    int sl = sl_of[p], r = p - sl_st[sl];
    long bl = sl_bl[sl], bu = sl_bu[sl];
    int el = 0, eu = 0;
    for (int t = aptr[l]; t < aptr[l + 1]; t++) {
        int h = adj[t];
        int gh = glob_nat[h];
        if (before(gh, g, n, order, phi)) {
            long k = ras_entry(bl, r, el++);
            lcol[k] = pos[h];
            lsrc[k] = asrc[t];
        } else {
            long k = ras_entry(bu, r, eu++);
            ucol[k] = pos[h];
            usrc[k] = asrc[t];
        }
    }
    for (int part = 0; part < 2; part++) {
        int cnt = part == 0 ? el : eu;
        long b = part == 0 ? bl : bu;
        int *col = part == 0 ? lcol : ucol;
        int *src = part == 0 ? lsrc : usrc;
        for (int u = 1; u < cnt; u++) {
            long ku = ras_entry(b, r, u);
            int vc = col[ku], vs = src[ku];
            int vg = glob[vc];
            int k = u - 1;
            while (k >= 0 && before(vg, glob[col[ras_entry(b, r, k)]], n, order, phi)) {
                col[ras_entry(b, r, k + 1)] = col[ras_entry(b, r, k)];
                src[ras_entry(b, r, k + 1)] = src[ras_entry(b, r, k)];
                k--;
            }
            col[ras_entry(b, r, k + 1)] = vc;
            src[ras_entry(b, r, k + 1)] = vs;
        }
    }
}

// Placement of every local row's couplings into its L (predecessors) and U
// (successors) entries, each part ascending in the local order.  A row with
// at most FE couplings (every cell row) sorts them in registers: the local
// order is a strict total order on global rows, so sorting all couplings at
// once puts the predecessors first, both parts ascending, and the result is
// the same as the per-part insertion sort that longer rows (wells) use.
constexpr int FE = 8;

// before() on values already loaded: cells ahead of wells, cells by
// decreasing potential then index, wells (or the natural order) by index.
__device__ __forceinline__ bool before_v(int h, double ph, int g, double pg, int n, int order) {
    bool hc = h < n, gc = g < n;
    if (hc != gc) return hc;
    if (!hc || order == R2P_ORDER_NATURAL) return h < g;
    return ph > pg || (ph == pg && h < g);
}

__global__ void k_fill_entries(int mtot, int n, int order, const double *phi, const int *permi,
                               const int *glob_nat, const int *aptr, const int *adj,
                               const int *asrc, const int *pos, const int *glob, const int *sl_of,
                               const int *sl_st, const int *sl_bl, const int *sl_bu, int *lcol,
                               int *lsrc, int *ucol, int *usrc) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= mtot) return;
    int l = permi[p];
    int t0 = aptr[l], deg = aptr[l + 1] - t0;
    if (deg > FE) {
        fill_row_long(p, n, order, phi, permi, glob_nat, aptr, adj, asrc, pos, glob, sl_of, sl_st,
                      sl_bl, sl_bu, lcol, lsrc, ucol, usrc);
        return;
    }
    const bool pot = order != R2P_ORDER_NATURAL;
    int g = glob_nat[l];
    double pg = (pot && g < n) ? phi[g] : 0.0;
    // INT_MAX pads the unused slots: it sorts after every row
    int gh[FE], ps[FE], sr[FE];
    double pv[FE];
#pragma unroll
    for (int k = 0; k < FE; k++) {
        gh[k] = 0x7fffffff; ps[k] = 0; sr[k] = 0; pv[k] = 0.0;
        if (k < deg) {
            int h = adj[t0 + k];
            gh[k] = glob_nat[h];
            ps[k] = pos[h];
            sr[k] = asrc[t0 + k];
        }
    }
#pragma unroll
    for (int k = 0; k < FE; k++)
        if (pot && gh[k] < n) pv[k] = phi[gh[k]];
    // odd-even transposition sort (FE rounds sort FE keys)
#pragma unroll
    for (int rd = 0; rd < FE; rd++) {
#pragma unroll
        for (int k = rd & 1; k + 1 < FE; k += 2) {
            if (before_v(gh[k + 1], pv[k + 1], gh[k], pv[k], n, order)) {
                int ti = gh[k]; gh[k] = gh[k + 1]; gh[k + 1] = ti;
                ti = ps[k]; ps[k] = ps[k + 1]; ps[k + 1] = ti;
                ti = sr[k]; sr[k] = sr[k + 1]; sr[k + 1] = ti;
                double td = pv[k]; pv[k] = pv[k + 1]; pv[k + 1] = td;
            }
        }
    }
    int sl = sl_of[p], r = p - sl_st[sl];
    long bl = sl_bl[sl], bu = sl_bu[sl];
    int el = 0, eu = 0;
#pragma unroll
    for (int k = 0; k < FE; k++) {
        if (k < deg) {
            if (before_v(gh[k], pv[k], g, pg, n, order)) {
                long e = ras_entry(bl, r, el++);
                lcol[e] = ps[k];
                lsrc[e] = sr[k];
            } else {
                long e = ras_entry(bu, r, eu++);
                ucol[e] = ps[k];
                usrc[e] = sr[k];
            }
        }
    }
}

// ---------------------------------------------------------- factorisation
// Block ILU(0) in IKJ form: for every predecessor q of row p, in local
// order, L_pq = A_pq U_qq^-1, then A_pj -= L_pq U_qj for every later entry j
// of row p that row q also holds.  The set-up splits this into
//   1. a gather of every row's blocks into the factor arrays (all rows at
//      once; the diagonal block goes where its inverse will be stored);
//   2. a symbolic pass (all rows at once) that finds, for each L entry
//      (p, q), where U_qp sits in row q, plus the rarer matches of other
//      later entries (they need a triangle p-q-j, which the 7-point grid
//      graph does not have; well couplings make them);
//   3. the numeric pass, one workgroup per subdomain, level by level, which
//      only follows the precomputed matches.
// The updates of every target happen in the same order as in the plain
// loop, with the same expressions, so the factors are the same.
struct FactArgs {
    BlkSrc B;
    const int *lbase, *nlev, *soff;
    const int *sl_st, *sl_cn, *sl_bl, *sl_bu, *sl_of;
    const int *nl, *nu, *dsrc, *lcol, *ucol, *lsrc, *usrc;
    int *ldiag;                  // per L entry: entry index of U_qp in row q
    int *xptr;                   // mtot+1: first extra match of every position
    int4 *xl;                    // extra matches: (e, e2, entry index in row q's U, 0)
    double *lval, *uval, *dinv;
    int *status;
};

// Entry e of position p in the L (sl_b = sl_bl) or U (sl_bu) arrays.
__device__ __forceinline__ long slice_entry(const int *sl_of, const int *sl_st, const int *sl_b,
                                            int p, int e) {
    int sl = sl_of[p];
    return ras_entry(sl_b[sl], p - sl_st[sl], e);
}

// Entry e of a row whose entry 0 sits at rb (rb = ras_entry(base, r, 0)).
__device__ __forceinline__ long ent(long rb, int e) {
    return rb + (long)(e >> 1) * RAS_SLICE + (e & 1);
}

__global__ void k_bilu_gather(int mtot, FactArgs A) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= mtot) return;
    int nlp = A.nl[p], nup = A.nu[p];
    long bl = slice_entry(A.sl_of, A.sl_st, A.sl_bl, p, 0);
    long bu = slice_entry(A.sl_of, A.sl_st, A.sl_bu, p, 0);
    for (int e = 0; e < nlp; e++) {
        long k = ent(bl, e);
        load_block(A.B, A.lsrc[k], &A.lval[4 * k]);
    }
    for (int e = 0; e < nup; e++) {
        long k = ent(bu, e);
        load_block(A.B, A.usrc[k], &A.uval[4 * k]);
    }
    load_block(A.B, A.dsrc[p], &A.dinv[4 * (long)p]);
}

// Pass 0 counts the extra matches of every position and records the
// diagonal match of every L entry; pass 1 writes the extra matches.
__device__ __forceinline__ void bilu_sym_long(const FactArgs &A, int p, int nlp, int nup, long bl,
                                              long bu, int pass) {
    int cnt = 0, out = pass ? A.xptr[p] : 0;
    for (int e = 0; e < nlp; e++) {
        long k = ent(bl, e);
        int q = A.lcol[k];
        long buq = slice_entry(A.sl_of, A.sl_st, A.sl_bu, q, 0);
        int nuq = A.nu[q];
        for (int e2 = e + 1; e2 <= nlp + nup; e2++) {
            int cj = e2 < nlp ? A.lcol[ent(bl, e2)]
                              : (e2 == nlp ? p : A.ucol[ent(bu, e2 - nlp - 1)]);
            for (int y = 0; y < nuq; y++) {
                long ky = ent(buq, y);
                if (A.ucol[ky] != cj) continue;
                if (e2 == nlp) {
                    if (pass == 0) A.ldiag[k] = (int)ky;
                } else {
                    if (pass) A.xl[out + cnt] = make_int4(e, e2, (int)ky, 0);
                    cnt++;
                }
                break;
            }
        }
    }
    if (pass == 0) A.xptr[p] = cnt;
}

// Rows whose own entries and whose predecessors' U parts each fit in SE
// slots (every cell row) hold them in registers: the predecessors' U column
// lists are all requested before the matching starts, and the matches come
// out in the same order (by L entry, then by later entry) as the general
// loop's.
constexpr int SE = 8;

__global__ void k_bilu_sym(int mtot, FactArgs A, int pass) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= mtot) return;
    int nlp = A.nl[p], nup = A.nu[p];
    long bl = slice_entry(A.sl_of, A.sl_st, A.sl_bl, p, 0);
    long bu = slice_entry(A.sl_of, A.sl_st, A.sl_bu, p, 0);
    if (nlp + nup > SE) {
        bilu_sym_long(A, p, nlp, nup, bl, bu, pass);
        return;
    }
    // the row's entries in order: L columns, p itself, U columns
    int c[SE + 1];
#pragma unroll
    for (int k = 0; k <= SE; k++) {
        c[k] = -1;
        if (k < nlp) c[k] = A.lcol[ent(bl, k)];
        else if (k == nlp) c[k] = p;
        else if (k <= nlp + nup) c[k] = A.ucol[ent(bu, k - nlp - 1)];
    }
    long buq[SE];
    int nuq[SE];
#pragma unroll
    for (int e = 0; e < SE; e++) {
        buq[e] = 0;
        nuq[e] = 0;
        if (e < nlp) {
            buq[e] = slice_entry(A.sl_of, A.sl_st, A.sl_bu, c[e], 0);
            nuq[e] = A.nu[c[e]];
        }
    }
    bool fits = true;
#pragma unroll
    for (int e = 0; e < SE; e++) fits = fits && nuq[e] <= SE;
    if (!fits) {
        bilu_sym_long(A, p, nlp, nup, bl, bu, pass);
        return;
    }
    int u[SE][SE];
#pragma unroll
    for (int e = 0; e < SE; e++)
#pragma unroll
        for (int y = 0; y < SE; y++)
            u[e][y] = (e < nlp && y < nuq[e]) ? A.ucol[ent(buq[e], y)] : -2;
    int cnt = 0, out = pass ? A.xptr[p] : 0;
#pragma unroll
    for (int e = 0; e < SE; e++) {
        if (e >= nlp) break;
#pragma unroll
        for (int e2 = e + 1; e2 <= SE; e2++) {
            if (e2 > nlp + nup) break;
            int y = -1;
#pragma unroll
            for (int yy = SE - 1; yy >= 0; yy--)
                if (u[e][yy] == c[e2]) y = yy;
            if (y < 0) continue;
            long ky = ent(buq[e], y);
            if (e2 == nlp) {
                if (pass == 0) A.ldiag[ent(bl, e)] = (int)ky;
            } else {
                if (pass) A.xl[out + cnt] = make_int4(e, e2, (int)ky, 0);
                cnt++;
            }
        }
    }
    if (pass == 0) A.xptr[p] = cnt;
}

__device__ __forceinline__ void sub_prod(double *t, const double *l, const double *u) {
    t[0] -= l[0] * u[0] + l[1] * u[2];
    t[1] -= l[0] * u[1] + l[1] * u[3];
    t[2] -= l[2] * u[0] + l[3] * u[2];
    t[3] -= l[2] * u[1] + l[3] * u[3];
}

__device__ __forceinline__ void ld4(double *v, const double *p) {
    const double2 a = ((const double2 *)p)[0], b = ((const double2 *)p)[1];
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}

// L entry e of row p (block a = A_pq, pivot dk = D_q^-1, ud = U_qp if kd >=
// 0): the multiplier l = A_pq D_q^-1 replaces A_pq, then every later entry of
// row p that row q's U part reaches loses l times that U block, in the row's
// order (the remaining L entries, the diagonal, the U entries).
__device__ __forceinline__ void bilu_entry(const FactArgs &A, long bl, long bu, int nlp, int e,
                                           const double *a, const double *dk, int kd,
                                           const double *ud, double *d, int &xi, int xe) {
    double l[4];
    l[0] = a[0] * dk[0] + a[1] * dk[2];
    l[1] = a[0] * dk[1] + a[1] * dk[3];
    l[2] = a[2] * dk[0] + a[3] * dk[2];
    l[3] = a[2] * dk[1] + a[3] * dk[3];
    double2 *o = (double2 *)&A.lval[4 * ent(bl, e)];
    o[0] = make_double2(l[0], l[1]);
    o[1] = make_double2(l[2], l[3]);
    for (; xi < xe; xi++) {
        int4 m = A.xl[xi];
        if (m.x != e || m.y > nlp) break;
        sub_prod(&A.lval[4 * ent(bl, m.y)], l, &A.uval[4 * (long)m.z]);
    }
    if (kd >= 0) sub_prod(d, l, ud);
    for (; xi < xe; xi++) {
        int4 m = A.xl[xi];
        if (m.x != e) break;
        sub_prod(&A.uval[4 * ent(bu, m.y - nlp - 1)], l, &A.uval[4 * (long)m.z]);
    }
}

// Rows of one level are factorised together, one lane per row, the levels in
// turn.  A row's wait on earlier rows is one round of loads: its own first
// LPF L blocks, their columns and U_qp slots (the row's own data, which no
// other row changes) are requested together, then together the pivots and
// U_qp blocks of the rows they name (final since those rows' levels), and
// only then is any of them used.  Entries past LPF load theirs in turn.
constexpr int LPF = 4;
constexpr int BWG = 512;              // 8 waves: registers for the prefetched blocks

__global__ __launch_bounds__(BWG) void k_bilu0(FactArgs A) {
    int s = blockIdx.x;
    int nlev = A.nlev[s], base = A.lbase[s];
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int L = 0; L < nlev; L++) {
        int s0 = A.soff[base + L], s1 = A.soff[base + L + 1];
        for (int sl = s0 + wave; sl < s1; sl += BWG / 64) {
            if (lane >= A.sl_cn[sl]) continue;
            int p = A.sl_st[sl] + lane;
            long bl = ras_entry(A.sl_bl[sl], lane, 0), bu = ras_entry(A.sl_bu[sl], lane, 0);
            int nlp = A.nl[p];
            int xi = A.xptr[p], xe = A.xptr[p + 1];
            // an extra match of an earlier entry may change a later L block
            bool reread = xi < xe;
            double *dp = &A.dinv[4 * (long)p];
            double d[4];
            ld4(d, dp);
            int q[LPF], kd[LPF];
            double a[LPF][4], dk[LPF][4], ud[LPF][4];
#pragma unroll
            for (int e = 0; e < LPF; e++) {
                if (e < nlp) {
                    long k = ent(bl, e);
                    q[e] = A.lcol[k];
                    kd[e] = A.ldiag[k];
                    ld4(a[e], &A.lval[4 * k]);
                }
            }
#pragma unroll
            for (int e = 0; e < LPF; e++) {
                if (e < nlp) {
                    ld4(dk[e], &A.dinv[4 * (long)q[e]]);
                    if (kd[e] >= 0) ld4(ud[e], &A.uval[4 * (long)kd[e]]);
                }
            }
#pragma unroll
            for (int e = 0; e < LPF; e++) {
                if (e < nlp) {
                    if (reread) ld4(a[e], &A.lval[4 * ent(bl, e)]);
                    bilu_entry(A, bl, bu, nlp, e, a[e], dk[e], kd[e], ud[e], d, xi, xe);
                }
            }
            for (int e = LPF; e < nlp; e++) {
                long k = ent(bl, e);
                int qe = A.lcol[k], kde = A.ldiag[k];
                double ae[4], dke[4], ude[4];
                ld4(ae, &A.lval[4 * k]);
                ld4(dke, &A.dinv[4 * (long)qe]);
                if (kde >= 0) ld4(ude, &A.uval[4 * (long)kde]);
                bilu_entry(A, bl, bu, nlp, e, ae, dke, kde, ude, d, xi, xe);
            }
            double det = d[0] * d[3] - d[1] * d[2];
            if (det == 0.0 || det != det) atomicOr(A.status, 1);
            dp[0] = d[3] / det; dp[1] = -d[1] / det; dp[2] = -d[2] / det; dp[3] = d[0] / det;
        }
        __syncthreads();
    }
}

template <class T>
__global__ void k_cast(long n, const double *a, T *b) {
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) b[i] = (T)a[i];
}

// ------------------------------------------------------------------ solve
// Restriction of r to the overlapped subdomains, into local (level) order:
// one thread per local row in natural order, so that the reads of r are
// contiguous along the tiles' rows; each row's pair lands at its position.
template <class T>
__global__ void k_ras_gather(int mtot, const int *glob_nat, const int *pos, const double *r,
                             T *rl, int *prog, int ns) {
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < ns) prog[PROG_STRIDE * l] = 0;   // the sweeps' progress counters (read by the helpers)
    if (l >= mtot) return;
    long g = glob_nat[l], p = pos[l];
    const double2 v = ((const double2 *)r)[g];
    rl[2 * p] = (T)v.x;
    rl[2 * p + 1] = (T)v.y;
}

// Restricted scatter: owned rows only; optional Pi_p addend on the pressure
// and accumulation into out (out = (out + Pi_p xp) + z, Algorithm 2's order).
// One thread per local row in natural order, like the gather, so that the
// writes to out are contiguous along the tiles' rows; each row reads its pair
// at its position.
template <class T>
__global__ void k_ras_scatter(int mtot, int n, const int *glob_nat, const unsigned char *owned_nat,
                              const int *pos, const T *y, const double *xp, int accumulate,
                              double *out) {
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= mtot || !owned_nat[l]) return;
    long g = glob_nat[l], p = pos[l];
    double o0 = (double)y[2 * p], o1 = (double)y[2 * p + 1];
    if (accumulate) {
        double v0 = out[2 * g];
        if (xp && g < n) v0 += xp[g];
        out[2 * g] = v0 + o0;
        out[2 * g + 1] += o1;
    } else {
        if (xp && g < n) o0 += xp[g];
        out[2 * g] = o0;
        out[2 * g + 1] = o1;
    }
}

template <class T>
struct SweepArgs {
    const int *lbase, *nlev, *soff, *lptr;
    const int4 *mL, *mU;         // per slice: (first position, rows | slot pairs << 8, entry base, level)
    const int *lcol, *ucol;
    const T *lval, *uval, *dinv, *rl;
    T *y;
    long lpad, upad;             // first entry of the L and U arrays' zero padding (columns -1)
    int *prog;                   // PROG_STRIDE ns: levels passed by each sweep (forward, then
                                 // nlev + backward), one counter per 256 bytes
    int mtot;                    // local rows over all subdomains: the extent of y
    int ns;                      // subdomains (sweep workgroups)
    int nhelp;                   // prefetch workgroups per subdomain (workgroups ns .. ns (1 + nhelp))
};

// LDS ring of the results of recently finished rows: position p sits in
// slot p mod RING.  While level L is being computed, a finished position q
// is still in the ring when no position written after it has the same slot.
// Positions written after q lie in q's own level (concurrently) or in later
// levels up to L, so with every level narrower than RING the test is
// forward q >= end(L) - RING, backward q < start(L) + RING; with a wider
// level the window is empty and such entries come from global memory.
constexpr int RING_BYTES = 128 * 1024;
template <class T>
struct RingSize {
    static constexpr int rows = RING_BYTES / (2 * (int)sizeof(T));
};

template <class T>
struct Vec2 {
    typedef T type __attribute__((ext_vector_type(2)));
};
template <class T>
struct Vec4 {
    typedef T type __attribute__((ext_vector_type(4)));
};

// The static data of one task (slice) held by the lane pair of each row:
// lane h holds entries e = h, h + 2 of the row (slot pairs k < MAXK),
// component h of the right-hand side and, backward, row h of the inverse
// diagonal block; y values of entries finished before the prefetch was
// issued arrive in yf.  st .. L are uniform.
template <class T>
struct Task {
    int st, cn, w, b, L;
    T a, d0, d1;
    T v[MAXK][4];
    T yf[MAXK][2];
};

// Slice of task j of a wavefront: the wavefronts take the slices of the
// subdomain in turn (forward from the first, backward from the last).  Past
// the wavefront's last task the last one is repeated (prefetches only).
template <bool FWD, int NCW>
__device__ __forceinline__ int task_slice(int sa, int sb, int wave, int j, int nt) {
    int jj = j < nt ? j : nt - 1;
    return FWD ? sa + wave + NCW * jj : sb - 1 - wave - NCW * jj;
}

template <class T, bool FWD>
__device__ __forceinline__ void load_cols(int (&c)[MAXK], const SweepArgs<T> &A, int4 m, int lane) {
    int w = __builtin_amdgcn_readfirstlane(m.y) >> 8, b = __builtin_amdgcn_readfirstlane(m.z);
    const int *cols = FWD ? A.lcol : A.ucol;
    // slot pairs past the slice's own read the arrays' padding (column -1,
    // block 0), so they add nothing and need no mask
    long pad = FWD ? A.lpad : A.upad;
#pragma unroll
    for (int k = 0; k < MAXK; k++)
        c[k] = cols[(k < w ? (long)b + (long)k * RAS_SLICE : pad) + lane];
}

template <class T, bool FWD>
__device__ __forceinline__ void load_task(Task<T> &R, const SweepArgs<T> &A, int4 m, int lane) {
    typedef typename Vec4<T>::type V4;
    typedef typename Vec2<T>::type V2;
    R.st = __builtin_amdgcn_readfirstlane(m.x);
    int cw = __builtin_amdgcn_readfirstlane(m.y);
    R.cn = cw & 255;
    R.w = cw >> 8;
    R.b = __builtin_amdgcn_readfirstlane(m.z);
    R.L = __builtin_amdgcn_readfirstlane(m.w);
    int r = lane >> 1;
    // rows past the slice's end read its last row (never stored)
    long p = R.st + (r < R.cn ? r : R.cn - 1);
    int h = lane & 1;
    R.a = FWD ? A.rl[2 * p + h] : A.y[2 * p + h];
    if (!FWD) {
        V2 d = *(const V2 *)&A.dinv[4 * p + 2 * h];
        R.d0 = d.x;
        R.d1 = d.y;
    }
    const T *vals = FWD ? A.lval : A.uval;
    long pad = FWD ? A.lpad : A.upad;
#pragma unroll
    for (int k = 0; k < MAXK; k++) {
        long e = (k < R.w ? (long)R.b + (long)k * RAS_SLICE : pad) + lane;
        V4 v = *(const V4 *)&vals[4 * e];
        R.v[k][0] = v.x; R.v[k][1] = v.y; R.v[k][2] = v.z; R.v[k][3] = v.w;
    }
}

// Load the y values of the task's entries marked F_PRE: finished before the
// level the wavefront is at when it issues this load (two steps before the
// task) and outside the LDS ring's window of the task's level.
template <class T, bool FWD>
__device__ __forceinline__ void prefetch_y(Task<T> &R, const int (&c)[MAXK], const T *y) {
    typedef typename Vec2<T>::type V2;
#pragma unroll
    for (int k = 0; k < MAXK; k++) {
        bool far = ((unsigned)c[k] >> COL_BITS) == (unsigned)F_PRE;
        // only the lanes with such an entry load (a few per task)
        if (far) {
            V2 v = *(const V2 *)&y[2 * (long)(c[k] & COL_MASK)];
            R.yf[k][0] = v.x;
            R.yf[k][1] = v.y;
        }
    }
}

// One step of a triangular sweep: task k of the wavefront (buffers U).
// The task's level barriers come first; then, with every earlier level
// finished, the y values of task k+2's finished entries are requested,
// task k's other entries are read from the ring (or, outside it, from
// global memory), and the metadata of task k+6, the columns of task k+4 and
// the values of task k+3 are requested; task k is then computed and its
// rows stored to y and the ring.  Every buffer is filled several steps
// before its use, so the waits of a step are for loads issued two or more
// steps earlier.
template <class T, bool FWD, int U>
__device__ __forceinline__ void sweep_step(const SweepArgs<T> &A, T *ring,
                                           int sa, int sb, int nlev, int wave, int lane, int nt, int k,
                                           Task<T> (&B)[4], int (&C)[4][MAXK], int4 (&M)[4],
                                           int &passed) {
    typedef typename Vec2<T>::type V2;
    constexpr int R = RingSize<T>::rows;
    const int4 *meta = FWD ? A.mL : A.mU;
    Task<T> &cur = B[U];
    int rank = FWD ? cur.L : nlev - 1 - cur.L;
    while (passed < rank) {
        __syncthreads();
        passed++;
    }
    // every wavefront, every step: a store the helpers poll (unconditional, so
    // the wait counts stay the same at every step).  Workgroup scope is enough:
    // the store goes through to the XCD's L2, where the helpers' polls read,
    // and nothing of the sweep's results depends on when they see it.
    __hip_atomic_store(&A.prog[PROG_STRIDE * blockIdx.x], (FWD ? 0 : nlev) + passed,
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    // marked entries of task k+2 (finished by now, outside its ring window)
    prefetch_y<T, FWD>(B[(U + 2) & 3], C[(U + 2) & 3], A.y);
    // task k's other entries: from the ring, or (rare) from y
    T y0[MAXK], y1[MAXK];
    bool slow = false;
#pragma unroll
    for (int kk = 0; kk < MAXK; kk++) {
        int c = C[U][kk];
        unsigned f = (unsigned)c >> COL_BITS;
        V2 rv = *(const V2 *)&ring[2 * (c & (R - 1))];
        y0[kk] = f == (unsigned)F_PRE ? cur.yf[kk][0] : rv.x;
        y1[kk] = f == (unsigned)F_PRE ? cur.yf[kk][1] : rv.y;
        slow |= f == (unsigned)F_SLOW;
    }
    if (__builtin_amdgcn_read_exec() & __ballot(slow)) {
#pragma unroll
        for (int kk = 0; kk < MAXK; kk++) {
            int c = C[U][kk];
            if (((unsigned)c >> COL_BITS) == (unsigned)F_SLOW) {
                V2 v = *(const V2 *)&A.y[2 * (long)(c & COL_MASK)];
                y0[kk] = v.x;
                y1[kk] = v.y;
            }
        }
        __builtin_amdgcn_s_waitcnt(0);      // nothing of this rare path stays in flight
    }
    __builtin_amdgcn_sched_barrier(0);
    // metadata of task k+6, columns of task k+4, values of task k+3
    M[(U + 2) & 3] = meta[task_slice<FWD, Sweep<T>::ncw>(sa, sb, wave, k + 6, nt)];
    load_cols<T, FWD>(C[U], A, M[U], lane);
    load_task<T, FWD>(B[(U + 3) & 3], A, M[(U + 3) & 3], lane);
    __builtin_amdgcn_sched_barrier(0);
    // t = a - sum_e B_e y_e over this lane's entries; the pair then adds
    int h = lane & 1;
    T t0 = h == 0 ? cur.a : (T)0, t1 = h == 0 ? (T)0 : cur.a;
#pragma unroll
    for (int kk = 0; kk < MAXK; kk++) {
        T d0 = cur.v[kk][0] * y0[kk] + cur.v[kk][1] * y1[kk];
        T d1 = cur.v[kk][2] * y0[kk] + cur.v[kk][3] * y1[kk];
        // padding entries hold a zero block (their y, from the ring, is finite)
        t0 -= d0;
        t1 -= d1;
    }
    if (cur.w > MAXK) {
        // rows with more than 2 MAXK entries (well rows and a few others): the
        // rest from memory
        const int *cols = FWD ? A.lcol : A.ucol;
        const T *vals = FWD ? A.lval : A.uval;
        // in rounds of LK slot pairs: the columns of a round, then its y values
        // and blocks, are requested together (two dependent loads per round);
        // pairs past the row's own re-read its last and are masked
        typedef typename Vec4<T>::type V4;
        for (int k0 = MAXK; k0 < cur.w; k0 += LK) {
            long idx[LK];
            int q[LK];
#pragma unroll
            for (int j = 0; j < LK; j++) {
                idx[j] = (long)cur.b + (long)min(k0 + j, cur.w - 1) * RAS_SLICE + lane;
                q[j] = cols[idx[j]];
            }
            V2 gv[LK], rv[LK];
            V4 bv[LK];
#pragma unroll
            for (int j = 0; j < LK; j++) {
                int qs = q[j] >= 0 ? q[j] & COL_MASK : 0;
                gv[j] = *(const V2 *)&A.y[2 * (long)qs];
                rv[j] = *(const V2 *)&ring[2 * (qs & (R - 1))];
                bv[j] = *(const V4 *)&vals[4 * idx[j]];
            }
#pragma unroll
            for (int j = 0; j < LK; j++) {
                bool ok = k0 + j < cur.w && q[j] >= 0;
                bool inwin = ((unsigned)q[j] >> COL_BITS) == (unsigned)F_RING;
                T a0 = inwin ? rv[j].x : gv[j].x, a1 = inwin ? rv[j].y : gv[j].y;
                T e0 = bv[j].x * a0 + bv[j].y * a1;
                T e1 = bv[j].z * a0 + bv[j].w * a1;
                t0 -= ok ? e0 : (T)0;
                t1 -= ok ? e1 : (T)0;
            }
        }
        __builtin_amdgcn_s_waitcnt(0);
    }
    t0 += __shfl_xor(t0, 1, 64);
    t1 += __shfl_xor(t1, 1, 64);
    T out = FWD ? (h == 0 ? t0 : t1) : cur.d0 * t0 + cur.d1 * t1;
    // lanes past the slice's end store its last row again, with that row's
    // value, so the store needs no branch
    int r = lane >> 1;
    int rr = r < cur.cn ? r : cur.cn - 1;
    out = __shfl(out, 2 * rr + h, 64);
    long p = (long)cur.st + rr;
    A.y[2 * p + h] = out;
    ring[2 * (p & (R - 1)) + h] = out;
}

// One triangular sweep of a subdomain: forward (L, unit diagonal) or
// backward (U, then the inverse diagonal block).  Every wavefront passes one
// workgroup barrier per level, in the same sequence, wherever it has work.
template <class T, bool FWD>
__device__ __forceinline__ void sweep_dir(const SweepArgs<T> &A, T *ring,
                                          int sa, int sb, int nlev, int wave, int lane) {
    int nsl = sb - sa;
    constexpr int NCW = Sweep<T>::ncw;
    int nt = nsl > wave ? (nsl - wave + NCW - 1) / NCW : 0;
    int passed = 0;
    if (nt > 0) {
        const int4 *meta = FWD ? A.mL : A.mU;
        Task<T> B[4];
        int C[4][MAXK];
        int4 M[4];
#pragma unroll
        for (int j = 0; j < 4; j++) M[j] = meta[task_slice<FWD, Sweep<T>::ncw>(sa, sb, wave, j, nt)];
#pragma unroll
        for (int j = 0; j < 4; j++) load_cols<T, FWD>(C[j], A, M[j], lane);
#pragma unroll
        for (int j = 0; j < 3; j++) load_task<T, FWD>(B[j], A, M[j], lane);
        M[0] = meta[task_slice<FWD, Sweep<T>::ncw>(sa, sb, wave, 4, nt)];
        M[1] = meta[task_slice<FWD, Sweep<T>::ncw>(sa, sb, wave, 5, nt)];
        // enter the loop with nothing in flight, so that the wait counts the
        // compiler derives at its head follow the steady state
        __builtin_amdgcn_s_waitcnt(0);
        // Steps past the wavefront's last task repeat it: its data were read
        // before its first computation stored anything (backward, y is read
        // as input and overwritten), its level barrier is already passed, and
        // it stores the same values again.  With no exit inside the unrolled
        // body the wait counts at every step follow the steady state.
        for (int k = 0; k < nt; k += 4) {
            sweep_step<T, FWD, 0>(A, ring, sa, sb, nlev, wave, lane, nt, k, B, C, M, passed);
            sweep_step<T, FWD, 1>(A, ring, sa, sb, nlev, wave, lane, nt, k + 1, B, C, M, passed);
            sweep_step<T, FWD, 2>(A, ring, sa, sb, nlev, wave, lane, nt, k + 2, B, C, M, passed);
            sweep_step<T, FWD, 3>(A, ring, sa, sb, nlev, wave, lane, nt, k + 3, B, C, M, passed);
        }
    }
    while (passed < nlev) {
        __syncthreads();
        passed++;
    }
    __hip_atomic_store(&A.prog[PROG_STRIDE * blockIdx.x], (FWD ? 0 : nlev) + passed,
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// ------------------------------------------------------- prefetch helpers
constexpr int PCH = 8;            // slices per helper chunk
constexpr int PDS = 128;          // slices a chunk is read ahead of the sweep (about 0.8 MB)
constexpr int PSPIN = 1 << 16;    // bound of a helper's wait for the sweep
constexpr int MAX_HELP = 4;       // helper workgroups per subdomain

// Read one dword of every 128-byte line of [p, p + bytes) (all addresses
// inside the range); the values are summed only so that the loads stay.
__device__ __forceinline__ unsigned touch(const void *p, long bytes) {
    if (bytes < 4) return 0;
    const char *c = (const char *)p;
    const char *line0 = (const char *)((unsigned long)c & ~127ul);
    long last = (long)(c + bytes - 4 - line0);          // offset of the range's last dword
    long lines = last / 128 + 1;
    unsigned acc = 0;
    for (long i = threadIdx.x; i < lines; i += blockDim.x) {
        const char *a = line0 + i * 128;
        a = a < c ? c : a;
        a = a > c + bytes - 4 ? c + bytes - 4 : a;
        acc += *(const unsigned *)((unsigned long)a & ~3ul);
    }
    return acc;
}

// Helper j of subdomain s, one direction: chunks j, j + H, ... of PCH
// slices in the sweep's order; each waits (bounded) until the sweep has
// finished all but PDS of the slices before it, then reads the chunk's
// metadata, columns, factor blocks and right-hand side (backward: the forward
// result and the inverse diagonal blocks).
template <class T, bool FWD>
__device__ unsigned prefetch_dir(const SweepArgs<T> &A, int s, int j, int H, int sa, int sb,
                                 int nlev, int base) {
    const int4 *meta = FWD ? A.mL : A.mU;
    const int *cols = FWD ? A.lcol : A.ucol;
    const T *vals = FWD ? A.lval : A.uval;
    int nsl = sb - sa;
    unsigned acc = 0;
    for (int c = j; c * PCH < nsl; c += H) {
        int i0 = c * PCH, i1 = min(i0 + PCH, nsl);
        int f = FWD ? sa + i0 : sb - i1;           // lowest and highest slice of the chunk
        int l = FWD ? sa + i1 - 1 : sb - 1 - i0;
        int4 mf = meta[f], ml = meta[l];
        // one lane polls (the counter's line is written at every step of the
        // sweep), the workgroup waits for it
        if (threadIdx.x == 0) {
            for (int spin = 0; spin < PSPIN; spin++) {
                int pr = __hip_atomic_load(&A.prog[PROG_STRIDE * s], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                // slices the sweep has finished in this direction
                int done;
                if (FWD)
                    done = pr >= nlev ? nsl : A.soff[base + max(pr, 0)] - sa;
                else
                    done = pr < nlev ? -1 : sb - A.soff[base + nlev - min(pr - nlev, nlev)];
                if (i0 - done <= PDS) break;
                __builtin_amdgcn_s_sleep(8);
            }
        }
        __syncthreads();
        long e0 = mf.z, e1 = (long)ml.z + (long)(ml.y >> 8) * RAS_SLICE;
        long p0 = mf.x, p1 = (long)ml.x + (ml.y & 255);
        acc += touch(meta + f, 16L * (l - f + 1));
        acc += touch(cols + e0, 4L * (e1 - e0));
        acc += touch(vals + 4 * e0, 4L * (long)sizeof(T) * (e1 - e0));
        acc += touch((FWD ? A.rl : (const T *)A.y) + 2 * p0, 2L * (long)sizeof(T) * (p1 - p0));
        if (!FWD) acc += touch(A.dinv + 4 * p0, 4L * (long)sizeof(T) * (p1 - p0));
    }
    return acc;
}

// Forward then backward substitution of one subdomain per workgroup on the
// gathered right-hand side; the result overwrites y in local order.
template <class T>
__global__ __launch_bounds__(Sweep<T>::wg) void k_ras_sweep(SweepArgs<T> A) {
    constexpr int R = RingSize<T>::rows;
    __shared__ __attribute__((aligned(16))) T ring[2 * R];
    if ((int)blockIdx.x >= A.ns) {
        // a helper: subdomain (b - ns) mod ns, on the same XCD as its sweep
        // (workgroup b goes to XCD b mod 8 and ns is a multiple of 8)
        int hb = blockIdx.x - A.ns, hs = hb % A.ns;
        int hn = A.nlev[hs], hbase = A.lbase[hs];
        int hsa = A.soff[hbase], hsb = A.soff[hbase + hn];
        unsigned acc = prefetch_dir<T, true>(A, hs, hb / A.ns, A.nhelp, hsa, hsb, hn, hbase);
        acc += prefetch_dir<T, false>(A, hs, hb / A.ns, A.nhelp, hsa, hsb, hn, hbase);
        if (A.nhelp < 0) A.prog[0] = (int)acc;     // never taken; keeps the reads
        return;
    }
    int s = blockIdx.x;
    int nlev = A.nlev[s], base = A.lbase[s];
    for (int i = threadIdx.x; i < 2 * R; i += Sweep<T>::wg) ring[i] = (T)0;
    int sa = A.soff[base], sb = A.soff[base + nlev];
    __syncthreads();
    int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int lane = threadIdx.x & 63;
    sweep_dir<T, true>(A, ring, sa, sb, nlev, wave, lane);
    sweep_dir<T, false>(A, ring, sa, sb, nlev, wave, lane);
}

// Ring window of every subdomain: positions [end(L) - ring, end(L)) forward
// ([start(L), start(L) + ring) backward) are still in the LDS ring while
// level L runs when every level is narrower than the ring; else none is.
__global__ void k_sub_window(const int *lbase, const int *nlevs, const int *lptr, int ring, int *win) {
    __shared__ int mw;
    int s = blockIdx.x, base = lbase[s], nlev = nlevs[s];
    if (threadIdx.x == 0) mw = 0;
    __syncthreads();
    int m = 0;
    for (int L = threadIdx.x; L < nlev; L += blockDim.x)
        m = max(m, lptr[base + L + 1] - lptr[base + L]);
    atomicMax(&mw, m);
    __syncthreads();
    if (threadIdx.x == 0) win[s] = mw <= ring ? ring : 0;
}

// Where the sweep finds each entry's y value, from the sweep's fixed
// schedule (ncw wavefronts take a subdomain's slices in turn, forward from
// the first, backward from the last; the early loads of task j are issued
// at task j - 2 of the same wavefront, when every level before that task's
// has finished): in the ring window of the entry's level -> F_RING; else
// finished before that bound -> F_PRE; else F_SLOW.  One workgroup per
// slice; the class goes into the column's top bits.
template <bool FWD>
__global__ void k_entry_class(int ns, const int *lbase, const int *nlevs, const int *soff,
                              const int *lptr, const int *win, const int4 *meta, int *cols,
                              int ncw) {
    int sl = blockIdx.x;
    int lo = 0, hi = ns - 1;                  // subdomain: the last one starting at or before sl
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (soff[lbase[mid]] <= sl) lo = mid; else hi = mid - 1;
    }
    int s = lo, base = lbase[s], nlev = nlevs[s];
    int sa = soff[base], sb = soff[base + nlev];
    if (sl < sa || sl >= sb) return;
    int4 m = meta[sl];
    int w = m.y >> 8, b = m.z, L = m.w;
    int idx = FWD ? sl - sa : sb - 1 - sl;
    int bound;
    if (idx / ncw < 2) {
        bound = FWD ? lptr[base] : lptr[base + nlev];      // nothing finished yet
    } else {
        int L2 = meta[FWD ? sl - 2 * ncw : sl + 2 * ncw].w;
        bound = FWD ? lptr[base + L2] : lptr[base + L2 + 1];
    }
    int ws = win[s], lev0 = lptr[base + L], lev1 = lptr[base + L + 1];
    for (int e = b + (int)threadIdx.x; e < b + w * RAS_SLICE; e += blockDim.x) {
        int q = cols[e];
        if (q < 0) continue;
        bool inwin = FWD ? q >= lev1 - ws : q < lev0 + ws;
        bool pre = (FWD ? q < bound : q >= bound) && !inwin;
        cols[e] = q | ((inwin ? F_RING : (pre ? F_PRE : F_SLOW)) << COL_BITS);
    }
}

__global__ void k_slice_meta(int nslice, const int *st, const int *cn, const int *wl,
                             const int *bl, const int *wu, const int *bu, const int *perm,
                             const int *lev, int4 *mL, int4 *mU) {
    int sl = blockIdx.x * blockDim.x + threadIdx.x;
    if (sl >= nslice) return;
    int L = lev[perm[st[sl]]];
    mL[sl] = make_int4(st[sl], cn[sl] | ((wl[sl] + 1) / 2) << 8, bl[sl], L);
    mU[sl] = make_int4(st[sl], cn[sl] | ((wu[sl] + 1) / 2) << 8, bu[sl], L);
}

// ----------------------------------------------------------------- set-up
int r2p_ras_setup(r2p_cpr *P, hipStream_t s) {
    double t0 = r2p_now_ms();
    R2P_TRY(r2p_ras_static(P, s));
    r2p_jacobian *J = P->J;
    r2p_model *m = J->m;
    const Phys &ph = m->ph;
    RasStatic &S = P->rs;
    RasDyn &D = P->rd;
    int mtot = S.mtot, ns = S.ns, order = P->o.order;
    R2P_TRY(D.lev.ensure(mtot));
    R2P_TRY(D.nlnat.ensure(mtot));
    R2P_TRY(D.nunat.ensure(mtot));
    R2P_TRY(D.pos.ensure(mtot));
    R2P_TRY(D.perm.ensure(mtot));
    R2P_TRY(D.glob.ensure(mtot));
    R2P_TRY(D.owned.ensure(mtot));
    R2P_TRY(D.nl.ensure(mtot));
    R2P_TRY(D.nu.ensure(mtot));
    R2P_TRY(D.sl_of.ensure(mtot));
    R2P_TRY(D.dsrc_pos.ensure(mtot));
    R2P_TRY(D.counters.ensure(64 + 2 * ns));
    R2P_TRY(D.prog.ensure(PROG_STRIDE * ns));
    R2P_TRY(P->pin.ensure(1 << 16));
    int nb = r2p_blocks(mtot, BS);
    // 1. levels of the dependency graph
    R2P_TRY(D.apred.ensure(S.nadj > 0 ? S.nadj : 1));
    k_pred_count<<<nb, BS, 0, s>>>(mtot, ph.n, order, J->phi_o.p, S.glob_nat.p, S.aptr.p, S.adj.p,
                                   D.apred.p, D.nlnat.p, D.nunat.p);
    R2P_LAUNCH();
    R2P_TRY(D.suboff.ensure(ns + 1));
    R2P_TRY(D.indeg.ensure(mtot));
    R2P_TRY(D.queue.ensure(mtot));
    R2P_HIP(hipMemcpyAsync(D.suboff.p, S.h_off.data(), sizeof(int) * (ns + 1), hipMemcpyHostToDevice, s));
    int *dnlev = D.counters.p + 64;
    int *hflag = (int *)P->pin.p;
    k_levels<<<ns, WG, 0, s>>>(D.suboff.p, S.aptr.p, S.adj.p, D.apred.p, D.nlnat.p, D.indeg.p,
                               D.queue.p, D.lev.p, dnlev);
    R2P_LAUNCH();
    // 2. level segments
    R2P_HIP(hipMemcpyAsync(hflag, dnlev, sizeof(int) * ns, hipMemcpyDeviceToHost, s));
    R2P_HIP(hipStreamSynchronize(s));
    D.h_nlev.assign(ns, 0);
    D.h_lbase.assign(ns + 1, 0);
    for (int t = 0; t < ns; t++) {
        D.h_nlev[t] = hflag[t];
        if (D.h_nlev[t] > MAXLEV) {
            r2p_set_error("subdomain %d has %d dependency levels (limit %d)", t, D.h_nlev[t], MAXLEV);
            return R2P_EINVAL;
        }
        D.h_lbase[t + 1] = D.h_lbase[t] + D.h_nlev[t];
    }
    int nseg = D.h_lbase[ns];
    D.nseg = nseg;
    R2P_TRY(D.lptr_dev.ensure(nseg + 1));
    R2P_TRY(D.soff.ensure(nseg + 1));
    R2P_TRY(D.sub_lbase.ensure(ns));
    R2P_TRY(D.sub_nlev.ensure(ns));
    R2P_HIP(hipMemcpyAsync(D.sub_lbase.p, D.h_lbase.data(), sizeof(int) * ns, hipMemcpyHostToDevice, s));
    R2P_HIP(hipMemcpyAsync(D.sub_nlev.p, D.h_nlev.data(), sizeof(int) * ns, hipMemcpyHostToDevice, s));
    R2P_HIP(hipMemsetAsync(D.lptr_dev.p, 0, sizeof(int) * (nseg + 1), s));
    k_level_count<<<nb, BS, 0, s>>>(mtot, S.sub_of.p, D.lev.p, D.sub_lbase.p, D.lptr_dev.p);
    R2P_LAUNCH();
    R2P_TRY(r2p_scan_int(D.lptr_dev.p, D.lptr_dev.p, nseg + 1, nullptr, P->iscratch, P->pin, s));
    // 3. positions: stable sort by (level segment, descending predecessor count)
    {
        DBuf<unsigned> &key = P->ws.u[0], &val = P->ws.u[1], &kt = P->ws.u[2], &vt = P->ws.u[3];
        DBuf<int> &hist = P->ws.i[0];
        R2P_TRY(key.ensure(mtot));
        R2P_TRY(val.ensure(mtot));
        R2P_TRY(kt.ensure(mtot));
        R2P_TRY(vt.ensure(mtot));
        k_order_keys<<<nb, BS, 0, s>>>(mtot, S.sub_of.p, D.lev.p, D.sub_lbase.p, D.nlnat.p, key.p, val.p);
        R2P_LAUNCH();
        R2P_TRY(r2p_sort_pairs(key.p, val.p, kt.p, vt.p, mtot, r2p_bits_for(nseg) + 3, hist,
                               P->iscratch, P->pin, s));
        k_perm_gather<<<nb, BS, 0, s>>>(mtot, val.p, S.glob_nat.p, S.owned_nat.p, D.nlnat.p,
                                        D.nunat.p, S.dsrc.p, D.pos.p, D.perm.p, D.glob.p,
                                        D.owned.p, D.nl.p, D.nu.p, D.dsrc_pos.p);
        R2P_LAUNCH();
        R2P_HIP(hipStreamSynchronize(s));
    }
    double t1 = r2p_now_ms();
    P->ms_order = t1 - t0;       // membership (when rebuilt), levels and the local order
    // 4. slices of 64 rows per level, entry bases
    k_slice_count<<<r2p_blocks(nseg + 1, BS), BS, 0, s>>>(nseg, D.lptr_dev.p, D.soff.p);
    R2P_LAUNCH();
    int nslice = 0;
    R2P_TRY(r2p_scan_int(D.soff.p, D.soff.p, nseg + 1, &nslice, P->iscratch, P->pin, s));
    D.nslice = nslice;
    R2P_TRY(D.sl_start.ensure(nslice));
    R2P_TRY(D.sl_cnt.ensure(nslice));
    R2P_TRY(D.sl_wl.ensure(nslice));
    R2P_TRY(D.sl_wu.ensure(nslice));
    R2P_TRY(D.sl_bl.ensure(nslice + 1));
    R2P_TRY(D.sl_bu.ensure(nslice + 1));
    k_slice_fill<<<nseg, 64, 0, s>>>(nseg, D.lptr_dev.p, D.soff.p, nslice, D.nl.p, D.nu.p,
                                     D.sl_start.p, D.sl_cnt.p, D.sl_wl.p, D.sl_wu.p, D.sl_of.p);
    R2P_LAUNCH();
    k_slice_size<<<r2p_blocks(nslice + 1, BS), BS, 0, s>>>(nslice, D.sl_wl.p, D.sl_bl.p);
    R2P_LAUNCH();
    k_slice_size<<<r2p_blocks(nslice + 1, BS), BS, 0, s>>>(nslice, D.sl_wu.p, D.sl_bu.p);
    R2P_LAUNCH();
    int nle = 0, nue = 0;
    R2P_TRY(r2p_scan_int(D.sl_bl.p, D.sl_bl.p, nslice + 1, &nle, P->iscratch, P->pin, s));
    R2P_TRY(r2p_scan_int(D.sl_bu.p, D.sl_bu.p, nslice + 1, &nue, P->iscratch, P->pin, s));
    R2P_TRY(D.meta_l.ensure(nslice));
    R2P_TRY(D.meta_u.ensure(nslice));
    k_slice_meta<<<r2p_blocks(nslice, BS), BS, 0, s>>>(nslice, D.sl_start.p, D.sl_cnt.p, D.sl_wl.p,
                                                       D.sl_bl.p, D.sl_wu.p, D.sl_bu.p, D.perm.p,
                                                       D.lev.p, D.meta_l.p, D.meta_u.p);
    R2P_LAUNCH();
    D.nlent = nle;
    D.nuent = nue;
    // RAS_PAD entries of padding after each array: the sweep reads MAXK slot
    // pairs of every slice (the ones past its own are ignored)
    R2P_TRY(D.lcol.ensure(nle + RAS_PAD));
    R2P_TRY(D.ucol.ensure(nue + RAS_PAD));
    R2P_TRY(D.lsrc.ensure(nle));
    R2P_TRY(D.usrc.ensure(nue));
    R2P_HIP(hipMemsetAsync(D.lcol.p, 0xff, sizeof(int) * (size_t)(nle + RAS_PAD), s));
    R2P_HIP(hipMemsetAsync(D.ucol.p, 0xff, sizeof(int) * (size_t)(nue + RAS_PAD), s));
    k_fill_entries<<<nb, BS, 0, s>>>(mtot, ph.n, order, J->phi_o.p, D.perm.p, S.glob_nat.p,
                                     S.aptr.p, S.adj.p, S.asrc.p, D.pos.p, D.glob.p, D.sl_of.p,
                                     D.sl_start.p, D.sl_bl.p, D.sl_bu.p, D.lcol.p, D.lsrc.p,
                                     D.ucol.p, D.usrc.p);
    R2P_LAUNCH();
    // 5. numeric factorisation in FP64
    R2P_TRY(D.f64.lval.ensure(4L * (nle + RAS_PAD)));
    R2P_TRY(D.f64.uval.ensure(4L * (nue + RAS_PAD)));
    R2P_TRY(D.f64.dinv.ensure(4L * mtot));
    // padding slots stay zero (they are loaded, never used)
    R2P_HIP(hipMemsetAsync(D.f64.lval.p, 0, sizeof(double) * 4 * (size_t)(nle + RAS_PAD), s));
    R2P_HIP(hipMemsetAsync(D.f64.uval.p, 0, sizeof(double) * 4 * (size_t)(nue + RAS_PAD), s));
    R2P_TRY(P->status.ensure(4));
    R2P_HIP(hipMemsetAsync(P->status.p, 0, sizeof(int), s));
    FactArgs F;
    F.B.vp = J->vp.p; F.B.vs = J->vs.p; F.B.cw = J->cw.p; F.B.wc = J->wc.p; F.B.wd = J->wd.p;
    F.B.nperf = ph.nperf;
    F.lbase = D.sub_lbase.p; F.nlev = D.sub_nlev.p; F.soff = D.soff.p;
    F.sl_st = D.sl_start.p; F.sl_cn = D.sl_cnt.p; F.sl_bl = D.sl_bl.p; F.sl_bu = D.sl_bu.p;
    F.sl_of = D.sl_of.p; F.nl = D.nl.p; F.nu = D.nu.p; F.dsrc = D.dsrc_pos.p;
    F.lcol = D.lcol.p; F.ucol = D.ucol.p; F.lsrc = D.lsrc.p; F.usrc = D.usrc.p;
    F.lval = D.f64.lval.p; F.uval = D.f64.uval.p; F.dinv = D.f64.dinv.p; F.status = P->status.p;
    R2P_TRY(D.ldiag.ensure(nle + RAS_PAD));
    R2P_TRY(D.xptr.ensure(mtot + 1));
    R2P_HIP(hipMemsetAsync(D.ldiag.p, 0xff, sizeof(int) * (size_t)(nle + RAS_PAD), s));
    R2P_HIP(hipMemsetAsync(D.xptr.p + mtot, 0, sizeof(int), s));
    F.ldiag = D.ldiag.p; F.xptr = D.xptr.p; F.xl = nullptr;
    k_bilu_gather<<<nb, BS, 0, s>>>(mtot, F);
    R2P_LAUNCH();
    k_bilu_sym<<<nb, BS, 0, s>>>(mtot, F, 0);
    R2P_LAUNCH();
    int nx = 0;
    R2P_TRY(r2p_scan_int(D.xptr.p, D.xptr.p, mtot + 1, &nx, P->iscratch, P->pin, s));
    R2P_TRY(D.xl.ensure(nx));
    F.xl = D.xl.p;
    k_bilu_sym<<<nb, BS, 0, s>>>(mtot, F, 1);
    R2P_LAUNCH();
    k_bilu0<<<ns, BWG, 0, s>>>(F);
    R2P_LAUNCH();
    if (P->o.precision == R2P_FP32) {
        long nlp = 4L * (nle + RAS_PAD), nup = 4L * (nue + RAS_PAD);
        R2P_TRY(D.f32.lval.ensure(nlp));
        R2P_TRY(D.f32.uval.ensure(nup));
        R2P_TRY(D.f32.dinv.ensure(4L * mtot));
        k_cast<float><<<r2p_blocks(nlp, BS), BS, 0, s>>>(nlp, D.f64.lval.p, D.f32.lval.p);
        R2P_LAUNCH();
        k_cast<float><<<r2p_blocks(nup, BS), BS, 0, s>>>(nup, D.f64.uval.p, D.f32.uval.p);
        R2P_LAUNCH();
        k_cast<float><<<r2p_blocks(4L * mtot, BS), BS, 0, s>>>(4L * mtot, D.f64.dinv.p, D.f32.dinv.p);
        R2P_LAUNCH();
        R2P_TRY(P->t_rasf.ensure(2L * mtot));
        R2P_TRY(P->t_rlf.ensure(2L * mtot));
        R2P_HIP(hipMemsetAsync(P->t_rasf.p, 0, sizeof(float) * 2 * (size_t)mtot, s));
    } else {
        R2P_TRY(P->t_ras.ensure(2L * mtot));
        R2P_TRY(P->t_rl.ensure(2L * mtot));
        R2P_HIP(hipMemsetAsync(P->t_ras.p, 0, sizeof(double) * 2 * (size_t)mtot, s));
    }
    // entry classes for the sweep of the precision set up
    {
        bool f32 = P->o.precision == R2P_FP32;
        int ring = f32 ? RingSize<float>::rows : RingSize<double>::rows;
        int ncw = f32 ? Sweep<float>::ncw : Sweep<double>::ncw;
        R2P_TRY(D.swin.ensure(ns));
        k_sub_window<<<ns, 256, 0, s>>>(D.sub_lbase.p, D.sub_nlev.p, D.lptr_dev.p, ring, D.swin.p);
        R2P_LAUNCH();
        if (D.nslice > 0) {
            k_entry_class<true><<<D.nslice, 64, 0, s>>>(ns, D.sub_lbase.p, D.sub_nlev.p, D.soff.p,
                                                        D.lptr_dev.p, D.swin.p, D.meta_l.p,
                                                        D.lcol.p, ncw);
            R2P_LAUNCH();
            k_entry_class<false><<<D.nslice, 64, 0, s>>>(ns, D.sub_lbase.p, D.sub_nlev.p, D.soff.p,
                                                         D.lptr_dev.p, D.swin.p, D.meta_u.p,
                                                         D.ucol.p, ncw);
            R2P_LAUNCH();
        }
    }
    R2P_HIP(hipMemcpyAsync(hflag, P->status.p, sizeof(int), hipMemcpyDeviceToHost, s));
    R2P_HIP(hipStreamSynchronize(s));
    P->ms_ras = r2p_now_ms() - t1;
    if (*hflag) { r2p_set_error("singular diagonal block in block ILU(0)"); return R2P_ESINGULAR; }
    D.maxlev = 0;
    for (int t = 0; t < ns; t++) D.maxlev = std::max(D.maxlev, D.h_nlev[t]);
    return 0;
}

template <class T>
static int ras_solve_t(r2p_cpr *P, const double *r, double *out, const double *xp,
                       int accumulate, T *y, T *rl, const RasFactors<T> &F, hipStream_t s) {
    RasDyn &D = P->rd;
    int mtot = P->rs.mtot;
    int nb = r2p_blocks(mtot, BS);
    int ns = P->rs.ns;
    k_ras_gather<T><<<nb, BS, 0, s>>>(mtot, P->rs.glob_nat.p, D.pos.p, r, rl, D.prog.p, ns);
    R2P_LAUNCH();
    SweepArgs<T> A;
    A.lbase = D.sub_lbase.p; A.nlev = D.sub_nlev.p; A.soff = D.soff.p; A.lptr = D.lptr_dev.p;
    A.mL = D.meta_l.p; A.mU = D.meta_u.p;
    A.lcol = D.lcol.p; A.ucol = D.ucol.p;
    A.lval = F.lval.p; A.uval = F.uval.p; A.dinv = F.dinv.p; A.rl = rl; A.y = y;
    A.mtot = mtot;
    A.lpad = D.nlent;
    A.upad = D.nuent;
    A.ns = ns;
    A.prog = D.prog.p;
    // helpers only where they fit beside the sweeps and share their XCDs
    A.nhelp = ns % 8 == 0 ? std::max(0, std::min(MAX_HELP, 256 / ns - 1)) : 0;
    k_ras_sweep<T><<<ns * (1 + A.nhelp), Sweep<T>::wg, 0, s>>>(A);
    R2P_LAUNCH();
    k_ras_scatter<T><<<nb, BS, 0, s>>>(mtot, P->J->m->ph.n, P->rs.glob_nat.p, P->rs.owned_nat.p,
                                       D.pos.p, y, xp,
                                       accumulate, out);
    R2P_LAUNCH();
    return 0;
}

int r2p_ras_solve(r2p_cpr *P, const double *r, double *out, const double *xp, int accumulate,
                  hipStream_t s) {
    if (P->o.precision == R2P_FP32)
        return ras_solve_t<float>(P, r, out, xp, accumulate, P->t_rasf.p, P->t_rlf.p, P->rd.f32, s);
    return ras_solve_t<double>(P, r, out, xp, accumulate, P->t_ras.p, P->t_rl.p, P->rd.f64, s);
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
        std::vector<int> nl(b - a), nu(b - a);
        R2P_HIP(hipMemcpy(nl.data(), P->rd.nl.p + a, sizeof(int) * (b - a), hipMemcpyDeviceToHost));
        R2P_HIP(hipMemcpy(nu.data(), P->rd.nu.p + a, sizeof(int) * (b - a), hipMemcpyDeviceToHost));
        long t = 0;
        for (int i = 0; i < b - a; i++) t += nl[i] + nu[i];
        *nblk = (int)t;
    }
    return 0;
}

extern "C" int r2p_ras_export(r2p_cpr *P, int sub, int *glob, int *level, unsigned char *owned,
                              double *dinv, int *erow, int *ecol, double *eval, void *stream) {
    if (!P || !P->ready) { r2p_set_error("CPR not set up"); return R2P_ESTATE; }
    if (sub < 0 || sub >= P->rs.ns) { r2p_set_error("bad subdomain"); return R2P_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    R2P_HIP(hipStreamSynchronize(s));
    RasDyn &D = P->rd;
    int mtot = P->rs.mtot, a = P->rs.h_off[sub], b = P->rs.h_off[sub + 1], m = b - a;
    auto pull = [&](const auto *src, size_t cnt, auto &dst) -> int {
        dst.resize(cnt);
        if (cnt) {
            hipError_t e = hipMemcpy(dst.data(), src, sizeof(dst[0]) * cnt, hipMemcpyDeviceToHost);
            if (e != hipSuccess) return r2p_hip_fail(e, "export", __FILE__, __LINE__);
        }
        return 0;
    };
    std::vector<int> g, pm, lv, nl, nu, slof, slst, slbl, slbu, lc, uc;
    std::vector<unsigned char> ow;
    std::vector<double> lvv, uvv, dv;
    R2P_TRY(pull(D.glob.p, mtot, g));
    R2P_TRY(pull(D.perm.p, mtot, pm));
    R2P_TRY(pull(D.lev.p, mtot, lv));
    R2P_TRY(pull(D.nl.p, mtot, nl));
    R2P_TRY(pull(D.nu.p, mtot, nu));
    R2P_TRY(pull(D.sl_of.p, mtot, slof));
    R2P_TRY(pull(D.sl_start.p, D.nslice, slst));
    R2P_TRY(pull(D.sl_bl.p, D.nslice, slbl));
    R2P_TRY(pull(D.sl_bu.p, D.nslice, slbu));
    R2P_TRY(pull(D.lcol.p, D.nlent, lc));
    R2P_TRY(pull(D.ucol.p, D.nuent, uc));
    R2P_TRY(pull(D.f64.lval.p, 4L * D.nlent, lvv));
    R2P_TRY(pull(D.f64.uval.p, 4L * D.nuent, uvv));
    R2P_TRY(pull(D.f64.dinv.p, 4L * mtot, dv));
    R2P_TRY(pull(D.owned.p, mtot, ow));
    long k = 0;
    for (int p = a; p < b; p++) {
        int i = p - a;
        if (glob) glob[i] = g[p];
        if (level) level[i] = lv[pm[p]];
        if (owned) owned[i] = ow[p];
        if (dinv) memcpy(dinv + 4L * i, dv.data() + 4L * p, 4 * sizeof(double));
        int sl = slof[p], r = p - slst[sl];
        for (int part = 0; part < 2; part++) {
            int cnt = part == 0 ? nl[p] : nu[p];
            long base = part == 0 ? slbl[sl] : slbu[sl];
            const std::vector<int> &cc = part == 0 ? lc : uc;
            const std::vector<double> &vv = part == 0 ? lvv : uvv;
            for (int e = 0; e < cnt; e++, k++) {
                long idx = ras_entry(base, r, e);
                if (erow) erow[k] = g[p];
                if (ecol) ecol[k] = g[cc[idx] & COL_MASK];
                if (eval) memcpy(eval + 4 * k, vv.data() + 4 * idx, 4 * sizeof(double));
            }
        }
    }
    (void)m;
    return 0;
}
