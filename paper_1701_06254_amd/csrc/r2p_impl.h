// Internal definitions of the r2p device library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "../../include/r2p.h"

// ------------------------------------------------------------------ errors
void r2p_set_error(const char *fmt, ...);
int r2p_hip_fail(hipError_t e, const char *what, const char *file, int line);

#define R2P_HIP(expr)                                                          \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess) return r2p_hip_fail(e_, #expr, __FILE__, __LINE__); \
    } while (0)

#define R2P_TRY(expr)                                                          \
    do {                                                                       \
        int rc_ = (expr);                                                      \
        if (rc_ < 0) return rc_;                                               \
    } while (0)

#define R2P_LAUNCH()  R2P_HIP(hipGetLastError())

// ------------------------------------------------------- device allocations
// Grow-only device buffer; contents are not preserved on growth.
struct DevMem {
    void *p = nullptr;
    size_t bytes = 0;
    int ensure(size_t nbytes);
    void release();
    ~DevMem() { release(); }
};

template <class T>
struct DBuf {
    DevMem mem;
    T *p = nullptr;
    size_t cap = 0;
    int ensure(size_t n) {
        size_t need = n > 0 ? n : 1;
        if (need <= cap && p) return 0;
        int rc = mem.ensure(need * sizeof(T));
        if (rc) return rc;
        p = (T *)mem.p;
        cap = need;
        return 0;
    }
    void release() { mem.release(); p = nullptr; cap = 0; }
};

// Pinned host staging for small read-backs.
struct HostPinned {
    void *p = nullptr;
    size_t bytes = 0;
    int ensure(size_t nbytes);
    ~HostPinned();
};

// --------------------------------------------------------------- physics
struct Phys {
    int nx, ny, nz, n, nw, nperf;
    double dx, dy, dz, top;
    double beta, alpha, rho_o, rho_w, p_ref, z_ref, c_o, c_w, c_r, mu_o, mu_w, grav;
};

struct NewtonWork;
void r2p_newton_work_free(NewtonWork *W);

struct r2p_model {
    int dev = 0;
    unsigned long long serial = 0;     // unique over the process: caches are keyed by it
    NewtonWork *newton = nullptr;      // workspace of r2p_newton_step, freed with the model
    Phys ph{};
    // device arrays
    DBuf<double> kx, ky, kz, phi;      // n
    DBuf<double> tx, ty, tz;           // n: geometric transmissibility to the +x/+y/+z neighbour
    DBuf<int> cell_perf;               // n: perforation index or -1
    DBuf<int> perf_cell, perf_well;    // nperf
    DBuf<double> perf_wi;              // nperf
    DBuf<int> w_ptr, w_kind, w_ctrl;   // nw(+1)
    DBuf<double> w_target, w_zb, w_rw, w_skin;
    // host copies of the well description
    std::vector<int> h_w_ptr, h_w_cell, h_w_kind, h_w_ctrl;
    std::vector<double> h_w_target;
    // reduction scratch
    DBuf<unsigned long long> red;
    HostPinned pin;
};

// Jacobian in a 7-slot stencil layout: slot 0 = the cell itself, 1/2 = -x/+x,
// 3/4 = -y/+y, 5/6 = -z/+z.  Columns are implied by the grid; a slot whose
// neighbour does not exist holds a zero block and a clamped column.  Each
// block [[a00 a01] [a10 a11]] is split into a pressure-column plane
// vp = (a00, a10) and a saturation-column plane vs = (a01, a11), slot-major:
// vp[slot*n + c].
struct r2p_jacobian {
    r2p_model *m = nullptr;
    unsigned long long serial = 0;      // serial of the model it was created for
    DBuf<double2> vp, vs;   // 7n
    DBuf<double2> cw;       // nperf: d(cell oil, water eq)/d p_b
    DBuf<double2> wc;       // nperf: d(well eq)/d(p_cell, s_cell)
    DBuf<double> wd;        // nw: d(well eq)/d p_b
    DBuf<double> phi_o;     // n: oil potential at the assembled state
    DBuf<double4> dec;      // n: decoupling row operator D_i^-1 (row-major)
    int state = 0;          // 0 empty, 1 assembled, 2 decoupled
    int dec_kind = 0;
};

__host__ __device__ inline int slot_offset(int s, int nx, int nxy) {
    switch (s) {
    case 1: return -1;
    case 2: return 1;
    case 3: return -nx;
    case 4: return nx;
    case 5: return -nxy;
    case 6: return nxy;
    default: return 0;
    }
}

// ------------------------------------------------------------------ RAS
// Block ILU(0) factors of every overlapped subdomain.  Rows ("positions" p,
// concatenated over subdomains) are stored in level order of each
// subdomain's dependency graph, rows of a level sorted by descending number
// of predecessors.  Every level is cut into slices of RAS_ROWS consecutive
// positions, one wavefront per slice and two lanes per row (lane 2r + h
// holds the entries e = h, h + 2, ... of row r).  A slice stores its L
// blocks (predecessors, ascending local order) and its U blocks (successors)
// in sliced-ELL form with RAS_SLICE entries per column: entry e of row r
// sits at base + (e / 2) RAS_SLICE + 2r + (e mod 2), so each load
// instruction of a wavefront is contiguous.  Padding entries (e >= the
// row's count) hold column -1 and zero blocks.
constexpr int RAS_SLICE = 64;
constexpr int RAS_ROWS = 32;
__host__ __device__ inline long ras_entry(long base, int r, int e) {
    return base + (long)(e >> 1) * RAS_SLICE + 2 * r + (e & 1);
}
template <class T>
struct RasFactors {
    DBuf<T> lval, uval;   // 4 per entry (row-major 2x2)
    DBuf<T> dinv;         // 4 per position: inverse of U's diagonal block
};

struct RasStatic {
    // membership and local adjacency (depend on model + px, py, overlap only)
    int ns = 0, px = 0, py = 0, overlap = -1;
    int mtot = 0;                         // total local rows over subdomains
    std::vector<int> h_off;               // ns+1 local row offsets per subdomain
    DBuf<int> glob_nat;                   // mtot: global row of local row (natural order)
    DBuf<unsigned char> owned_nat;        // mtot
    DBuf<int> aptr, adj, asrc;            // local adjacency: neighbour local index, block source
    int nadj = 0;
    DBuf<int> dsrc;                       // mtot: source of the diagonal block
    DBuf<int> sub_of;                     // mtot: subdomain of local row
};

struct RasDyn {
    int maxlev = 0;
    int nseg = 0, nslice = 0, nlent = 0, nuent = 0;
    std::vector<int> h_nlev;              // levels per subdomain
    std::vector<int> h_lbase;             // first segment (level) index per subdomain
    DBuf<int> lev;                        // mtot: level of local row (natural)
    DBuf<int> suboff;                     // ns+1: first local row of every subdomain
    DBuf<int> indeg, queue;               // mtot: level computation (set-up only)
    DBuf<unsigned char> apred;            // nadj: coupling e of row l is a predecessor of l
    DBuf<int> nlnat, nunat;               // mtot: predecessor / successor counts (natural)
    DBuf<int> pos;                        // mtot: position of local row
    DBuf<int> perm;                       // mtot: local row (natural) at position
    DBuf<int> glob;                       // mtot: global row at position
    DBuf<unsigned char> owned;            // mtot
    DBuf<int> nl, nu;                     // mtot: counts per position
    DBuf<int> lptr_dev;                   // nseg+1: first position of every level
    DBuf<int> soff;                       // nseg+1: first slice of every level
    DBuf<int> sl_start, sl_cnt, sl_wl, sl_wu, sl_bl, sl_bu;   // per slice
    DBuf<int> sl_of;                      // mtot: slice of every position
    DBuf<int4> meta_l, meta_u;            // per slice: (start, rows | slot pairs << 8, entry base, level) of L / U
    DBuf<int> lcol, ucol;                 // entries: column position (-1 padding)
    DBuf<int> lsrc, usrc;                 // entries: block source (set-up only)
    DBuf<int> dsrc_pos;                   // mtot: diagonal block source per position
    DBuf<int> ldiag;                      // L entries: entry of U_qp in row q (set-up only)
    DBuf<int> xptr;                       // mtot+1: extra ILU(0) matches per position
    DBuf<int4> xl;                        // extra matches (set-up only)
    DBuf<int> sub_lbase;                  // ns: first segment of the subdomain
    DBuf<int> sub_nlev;                   // ns
    DBuf<int> counters;                   // scratch
    DBuf<int> prog;                       // ns: sweep progress read by the prefetch helpers
    DBuf<int> swin;                       // ns: ring window of every subdomain's sweep
    RasFactors<double> f64;
    RasFactors<float> f32;
};

// ------------------------------------------------------------------ AMG
template <class T>
struct AmgLevelT {
    DBuf<T> val;
    DBuf<T> l1;
};

struct AmgLevel {
    int n = 0, nnz = 0;
    DBuf<int> rp, col;
    DBuf<double> val, l1;
    DBuf<int> agg;           // n: row of the next level
    DBuf<int> mptr, mem;     // next level's member lists (n_next+1, n)
    DBuf<int> big;           // next-level rows with many members (restricted by a wavefront)
    int nbig = 0;
    DBuf<int> heavy;         // rows with many entries (smoothed by a wavefront)
    int nheavy = 0;
    DBuf<double> v7;         // level 0 only: A_pp in the 7-slot stencil layout (slot-major)
    DBuf<float> v7f;
    AmgLevelT<float> f32;
    DBuf<double> b, x, xo;   // work vectors (fp64)
    DBuf<float> bf, xf, xof; // work vectors (fp32)
    DBuf<double> kv;         // K-cycle level: p1, p2, q1, q2 (4n, fp64)
    DBuf<float> kvf;         // the same in fp32
};

// Scratch of the set-up kept in the handle, so that repeated set-ups at the
// same size allocate nothing.  Each helper names which entries it uses; no
// two helpers that use the same entry are live at once.
struct SetupWork {
    DBuf<unsigned> u[6];
    DBuf<int> i[4];
    DBuf<double> d[2];
    DBuf<int> agg;                        // aggregates of the current pass
    DBuf<int> crp[2], ccol[2];            // intermediate Galerkin products
    DBuf<double> cval[2];
};

struct Krylov;

struct r2p_cpr {
    r2p_cpr_opts o{};
    Krylov *kry = nullptr;   // Krylov basis and work vectors of the solves with this handle
    SetupWork ws;
    r2p_jacobian *J = nullptr;
    int ready = 0;
    RasStatic rs;
    RasDyn rd;
    int nlev = 0;
    AmgLevel lv[24];
    int ncoarse = 0;
    DBuf<double> cinv;       // coarsest inverse, column-major: cinv[c*n + i] = (A^-1)_ic
    DBuf<float> cinvf;
    DBuf<double> lu;         // coarsest dense LU scratch
    DBuf<int> piv;
    DBuf<double> kscal;      // K-cycle scalars {q1.q1, a1, beta, a2} per level
    DBuf<double> kpart;      // K-cycle dot-product partial sums
    DBuf<double> t_ares;           // pressure stage: residual for the later cycles
    DBuf<int> status;        // device status flags
    // level-0 structure cache, and the model the cached structures belong to
    int app_n = -1;
    unsigned long long serial = 0;
    // work vectors
    DBuf<double> t_r, t_y, t_xp, t_ras, t_rl;
    DBuf<float> t_rasf, t_rlf;
    DBuf<int> iscratch;
    DBuf<int> iscratch2;
    DBuf<double> dscratch;
    HostPinned pin;
    // The AMG set-up runs on a host thread and stream of its own beside the
    // RAS set-up, so it owns its scratch, pinned word and status flag.
    SetupWork aws;
    DBuf<int> aiscratch;
    DBuf<int> astatus;
    HostPinned apin;
    hipStream_t as = nullptr;            // non-blocking, default priority
    hipEvent_t aev[2] = {nullptr, nullptr};
    // host wall times of the last set-up's stages (ms): decoupling; reordering
    // (levels and local order); block ILU(0); AMG (on its own thread, beside
    // the two before it)
    double ms_dec = 0, ms_order = 0, ms_ras = 0, ms_amg = 0;
    ~r2p_cpr();
};

// ------------------------------------------------------------ utilities
// Exclusive scan of n ints (in may equal out); returns the total if
// total_host != NULL (synchronises the stream).
// Stable radix sort of n (key, value) pairs on the low key_bits bits of the
// key, in place (ktmp/vtmp: scratch of n each).
int r2p_sort_pairs(unsigned *key, unsigned *val, unsigned *ktmp, unsigned *vtmp, int n,
                   int key_bits, DBuf<int> &hist, DBuf<int> &tmp, HostPinned &pin, hipStream_t s);
inline int r2p_bits_for(long n) {
    int b = 1;
    while ((1L << b) < n) b++;
    return b;
}
int r2p_scan_int(const int *in, int *out, int n, int *total_host, DBuf<int> &tmp,
                 HostPinned &pin, hipStream_t s);

inline int r2p_blocks(long n, int bs) { return (int)((n + bs - 1) / bs); }

// Host wall clock in ms (steady).
double r2p_now_ms();

// Compute units of the current device (cached per device).
int r2p_cu_count();

// Workgroups are dealt to the 8 XCDs in turn (workgroup b runs on XCD
// b mod 8), each XCD with its own L2.  This renumbering gives XCD x a
// contiguous range of the nb logical blocks, so grid neighbours read by a
// stencil (the x vector at +-nx and +-nx*ny) are found in that XCD's L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    int q = nb >> 3, rem = nb & 7, x = b & 7, k = b >> 3;
    return x < rem ? x * (q + 1) + k : rem * (q + 1) + (x - rem) * q + k;
}

// Streaming load of a 16-byte pair that is read once per launch: marked
// non-temporal so it does not displace reused data from the caches.
__device__ __forceinline__ double2 ld_stream2(const double2 *p) {
    typedef double v2 __attribute__((ext_vector_type(2)));
    v2 v = __builtin_nontemporal_load((const v2 *)p);
    return make_double2(v.x, v.y);
}
template <class T>
__device__ __forceinline__ T ld_stream(const T *p) {
    return __builtin_nontemporal_load(p);
}

// Source of a Jacobian block for the subdomain matrices: >= 0 is a slot block
// index (slot*n + row) into vp/vs; -(1+q) the cell row's well column cw[q];
// -(1+nperf+q) the well row's cell block wc[q]; -(1+2*nperf+w) the well
// diagonal [[wd[w], 0], [0, 1]].
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

// Internal entry points shared between translation units.
int r2p_ras_static(r2p_cpr *P, hipStream_t s);
int r2p_cpr_apply_impl(r2p_cpr *P, const double *f, double *z, hipStream_t s);
int r2p_spmv_impl(r2p_jacobian *J, const double *x, double *y, const double *f, hipStream_t s);
int r2p_decouple_rhs(r2p_jacobian *J, const double *b, double *bd, hipStream_t s);
int r2p_ras_setup(r2p_cpr *P, hipStream_t s);
int r2p_amg_setup(r2p_cpr *P, hipStream_t s);
int r2p_ras_solve(r2p_cpr *P, const double *r, double *out, const double *xp, int accumulate,
                  hipStream_t s);
int r2p_amg_cycle(r2p_cpr *P, const double *f, int fstride, double *xp, hipStream_t s);
int r2p_amg_apply(r2p_cpr *P, const double *f, int fstride, double *xp, hipStream_t s);
int r2p_pcol_residual(r2p_jacobian *J, const double *f, const double *xp, double *r,
                      hipStream_t s);
int r2p_decouple_jacobian(r2p_jacobian *J, int kind, hipStream_t s);
int r2p_newton_update(r2p_model *m, const double *y, double *x, double ds_max, hipStream_t s);
