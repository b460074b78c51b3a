// Learned warm start: a 3D convolutional network that predicts the Newton
// increment of a time step from the state at its start (an extension of the
// paper's Newton iteration, Algorithm 1: the prediction is only a first
// iterate, taken when it lowers the residual).
//
// Network (channels-last, [crop][z][y][x][channel], zero padding per crop):
//     h_0 = relu(conv(f, W_in)),  a_k = relu(conv(h_k, W_a,k)),
//     h_k+1 = h_k + conv(a_k, W_b,k)  (k < K),  out = conv(h_K, W_out),
// 3x3x3 taps, 32 channels.  Activations and weights are bfloat16 (rounded to
// nearest, ties to even), products accumulate in FP32; the input (6 feature
// channels) and output (2 channels) layers are stored padded to 32 channels
// with zero weights, so every layer is the same 32 -> 32 kernel.
//
// Device design.  A convolution is an implicit GEMM: for each of the 27 taps
// a wavefront multiplies 16-voxel x 32-channel blocks of shifted inputs by
// the tap's 32 x 32 weight block on the matrix cores
// (v_mfma_f32_16x16x32_bf16); a persistent workgroup per CU stages the
// weights once and each 2 x 8 x 32 output tile's input with its halo in
// LDS.  The input gradient is the same kernel
// on mirrored taps with per-tap transposed weights.  The weight gradient is a
// GEMM over voxels: each wavefront stages 32-voxel chunks of the output
// gradient and of the tap-shifted input, transposed, in LDS and accumulates
// the tap's 32 x 32 block; workgroup partials are summed in a fixed order.
// Training keeps FP32 master weights with Adam moments.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "r2p_impl.h"

namespace {

constexpr int CH = 32;                      // channels of every layer (padded)
constexpr int TAPS = 27;
constexpr int WLAYER = TAPS * CH * CH;      // weights of one padded layer
constexpr int CBS = 256;                    // conv workgroup: 4 wavefronts
constexpr int DW_VPB = 2048;                // voxels per weight-gradient workgroup
constexpr int NIN = 6, NOUT = 2;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

__host__ __device__ inline u16 to_bf16(float f) {
    unsigned u;
    memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}
__host__ __device__ inline float from_bf16(u16 h) {
    unsigned u = (unsigned)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

struct Geo {
    int nx, ny, nz, nb;
    __host__ __device__ long V() const { return (long)nx * ny * nz * nb; }
};

__device__ __forceinline__ void tap_off(int t, int &dz, int &dy, int &dx) {
    dz = t / 9 - 1;
    dy = (t / 3) % 3 - 1;
    dx = t % 3 - 1;
}

// Index of the neighbour (dz, dy, dx) of voxel v inside its own crop, or -1.
__device__ __forceinline__ long neighbour(long v, int x, int y, int z, int dz, int dy, int dx,
                                          const Geo &g) {
    int xx = x + dx, yy = y + dy, zz = z + dz;
    if (xx < 0 || xx >= g.nx || yy < 0 || yy >= g.ny || zz < 0 || zz >= g.nz) return -1;
    return v + ((long)dz * g.ny + dy) * g.nx + dx;
}

struct ConvArgs {
    const u16 *x;         // [V][32] input
    Geo g;
    const u16 *w;         // [27][32 out][32 in]
    const float *bias;    // [32] or NULL
    const u16 *addend;    // [V][32] or NULL: added to the result
    const u16 *mask;      // [V][32] or NULL: result kept where mask > 0
    int relu, flip;       // flip: taps mirrored (input-gradient form)
    u16 *out;             // [V][32] bf16 result, or NULL
    float *outf;          // [V][32] fp32 result, or NULL
};

// out[v, o] = epilogue(bias[o] + sum_t sum_i x[v + s off_t, i] w[t, o, i]),
// s = -1 when flip.  A workgroup takes tiles of TZ x TY x TX output voxels of
// one crop in turn: it stages the tile's input with its one-voxel halo (zero
// outside the crop) in LDS, next to the 27 weight blocks staged once, so the
// taps read their shifted inputs from LDS with no bounds tests.  The tile's
// 16 rows of TX voxels make 32 pieces of 16 voxels; each of the 8 wavefronts owns 4
// pieces and, per tap, multiplies each piece's 16 x 32 input block by the
// tap's 32 x 32 weight block on the matrix cores (v_mfma_f32_16x16x32_bf16,
// two 16-channel halves).  A tile reads 1,360 halo voxels for 512 outputs,
// so each input voxel is fetched from memory about 2.7 times instead of 27.
constexpr int TZ = 2, TY = 8, TX = 32;
constexpr int HZ = TZ + 2, HY = TY + 2, HX = TX + 2, HV = HZ * HY * HX;
constexpr int CWG = 512;                        // convolution workgroup: 8 wavefronts
constexpr int PIECES = TZ * TY * TX / 16;       // 16-voxel pieces per tile
constexpr int MT = PIECES / (CWG / 64);         // pieces per wavefront
constexpr int HCH = (HV * 4 + CWG - 1) / CWG;   // 16-byte halo chunks per thread

struct TileAt {
    long cb;            // first voxel of the tile's crop
    int x0, y0, z0;
};
// (32-bit arithmetic: the tile count is checked against 2^31 at launch)
__device__ __forceinline__ TileAt tile_at(int tile, const Geo &g) {
    const int ntx = (g.nx + TX - 1) / TX, nty = (g.ny + TY - 1) / TY, ntz = (g.nz + TZ - 1) / TZ;
    int rr = tile;
    TileAt T;
    T.x0 = (rr % ntx) * TX;
    rr /= ntx;
    T.y0 = (rr % nty) * TY;
    rr /= nty;
    T.z0 = (rr % ntz) * TZ;
    rr /= ntz;
    T.cb = (long)rr * ((long)g.nx * g.ny * g.nz);
    return T;
}

// This thread's chunks of a tile's input with halo (zero outside the crop).
__device__ __forceinline__ void fetch_halo(uint4 (&h)[HCH], const u16 *x, const TileAt &T,
                                           const Geo &g) {
#pragma unroll
    for (int u = 0; u < HCH; u++) {
        int c = (int)threadIdx.x + u * CWG;
        int hv = c >> 2, part = c & 3;
        int hx = hv % HX, hy = (hv / HX) % HY, hz = hv / (HX * HY);
        int gx = T.x0 + hx - 1, gy = T.y0 + hy - 1, gz = T.z0 + hz - 1;
        bool in = c < HV * 4 && gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny && gz >= 0 &&
                  gz < g.nz;
        long at = in ? (T.cb + ((long)gz * g.ny + gy) * g.nx + gx) * CH + 8 * part : 0;
        uint4 v = *reinterpret_cast<const uint4 *>(x + at);
        h[u] = in ? v : uint4{0u, 0u, 0u, 0u};
    }
}

__global__ __launch_bounds__(CWG) void k_conv(ConvArgs A) {
    __shared__ __attribute__((aligned(16))) u16 wl[WLAYER];
    __shared__ __attribute__((aligned(16))) u16 xl[HV * CH];
    for (int e = threadIdx.x; e < WLAYER / 8; e += CWG)
        reinterpret_cast<uint4 *>(wl)[e] = reinterpret_cast<const uint4 *>(A.w)[e];
    const Geo g = A.g;
    const int ntile = g.nb * ((g.nz + TZ - 1) / TZ) * ((g.ny + TY - 1) / TY) *
                      ((g.nx + TX - 1) / TX);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, kg = lane >> 4;
    // the next tile's input is requested into registers before the current
    // tile is computed, so its memory latency overlaps the matrix work
    uint4 hreg[HCH];
    // bias of this thread's eight epilogue channels
    const int part = threadIdx.x & 3;
    float bz[8];
#pragma unroll
    for (int u = 0; u < 8; u++) bz[u] = A.bias ? A.bias[8 * part + u] : 0.f;
    if ((int)blockIdx.x < ntile) fetch_halo(hreg, A.x, tile_at(blockIdx.x, g), g);
    for (int tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
        const TileAt T = tile_at(tile, g);
        const long cb = T.cb;
        const int x0 = T.x0, y0 = T.y0, z0 = T.z0;
        __syncthreads();            // weights staged; the previous tile's reads are done
#pragma unroll
        for (int u = 0; u < HCH; u++) {
            int c = (int)threadIdx.x + u * CWG;
            if (c < HV * 4) reinterpret_cast<uint4 *>(xl)[c] = hreg[u];
        }
        __syncthreads();
        if (tile + (int)gridDim.x < ntile) fetch_halo(hreg, A.x, tile_at(tile + gridDim.x, g), g);
        f32x4 acc[MT][2];
#pragma unroll
        for (int j = 0; j < MT; j++) acc[j][0] = acc[j][1] = f32x4{0.f, 0.f, 0.f, 0.f};
        // every piece is computed (pieces past the crop's edge read zeros and
        // are not stored), so a tap is straight-line code: its ten LDS reads
        // are issued ahead of its sixteen matrix instructions
#pragma unroll 3
        for (int t = 0; t < TAPS; t++) {
            int dz, dy, dx;
            tap_off(t, dz, dy, dx);
            if (A.flip) { dz = -dz; dy = -dy; dx = -dx; }
            bf16x8 b[2];
#pragma unroll
            for (int n = 0; n < 2; n++)
                b[n] = __builtin_bit_cast(
                    bf16x8, *reinterpret_cast<const uint4 *>(&wl[(t * CH + 16 * n + i) * CH + 8 * kg]));
#pragma unroll
            for (int j = 0; j < MT; j++) {
                int pc = wave * MT + j, row = pc >> 1;
                int hv = ((row / TY + 1 + dz) * HY + (row % TY + 1 + dy)) * HX + (pc & 1) * 16 + i + 1 + dx;
                bf16x8 a = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(&xl[hv * CH + 8 * kg]));
                acc[j][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[0], acc[j][0], 0, 0, 0);
                acc[j][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[1], acc[j][1], 0, 0, 0);
            }
        }
        // The results go through LDS (the halo buffer is free once every
        // wavefront has finished its taps): element (voxel 4 kg + r of piece
        // pc, channel 16 n + i) is stored at float [16 pc + 4 kg + r][32];
        // then each thread takes eight channels of a voxel, so the addend and
        // mask are read and the result written 16 bytes per lane.
        float *st = reinterpret_cast<float *>(xl);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < MT; j++) {
            int pc = wave * MT + j;
#pragma unroll
            for (int n = 0; n < 2; n++)
#pragma unroll
                for (int r = 0; r < 4; r++) st[(16 * pc + 4 * kg + r) * CH + 16 * n + i] = acc[j][n][r];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PIECES * 16 * 4 / CWG; q++) {
            int tv = q * (CWG / 4) + (int)(threadIdx.x >> 2);     // voxel of the tile
            int pc = tv >> 4, row = pc >> 1;
            int xo = x0 + (pc & 1) * 16 + (tv & 15), yo = y0 + row % TY, zo = z0 + row / TY;
            if (xo >= g.nx || yo >= g.ny || zo >= g.nz) continue;
            long vo = cb + ((long)zo * g.ny + yo) * g.nx + xo;
            float4 r0 = *reinterpret_cast<const float4 *>(&st[tv * CH + 8 * part]);
            float4 r1 = *reinterpret_cast<const float4 *>(&st[tv * CH + 8 * part + 4]);
            float val[8] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
#pragma unroll
            for (int u = 0; u < 8; u++) val[u] += bz[u];
            if (A.addend) {
                uint4 ad = *reinterpret_cast<const uint4 *>(A.addend + vo * CH + 8 * part);
                const u16 *ah = reinterpret_cast<const u16 *>(&ad);
#pragma unroll
                for (int u = 0; u < 8; u++) val[u] += from_bf16(ah[u]);
            }
            if (A.mask) {
                uint4 mk = *reinterpret_cast<const uint4 *>(A.mask + vo * CH + 8 * part);
                const u16 *mh = reinterpret_cast<const u16 *>(&mk);
#pragma unroll
                for (int u = 0; u < 8; u++) val[u] = from_bf16(mh[u]) > 0.f ? val[u] : 0.f;
            }
            if (A.relu) {
#pragma unroll
                for (int u = 0; u < 8; u++) val[u] = val[u] > 0.f ? val[u] : 0.f;
            }
            if (A.out) {
                uint4 o;
                u16 *oh = reinterpret_cast<u16 *>(&o);
#pragma unroll
                for (int u = 0; u < 8; u++) oh[u] = to_bf16(val[u]);
                *reinterpret_cast<uint4 *>(A.out + vo * CH + 8 * part) = o;
            }
            if (A.outf) {
                *reinterpret_cast<float4 *>(A.outf + vo * CH + 8 * part) =
                    make_float4(val[0], val[1], val[2], val[3]);
                *reinterpret_cast<float4 *>(A.outf + vo * CH + 8 * part + 4) =
                    make_float4(val[4], val[5], val[6], val[7]);
            }
        }
    }
}

// Weight gradient of one tap (blockIdx.y): dW[t, o, i] = sum_v gy[v, o] x[v + off_t, i]
// over the workgroup's voxels; one partial 32 x 32 block per workgroup.
constexpr int DW_ROW = 40;                  // LDS row (32 voxels) padded to 80 bytes
__global__ __launch_bounds__(CBS) void k_conv_dw(const u16 *gy, const u16 *x, Geo g, float *part) {
    __shared__ __attribute__((aligned(16))) u16 st[4][2][CH * DW_ROW];
    __shared__ float red[4][CH * CH];
    const long V = g.V();
    const int t = blockIdx.y;
    int dz, dy, dx;
    tap_off(t, dz, dy, dx);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, kg = lane >> 4;
    u16 *GT = st[wave][0], *XT = st[wave][1];
    f32x4 acc[2][2];
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    const long v0 = (long)blockIdx.x * DW_VPB;
    for (long c0 = v0 + 32 * wave; c0 < v0 + DW_VPB && c0 < V; c0 += 32 * 4) {
        // stage the chunk transposed: GT[o][q] = gy[c0+q, o], XT[i][q] = x[nb(c0+q), i]
        for (int e = lane; e < 128; e += 64) {
            int q = e >> 2, cq = e & 3;
            long vq = c0 + q;
            uint4 gr{0u, 0u, 0u, 0u}, xr{0u, 0u, 0u, 0u};
            if (vq < V) {
                gr = *reinterpret_cast<const uint4 *>(gy + vq * CH + 8 * cq);
                long r = vq;
                int xx = (int)(r % g.nx);
                r /= g.nx;
                int yy = (int)(r % g.ny);
                r /= g.ny;
                int zz = (int)(r % g.nz);
                long nb = neighbour(vq, xx, yy, zz, dz, dy, dx, g);
                if (nb >= 0) xr = *reinterpret_cast<const uint4 *>(x + nb * CH + 8 * cq);
            }
            const u16 *gs = reinterpret_cast<const u16 *>(&gr);
            const u16 *xs = reinterpret_cast<const u16 *>(&xr);
#pragma unroll
            for (int u = 0; u < 8; u++) {
                GT[(8 * cq + u) * DW_ROW + q] = gs[u];
                XT[(8 * cq + u) * DW_ROW + q] = xs[u];
            }
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);      // this wavefront's LDS writes done
        __builtin_amdgcn_wave_barrier();
        bf16x8 a[2], b[2];
#pragma unroll
        for (int mi = 0; mi < 2; mi++)
            a[mi] = __builtin_bit_cast(
                bf16x8, *reinterpret_cast<const uint4 *>(&GT[(16 * mi + i) * DW_ROW + 8 * kg]));
#pragma unroll
        for (int nj = 0; nj < 2; nj++)
            b[nj] = __builtin_bit_cast(
                bf16x8, *reinterpret_cast<const uint4 *>(&XT[(16 * nj + i) * DW_ROW + 8 * kg]));
#pragma unroll
        for (int mi = 0; mi < 2; mi++)
#pragma unroll
            for (int nj = 0; nj < 2; nj++)
                acc[mi][nj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mi], b[nj], acc[mi][nj], 0, 0, 0);
        __builtin_amdgcn_wave_barrier();
    }
#pragma unroll
    for (int mi = 0; mi < 2; mi++)
#pragma unroll
        for (int nj = 0; nj < 2; nj++)
#pragma unroll
            for (int r = 0; r < 4; r++)
                red[wave][(16 * mi + 4 * kg + r) * CH + 16 * nj + i] = acc[mi][nj][r];
    __syncthreads();
    float *out = part + ((long)blockIdx.x * TAPS + t) * CH * CH;
    for (int e = threadIdx.x; e < CH * CH; e += CBS)
        out[e] = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
}

// dst[k] = sum over nparts of part[p * stride + k], in order.
__global__ void k_sum_parts(const float *part, int nparts, long stride, long n, float *dst,
                            int accumulate) {
    long k = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (k >= n) return;
    float s = 0.f;
    for (int p = 0; p < nparts; p++) s += part[p * stride + k];
    dst[k] = accumulate ? dst[k] + s : s;
}

// Column sums of gy ([V][32]): one partial row per workgroup.
constexpr int CS_VPB = 4096;
__global__ __launch_bounds__(CBS) void k_colsum(const u16 *gy, long V, float *part) {
    __shared__ float red[CBS];
    int c = threadIdx.x & 31, r = threadIdx.x >> 5;
    long v0 = (long)blockIdx.x * CS_VPB;
    float s = 0.f;
    for (long v = v0 + r; v < v0 + CS_VPB && v < V; v += CBS / 32) s += from_bf16(gy[v * CH + c]);
    red[threadIdx.x] = s;
    __syncthreads();
    if (r == 0) {
        float t = red[c];
        for (int q = 1; q < CBS / 32; q++) t += red[q * 32 + c];
        part[(long)blockIdx.x * CH + c] = t;
    }
}

// Mean squared error over voxels and the NOUT output channels: gradient
// (bf16, padded to 32 channels) and per-workgroup partial loss sums.
__global__ __launch_bounds__(CBS) void k_mse(const float *out, const float *tgt, long V, float scale,
                                             u16 *gy, double *part) {
    __shared__ double red[CBS];
    long v = blockIdx.x * (long)CBS + threadIdx.x;
    double s = 0.0;
    if (v < V) {
        for (int c = 0; c < CH; c++) {
            float gv = 0.f;
            if (c < NOUT) {
                float d = out[v * CH + c] - tgt[v * NOUT + c];
                s += (double)d * d;
                gv = 2.f * d * scale;
            }
            gy[v * CH + c] = to_bf16(gv);
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = CBS / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_take2(const float *outf, long V, float *out2) {
    long v = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (v >= V) return;
    out2[2 * v] = outf[v * CH];
    out2[2 * v + 1] = outf[v * CH + 1];
}

// Adam on the padded FP32 master weights; then bf16 copies in the forward
// layout [t][o][i] and the input-gradient layout [t][i][o].
__global__ void k_adam(long n, float *p, const float *g, float *m, float *vv, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
    long k = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (k >= n) return;
    float gk = g[k];
    float mk = b1 * m[k] + (1.f - b1) * gk;
    float vk = b2 * vv[k] + (1.f - b2) * gk * gk;
    m[k] = mk;
    vv[k] = vk;
    p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

__global__ void k_weights_bf16(long nl, const float *w, u16 *wf, u16 *wt) {
    long k = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (k >= nl * WLAYER) return;
    long l = k / WLAYER;
    int r = (int)(k % WLAYER);
    int t = r / (CH * CH), o = (r / CH) % CH, i = r % CH;
    u16 h = to_bf16(w[k]);
    wf[k] = h;
    wt[l * WLAYER + (t * CH + i) * CH + o] = h;
}

// -------------------------------------------------------------- features
// Per cell of a state x at the start of a step of length dt (channels 0..5;
// 6..31 zero): scaled pressure, water saturation, scaled ln kh, scaled
// porosity, a well source term, ln dt.  The source of a perforated cell is
// log(1 + V) with V the pore-volume fraction its well could move in the
// step: the injected volume per perforation for a rate injector, the
// drawdown-driven volume W_i dt (p - p_bhp)^+ / PV for a BHP producer; signs
// mark injection (+) and production (-).
__global__ void k_features(int n, const double *x, double dt, const double *kx, const double *phi,
                           const int *cell_perf, const int *perf_well, const double *perf_wi,
                           const int *w_ptr, const int *w_kind, const int *w_ctrl,
                           const double *w_target, double vol, double alpha, u16 *feat) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    float f[CH];
    for (int k = 0; k < CH; k++) f[k] = 0.f;
    double p = x[2 * c], s = x[2 * c + 1];
    double pv = phi[c] * vol / alpha;
    f[0] = (float)((p - 4800.0) / 1000.0);
    f[1] = (float)s;
    f[2] = (float)((log(kx[c]) - 4.6) / 2.0);
    f[3] = (float)((phi[c] - 0.2) / 0.1);
    int pf = cell_perf[c];
    if (pf >= 0) {
        int w = perf_well[pf];
        int np = w_ptr[w + 1] - w_ptr[w];
        double q;
        if (w_ctrl[w] != R2P_BHP) q = fabs(w_target[w]) / np * dt / pv;
        else q = perf_wi[pf] * dt * fmax(fabs(p - w_target[w]), 0.0) / pv / 1000.0;
        f[4] = (float)((w_kind[w] == R2P_INJECTOR ? 1.0 : -1.0) * log1p(q));
    }
    f[5] = (float)log(dt);
    for (int k = 0; k < CH; k++) feat[(long)c * CH + k] = to_bf16(f[k]);
}

// Training target of a step x_old -> x_new: (dp / P_SCALE, ds_w / S_SCALE),
// so both channels are of order one.
constexpr double P_SCALE = 100.0, S_SCALE = 0.1;
__global__ void k_targets(int n, const double *xo, const double *xn, float *tgt) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    tgt[2 * c] = (float)((xn[2 * c] - xo[2 * c]) / P_SCALE);
    tgt[2 * c + 1] = (float)((xn[2 * c + 1] - xo[2 * c + 1]) / S_SCALE);
}

// First Newton iterate from a prediction: p += P_SCALE dp, s_w += S_SCALE ds
// (clipped to [0, 1]); a rate well's bottom-hole pressure moves by the mean
// pressure change of its perforated cells, a BHP well's stays at its target.
__global__ void k_apply_guess(int n, int nw, const double *x, const float *pred, const int *w_ptr,
                              const int *perf_cell, double *xg) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) {
        xg[2 * c] = x[2 * c] + P_SCALE * (double)pred[2 * c];
        double s = x[2 * c + 1] + S_SCALE * (double)pred[2 * c + 1];
        xg[2 * c + 1] = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
    } else if (c < n + nw) {
        int w = c - n;
        double d = 0.0;
        for (int k = w_ptr[w]; k < w_ptr[w + 1]; k++) d += P_SCALE * (double)pred[2 * perf_cell[k]];
        int np = w_ptr[w + 1] - w_ptr[w];
        xg[2 * c] = x[2 * c] + (np > 0 ? d / np : 0.0);
        xg[2 * c + 1] = x[2 * c + 1];
    }
}

// out = a where mask > 0, else 0 (bf16 tensors of n elements).
__global__ void k_mask_mul(const u16 *a, const u16 *mask, long n, u16 *out) {
    long k = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (k >= n) return;
    out[k] = from_bf16(mask[k]) > 0.f ? a[k] : (u16)0;
}

int launch_conv(const ConvArgs &A, hipStream_t s) {
    const Geo &g = A.g;
    long tiles = (long)g.nb * ((g.nz + TZ - 1) / TZ) * ((g.ny + TY - 1) / TY) * ((g.nx + TX - 1) / TX);
    if (tiles >= (1L << 31)) { r2p_set_error("convolution grid too large"); return R2P_EINVAL; }
    // one workgroup per CU (the staged weights and halo take 139 KB of LDS)
    int grid = (int)std::min<long>(tiles, r2p_cu_count());
    if (grid < 1) grid = 1;
    k_conv<<<grid, CWG, 0, s>>>(A);
    R2P_LAUNCH();
    return 0;
}

}  // namespace

// ----------------------------------------------------------------- handle
struct r2p_cnn {
    int K = 4;                  // residual blocks
    int L = 0;                  // layers = 2K + 2
    DBuf<float> w, gw, mw, vw;  // padded FP32 master weights, gradients, Adam moments
    DBuf<float> b, gb, mb, vb;  // biases [L][32]
    DBuf<u16> wf, wt;           // bf16 weights: forward and input-gradient layouts
    long step = 0;
    // activations of the last forward pass ([V][32] each) and gradients
    std::vector<DBuf<u16>> act; // f, h0, a0, h1, a1, h2, ..., h_K
    DBuf<float> outf;           // [V][32]
    DBuf<u16> g0, g1, g2;       // gradient work tensors
    DBuf<float> part, bpart;
    DBuf<double> lpart;
    DBuf<float> pred;
    DBuf<u16> feat;
    HostPinned pin;
};

namespace {

int ensure_acts(r2p_cnn *C, long V) {
    C->act.resize(2 * C->K + 2);
    for (auto &a : C->act) R2P_TRY(a.ensure((size_t)V * CH));
    R2P_TRY(C->outf.ensure((size_t)V * CH));
    R2P_TRY(C->g0.ensure((size_t)V * CH));
    R2P_TRY(C->g1.ensure((size_t)V * CH));
    R2P_TRY(C->g2.ensure((size_t)V * CH));
    return 0;
}

// Layer l: weights at wf + l * WLAYER, bias at b + l * 32.  Activation
// slots: act[0] = f, act[1] = h0, then a_k at 2 + 2k, h_{k+1} at 3 + 2k.
int forward_impl(r2p_cnn *C, const u16 *feat, Geo g, hipStream_t s) {
    long V = g.V();
    R2P_HIP(hipMemcpyAsync(C->act[0].p, feat, sizeof(u16) * V * CH, hipMemcpyDeviceToDevice, s));
    ConvArgs A{};
    A.g = g;
    A.x = C->act[0].p; A.w = C->wf.p; A.bias = C->b.p; A.relu = 1; A.out = C->act[1].p;
    R2P_TRY(launch_conv(A, s));
    for (int k = 0; k < C->K; k++) {
        int la = 1 + 2 * k, lb = 2 + 2 * k;
        ConvArgs Aa{};
        Aa.g = g;
        Aa.x = C->act[1 + 2 * k].p; Aa.w = C->wf.p + (long)la * WLAYER; Aa.bias = C->b.p + la * CH;
        Aa.relu = 1; Aa.out = C->act[2 + 2 * k].p;
        R2P_TRY(launch_conv(Aa, s));
        ConvArgs Ab{};
        Ab.g = g;
        Ab.x = C->act[2 + 2 * k].p; Ab.w = C->wf.p + (long)lb * WLAYER; Ab.bias = C->b.p + lb * CH;
        Ab.addend = C->act[1 + 2 * k].p; Ab.out = C->act[3 + 2 * k].p;
        R2P_TRY(launch_conv(Ab, s));
    }
    int lo = C->L - 1;
    ConvArgs Ao{};
    Ao.g = g;
    Ao.x = C->act[2 * C->K + 1].p; Ao.w = C->wf.p + (long)lo * WLAYER; Ao.bias = C->b.p + lo * CH;
    Ao.outf = C->outf.p;
    return launch_conv(Ao, s);
}

int weight_grad(r2p_cnn *C, const u16 *gy, const u16 *x, Geo g, int layer, hipStream_t s) {
    long V = g.V();
    int nwg = (int)((V + DW_VPB - 1) / DW_VPB);
    R2P_TRY(C->part.ensure((size_t)nwg * TAPS * CH * CH));
    k_conv_dw<<<dim3(nwg, TAPS), CBS, 0, s>>>(gy, x, g, C->part.p);
    R2P_LAUNCH();
    long n = (long)TAPS * CH * CH;
    k_sum_parts<<<r2p_blocks(n, 256), 256, 0, s>>>(C->part.p, nwg, n, n,
                                                   C->gw.p + (long)layer * WLAYER, 0);
    R2P_LAUNCH();
    int ncs = (int)((V + CS_VPB - 1) / CS_VPB);
    R2P_TRY(C->bpart.ensure((size_t)ncs * CH));
    k_colsum<<<ncs, CBS, 0, s>>>(gy, V, C->bpart.p);
    R2P_LAUNCH();
    k_sum_parts<<<1, CH, 0, s>>>(C->bpart.p, ncs, CH, CH, C->gb.p + layer * CH, 0);
    R2P_LAUNCH();
    return 0;
}

// Input gradient of layer l applied to gy, with an optional mask and addend.
int input_grad(r2p_cnn *C, const u16 *gy, Geo g, int layer, const u16 *mask, const u16 *addend,
               u16 *out, hipStream_t s) {
    ConvArgs A{};
    A.g = g;
    A.x = gy; A.w = C->wt.p + (long)layer * WLAYER; A.flip = 1;
    A.mask = mask; A.addend = addend; A.out = out;
    return launch_conv(A, s);
}

int refresh_bf16(r2p_cnn *C, hipStream_t s) {
    long n = (long)C->L * WLAYER;
    k_weights_bf16<<<r2p_blocks(n, 256), 256, 0, s>>>(C->L, C->w.p, C->wf.p, C->wt.p);
    R2P_LAUNCH();
    return 0;
}

Geo make_geo(int nb, int nz, int ny, int nx) { return Geo{nx, ny, nz, nb}; }

int check_geo(int nb, int nz, int ny, int nx) {
    if (nb < 1 || nz < 1 || ny < 1 || nx < 1 || (long)nb * nz * ny * nx > (1L << 31) / CH) {
        r2p_set_error("invalid network input shape");
        return R2P_EINVAL;
    }
    return 0;
}

// Compact parameter order: per layer W[t][cout][cin] then b[cout], with
// (cin, cout) = (6, 32) for the input layer, (32, 32) inside, (32, 2) last.
void layer_dims(const r2p_cnn *C, int l, int &cin, int &cout) {
    cin = l == 0 ? NIN : CH;
    cout = l == C->L - 1 ? NOUT : CH;
}

}  // namespace

extern "C" int r2p_cnn_param_count(int blocks, long *n_host) {
    if (blocks < 1 || blocks > 16 || !n_host) { r2p_set_error("invalid arguments"); return R2P_EINVAL; }
    *n_host = (long)TAPS * CH * NIN + CH + (long)blocks * 2 * (TAPS * CH * CH + CH) + TAPS * NOUT * CH + NOUT;
    return 0;
}

extern "C" int r2p_cnn_create(int blocks, r2p_cnn **out) {
    if (!out || blocks < 1 || blocks > 16) { r2p_set_error("invalid arguments"); return R2P_EINVAL; }
    r2p_cnn *C = new r2p_cnn();
    C->K = blocks;
    C->L = 2 * blocks + 2;
    long nw = (long)C->L * WLAYER, nb = (long)C->L * CH;
    int rc = 0;
    if ((rc = C->w.ensure(nw)) || (rc = C->gw.ensure(nw)) || (rc = C->mw.ensure(nw)) ||
        (rc = C->vw.ensure(nw)) || (rc = C->b.ensure(nb)) || (rc = C->gb.ensure(nb)) ||
        (rc = C->mb.ensure(nb)) || (rc = C->vb.ensure(nb)) || (rc = C->wf.ensure(nw)) ||
        (rc = C->wt.ensure(nw)) || (rc = C->pin.ensure(1 << 16))) {
        delete C;
        return rc;
    }
    hipMemset(C->w.p, 0, sizeof(float) * nw);
    hipMemset(C->b.p, 0, sizeof(float) * nb);
    hipMemset(C->mw.p, 0, sizeof(float) * nw);
    hipMemset(C->vw.p, 0, sizeof(float) * nw);
    hipMemset(C->mb.p, 0, sizeof(float) * nb);
    hipMemset(C->vb.p, 0, sizeof(float) * nb);
    hipMemset(C->gw.p, 0, sizeof(float) * nw);
    hipMemset(C->gb.p, 0, sizeof(float) * nb);
    if (refresh_bf16(C, nullptr)) { delete C; return R2P_EHIP; }
    if (hipDeviceSynchronize() != hipSuccess) { delete C; r2p_set_error("HIP error"); return R2P_EHIP; }
    *out = C;
    return 0;
}

extern "C" int r2p_cnn_destroy(r2p_cnn *C) {
    delete C;
    return 0;
}

extern "C" int r2p_cnn_set_params(r2p_cnn *C, const float *theta) {
    if (!C || !theta) { r2p_set_error("NULL argument"); return R2P_EINVAL; }
    std::vector<float> w((size_t)C->L * WLAYER, 0.f), b((size_t)C->L * CH, 0.f);
    long o = 0;
    for (int l = 0; l < C->L; l++) {
        int cin, cout;
        layer_dims(C, l, cin, cout);
        for (int t = 0; t < TAPS; t++)
            for (int co = 0; co < cout; co++)
                for (int ci = 0; ci < cin; ci++) w[(size_t)l * WLAYER + (t * CH + co) * CH + ci] = theta[o++];
        for (int co = 0; co < cout; co++) b[(size_t)l * CH + co] = theta[o++];
    }
    R2P_HIP(hipMemcpy(C->w.p, w.data(), sizeof(float) * w.size(), hipMemcpyHostToDevice));
    R2P_HIP(hipMemcpy(C->b.p, b.data(), sizeof(float) * b.size(), hipMemcpyHostToDevice));
    R2P_HIP(hipMemset(C->mw.p, 0, sizeof(float) * w.size()));
    R2P_HIP(hipMemset(C->vw.p, 0, sizeof(float) * w.size()));
    R2P_HIP(hipMemset(C->mb.p, 0, sizeof(float) * b.size()));
    R2P_HIP(hipMemset(C->vb.p, 0, sizeof(float) * b.size()));
    C->step = 0;
    R2P_TRY(refresh_bf16(C, nullptr));
    R2P_HIP(hipDeviceSynchronize());
    return 0;
}

static int pull_compact(r2p_cnn *C, const float *wdev, const float *bdev, float *theta) {
    std::vector<float> w((size_t)C->L * WLAYER), b((size_t)C->L * CH);
    R2P_HIP(hipDeviceSynchronize());
    R2P_HIP(hipMemcpy(w.data(), wdev, sizeof(float) * w.size(), hipMemcpyDeviceToHost));
    R2P_HIP(hipMemcpy(b.data(), bdev, sizeof(float) * b.size(), hipMemcpyDeviceToHost));
    long o = 0;
    for (int l = 0; l < C->L; l++) {
        int cin, cout;
        layer_dims(C, l, cin, cout);
        for (int t = 0; t < TAPS; t++)
            for (int co = 0; co < cout; co++)
                for (int ci = 0; ci < cin; ci++) theta[o++] = w[(size_t)l * WLAYER + (t * CH + co) * CH + ci];
        for (int co = 0; co < cout; co++) theta[o++] = b[(size_t)l * CH + co];
    }
    return 0;
}

extern "C" int r2p_cnn_get_params(r2p_cnn *C, float *theta) {
    if (!C || !theta) { r2p_set_error("NULL argument"); return R2P_EINVAL; }
    return pull_compact(C, C->w.p, C->b.p, theta);
}

extern "C" int r2p_cnn_get_grads(r2p_cnn *C, float *grad) {
    if (!C || !grad) { r2p_set_error("NULL argument"); return R2P_EINVAL; }
    return pull_compact(C, C->gw.p, C->gb.p, grad);
}

extern "C" int r2p_cnn_forward(r2p_cnn *C, const uint16_t *feat, int nb, int nz, int ny, int nx,
                               float *out, void *stream) {
    if (!C || !feat || !out) { r2p_set_error("NULL argument"); return R2P_EINVAL; }
    R2P_TRY(check_geo(nb, nz, ny, nx));
    hipStream_t s = (hipStream_t)stream;
    Geo g = make_geo(nb, nz, ny, nx);
    R2P_TRY(ensure_acts(C, g.V()));
    R2P_TRY(forward_impl(C, feat, g, s));
    k_take2<<<r2p_blocks(g.V(), 256), 256, 0, s>>>(C->outf.p, g.V(), out);
    R2P_LAUNCH();
    return 0;
}

extern "C" int r2p_cnn_backward(r2p_cnn *C, const uint16_t *feat, const float *target, int nb,
                                int nz, int ny, int nx, double *loss_host, void *stream) {
    if (!C || !feat || !target) { r2p_set_error("NULL argument"); return R2P_EINVAL; }
    R2P_TRY(check_geo(nb, nz, ny, nx));
    hipStream_t s = (hipStream_t)stream;
    Geo g = make_geo(nb, nz, ny, nx);
    long V = g.V();
    R2P_TRY(ensure_acts(C, V));
    R2P_TRY(forward_impl(C, feat, g, s));
    int nbl = r2p_blocks(V, CBS);
    R2P_TRY(C->lpart.ensure(nbl));
    k_mse<<<nbl, CBS, 0, s>>>(C->outf.p, target, V, 1.0f / (float)(V * NOUT), C->g0.p, C->lpart.p);
    R2P_LAUNCH();
    // output layer
    int lo = C->L - 1, K = C->K;
    R2P_TRY(weight_grad(C, C->g0.p, C->act[2 * K + 1].p, g, lo, s));
    R2P_TRY(input_grad(C, C->g0.p, g, lo, nullptr, nullptr, C->g1.p, s));   // gh
    u16 *gh = C->g1.p, *ga = C->g2.p, *spare = C->g0.p;
    for (int k = K - 1; k >= 0; k--) {
        int la = 1 + 2 * k, lb = 2 + 2 * k;
        const u16 *a = C->act[2 + 2 * k].p, *h = C->act[1 + 2 * k].p;
        R2P_TRY(weight_grad(C, gh, a, g, lb, s));
        R2P_TRY(input_grad(C, gh, g, lb, a, nullptr, ga, s));               // ga = (W_b^T gh) (a > 0)
        R2P_TRY(weight_grad(C, ga, h, g, la, s));
        R2P_TRY(input_grad(C, ga, g, la, nullptr, gh, spare, s));          // gh' = gh + W_a^T ga
        std::swap(gh, spare);
    }
    // input layer: g0 = gh (h0 > 0)
    u16 *g0m = spare;
    k_mask_mul<<<r2p_blocks(V * CH, 256), 256, 0, s>>>(gh, C->act[1].p, V * CH, g0m);
    R2P_LAUNCH();
    R2P_TRY(weight_grad(C, g0m, C->act[0].p, g, 0, s));
    if (loss_host) {
        std::vector<double> lp(nbl);
        R2P_HIP(hipStreamSynchronize(s));
        R2P_HIP(hipMemcpy(lp.data(), C->lpart.p, sizeof(double) * nbl, hipMemcpyDeviceToHost));
        double t = 0.0;
        for (int i = 0; i < nbl; i++) t += lp[i];
        *loss_host = t / (double)(V * NOUT);
    }
    return 0;
}

extern "C" int r2p_cnn_sgd_step(r2p_cnn *C, float lr, void *stream) {
    if (!C || !(lr > 0.f)) { r2p_set_error("invalid arguments"); return R2P_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    C->step++;
    float c1 = 1.f - powf(b1, (float)C->step), c2 = 1.f - powf(b2, (float)C->step);
    long nw = (long)C->L * WLAYER, nb = (long)C->L * CH;
    k_adam<<<r2p_blocks(nw, 256), 256, 0, s>>>(nw, C->w.p, C->gw.p, C->mw.p, C->vw.p, lr, b1, b2,
                                               eps, c1, c2);
    R2P_LAUNCH();
    k_adam<<<r2p_blocks(nb, 256), 256, 0, s>>>(nb, C->b.p, C->gb.p, C->mb.p, C->vb.p, lr, b1, b2,
                                               eps, c1, c2);
    R2P_LAUNCH();
    return refresh_bf16(C, s);
}

extern "C" int r2p_cnn_conv(const uint16_t *x, int nb, int nz, int ny, int nx, const uint16_t *w,
                            const float *bias, const uint16_t *addend, const uint16_t *mask,
                            int relu, int flip, uint16_t *out, float *outf, void *stream) {
    if (!x || !w || (!out && !outf)) { r2p_set_error("NULL argument"); return R2P_EINVAL; }
    R2P_TRY(check_geo(nb, nz, ny, nx));
    ConvArgs A{};
    A.x = x; A.g = make_geo(nb, nz, ny, nx); A.w = w; A.bias = bias; A.addend = addend;
    A.mask = mask; A.relu = relu; A.flip = flip; A.out = out; A.outf = outf;
    return launch_conv(A, (hipStream_t)stream);
}

extern "C" int r2p_cnn_conv_dw(const uint16_t *gy, const uint16_t *x, int nb, int nz, int ny,
                               int nx, float *dw, float *db, void *stream) {
    if (!gy || !x || !dw || !db) { r2p_set_error("NULL argument"); return R2P_EINVAL; }
    R2P_TRY(check_geo(nb, nz, ny, nx));
    hipStream_t s = (hipStream_t)stream;
    Geo g = make_geo(nb, nz, ny, nx);
    long V = g.V();
    int nwg = (int)((V + DW_VPB - 1) / DW_VPB);
    DBuf<float> part, bpart;
    R2P_TRY(part.ensure((size_t)nwg * TAPS * CH * CH));
    k_conv_dw<<<dim3(nwg, TAPS), CBS, 0, s>>>(gy, x, g, part.p);
    R2P_LAUNCH();
    long n = (long)TAPS * CH * CH;
    k_sum_parts<<<r2p_blocks(n, 256), 256, 0, s>>>(part.p, nwg, n, n, dw, 0);
    R2P_LAUNCH();
    int ncs = (int)((V + CS_VPB - 1) / CS_VPB);
    R2P_TRY(bpart.ensure((size_t)ncs * CH));
    k_colsum<<<ncs, CBS, 0, s>>>(gy, V, bpart.p);
    R2P_LAUNCH();
    k_sum_parts<<<1, CH, 0, s>>>(bpart.p, ncs, CH, CH, db, 0);
    R2P_LAUNCH();
    R2P_HIP(hipStreamSynchronize(s));
    return 0;
}

extern "C" int r2p_cnn_features(r2p_model *m, const double *x, double dt, uint16_t *feat,
                                void *stream) {
    if (!m || !x || !feat || !(dt > 0)) { r2p_set_error("invalid arguments"); return R2P_EINVAL; }
    const Phys &ph = m->ph;
    k_features<<<r2p_blocks(ph.n, 256), 256, 0, (hipStream_t)stream>>>(
        ph.n, x, dt, m->kx.p, m->phi.p, m->cell_perf.p, m->perf_well.p, m->perf_wi.p, m->w_ptr.p,
        m->w_kind.p, m->w_ctrl.p, m->w_target.p, ph.dx * ph.dy * ph.dz, ph.alpha, feat);
    R2P_LAUNCH();
    return 0;
}

extern "C" int r2p_cnn_targets(r2p_model *m, const double *x_old, const double *x_new,
                               float *target, void *stream) {
    if (!m || !x_old || !x_new || !target) { r2p_set_error("NULL argument"); return R2P_EINVAL; }
    k_targets<<<r2p_blocks(m->ph.n, 256), 256, 0, (hipStream_t)stream>>>(m->ph.n, x_old, x_new,
                                                                          target);
    R2P_LAUNCH();
    return 0;
}

extern "C" int r2p_cnn_warm_start(r2p_model *m, r2p_cnn *C, const double *x, double dt,
                                  double *x_guess, void *stream) {
    if (!m || !C || !x || !x_guess || !(dt > 0)) { r2p_set_error("invalid arguments"); return R2P_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    const Phys &ph = m->ph;
    R2P_TRY(C->feat.ensure((size_t)ph.n * CH));
    R2P_TRY(C->pred.ensure(2L * ph.n));
    R2P_TRY(r2p_cnn_features(m, x, dt, C->feat.p, stream));
    R2P_TRY(r2p_cnn_forward(C, C->feat.p, 1, ph.nz, ph.ny, ph.nx, C->pred.p, stream));
    k_apply_guess<<<r2p_blocks(ph.n + ph.nw, 256), 256, 0, s>>>(ph.n, ph.nw, x, C->pred.p,
                                                                 m->w_ptr.p, m->perf_cell.p, x_guess);
    R2P_LAUNCH();
    return 0;
}
