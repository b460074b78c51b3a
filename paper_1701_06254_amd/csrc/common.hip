// Error reporting, device/pinned buffers and a device exclusive scan.
#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstring>

#include "r2p_impl.h"

static thread_local char g_err[512] = "";

void r2p_set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int r2p_hip_fail(hipError_t e, const char *what, const char *file, int line) {
    r2p_set_error("HIP error %d (%s) in %s at %s:%d", (int)e, hipGetErrorString(e), what, file,
                  line);
    return e == hipErrorOutOfMemory ? R2P_ENOMEM : R2P_EHIP;
}

extern "C" const char *r2p_last_error(void) { return g_err; }

int DevMem::ensure(size_t nbytes) {
    if (nbytes <= bytes && p) return 0;
    release();
    hipError_t e = hipMalloc(&p, nbytes);
    if (e != hipSuccess) {
        p = nullptr;
        bytes = 0;
        (void)hipGetLastError();
        r2p_set_error("hipMalloc(%zu bytes) failed: %s", nbytes, hipGetErrorString(e));
        return R2P_ENOMEM;
    }
    bytes = nbytes;
    return 0;
}

void DevMem::release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

int HostPinned::ensure(size_t nbytes) {
    if (nbytes <= bytes && p) return 0;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
    hipError_t e = hipHostMalloc(&p, nbytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        p = nullptr;
        r2p_set_error("hipHostMalloc(%zu) failed: %s", nbytes, hipGetErrorString(e));
        return R2P_ENOMEM;
    }
    bytes = nbytes;
    return 0;
}

HostPinned::~HostPinned() {
    if (p) (void)hipHostFree(p);
}

// ------------------------------------------------------------------ scan
// Three passes: per-tile sums, a scan of the tile sums by one workgroup, then
// per-tile scans offset by the scanned sums.  Tiles of 4096 ints (1024 lanes
// x 4), fixed summation order, so the result is deterministic.
constexpr int SCAN_BS = 1024;
constexpr int SCAN_PER = 4;
constexpr int SCAN_TILE = SCAN_BS * SCAN_PER;

__device__ inline int block_excl_scan(int v, int *lds, int *total) {
    // inclusive within the wavefront
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int x = v;
    for (int d = 1; d < 64; d <<= 1) {
        int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) lds[wid] = x;
    __syncthreads();
    int nw = blockDim.x >> 6;
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int w = 0; w < nw; w++) {
            int t = lds[w];
            lds[w] = acc;
            acc += t;
        }
        lds[nw] = acc;
    }
    __syncthreads();
    int r = x - v + lds[wid];
    if (total) *total = lds[nw];
    __syncthreads();
    return r;
}

__global__ void k_scan_tiles(const int *in, int n, int *tsum) {
    __shared__ int lds[SCAN_BS / 64 + 1];
    long base = (long)blockIdx.x * SCAN_TILE + (long)threadIdx.x * SCAN_PER;
    int s = 0;
    for (int k = 0; k < SCAN_PER; k++)
        if (base + k < n) s += in[base + k];
    int tot;
    block_excl_scan(s, lds, &tot);
    if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

__global__ void k_scan_sums(int *tsum, int nt, int *total) {
    __shared__ int lds[SCAN_BS / 64 + 1];
    int per = (nt + SCAN_BS - 1) / SCAN_BS;
    long base = (long)threadIdx.x * per;
    int s = 0;
    for (int k = 0; k < per; k++)
        if (base + k < nt) s += tsum[base + k];
    int tot;
    int off = block_excl_scan(s, lds, &tot);
    for (int k = 0; k < per; k++)
        if (base + k < nt) {
            int t = tsum[base + k];
            tsum[base + k] = off;
            off += t;
        }
    if (threadIdx.x == 0) *total = tot;
}

__global__ void k_scan_apply(const int *in, int *out, int n, const int *tsum) {
    __shared__ int lds[SCAN_BS / 64 + 1];
    long base = (long)blockIdx.x * SCAN_TILE + (long)threadIdx.x * SCAN_PER;
    int v[SCAN_PER];
    int s = 0;
    for (int k = 0; k < SCAN_PER; k++) {
        v[k] = base + k < n ? in[base + k] : 0;
        s += v[k];
    }
    int off = block_excl_scan(s, lds, nullptr) + tsum[blockIdx.x];
    for (int k = 0; k < SCAN_PER; k++)
        if (base + k < n) {
            out[base + k] = off;
            off += v[k];
        }
}

// ------------------------------------------------------------ radix sort
// Stable least-significant-digit radix sort of (key, value) pairs, 8 bits per
// pass.  Each pass: per-tile digit histograms (digit-major, so one exclusive
// scan gives every tile's start for every digit in stable order), then a
// scatter in which every element's rank among equal digits of its tile is
// found with wavefront ballots and carried across the tile's rounds in LDS.
// Fixed tiles and fixed order: the result is deterministic.
constexpr int RS_BS = 256;
constexpr int RS_ROUNDS = 16;
constexpr int RS_TILE = RS_BS * RS_ROUNDS;

__global__ __launch_bounds__(RS_BS) void k_rs_hist(const unsigned *key, int n, int shift,
                                                   int ntiles, int *hist) {
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    long base = (long)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ROUNDS; r++) {
        long i = base + (long)r * RS_BS + threadIdx.x;
        if (i < n) atomicAdd(&h[(key[i] >> shift) & 255u], 1);
    }
    __syncthreads();
    hist[(long)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Scatter of one pass.  Every element's stable rank among the equal digits
// of its tile comes from wavefront ballots, carried across the tile's
// rounds in LDS; the tile is then placed in LDS in digit order and written
// out from there, so each digit's run of the tile leaves as consecutive
// addresses instead of one element per digit per round.
__global__ __launch_bounds__(RS_BS) void k_rs_scatter(const unsigned *key, const unsigned *val,
                                                      int n, int shift, int ntiles,
                                                      const int *off, unsigned *okey,
                                                      unsigned *oval) {
    __shared__ int run[256];
    __shared__ int wc[RS_BS / 64][256];
    __shared__ int toff[256], goff[256];
    __shared__ unsigned sk[RS_TILE], sv[RS_TILE];
    int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    run[threadIdx.x] = 0;
    goff[threadIdx.x] = off[(long)threadIdx.x * ntiles + blockIdx.x];
    long base = (long)blockIdx.x * RS_TILE;
    int cnt = (int)min((long)RS_TILE, (long)n - base);
    unsigned long long lt = (1ull << lane) - 1ull;
    unsigned kr[RS_ROUNDS], vr[RS_ROUNDS];
    int rk[RS_ROUNDS];
#pragma unroll
    for (int r = 0; r < RS_ROUNDS; r++) {
        int j = r * RS_BS + threadIdx.x;
        bool valid = j < cnt;
        kr[r] = valid ? key[base + j] : 0u;
        vr[r] = valid ? val[base + j] : 0u;
    }
#pragma unroll
    for (int r = 0; r < RS_ROUNDS; r++) {
        for (int w = 0; w < RS_BS / 64; w++) wc[w][threadIdx.x] = 0;
        __syncthreads();
        bool valid = r * RS_BS + (int)threadIdx.x < cnt;
        unsigned d = (kr[r] >> shift) & 255u;
        unsigned long long peers = __ballot(valid);
        for (int b = 0; b < 8; b++) {
            unsigned long long bb = __ballot(valid && ((d >> b) & 1u));
            peers &= ((d >> b) & 1u) ? bb : ~bb;
        }
        int rank_w = __popcll(peers & lt);
        if (valid && rank_w == 0) wc[wid][d] = __popcll(peers);
        __syncthreads();
        int before = 0;
        for (int w = 0; w < wid; w++) before += wc[w][d];
        rk[r] = run[d] + before + rank_w;
        __syncthreads();
        int add = 0;
        for (int w = 0; w < RS_BS / 64; w++) add += wc[w][threadIdx.x];
        run[threadIdx.x] += add;
    }
    __syncthreads();
    // exclusive scan of the tile's digit counts (one wavefront)
    if (wid == 0) {
        int c0 = run[4 * lane], c1 = run[4 * lane + 1], c2 = run[4 * lane + 2],
            c3 = run[4 * lane + 3];
        int sum = c0 + c1 + c2 + c3, inc = sum;
        for (int o = 1; o < 64; o <<= 1) {
            int t = __shfl_up(inc, o, 64);
            if (lane >= o) inc += t;
        }
        int ex = inc - sum;
        toff[4 * lane] = ex;
        toff[4 * lane + 1] = ex + c0;
        toff[4 * lane + 2] = ex + c0 + c1;
        toff[4 * lane + 3] = ex + c0 + c1 + c2;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RS_ROUNDS; r++) {
        if (r * RS_BS + (int)threadIdx.x < cnt) {
            int q = toff[(kr[r] >> shift) & 255u] + rk[r];
            sk[q] = kr[r];
            sv[q] = vr[r];
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < cnt; j += RS_BS) {
        unsigned k = sk[j];
        unsigned d = (k >> shift) & 255u;
        long pos = (long)goff[d] + (j - toff[d]);
        okey[pos] = k;
        oval[pos] = sv[j];
    }
}

int r2p_sort_pairs(unsigned *key, unsigned *val, unsigned *ktmp, unsigned *vtmp, int n,
                   int key_bits, DBuf<int> &hist, DBuf<int> &tmp, HostPinned &pin, hipStream_t s) {
    if (n <= 1) return 0;
    int ntiles = r2p_blocks(n, RS_TILE);
    R2P_TRY(hist.ensure(256L * ntiles + 1));
    unsigned *ka = key, *va = val, *kb = ktmp, *vb = vtmp;
    int passes = (key_bits + 7) / 8;
    for (int p = 0; p < passes; p++) {
        int shift = 8 * p;
        k_rs_hist<<<ntiles, RS_BS, 0, s>>>(ka, n, shift, ntiles, hist.p);
        R2P_LAUNCH();
        R2P_TRY(r2p_scan_int(hist.p, hist.p, 256 * ntiles, nullptr, tmp, pin, s));
        k_rs_scatter<<<ntiles, RS_BS, 0, s>>>(ka, va, n, shift, ntiles, hist.p, kb, vb);
        R2P_LAUNCH();
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != key) {
        R2P_HIP(hipMemcpyAsync(key, ka, sizeof(unsigned) * (size_t)n, hipMemcpyDeviceToDevice, s));
        R2P_HIP(hipMemcpyAsync(val, va, sizeof(unsigned) * (size_t)n, hipMemcpyDeviceToDevice, s));
    }
    return 0;
}

int r2p_scan_int(const int *in, int *out, int n, int *total_host, DBuf<int> &tmp, HostPinned &pin,
                 hipStream_t s) {
    int nt = r2p_blocks(n > 0 ? n : 1, SCAN_TILE);
    R2P_TRY(tmp.ensure(nt + 1));
    if (n > 0) {
        k_scan_tiles<<<nt, SCAN_BS, 0, s>>>(in, n, tmp.p);
        R2P_LAUNCH();
        k_scan_sums<<<1, SCAN_BS, 0, s>>>(tmp.p, nt, tmp.p + nt);
        R2P_LAUNCH();
        k_scan_apply<<<nt, SCAN_BS, 0, s>>>(in, out, n, tmp.p);
        R2P_LAUNCH();
    } else {
        R2P_HIP(hipMemsetAsync(tmp.p + nt, 0, sizeof(int), s));
    }
    if (total_host) {
        R2P_TRY(pin.ensure(64));
        R2P_HIP(hipMemcpyAsync(pin.p, tmp.p + nt, sizeof(int), hipMemcpyDeviceToHost, s));
        R2P_HIP(hipStreamSynchronize(s));
        *total_host = *(int *)pin.p;
    }
    return 0;
}

int r2p_cu_count() {
    static std::atomic<int> cache[64];   // zero-initialised (static storage)
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    int c = cache[dev].load(std::memory_order_relaxed);
    if (!c) {
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) c = 0;
        cache[dev].store(c, std::memory_order_relaxed);
    }
    return c;
}
