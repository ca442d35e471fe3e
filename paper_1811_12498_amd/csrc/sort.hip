// Stable LSD radix sort of (uint64 key, int32 value) pairs and a single-block scan.
//
// Each pass handles 8 key bits: (1) per-tile digit histograms, (2) an exclusive scan of
// each digit's row of tile counts, (3) a stable scatter in which every tile first scans the
// 256 digit totals itself, then ranks its keys round by round (256 keys per round, wave64
// ballots find the lanes sharing a digit, wave counts are combined in LDS in wave order),
// lays the tile out in digit order in LDS and writes each digit's run contiguously.  Ties
// keep their input order, so sorting (key, index) pairs yields the order of a
// lexicographic (key, index) sort.
#include "stk_internal.hpp"

namespace stk {
namespace {

constexpr int RB = 8;                 // bits per pass
constexpr int RADIX = 1 << RB;
constexpr int ST = 256;               // threads per block (4 waves)
constexpr int ITEMS = 8;              // rounds per tile
constexpr int TILE = ST * ITEMS;
constexpr int NWAVE = ST / 64;

__global__ __launch_bounds__(ST) void k_hist(const uint64_t *__restrict__ keys, int64_t n, int shift,
                                             int32_t *__restrict__ hist, int32_t ntiles) {
    __shared__ int32_t cnt[RADIX];
    const int tid = threadIdx.x;
    cnt[tid] = 0;
    __syncthreads();
    const int64_t base = int64_t(blockIdx.x) * TILE;
    for (int it = 0; it < ITEMS; ++it) {
        const int64_t i = base + int64_t(it) * ST + tid;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & (RADIX - 1)], 1);
    }
    __syncthreads();
    hist[int64_t(tid) * ntiles + blockIdx.x] = cnt[tid];
}

// exclusive scan over the RADIX (= ST) values v of the block's threads, in thread order
__device__ inline int32_t block_excl_radix(int32_t v, int32_t *ws) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) ws[wave] = x;
    __syncthreads();
    int32_t before = 0;
    for (int w = 0; w < wave; ++w) before += ws[w];
    return before + x - v;
}

// One tile per block.  The keys are ranked round by round as in a direct scatter (stable),
// but placed at their position within the tile's digit-ordered layout in LDS; the tile is
// then written out in that order, so each digit's run goes to consecutive addresses.
__global__ __launch_bounds__(ST) void k_scatter(const uint64_t *__restrict__ kin, const int32_t *__restrict__ vin,
                                                uint64_t *__restrict__ kout, int32_t *__restrict__ vout, int64_t n,
                                                int shift, const int32_t *__restrict__ off, int32_t ntiles,
                                                const int32_t *__restrict__ dtot) {
    static_assert(RADIX == ST, "one thread per digit");
    __shared__ uint64_t lk[TILE];
    __shared__ int32_t lv[TILE];
    __shared__ int32_t gbase[RADIX];   // global start of this tile's run of each digit
    __shared__ int32_t tstart[RADIX];  // start of each digit's run within the tile
    __shared__ int32_t run[RADIX];     // keys of each digit placed so far
    __shared__ int32_t wcnt[NWAVE][RADIX];
    __shared__ int32_t ws[NWAVE], ws2[NWAVE];
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int32_t tile = blockIdx.x;
    const int64_t tbase = int64_t(tile) * TILE;
    const int32_t tn = int32_t(n - tbase < TILE ? n - tbase : TILE);
    // digit tid: its total over all tiles, their exclusive scan (every block scans the 256
    // totals itself), and this tile's count, the difference of the scanned histogram row
    // (the last tile against the digit's total)
    const int32_t total_d = dtot[tid];
    const int32_t dbase = block_excl_radix(total_d, ws2);
    const int32_t o = off[int64_t(tid) * ntiles + tile];
    const int32_t cnt = (tile + 1 < ntiles ? off[int64_t(tid) * ntiles + tile + 1] : total_d) - o;
    gbase[tid] = dbase + o;
    tstart[tid] = block_excl_radix(cnt, ws);
    run[tid] = 0;
    for (int w = 0; w < NWAVE; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int it = 0; it < ITEMS; ++it) {
        const int32_t li = it * ST + tid;
        const bool valid = li < tn;
        uint64_t key = 0;
        int32_t val = 0;
        int dig = 0;
        if (valid) {
            key = kin[tbase + li];
            val = vin[tbase + li];
            dig = int((key >> shift) & (RADIX - 1));
        }
        uint64_t match = __ballot(valid);
#pragma unroll
        for (int bt = 0; bt < RB; ++bt) {
            const bool bit = (dig >> bt) & 1;
            const uint64_t bb = __ballot(bit);
            match &= bit ? bb : ~bb;
        }
        const int rank = __popcll(match & lt);
        if (valid && rank == 0) wcnt[wave][dig] = __popcll(match);
        __syncthreads();
        if (valid) {
            int before = 0;
            for (int w = 0; w < wave; ++w) before += wcnt[w][dig];
            const int32_t lp = tstart[dig] + run[dig] + before + rank;
            lk[lp] = key;
            lv[lp] = val;
        }
        __syncthreads();
        {
            int tot = 0;
            for (int w = 0; w < NWAVE; ++w) {
                tot += wcnt[w][tid];
                wcnt[w][tid] = 0;
            }
            run[tid] += tot;
        }
        __syncthreads();
    }
    // the tile in digit order: consecutive positions of one digit go to consecutive
    // addresses
    for (int it = 0; it < ITEMS; ++it) {
        const int32_t li = it * ST + tid;
        if (li < tn) {
            const uint64_t key = lk[li];
            const int dig = int((key >> shift) & (RADIX - 1));
            const int64_t dest = int64_t(gbase[dig]) + (li - tstart[dig]);
            kout[dest] = key;
            vout[dest] = lv[li];
        }
    }
}

// Exclusive scan of in[0..n) into out[0..n) by one block of NT threads, tiles of 4 NT
// elements (each thread 4 consecutive), carrying the running total; returns the total.
template <int NT>
__device__ int32_t block_scan_excl(const int32_t *in, int32_t *out, int64_t n, int32_t carry = 0) {  // in may equal out
    constexpr int NW = NT / 64;
    __shared__ int32_t wsum[NW];
    __shared__ int32_t tile_total;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int64_t base = 0; base < n; base += int64_t(NT) * 4) {
        const int64_t i0 = base + int64_t(tid) * 4;
        int32_t v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = (i0 + j < n) ? in[i0 + j] : 0;
        const int32_t tsum = v[0] + v[1] + v[2] + v[3];
        int32_t x = tsum;  // inclusive scan over the wave
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        if (tid == 0) {
            int32_t run = 0;
            for (int w = 0; w < NW; ++w) {
                const int32_t t = wsum[w];
                wsum[w] = run;
                run += t;
            }
            tile_total = run;
        }
        __syncthreads();
        int32_t e = carry + wsum[wave] + (x - tsum);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (i0 + j < n) out[i0 + j] = e;
            e += v[j];
        }
        carry += tile_total;
        __syncthreads();
    }
    return carry;
}

constexpr int SCAN_T = 1024;

__global__ __launch_bounds__(SCAN_T) void k_scan(const int32_t *__restrict__ in, int32_t *__restrict__ out,
                                                 int64_t n) {
    const int32_t tot = block_scan_excl<SCAN_T>(in, out, n);
    if (threadIdx.x == 0) out[n] = tot;
}

// Blocks base + blockIdx.x: 0 scans a into oa (oa[n] = its total), 1 scans b into ob, 2
// writes stats = {sum of c, sum of d (int64), max of a, max of b}.
__global__ __launch_bounds__(SCAN_T) void k_scan2_stats(const int32_t *__restrict__ a, int32_t *__restrict__ oa,
                                                        const int32_t *__restrict__ b, int32_t *__restrict__ ob,
                                                        const int32_t *__restrict__ c, const int32_t *__restrict__ d,
                                                        int64_t n, int base, long long *__restrict__ stats) {
    const int role = base + int(blockIdx.x);
    if (role < 2) {
        const int32_t *in = role == 0 ? a : b;
        int32_t *out = role == 0 ? oa : ob;
        const int32_t tot = block_scan_excl<SCAN_T>(in, out, n);
        if (threadIdx.x == 0) out[n] = tot;
        return;
    }
    __shared__ long long red[4][SCAN_T];
    long long sc = 0, sd = 0, ma = 0, mb = 0;
    for (int64_t i = threadIdx.x; i < n; i += SCAN_T) {
        sc += c[i];
        sd += d[i];
        ma = a[i] > ma ? a[i] : ma;
        mb = b[i] > mb ? b[i] : mb;
    }
    red[0][threadIdx.x] = sc;
    red[1][threadIdx.x] = sd;
    red[2][threadIdx.x] = ma;
    red[3][threadIdx.x] = mb;
    __syncthreads();
    for (int o = SCAN_T / 2; o > 0; o >>= 1) {
        if (int(threadIdx.x) < o) {
            red[0][threadIdx.x] += red[0][threadIdx.x + o];
            red[1][threadIdx.x] += red[1][threadIdx.x + o];
            red[2][threadIdx.x] = red[2][threadIdx.x + o] > red[2][threadIdx.x] ? red[2][threadIdx.x + o]
                                                                                 : red[2][threadIdx.x];
            red[3][threadIdx.x] = red[3][threadIdx.x + o] > red[3][threadIdx.x] ? red[3][threadIdx.x + o]
                                                                                 : red[3][threadIdx.x];
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) stats[threadIdx.x] = red[threadIdx.x][0];
}

// device-wide scan for long inputs: tile sums, a single-block scan of them, then each
// tile scanned from its offset
constexpr int STILE_T = 256;
constexpr int STILE = 4 * STILE_T;

__global__ __launch_bounds__(STILE_T) void k_tile_sums(const int32_t *__restrict__ in, int64_t n,
                                                       int32_t *__restrict__ sums) {
    __shared__ int32_t ws[STILE_T / 64];
    const int64_t base = int64_t(blockIdx.x) * STILE + int64_t(threadIdx.x) * 4;
    int32_t v = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (base + j < n) v += in[base + j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t tot = 0;
        for (int w = 0; w < STILE_T / 64; ++w) tot += ws[w];
        sums[blockIdx.x] = tot;
    }
}

// each tile scanned from its offset; the first block also writes the total, out[n]
__global__ __launch_bounds__(STILE_T) void k_tile_scan(const int32_t *__restrict__ in, int64_t n,
                                                       const int32_t *__restrict__ offs, int32_t *__restrict__ out) {
    const int64_t base = int64_t(blockIdx.x) * STILE;
    const int64_t len = n - base < STILE ? n - base : STILE;
    block_scan_excl<STILE_T>(in + base, out + base, len, offs[blockIdx.x]);
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = offs[gridDim.x];
}

// radix histogram table hist[digit * ntiles + tile]: block d scans row d in place and
// writes the row total
__global__ __launch_bounds__(256) void k_scan_rows(int32_t *__restrict__ hist, int32_t ntiles,
                                                   int32_t *__restrict__ tot) {
    int32_t *row = hist + int64_t(blockIdx.x) * ntiles;
    const int32_t t = block_scan_excl<256>(row, row, ntiles);
    if (threadIdx.x == 0) tot[blockIdx.x] = t;
}

}  // namespace

void scan_exclusive_i32(const int32_t *in, int32_t *out, int64_t n, DBuf &scratch, hipStream_t s) {
    if (n <= 16 * 4 * SCAN_T) {
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(SCAN_T), 0, s, in, out, n);
        STK_CHECK_LAUNCH();
        return;
    }
    const int64_t ntiles = (n + STILE - 1) / STILE;
    int32_t *sums = reserve<int32_t>(scratch, size_t(2 * ntiles + 1));
    int32_t *offs = sums + ntiles;
    hipLaunchKernelGGL(k_tile_sums, dim3(unsigned(ntiles)), dim3(STILE_T), 0, s, in, n, sums);
    STK_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(SCAN_T), 0, s, sums, offs, ntiles);  // offs[ntiles] = total
    STK_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_tile_scan, dim3(unsigned(ntiles)), dim3(STILE_T), 0, s, in, n, offs, out);
    STK_CHECK_LAUNCH();
}

namespace {
struct PeekArgs {
    const void *p[PEEK_MAX];
    int32_t bytes[PEEK_MAX];
    int32_t n;
};

__global__ void k_peek(PeekArgs a, int64_t *__restrict__ dst) {
    const int i = threadIdx.x;
    if (i < a.n)
        dst[i] = a.bytes[i] == 8 ? *static_cast<const int64_t *>(a.p[i])
                                 : int64_t(*static_cast<const int32_t *>(a.p[i]));
}
}  // namespace

int64_t *peek_slots(HostPeek &pk) {
    if (!pk.h) {
        void *h = nullptr, *d = nullptr;
        STK_HIP(hipHostMalloc(&h, sizeof(int64_t) * PEEK_MAX, hipHostMallocMapped | hipHostMallocCoherent));
        const hipError_t e = hipHostGetDevicePointer(&d, h, 0);
        if (e != hipSuccess) {
            (void)hipHostFree(h);
            STK_HIP(e);
        }
        pk.h = static_cast<int64_t *>(h);
        pk.d = static_cast<int64_t *>(d);
    }
    return pk.d;
}

void peek_wait(HostPeek &pk, hipStream_t s, int n, int64_t *out) {
    if (n < 1 || n > PEEK_MAX || !pk.h) throw Error(STK_EINVAL, "peek_wait: 1 to PEEK_MAX allocated slots");
    STK_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < n; ++i) out[i] = pk.h[i];
}

void peek(HostPeek &pk, hipStream_t s, int n, const PeekSrc *src, int64_t *out) {
    peek_start(pk, s, n, src);
    peek_wait(pk, s, n, out);
}

void peek_start(HostPeek &pk, hipStream_t s, int n, const PeekSrc *src) {
    if (n < 1 || n > PEEK_MAX) throw Error(STK_EINVAL, "peek: 1 to PEEK_MAX values");
    peek_slots(pk);
    PeekArgs a{};
    a.n = n;
    for (int i = 0; i < n; ++i) {
        if (src[i].bytes != 4 && src[i].bytes != 8) throw Error(STK_EINVAL, "peek: 4- or 8-byte values");
        a.p[i] = src[i].p;
        a.bytes[i] = src[i].bytes;
    }
    hipLaunchKernelGGL(k_peek, dim3(1), dim3(64), 0, s, a, pk.d);
    STK_CHECK_LAUNCH();
}

void scan2_stats(const int32_t *a, int32_t *oa, const int32_t *b, int32_t *ob, const int32_t *c, const int32_t *d,
                 int64_t n, long long *stats, DBuf &scratch, hipStream_t s) {
    if (n <= 16 * 4 * SCAN_T) {  // the two scans and the statistics in one launch
        hipLaunchKernelGGL(k_scan2_stats, dim3(3), dim3(SCAN_T), 0, s, a, oa, b, ob, c, d, n, 0, stats);
        STK_CHECK_LAUNCH();
        return;
    }
    scan_exclusive_i32(a, oa, n, scratch, s);
    scan_exclusive_i32(b, ob, n, scratch, s);
    hipLaunchKernelGGL(k_scan2_stats, dim3(1), dim3(SCAN_T), 0, s, a, oa, b, ob, c, d, n, 2, stats);
    STK_CHECK_LAUNCH();
}

void radix_sort_pairs(Tree &t, uint64_t *keys, int32_t *vals, int64_t n, int bits, hipStream_t s) {
    radix_sort_pairs(t.s_keys2, t.s_vals2, t.s_hist, keys, vals, n, bits, s);
}

void radix_sort_pairs(DBuf &keys2, DBuf &vals2, DBuf &hbuf, uint64_t *keys, int32_t *vals, int64_t n, int bits,
                      hipStream_t s) {
    if (n <= 1) return;
    const int32_t ntiles = int32_t((n + TILE - 1) / TILE);
    uint64_t *k2 = reserve<uint64_t>(keys2, size_t(n));
    int32_t *v2 = reserve<int32_t>(vals2, size_t(n));
    const int64_t hn = int64_t(RADIX) * ntiles;
    int32_t *hist = reserve<int32_t>(hbuf, size_t(hn + RADIX));
    int32_t *dtot = hist + hn;  // the digits' totals
    uint64_t *ka = keys, *kb = k2;
    int32_t *va = vals, *vb = v2;
    const int passes = (bits + RB - 1) / RB;
    for (int ps = 0; ps < passes; ++ps) {
        const int shift = ps * RB;
        hipLaunchKernelGGL(k_hist, dim3(ntiles), dim3(ST), 0, s, ka, n, shift, hist, ntiles);
        STK_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_scan_rows, dim3(RADIX), dim3(256), 0, s, hist, ntiles, dtot);
        STK_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_scatter, dim3(ntiles), dim3(ST), 0, s, ka, va, kb, vb, n, shift, hist, ntiles, dtot);
        STK_CHECK_LAUNCH();
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        STK_HIP(hipMemcpyAsync(keys, ka, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
        STK_HIP(hipMemcpyAsync(vals, va, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    }
}

}  // namespace stk
