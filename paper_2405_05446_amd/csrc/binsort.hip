// Tile binning and compositing order (the front-to-back order of the alpha
// blend, GDGS Sec. 1.2 Eq. 11, "sorted from the view direction").
//
// 1. key each splat by the bits of its FP32 depth (culled splats last) and
//    stable-radix-sort the splat indices: order[s] = splat of depth rank s;
// 2. exclusive scan of the tile counts in rank order, then one (tile, splat)
//    pair per tile of each splat's rectangle, written in rank order;
// 3. stable radix sort of the pairs by tile id, then each tile's range.
// Because step 2 emits pairs in depth-rank order and step 3 is stable, the
// final order equals a lexicographic sort by (tile, depth bits, splat index).
//
// The radix sort is a reduce-then-scan LSD sort with digits of equal width,
// at most 8 bits, on a fixed grid (the element count may live on the
// device): per pass an upsweep digit
// histogram per block, a scan of every digit's row of block counts, and a
// downsweep that ranks each 2048-key tile in LDS with wave64 ballots (lanes
// holding equal digits are matched bit by bit; a lane's rank is the popcount
// of lower matched lanes), stages the tile in LDS in sorted order and writes
// coalesced runs.
#include "internal.hpp"

namespace gdgs {
namespace {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;  // keys per block iteration
constexpr int kWaves = kSortThreads / 64;
constexpr int kRadix = 256;
constexpr int kMaxGrid = 1024;

__device__ __forceinline__ int64_t clamp_n(const int64_t* n_dev, int64_t n_host, int64_t cap) {
    int64_t n = n_dev ? *n_dev : n_host;
    if (n > cap) n = cap;
    if (n < 0) n = 0;
    return n;
}

// Contiguous key range of block b: chunks are whole multiples of kSortTile.
__device__ __forceinline__ void block_range(int64_t n, int G, int b, int64_t* lo, int64_t* hi) {
    int64_t chunk = (n + G - 1) / G;
    chunk = (chunk + kSortTile - 1) / kSortTile * kSortTile;
    int64_t l = (int64_t)b * chunk;
    if (l > n) l = n;
    int64_t h = l + chunk;
    if (h > n) h = n;
    *lo = l;
    *hi = h;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Mask of the valid lanes of this wave whose digit equals this lane's digit.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid, int bits) {
    uint64_t m = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// Exclusive scan of one value per thread over a 256-thread block.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* s_tmp, uint32_t* total) {
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_scan(x);
    if (lane == 63) s_tmp[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) {
        const uint32_t v = s_tmp[i];
        off += (i < w) ? v : 0u;
        tot += v;
    }
    __syncthreads();
    *total = tot;
    return off + inc - x;
}

// gate (the first depth pass only): key i is keys[i] where gate[i] != 0 and
// 0xFFFFFFFF (last) where it is 0, i.e. the depth bits of the splats with
// tiles and the culled splats after them, read straight from the projection.
__device__ __forceinline__ uint32_t gated_key(const uint32_t* __restrict__ keys,
                                              const uint32_t* __restrict__ gate, int64_t i) {
    const uint32_t k = keys[i];
    return gate ? (gate[i] ? k : 0xFFFFFFFFu) : k;
}

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(
    const uint32_t* __restrict__ keys, const uint32_t* __restrict__ gate, const int64_t* n_dev,
    int64_t n_host, int64_t cap, int shift, int bits, uint32_t* __restrict__ hist) {
    __shared__ uint32_t s_h[kWaves][kRadix];  // one row per wave: fewer colliding atomics
    const int G = gridDim.x, b = blockIdx.x, t = threadIdx.x, w = t >> 6;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) s_h[i][t] = 0;
    __syncthreads();
    int64_t lo, hi;
    block_range(clamp_n(n_dev, n_host, cap), G, b, &lo, &hi);
    const uint32_t mask = (1u << bits) - 1u;
    for (int64_t base = lo; base < hi; base += kSortTile) {
        uint32_t d[kSortItems];
#pragma unroll
        for (int r = 0; r < kSortItems; ++r) {
            const int64_t i = base + r * kSortThreads + t;
            d[r] = i < hi ? (gated_key(keys, gate, i) >> shift) & mask : 0u;
        }
#pragma unroll
        for (int r = 0; r < kSortItems; ++r)
            if (base + r * kSortThreads + t < hi) atomicAdd(&s_h[w][d[r]], 1u);
    }
    __syncthreads();
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) sum += s_h[i][t];
    hist[(size_t)t * G + b] = sum;
}

// Block d: exclusive scan of digit d's block counts (in place) and its total.
__global__ __launch_bounds__(256) void k_radix_scan(uint32_t* __restrict__ hist, int G,
                                                    uint32_t* __restrict__ digit_tot) {
    __shared__ uint32_t s_tmp[kWaves];
    constexpr int IT = kMaxGrid / 256;
    const int d = blockIdx.x, t = threadIdx.x;
    uint32_t* row = hist + (size_t)d * G;
    uint32_t v[IT], sum = 0;
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const int idx = t * IT + i;
        v[i] = idx < G ? row[idx] : 0u;
        sum += v[i];
    }
    uint32_t tot;
    uint32_t off = block_excl_scan(sum, s_tmp, &tot);
#pragma unroll
    for (int i = 0; i < IT; ++i) {
        const int idx = t * IT + i;
        if (idx < G) row[idx] = off;
        off += v[i];
    }
    if (t == 0) digit_tot[d] = tot;
}

// Up to three value arrays travel with the keys.
struct Vals {
    const uint32_t* in[3];
    uint32_t* out[3];
};

// Value array v with in[v] null carries the element's index.
template <int NV>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ gate,
    uint32_t* __restrict__ kout, Vals vals, const int64_t* n_dev, int64_t n_host, int64_t cap,
    int shift, int bits,
    const uint32_t* __restrict__ hist, const uint32_t* __restrict__ digit_tot) {
    __shared__ uint32_t s_base[kRadix];
    __shared__ uint32_t s_wcnt[kWaves][kRadix];
    __shared__ uint32_t s_tstart[kRadix];
    __shared__ uint32_t s_key[kSortTile];
    __shared__ uint32_t s_val[NV][kSortTile];
    __shared__ uint32_t s_tmp[kWaves];
    const int G = gridDim.x, b = blockIdx.x, t = threadIdx.x, lane = __lane_id(), w = t >> 6;
    const uint32_t mask = (1u << bits) - 1u;
    const uint64_t lt = lanemask_lt();
    {
        uint32_t all;
        const uint32_t start = block_excl_scan(digit_tot[t], s_tmp, &all);
        s_base[t] = start + hist[(size_t)t * G + b];
    }
    int64_t lo, hi;
    block_range(clamp_n(n_dev, n_host, cap), G, b, &lo, &hi);
    for (int64_t tlo = lo; tlo < hi; tlo += kSortTile) {
        for (int i = t; i < kWaves * kRadix; i += kSortThreads) (&s_wcnt[0][0])[i] = 0u;
        __syncthreads();
        uint32_t key[kSortItems], val[NV][kSortItems], rank[kSortItems];
        const int64_t wbase = tlo + (int64_t)w * 64 * kSortItems;
#pragma unroll
        for (int r = 0; r < kSortItems; ++r) {
            const int64_t i = wbase + r * 64 + lane;
            const bool valid = i < hi;
            key[r] = valid ? gated_key(kin, gate, i) : 0u;
#pragma unroll
            for (int v = 0; v < NV; ++v)
                val[v][r] = valid ? (vals.in[v] ? vals.in[v][i] : (uint32_t)i) : 0u;
        }
#pragma unroll
        for (int r = 0; r < kSortItems; ++r) {
            const bool valid = wbase + r * 64 + lane < hi;
            const uint32_t d = (key[r] >> shift) & mask;
            const uint64_t peers = match_digit(d, valid, bits);
            const uint32_t prev = s_wcnt[w][d];
            const uint32_t rr = (uint32_t)__popcll(peers & lt);
            if (valid && rr == 0) s_wcnt[w][d] = prev + (uint32_t)__popcll(peers);
            rank[r] = prev + rr;
        }
        __syncthreads();
        uint32_t tot_t;
        {
            const uint32_t c0 = s_wcnt[0][t], c1 = s_wcnt[1][t], c2 = s_wcnt[2][t],
                           c3 = s_wcnt[3][t];
            tot_t = c0 + c1 + c2 + c3;
            s_wcnt[0][t] = 0u;
            s_wcnt[1][t] = c0;
            s_wcnt[2][t] = c0 + c1;
            s_wcnt[3][t] = c0 + c1 + c2;
            uint32_t all;
            s_tstart[t] = block_excl_scan(tot_t, s_tmp, &all);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kSortItems; ++r) {
            if (wbase + r * 64 + lane < hi) {
                const uint32_t d = (key[r] >> shift) & mask;
                const uint32_t pos = s_tstart[d] + s_wcnt[w][d] + rank[r];
                s_key[pos] = key[r];
#pragma unroll
                for (int v = 0; v < NV; ++v) s_val[v][pos] = val[v][r];
            }
        }
        __syncthreads();
        const int ntile = (int)min((int64_t)kSortTile, hi - tlo);
        for (int p = t; p < ntile; p += kSortThreads) {
            const uint32_t k = s_key[p];
            const uint32_t d = (k >> shift) & mask;
            const uint32_t g = s_base[d] + ((uint32_t)p - s_tstart[d]);
            kout[g] = k;
#pragma unroll
            for (int v = 0; v < NV; ++v) vals.out[v][g] = s_val[v][p];
        }
        __syncthreads();
        s_base[t] += tot_t;
    }
}

// ---------------------------------------------------------------- binning
constexpr int kScanThreads = 256;
constexpr int kScanItems = 2;   // 512 splats per block: enough blocks to hide the emission's latency
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ uint32_t rect_count(uint32_t r0, uint32_t r1) {
    return ((r0 >> 16) - (r0 & 0xFFFFu)) * ((r1 >> 16) - (r1 & 0xFFFFu));
}

// Block sums of the tile counts in depth-rank order (rect0/rect1: the
// rectangles permuted into rank order by the depth sort; count = area).
__global__ __launch_bounds__(kScanThreads) void k_count_reduce(const uint32_t* __restrict__ rect0,
                                                               const uint32_t* __restrict__ rect1,
                                                               int64_t K,
                                                               unsigned long long* __restrict__ bsum) {
    __shared__ uint32_t s_tmp[kWaves];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)t * kScanItems;
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t s = base + i;
        if (s < K) sum += rect_count(rect0[s], rect1[s]);
    }
    uint32_t tot;
    block_excl_scan(sum, s_tmp, &tot);
    if (t == 0) bsum[blockIdx.x] = tot;
}

// One block: exclusive scan of nb block sums in place; writes the total.
__global__ __launch_bounds__(1024) void k_scan_bsums(unsigned long long* __restrict__ bsum,
                                                     int64_t nb, int64_t* __restrict__ total) {
    __shared__ unsigned long long s_w[16];
    __shared__ unsigned long long s_carry;
    const int t = threadIdx.x, lane = __lane_id(), w = t >> 6;
    if (t == 0) s_carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += 1024) {
        const int64_t i = base + t;
        const unsigned long long x = i < nb ? bsum[i] : 0ull;
        unsigned long long inc = x;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const unsigned long long y = __shfl_up(inc, d, 64);
            if (lane >= d) inc += y;
        }
        if (lane == 63) s_w[w] = inc;
        __syncthreads();
        unsigned long long off = s_carry, tot = 0;
        for (int j = 0; j < 16; ++j) {
            off += (j < w) ? s_w[j] : 0ull;
            tot += s_w[j];
        }
        if (i < nb) bsum[i] = off + inc - x;
        __syncthreads();
        if (t == 0) s_carry += tot;
        __syncthreads();
    }
    if (t == 0) *total = (int64_t)s_carry;
}

// Pair emission for the splats of depth ranks [b * kScanTile, (b+1) * kScanTile):
// each splat's block-local pair offset comes from a block scan of the tile
// counts; then the block's pairs are written cooperatively and coalesced,
// pair p finding its splat by binary search over the offsets in LDS.
__global__ __launch_bounds__(kScanThreads) void k_emit_pairs(
    const uint32_t* __restrict__ order, const uint32_t* __restrict__ rect0,
    const uint32_t* __restrict__ rect1, int64_t K, const unsigned long long* __restrict__ bsum,
    int64_t cap, int nx, uint32_t* __restrict__ tile_out, uint32_t* __restrict__ splat_out) {
    __shared__ uint32_t s_tmp[kWaves];
    __shared__ uint32_t s_off[kScanTile + 1];
    __shared__ uint32_t s_k[kScanTile];
    __shared__ uint32_t s_org[kScanTile];  // tx0 | ty0 << 16
    __shared__ uint32_t s_w[kScanTile];    // rectangle width in tiles
    const int t = threadIdx.x;
    const int64_t sbase = (int64_t)blockIdx.x * kScanTile;
    uint32_t c[kScanItems], ks[kScanItems], r0[kScanItems], r1[kScanItems], sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t s = sbase + (int64_t)t * kScanItems + i;
        ks[i] = s < K ? order[s] : 0u;
        r0[i] = s < K ? rect0[s] : 0u;
        r1[i] = s < K ? rect1[s] : 0u;
    }
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        c[i] = ks[i] < (uint64_t)K ? rect_count(r0[i], r1[i]) : 0u;
        sum += c[i];
    }
    uint32_t tot;
    uint32_t off = block_excl_scan(sum, s_tmp, &tot);
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int j = t * kScanItems + i;
        s_off[j] = off;
        s_k[j] = ks[i];
        uint32_t org = 0, w = 1;
        if (c[i]) {
            org = (r0[i] & 0xFFFF) | ((r1[i] & 0xFFFF) << 16);
            w = (r0[i] >> 16) - (r0[i] & 0xFFFF);
        }
        s_org[j] = org;
        s_w[j] = w;
        off += c[i];
    }
    if (t == 0) s_off[kScanTile] = tot;
    __syncthreads();
    const int64_t gbase = (int64_t)bsum[blockIdx.x];
    // thread t writes pairs 4t..4t+3 of each 1024-pair window: one binary search
    // per four pairs, then a forward walk; the four stores are contiguous
    for (uint32_t p0 = 4u * t; p0 < tot; p0 += 4u * kScanThreads) {
        int lo = 0, hi = kScanTile;  // last j with s_off[j] <= p0
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_off[mid] <= p0)
                lo = mid;
            else
                hi = mid;
        }
        int j = lo;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t p = p0 + q;
            if (p >= tot) break;
            while (s_off[j + 1] <= p) ++j;  // s_off[kScanTile] = tot > p ends the walk
            const uint32_t k = s_k[j];
            const uint32_t local = p - s_off[j];
            const uint32_t org = s_org[j], w = s_w[j];
            const uint32_t tx0 = org & 0xFFFF, ty0 = org >> 16;
            const uint32_t dy = local / w;
            const int64_t g = gbase + p;
            if (g < cap) {
                tile_out[g] = (ty0 + dy) * (uint32_t)nx + tx0 + (local - dy * w);
                splat_out[g] = k;
            }
        }
    }
}

// Tile ranges from the sorted tile ids: block b covers pairs
// b * 256 * kRangeItems .., thread t every 256th of them (coalesced); all of
// a thread's loads, with each pair's two neighbours, are issued before any
// comparison.
constexpr int kRangeItems = 8;
__global__ __launch_bounds__(256) void k_tile_ranges(const uint32_t* __restrict__ tiles,
                                                     const int64_t* n_dev, int64_t cap,
                                                     uint32_t* __restrict__ ranges, int T) {
    const int64_t n = clamp_n(n_dev, 0, cap);
    const int64_t base = (int64_t)blockIdx.x * 256 * kRangeItems + threadIdx.x;
    if (base >= n) return;
    uint32_t prev[kRangeItems], cur[kRangeItems], next[kRangeItems];
#pragma unroll
    for (int k = 0; k < kRangeItems; ++k) {
        const int64_t i = base + 256 * k;
        const bool in = i < n;
        cur[k] = in ? tiles[i] : 0xFFFFFFFFu;
        prev[k] = (in && i > 0) ? tiles[i - 1] : 0xFFFFFFFFu;
        next[k] = (i + 1 < n) ? tiles[i + 1] : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int k = 0; k < kRangeItems; ++k) {
        const int64_t i = base + 256 * k;
        const uint32_t tl = cur[k];
        if (i >= n || tl >= (uint32_t)T) continue;
        if (prev[k] != tl) ranges[tl] = (uint32_t)i;
        if (next[k] != tl) ranges[T + tl] = (uint32_t)(i + 1);
    }
}

// Heaviest-first schedule of the tiles for the compositing kernels: a stable
// counting sort of the tile ids by floor(log2(pairs)), largest first, empty
// tiles last.  A tile's compositing time grows with its pair count, and the
// hardware dispatches blocks in launch order, so starting the long tiles
// first keeps them from finishing alone at the end of the launch.  Two
// passes over blocks of kOrdThreads tiles: per-block key counts, then each
// block places its tiles after those of every larger key and of the earlier
// blocks with the same key.
constexpr int kOrdThreads = 256;
constexpr int kOrdWaves = kOrdThreads / 64;
constexpr int kOrdKeys = 33;  // key 32 - bitlen(pairs): 0 (most) ... 32 (empty)
constexpr int kOrdGroups = kOrdThreads / kOrdKeys;

int tile_blocks(int64_t T) { return (int)((T + kOrdThreads - 1) / kOrdThreads); }

__device__ __forceinline__ int tile_key(const uint32_t* __restrict__ ranges, int T, int i) {
    const uint32_t n = ranges[T + i] - ranges[i];
    return n == 0 ? 32 : __clz(n);  // __clz(n) = 32 - bitlen(n)
}

// Rank of this lane among the wave's valid lanes with the same key (lane
// order); wc[key] receives the wave's count of each key present.
__device__ __forceinline__ uint32_t wave_key_rank(int k, bool valid, uint32_t* wc) {
    const uint64_t lt = lanemask_lt();
    uint32_t rank = 0;
    uint64_t rest = __ballot(valid);
    while (rest) {
        const int lk = __shfl(k, __ffsll((unsigned long long)rest) - 1);
        const uint64_t m = __ballot(valid && k == lk);
        if (valid && k == lk) rank = (uint32_t)__popcll(m & lt);
        if (__lane_id() == 0) wc[lk] = (uint32_t)__popcll(m);
        rest &= ~m;
    }
    return rank;
}

__global__ __launch_bounds__(kOrdThreads) void k_tile_hist(const uint32_t* __restrict__ ranges,
                                                            int T, uint32_t* __restrict__ bh) {
    __shared__ uint32_t s_wc[kOrdWaves][kOrdKeys];
    const int t = threadIdx.x, wv = t >> 6;
    const int i = blockIdx.x * kOrdThreads + t;
    for (int j = t; j < kOrdWaves * kOrdKeys; j += kOrdThreads) (&s_wc[0][0])[j] = 0;
    __syncthreads();
    const bool valid = i < T;
    wave_key_rank(valid ? tile_key(ranges, T, i) : 0, valid, s_wc[wv]);
    __syncthreads();
    if (t < kOrdKeys) {
        uint32_t c = 0;
        for (int w = 0; w < kOrdWaves; ++w) c += s_wc[w][t];
        bh[(size_t)blockIdx.x * kOrdKeys + t] = c;
    }
}

__global__ __launch_bounds__(kOrdThreads) void k_tile_place(const uint32_t* __restrict__ ranges,
                                                             int T, const uint32_t* __restrict__ bh,
                                                             uint32_t* __restrict__ order) {
    __shared__ uint32_t s_wc[kOrdWaves][kOrdKeys];
    __shared__ uint32_t s_tot[kOrdGroups][kOrdKeys], s_pre[kOrdGroups][kOrdKeys];
    __shared__ uint32_t s_base[kOrdKeys];
    const int t = threadIdx.x, wv = t >> 6, b = blockIdx.x, nb = gridDim.x;
    const int i = b * kOrdThreads + t;
    for (int j = t; j < kOrdWaves * kOrdKeys; j += kOrdThreads) (&s_wc[0][0])[j] = 0;
    // per key: tiles in all blocks and in the blocks before this one, summed
    // by kOrdGroups groups of kOrdKeys threads over strided blocks
    if (t < kOrdGroups * kOrdKeys) {
        const int q = t / kOrdKeys, k = t - q * kOrdKeys;
        uint32_t tot = 0, pre = 0;
        for (int g = q; g < nb; g += kOrdGroups) {
            const uint32_t v = bh[(size_t)g * kOrdKeys + k];
            tot += v;
            pre += g < b ? v : 0u;
        }
        s_tot[q][k] = tot;
        s_pre[q][k] = pre;
    }
    __syncthreads();
    const bool valid = i < T;
    const int key = valid ? tile_key(ranges, T, i) : 0;
    const uint32_t rank = wave_key_rank(key, valid, s_wc[wv]);
    if (t < 64) {  // wave 0: exclusive scan of the key totals
        uint32_t tot = 0, pre = 0;
        if (t < kOrdKeys)
            for (int q = 0; q < kOrdGroups; ++q) {
                tot += s_tot[q][t];
                pre += s_pre[q][t];
            }
        uint32_t inc = tot;
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t v = __shfl_up(inc, d);
            if (t >= d) inc += v;
        }
        if (t < kOrdKeys) s_base[t] = inc - tot + pre;
    }
    __syncthreads();
    if (valid) {
        uint32_t slot = s_base[key] + rank;
        for (int w = 0; w < wv; ++w) slot += s_wc[w][key];
        order[slot] = (uint32_t)i;
    }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, size_t n, uint32_t v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

int bitlen(uint64_t x) {
    int b = 0;
    while (x) {
        ++b;
        x >>= 1;
    }
    return b;
}

// One full LSD sort of keys with NV value arrays over `key_bits` key bits.
// Pass 0 reads (kin0, vin0[]), its keys gated by gate0 if that is not null
// (see gated_key) and a null vin0[v] standing for the element indices; pass
// p > 0 reads buffer set (p + 1) & 1 ... as
// written by pass p - 1: pass p writes set (p + 1) & 1, the last pass writes
// (kfin, vfin[]).  buf sets: (kb[i], vb[v][i]).
template <int NV>
gdgs_status radix_sort(const uint32_t* kin0, const uint32_t* gate0, const uint32_t* const* vin0,
                       uint32_t* const* kb,
                       uint32_t* const (*vb)[2], uint32_t* kfin, uint32_t* const* vfin,
                       const int64_t* n_dev, int64_t n_host, int64_t cap, int key_bits,
                       uint32_t* hist, uint32_t* digit_tot, hipStream_t st) {
    const int G = sort_grid(cap);
    const int passes = (key_bits + 7) / 8;
    // digits of equal width (13 tile bits at 1080p: 7 + 6, whose first pass
    // writes longer runs than an 8-bit one; 2% faster than 8 + 5)
    const int per = (key_bits + passes - 1) / passes;
    for (int p = 0; p < passes; ++p) {
        const int shift = per * p;
        const int bits = key_bits - shift < per ? key_bits - shift : per;
        const bool last = p == passes - 1;
        const uint32_t* kin = p == 0 ? kin0 : kb[p & 1];
        uint32_t* kout = last ? kfin : kb[(p + 1) & 1];
        Vals vals{};
        for (int v = 0; v < NV; ++v) {
            vals.in[v] = p == 0 ? vin0[v] : vb[v][p & 1];
            vals.out[v] = last ? vfin[v] : vb[v][(p + 1) & 1];
        }
        const uint32_t* gate = p == 0 ? gate0 : nullptr;
        hipLaunchKernelGGL(k_radix_hist, dim3(G), dim3(kSortThreads), 0, st, kin, gate, n_dev,
                           n_host, cap, shift, bits, hist);
        hipLaunchKernelGGL(k_radix_scan, dim3(kRadix), dim3(256), 0, st, hist, G, digit_tot);
        hipLaunchKernelGGL(k_radix_scatter<NV>, dim3(G), dim3(kSortThreads), 0, st, kin, gate,
                           kout, vals, n_dev, n_host, cap, shift, bits, hist, digit_tot);
    }
    GDGS_LAUNCH_CHECK();
    return GDGS_OK;
}

}  // namespace

int sort_grid(int64_t cap) {
    int64_t g = (cap + kSortTile - 1) / kSortTile;
    if (g < 1) g = 1;
    if (g > kMaxGrid) g = kMaxGrid;
    return (int)g;
}

size_t bin_ws_layout(int64_t K, int64_t cap, int64_t T, void* ws, BinWs* out) {
    Carver c(ws);
    BinWs b;
    const int64_t Kp = K > 0 ? K : 1;
    const int64_t cp = cap > 0 ? cap : 1;
    for (int i = 0; i < 2; ++i) {
        b.dkey[i] = c.take<uint32_t>(Kp);
        b.dval[i] = c.take<uint32_t>(Kp);
        b.drect[0][i] = c.take<uint32_t>(Kp);
        b.drect[1][i] = c.take<uint32_t>(Kp);
        b.pkey[i] = c.take<uint32_t>(cp);
        b.pval[i] = c.take<uint32_t>(cp);
    }
    const int G = sort_grid(Kp > cp ? Kp : cp);
    b.hist = c.take<uint32_t>((size_t)kRadix * G);
    b.digit_tot = c.take<uint32_t>(kRadix);
    b.bsum = c.take<uint32_t>(2 * ((Kp + kScanTile - 1) / kScanTile + 1));
    b.tile_bh = c.take<uint32_t>((size_t)kOrdKeys * tile_blocks(T > 0 ? T : 1));
    if (out) *out = b;
    return c.off + 256;
}

gdgs_status launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t st) {
    if (n == 0) return GDGS_OK;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
    GDGS_LAUNCH_CHECK();
    return GDGS_OK;
}

namespace {
gdgs_status launch_tile_order(const uint32_t* ranges, int T, uint32_t* bh, uint32_t* order,
                              hipStream_t st) {
    const int nb = tile_blocks(T);
    hipLaunchKernelGGL(k_tile_hist, dim3(nb), dim3(kOrdThreads), 0, st, ranges, T, bh);
    hipLaunchKernelGGL(k_tile_place, dim3(nb), dim3(kOrdThreads), 0, st, ranges, T, bh, order);
    GDGS_LAUNCH_CHECK();
    return GDGS_OK;
}
}  // namespace

gdgs_status launch_bin_sort(const gdgs_proj& proj, int64_t K, int W, int H, const gdgs_bins& bins,
                            const BinWs& ws, hipStream_t st) {
    const int nx = tiles_x(W), T = nx * tiles_y(H);
    gdgs_status s = launch_fill_u32(bins.ranges, 2 * (size_t)T, 0u, st);
    if (s != GDGS_OK) return s;
    if (K == 0) {
        // no splats: zero pairs
        hipLaunchKernelGGL(k_scan_bsums, dim3(1), dim3(1024), 0, st,
                           reinterpret_cast<unsigned long long*>(ws.bsum), (int64_t)0,
                           bins.num_pairs);
        if (bins.tile_order) {  // every tile empty: the order by id
            s = launch_tile_order(bins.ranges, T, ws.tile_bh, bins.tile_order, st);
            if (s != GDGS_OK) return s;
        }
        GDGS_LAUNCH_CHECK();
        return GDGS_OK;
    }
    // 1. depth order of the splats; their rectangles ride along, so that the
    //    scan and the emission read them in rank order without gathers.  The
    //    first pass keys the splats straight from the projection's depth and
    //    tile count, with the splat indices as the first values
    {
        const uint32_t* vin0[3] = {nullptr, proj.rect, proj.rect + K};
        uint32_t* const kb[2] = {ws.dkey[0], ws.dkey[1]};
        uint32_t* const vb[3][2] = {{ws.dval[0], ws.dval[1]},
                                    {ws.drect[0][0], ws.drect[0][1]},
                                    {ws.drect[1][0], ws.drect[1][1]}};
        uint32_t* const vfin[3] = {bins.order, ws.drect[0][0], ws.drect[1][0]};
        s = radix_sort<3>(reinterpret_cast<const uint32_t*>(proj.depth), proj.count, vin0, kb, vb,
                          ws.dkey[0], vfin, nullptr, K, K, 32, ws.hist, ws.digit_tot, st);
        if (s != GDGS_OK) return s;
    }
    const uint32_t* rect0 = ws.drect[0][0];
    const uint32_t* rect1 = ws.drect[1][0];
    // 2. scan of tile counts in rank order, pair emission
    const int64_t nb = (K + kScanTile - 1) / kScanTile;
    unsigned long long* bsum = reinterpret_cast<unsigned long long*>(ws.bsum);
    hipLaunchKernelGGL(k_count_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, st, rect0,
                       rect1, K, bsum);
    hipLaunchKernelGGL(k_scan_bsums, dim3(1), dim3(1024), 0, st, bsum, nb, bins.num_pairs);
    hipLaunchKernelGGL(k_emit_pairs, dim3((unsigned)nb), dim3(kScanThreads), 0, st, bins.order,
                       rect0, rect1, K, bsum, bins.capacity, nx, ws.pkey[0], ws.pval[0]);
    GDGS_LAUNCH_CHECK();
    // 3. stable sort of the pairs by tile, then the ranges
    const int tbits = bitlen((uint64_t)(T > 1 ? T - 1 : 1));
    {
        const uint32_t* vin0[1] = {ws.pval[0]};
        uint32_t* const kb[2] = {ws.pkey[0], ws.pkey[1]};
        uint32_t* const vb[1][2] = {{ws.pval[0], ws.pval[1]}};
        uint32_t* const vfin[1] = {bins.splat_of_pair};
        s = radix_sort<1>(ws.pkey[0], nullptr, vin0, kb, vb, bins.tile_of_pair, vfin,
                          bins.num_pairs, 0, bins.capacity, tbits, ws.hist, ws.digit_tot, st);
        if (s != GDGS_OK) return s;
    }
    const int64_t rblocks = (bins.capacity + 256 * kRangeItems - 1) / (256 * kRangeItems);
    hipLaunchKernelGGL(k_tile_ranges, dim3((unsigned)rblocks), dim3(256), 0, st,
                       bins.tile_of_pair,
                       bins.num_pairs, bins.capacity, bins.ranges, T);
    GDGS_LAUNCH_CHECK();
    if (bins.tile_order) return launch_tile_order(bins.ranges, T, ws.tile_bh, bins.tile_order, st);
    return GDGS_OK;
}

}  // namespace gdgs
