// Stable LSD radix sort of (key, u32 value) pairs on gfx950.
//
// Section IV sorts DC3's sample and non-sample keys with a radix sort that
// walks the digits from least to most significant, each pass a stable split
// computed with a prefix scan (one bit per pass in the paper's kernel).
// Here a pass handles a digit of up to 8 bits (the width and the tile size
// come from the tuning plan) and runs as follows, one workgroup per tile:
//   1. count  : the digit histogram of every tile, built in LDS (one
//               sub-histogram per wave) and stored tile-major;
//   2. scan   : a column scan of the tile-major table gives every (tile,
//               digit) its output offset: all smaller digits first, then
//               digit d of the earlier tiles;
//   3. scatter: each wave ranks its elements by digit (below), the tile is
//               reordered by digit in LDS and written out, so runs of equal
//               digits leave as contiguous stores.
// Ranking without ballots: for every item, each lane ORs its lane bit into
// its wave's 64-bit word for its digit in LDS, reads the word back (the
// wave's LDS instructions run in order, so the word then holds exactly the
// lanes of this item with that digit) and clears it. The rank is the number
// of those lanes below the calling lane plus the wave's running count for
// the digit, which the lowest of them advances.
// Element order inside a tile is wave-major, then item, then lane, so ranks
// follow input order and every pass is stable.
//
// Tiles are dealt to the 8 XCDs in contiguous eighths of the array (tile
// order inside each eighth follows the workgroup index). The tiles in flight
// on one XCD are then neighbours, their runs of a digit are adjacent in the
// output, and the cache lines the runs share are completed in that XCD's L2
// instead of leaving it part-written.
#include "lor_internal.hpp"

namespace lor {

namespace {

constexpr int kDigitBits = 8;
constexpr int kBins = 1 << kDigitBits;
constexpr uint32_t kMinTile = kBlock * 8;   // smallest tile of any plan (sizes the count table)
constexpr uint32_t kColChunks = 2048;       // row chunks of the column scan (8 per scan thread)

// Tile handled by this workgroup: XCD x = blockIdx mod 8 takes the x-th
// eighth of the tiles, in workgroup order. Returns false for the padding
// workgroups of the last eighth.
__device__ __forceinline__ bool xcd_tile(uint32_t tiles, uint32_t *tile) {
    const uint32_t per = (tiles + kXcds - 1) / kXcds;
    const uint32_t x = blockIdx.x % kXcds, j = blockIdx.x / kXcds;
    *tile = x * per + j;
    return j < per && *tile < tiles;
}

inline uint32_t xcd_tile_grid(uint32_t tiles) { return kXcds * ((tiles + kXcds - 1) / kXcds); }

template <typename K, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_radix_count(const K *__restrict__ keys, uint32_t n, uint32_t tiles,
                                                        int shift, uint32_t mask, uint32_t *__restrict__ table) {
    constexpr uint32_t TILE = kBlock * ITEMS;
    __shared__ uint32_t hist[kBlock / kWave][kBins];
    const unsigned tid = threadIdx.x, w = tid >> 6;
    uint32_t t;
    if (!xcd_tile(tiles, &t)) return;
#pragma unroll
    for (int i = 0; i < kBlock / kWave; ++i) hist[i][tid] = 0;
    __syncthreads();
    const uint32_t base = t * TILE + tid;
    K k[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t e = base + r * kBlock;
        k[r] = (e < n) ? keys[e] : K(0);
    }
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t e = base + r * kBlock;
        if (e < n) atomicAdd(&hist[w][(uint32_t)(k[r] >> shift) & mask], 1u);
    }
    __syncthreads();
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < kBlock / kWave; ++i) c += hist[i][tid];
    table[(size_t)t * kBins + tid] = c;
}

// Column scan of the tile-major table (rows = tiles, 256 columns = digits),
// in three fully parallel kernels: per-chunk column sums; per digit, an
// exclusive scan of its chunk sums (one workgroup per digit, one thread per
// chunk) and the digit total; then every chunk rescans its rows from its
// base, where digit d starts after the totals of all smaller digits.
__device__ __forceinline__ void col_chunk(uint32_t rows, uint32_t chunks, uint32_t c, uint32_t *r0, uint32_t *r1) {
    *r0 = (uint32_t)((uint64_t)rows * c / chunks);
    *r1 = (uint32_t)((uint64_t)rows * (c + 1) / chunks);
}

__global__ __launch_bounds__(kBlock) void k_col_reduce(const uint32_t *__restrict__ table, uint32_t rows,
                                                       uint32_t chunks, uint32_t *__restrict__ csum) {
    uint32_t r0, r1;
    col_chunk(rows, chunks, blockIdx.x, &r0, &r1);
    uint32_t acc = 0;
    for (uint32_t r = r0; r < r1; ++r) acc += table[(size_t)r * kBins + threadIdx.x];
    csum[(size_t)blockIdx.x * kBins + threadIdx.x] = acc;
}

// Workgroup d: csum[c][d] becomes the sum over chunks < c; dtot[d] the total.
// Thread j owns chunks 4j .. 4j+3.
constexpr uint32_t kColPer = kColChunks / kBlock;
__global__ __launch_bounds__(kBlock) void k_col_scan(uint32_t *__restrict__ csum, uint32_t chunks,
                                                     uint32_t *__restrict__ dtot) {
    __shared__ uint32_t s_tmp[kBlock / kWave];
    const uint32_t d = blockIdx.x, c0 = threadIdx.x * kColPer;
    uint32_t x[kColPer], sum = 0;
#pragma unroll
    for (uint32_t q = 0; q < kColPer; ++q) {
        x[q] = c0 + q < chunks ? csum[(size_t)(c0 + q) * kBins + d] : 0u;
        sum += x[q];
    }
    uint32_t total;
    uint32_t run = dev::block_exclusive_sum(sum, s_tmp, &total);
#pragma unroll
    for (uint32_t q = 0; q < kColPer; ++q) {
        if (c0 + q < chunks) csum[(size_t)(c0 + q) * kBins + d] = run;
        run += x[q];
    }
    if (threadIdx.x == 0) dtot[d] = total;
}

__global__ __launch_bounds__(kBlock) void k_col_down(uint32_t *__restrict__ table, uint32_t rows, uint32_t chunks,
                                                     const uint32_t *__restrict__ csum,
                                                     const uint32_t *__restrict__ dtot) {
    __shared__ uint32_t s_tmp[kBlock / kWave];
    uint32_t r0, r1;
    col_chunk(rows, chunks, blockIdx.x, &r0, &r1);
    uint32_t all;
    const uint32_t dstart = dev::block_exclusive_sum(dtot[threadIdx.x], s_tmp, &all);
    uint32_t run = dstart + csum[(size_t)blockIdx.x * kBins + threadIdx.x];
    for (uint32_t r = r0; r < r1; ++r) {
        const size_t i = (size_t)r * kBins + threadIdx.x;
        const uint32_t x = table[i];
        table[i] = run;
        run += x;
    }
}

// IMPLICIT: the value of input element e is e + voff (vin unused).
template <typename K, int ITEMS, bool IMPLICIT>
__global__ __launch_bounds__(kBlock, 2) void k_radix_scatter(const K *__restrict__ kin,
                                                          const uint32_t *__restrict__ vin,
                                                          K *__restrict__ kout,
                                                          uint32_t *__restrict__ vout, uint32_t n,
                                                          uint32_t tiles, int shift, int nbits,
                                                          const uint32_t *__restrict__ table, uint32_t voff) {
    constexpr uint32_t TILE = kBlock * ITEMS;
    constexpr int W = kBlock / kWave;
    __shared__ uint32_t s_cnt[W][kBins];     // per-wave digit counters, then per-wave digit bases
    __shared__ uint32_t s_delta[kBins];      // global index minus tile slot, per digit
    __shared__ uint32_t s_tmp[W];
    // The per-wave lane masks of one item's digit are dead once the ranks are
    // known, before the tile is reordered: they share LDS with the tile, which
    // is reordered in two rounds (keys, then values) through the same bytes,
    // so a workgroup of 64-bit keys takes 38 KB of LDS instead of 54 KB.
    constexpr size_t kMatchBytes = sizeof(uint64_t) * W * kBins;
    constexpr size_t kTileBytes = sizeof(K) * TILE;
    __shared__ __align__(16) unsigned char s_raw[kMatchBytes > kTileBytes ? kMatchBytes : kTileBytes];
    uint64_t(*s_match)[kBins] = reinterpret_cast<uint64_t(*)[kBins]>(s_raw);
    K *s_key = reinterpret_cast<K *>(s_raw);
    uint32_t *s_val = reinterpret_cast<uint32_t *>(s_raw);

    uint32_t t;
    if (!xcd_tile(tiles, &t)) return;
    const unsigned tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
    const uint32_t mask = (1u << nbits) - 1u;
    const uint32_t gbase = table[(size_t)t * kBins + tid];   // output offset of digit tid for this tile
#pragma unroll
    for (int i = 0; i < W; ++i) {
        s_cnt[i][tid] = 0;
        s_match[i][tid] = 0;
    }
    const uint32_t base = t * TILE;
    const uint32_t nvalid = min(TILE, n - base);
    const uint32_t first = base + w * (kWave * ITEMS) + lane;
    K k[ITEMS];
    uint32_t v[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t e = first + r * kWave;
        const bool ok = e < n;
        k[r] = ok ? kin[e] : K(0);
        if constexpr (IMPLICIT) v[r] = e + voff;
        else v[r] = ok ? vin[e] : 0u;
    }
    __syncthreads();

    // Peer masks of every item: OR, read back, clear (no waits in between).
    // dr[r] holds the item's digit (kBins for a slot past the end) in its low
    // 9 bits and, once known, its rank among the wave's items of that digit
    // above them (digit and rank share a register).
    uint32_t dr[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r)
        dr[r] = (first + r * kWave < n) ? ((uint32_t)(k[r] >> shift) & mask) : (uint32_t)kBins;
    uint32_t *mw = reinterpret_cast<uint32_t *>(&s_match[w][0]);
    const uint32_t lbit = 1u << (lane & 31u), half = lane >> 5;
    // Items go in chunks: the mask operations of a whole chunk are issued
    // back to back, then its count operations, so LDS latency is paid once
    // per chunk and few masks are live at a time.
    constexpr int CH = (ITEMS % 8 == 0) ? 8 : 4;
#pragma unroll
    for (int c0 = 0; c0 < ITEMS; c0 += CH) {
        uint64_t pm[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int r = c0 + j;
            pm[j] = 0;
            if (dr[r] < kBins) {
                uint32_t *word = &mw[2 * dr[r]];
                __hip_atomic_fetch_or(word + half, lbit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                pm[j] = __hip_atomic_load(reinterpret_cast<uint64_t *>(word), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_WORKGROUP);
                __hip_atomic_store(reinterpret_cast<uint64_t *>(word), (uint64_t)0, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        // Ranks: the wave's running count of the digit (read before the
        // lowest peer advances it) plus the peers below.
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int r = c0 + j;
            const uint32_t below = dev::count_below(pm[j]);
            uint32_t old = 0;
            if (dr[r] < kBins) {
                uint32_t *cnt = &s_cnt[w][dr[r]];
                old = __hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                if (below == 0)
                    __hip_atomic_fetch_add(cnt, (uint32_t)__popcll(pm[j]), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            dr[r] |= (old + below) << 9;
        }
    }
    __syncthreads();

    uint32_t c[W], tot = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        c[i] = s_cnt[i][tid];
        tot += c[i];
    }
    uint32_t all;
    const uint32_t start = dev::block_exclusive_sum(tot, s_tmp, &all);
    uint32_t run = start;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        s_cnt[i][tid] = run;
        run += c[i];
    }
    s_delta[tid] = gbase - start;
    __syncthreads();

    uint32_t lp[ITEMS];   // tile slot of each item, TILE when it has none
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t d = dr[r] & 511u;
        const uint32_t x = s_cnt[w][min(d, (uint32_t)kBins - 1u)] + (dr[r] >> 9);
        lp[r] = (d < kBins && x < TILE) ? x : TILE;   // always a slot for a consistent ranking
        if (lp[r] < TILE) s_key[lp[r]] = k[r];
    }
    __syncthreads();

    // Slot i holds the element that goes to s_delta[digit] + i.
    uint32_t go[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t i = r * kBlock + tid;
        go[r] = 0xffffffffu;
        if (i < nvalid) {
            const K key = s_key[i];
            const uint32_t d = (uint32_t)(key >> shift) & mask;
            const uint32_t g = s_delta[d] + i;
            if (g < n) {                    // always true for a consistent count table
                kout[g] = key;
                go[r] = g;
            }
        }
    }
    __syncthreads();   // every key has left the tile: the values take its place
#pragma unroll
    for (int r = 0; r < ITEMS; ++r)
        if (lp[r] < TILE) s_val[lp[r]] = v[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r)
        if (go[r] != 0xffffffffu) vout[go[r]] = s_val[r * kBlock + tid];
}

// Exclusive scan of `count` words in place by one 1024-thread workgroup;
// each thread owns a contiguous slice.
__global__ __launch_bounds__(1024) void k_scan_inplace(uint32_t *__restrict__ vals, uint32_t count,
                                                       uint32_t *__restrict__ total) {
    __shared__ uint32_t s_w[16];
    const unsigned tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
    const uint32_t per = (count + 1023u) / 1024u;
    const uint32_t b = min(count, tid * per), e = min(count, b + per);
    uint32_t s = 0;
    for (uint32_t i = b; i < e; ++i) s += vals[i];
    uint32_t inc = dev::wave_inclusive_sum(s);
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    uint32_t wb = 0, tot = 0;
    for (int i = 0; i < 16; ++i) {
        uint32_t x = s_w[i];
        wb += (i < (int)w) ? x : 0u;
        tot += x;
    }
    uint32_t run = wb + inc - s;
    for (uint32_t i = b; i < e; ++i) {
        uint32_t x = vals[i];
        vals[i] = run;
        run += x;
    }
    if (tid == 0 && total) *total = tot;
}

// Device-wide exclusive scan: per-group sums of contiguous ranges, a scan of
// the sums, then each group rescans its range from its base.
constexpr int kScanItems = 8;
constexpr uint32_t kScanTile = kBlock * kScanItems;
constexpr uint32_t kScanGroups = 1024;

__device__ __forceinline__ void scan_range(uint32_t count, uint32_t groups, uint32_t g, uint32_t *b,
                                           uint32_t *e) {
    const uint32_t tiles = (count + kScanTile - 1) / kScanTile;
    *b = min(count, (uint32_t)((uint64_t)tiles * g / groups) * kScanTile);
    *e = min(count, (uint32_t)((uint64_t)tiles * (g + 1) / groups) * kScanTile);
}

__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t *__restrict__ data, uint32_t count,
                                                        uint32_t groups, uint32_t *__restrict__ sums) {
    __shared__ uint32_t s_tmp[kBlock / kWave];
    uint32_t b, e;
    scan_range(count, groups, blockIdx.x, &b, &e);
    uint32_t acc = 0;
    for (uint32_t i = b + threadIdx.x; i < e; i += kBlock) acc += data[i];
    uint32_t tot;
    dev::block_exclusive_sum(acc, s_tmp, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_scan_down(uint32_t *__restrict__ data, uint32_t count, uint32_t groups,
                                                      const uint32_t *__restrict__ sums) {
    __shared__ uint32_t s_tmp[kBlock / kWave];
    uint32_t b, e;
    scan_range(count, groups, blockIdx.x, &b, &e);
    uint32_t base = sums[blockIdx.x];
    for (uint32_t t0 = b; t0 < e; t0 += kScanTile) {
        const uint32_t i0 = t0 + threadIdx.x * kScanItems;
        uint32_t v[kScanItems];
        uint32_t c = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            v[i] = (i0 + i < e) ? data[i0 + i] : 0u;
            c += v[i];
        }
        uint32_t tot;
        uint32_t run = base + dev::block_exclusive_sum(c, s_tmp, &tot);
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            if (i0 + i < e) data[i0 + i] = run;
            run += v[i];
        }
        base += tot;
    }
}

template <typename K, int ITEMS>
lor_status radix_pass_items(const K *ki, const uint32_t *vi, uint32_t voff, K *ko, uint32_t *vo, uint32_t n,
                            int shift, int nbits, uint32_t *counts, hipStream_t s) {
    constexpr uint32_t TILE = kBlock * ITEMS;
    static_assert(TILE >= kMinTile, "tile below the size the count table is laid out for");
    const uint32_t tiles = div_up(n, TILE);
    const uint32_t grid = xcd_tile_grid(tiles);
    const uint32_t mask = (1u << nbits) - 1u;
    const uint32_t chunks = tiles < kColChunks ? tiles : kColChunks;
    uint32_t *table = counts;
    uint32_t *csum = counts + (size_t)kBins * div_up(n, kMinTile);
    const double tbytes = 4.0 * kBins * tiles;
    LOR_LAUNCH("k_radix_count", (double)n * sizeof(K) + tbytes, s,
               hipLaunchKernelGGL((k_radix_count<K, ITEMS>), dim3(grid), dim3(kBlock), 0, s, ki, n, tiles, shift,
                                  mask, table));
    LOR_LAUNCH("k_col_reduce", tbytes, s,
               hipLaunchKernelGGL(k_col_reduce, dim3(chunks), dim3(kBlock), 0, s, table, tiles, chunks, csum));
    uint32_t *dtot = csum + (size_t)kBins * kColChunks;
    LOR_LAUNCH("k_col_scan", 8.0 * kBins * chunks, s,
               hipLaunchKernelGGL(k_col_scan, dim3(kBins), dim3(kBlock), 0, s, csum, chunks, dtot));
    LOR_LAUNCH("k_col_down", 2.0 * tbytes, s,
               hipLaunchKernelGGL(k_col_down, dim3(chunks), dim3(kBlock), 0, s, table, tiles, chunks, csum,
                                  dtot));
    const double sbytes = (double)n * ((vi ? 2.0 : 1.0) * (sizeof(K) + 4) + (vi ? 0.0 : sizeof(K))) + tbytes;
    if (vi)
        LOR_LAUNCH("k_radix_scatter", sbytes, s,
                   hipLaunchKernelGGL((k_radix_scatter<K, ITEMS, false>), dim3(grid), dim3(kBlock), 0, s, ki, vi, ko,
                                      vo, n, tiles, shift, nbits, table, voff));
    else
        LOR_LAUNCH("k_radix_scatter", sbytes, s,
                   hipLaunchKernelGGL((k_radix_scatter<K, ITEMS, true>), dim3(grid), dim3(kBlock), 0, s, ki, vi, ko,
                                      vo, n, tiles, shift, nbits, table, voff));
    return LOR_OK;
}

}  // namespace

// Tile-major count table sized for the smallest tile, then the chunk sums
// and the digit totals of the column scan (workspace sizes do not depend on
// the plan).
size_t radix_counts_words(uint64_t n) {
    return (size_t)kBins * (div_up(n ? n : 1, kMinTile) + kColChunks + 1) + 64;
}

lor_status scan_exclusive(uint32_t *data, uint32_t count, uint32_t *tmp, uint32_t *total, hipStream_t s) {
    if (count == 0) return LOR_OK;
    uint32_t tiles = div_up(count, kScanTile);
    const uint32_t groups = tiles < kScanGroups ? tiles : kScanGroups;
    if (groups == 1) return scan_block_totals(data, count, total, s);
    LOR_LAUNCH("k_scan_reduce", 4.0 * count, s,
               hipLaunchKernelGGL(k_scan_reduce, dim3(groups), dim3(kBlock), 0, s, data, count, groups, tmp));
    LOR_TRY(scan_block_totals(tmp, groups, total, s));
    LOR_LAUNCH("k_scan_down", 8.0 * count, s,
               hipLaunchKernelGGL(k_scan_down, dim3(groups), dim3(kBlock), 0, s, data, count, groups, tmp));
    return LOR_OK;
}

int radix_passes(int bit_lo, int bit_hi) {
    const int step = plan().digit_bits;
    return bit_hi > bit_lo ? (bit_hi - bit_lo + step - 1) / step : 0;
}

lor_status scan_block_totals(uint32_t *vals, uint32_t count, uint32_t *total, hipStream_t s) {
    LOR_LAUNCH("k_scan_inplace", 8.0 * count, s,
               hipLaunchKernelGGL(k_scan_inplace, dim3(1), dim3(1024), 0, s, vals, count, total));
    return LOR_OK;
}

template <typename K>
lor_status radix_pass(const K *ki, const uint32_t *vi, uint32_t voff, K *ko, uint32_t *vo, uint32_t n, int shift,
                      int nbits, uint32_t *counts, hipStream_t s) {
    if (n == 0) return LOR_OK;
    const int items = sizeof(K) == 4 ? plan().items_u32 : plan().items_u64;
    if constexpr (sizeof(K) == 4) {
        switch (items) {
            case 8: return radix_pass_items<K, 8>(ki, vi, voff, ko, vo, n, shift, nbits, counts, s);
            case 12: return radix_pass_items<K, 12>(ki, vi, voff, ko, vo, n, shift, nbits, counts, s);
            case 24: return radix_pass_items<K, 24>(ki, vi, voff, ko, vo, n, shift, nbits, counts, s);
            default: return radix_pass_items<K, 16>(ki, vi, voff, ko, vo, n, shift, nbits, counts, s);
        }
    } else {
        switch (items) {
            case 12: return radix_pass_items<K, 12>(ki, vi, voff, ko, vo, n, shift, nbits, counts, s);
            case 16: return radix_pass_items<K, 16>(ki, vi, voff, ko, vo, n, shift, nbits, counts, s);
            default: return radix_pass_items<K, 8>(ki, vi, voff, ko, vo, n, shift, nbits, counts, s);
        }
    }
}

template <typename K>
lor_status radix_sort(K *k0, uint32_t *v0, K *k1, uint32_t *v1, uint32_t n, int bit_lo, int bit_hi,
                      uint32_t *counts, hipStream_t s, bool *in_alt) {
    *in_alt = false;
    if (n <= 1 || bit_hi <= bit_lo) return LOR_OK;
    K *ki = k0, *ko = k1;
    uint32_t *vi = v0, *vo = v1;
    const int step = plan().digit_bits;
    for (int shift = bit_lo; shift < bit_hi; shift += step) {
        const int nbits = min(step, bit_hi - shift);
        LOR_TRY(radix_pass<K>(ki, vi, 0, ko, vo, n, shift, nbits, counts, s));
        K *tk = ki; ki = ko; ko = tk;
        uint32_t *tv = vi; vi = vo; vo = tv;
        *in_alt = !*in_alt;
    }
    return LOR_OK;
}

template lor_status radix_pass<uint32_t>(const uint32_t *, const uint32_t *, uint32_t, uint32_t *, uint32_t *, uint32_t,
                                         int, int, uint32_t *, hipStream_t);
template lor_status radix_pass<uint64_t>(const uint64_t *, const uint32_t *, uint32_t, uint64_t *, uint32_t *, uint32_t,
                                         int, int, uint32_t *, hipStream_t);

template lor_status radix_sort<uint32_t>(uint32_t *, uint32_t *, uint32_t *, uint32_t *, uint32_t, int, int,
                                         uint32_t *, hipStream_t, bool *);
template lor_status radix_sort<uint64_t>(uint64_t *, uint32_t *, uint64_t *, uint32_t *, uint32_t, int, int,
                                         uint32_t *, hipStream_t, bool *);

}  // namespace lor
