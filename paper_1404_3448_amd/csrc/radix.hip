// Stable LSD radix sort of (key, u32 value) pairs on gfx950.
//
// Section IV sorts DC3's sample and non-sample keys with a radix sort that
// walks the digits from least to most significant, each pass a stable split
// computed with a prefix scan (one bit per pass in the paper's kernel).
// Here a pass handles a digit of up to 8 bits (the width and the tile size
// come from the tuning plan) and runs as three kernels:
//   1. count  : every workgroup owns a contiguous run of tiles and builds the
//               digit histogram of its run in LDS (per-wave sub-histograms);
//   2. scan   : a device-wide exclusive scan turns the digit-major table
//               counts[d][g] into global offsets (digit d of group g starts
//               after every smaller digit and after digit d of groups < g);
//   3. scatter: every workgroup walks its tiles in order; inside a tile each
//               wave ranks its elements by digit with 8 ballots per round
//               (lanes with the same digit form a peer mask; the rank is the
//               number of peers in lower lanes), the tile is reordered by
//               digit in LDS, and written out so that runs of equal digits
//               leave as contiguous stores.
// Element order inside a tile is wave-major then round-major then lane, so
// ranks follow input order and every pass is stable.
#include "lor_internal.hpp"

namespace lor {

namespace {

constexpr int kDigitBits = 8;
constexpr int kBins = 1 << kDigitBits;
constexpr uint32_t kMaxGroups = 1024;     // workgroups per pass (fixed: workspace sizes are device-independent)


__device__ __forceinline__ void tile_range(uint32_t tiles, uint32_t groups, uint32_t g, uint32_t *t0,
                                           uint32_t *t1) {
    *t0 = (uint32_t)((uint64_t)tiles * g / groups);
    *t1 = (uint32_t)((uint64_t)tiles * (g + 1) / groups);
}

template <typename K, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_radix_count(const K *__restrict__ keys, uint32_t n,
                                                        uint32_t tiles, uint32_t groups, int shift,
                                                        uint32_t mask, uint32_t *__restrict__ counts) {
    constexpr uint32_t TILE = kBlock * ITEMS;
    __shared__ uint32_t hist[kBlock / kWave][kBins];
    const unsigned tid = threadIdx.x, w = tid >> 6;
#pragma unroll
    for (int i = 0; i < kBlock / kWave; ++i) hist[i][tid] = 0;
    __syncthreads();
    uint32_t t0, t1;
    tile_range(tiles, groups, blockIdx.x, &t0, &t1);
    for (uint32_t t = t0; t < t1; ++t) {
        const uint32_t base = t * TILE + tid;
        K k[ITEMS];
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            uint32_t e = base + r * kBlock;
            k[r] = (e < n) ? keys[e] : K(0);
        }
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            uint32_t e = base + r * kBlock;
            if (e < n) atomicAdd(&hist[w][(uint32_t)(k[r] >> shift) & mask], 1u);
        }
    }
    __syncthreads();
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kBlock / kWave; ++i) s += hist[i][tid];
    counts[(size_t)tid * groups + blockIdx.x] = s;
}

// vin == nullptr: the value of input element e is e + voff.
template <typename K, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_radix_scatter(const K *__restrict__ kin,
                                                          const uint32_t *__restrict__ vin,
                                                          K *__restrict__ kout,
                                                          uint32_t *__restrict__ vout, uint32_t n,
                                                          uint32_t tiles, uint32_t groups, int shift,
                                                          int nbits,
                                                          const uint32_t *__restrict__ offs, uint32_t voff) {
    constexpr uint32_t TILE = kBlock * ITEMS;
    constexpr int W = kBlock / kWave;
    __shared__ uint32_t s_cnt[W][kBins];   // per-wave digit counters, then digit bases per wave
    __shared__ uint32_t s_base[kBins];     // global output base of every digit for this group
    __shared__ uint32_t s_start[kBins];    // first tile-local slot of every digit
    __shared__ uint32_t s_tmp[W];
    __shared__ K s_key[TILE];
    __shared__ uint32_t s_val[TILE];

    const unsigned tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
    const uint32_t mask = (1u << nbits) - 1u;
    s_base[tid] = offs[(size_t)tid * groups + blockIdx.x];
    uint32_t t0, t1;
    tile_range(tiles, groups, blockIdx.x, &t0, &t1);

    // The next tile's keys and values are loaded while the current tile is
    // ranked and stored, so global-memory latency overlaps the LDS work.
    K kn[ITEMS];
    uint32_t vn[ITEMS];
    auto load_tile = [&](uint32_t t) {
        const uint32_t first = t * TILE + w * (kWave * ITEMS) + lane;
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            const uint32_t e = first + r * kWave;
            const bool ok = e < n;
            kn[r] = ok ? kin[e] : K(0);
            vn[r] = ok ? (vin ? vin[e] : e + voff) : 0u;
        }
    };
    if (t0 < t1) load_tile(t0);

    for (uint32_t t = t0; t < t1; ++t) {
        const uint32_t base = t * TILE;
        const uint32_t nvalid = min(TILE, n - base);
#pragma unroll
        for (int i = 0; i < W; ++i) s_cnt[i][tid] = 0;
        __syncthreads();

        const uint32_t wfirst = base + w * (kWave * ITEMS) + lane;
        K k[ITEMS];
        uint32_t v[ITEMS];
        uint32_t rk[ITEMS];
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            k[r] = kn[r];
            v[r] = vn[r];
        }
        if (t + 1 < t1) load_tile(t + 1);
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            const bool ok = (wfirst + r * kWave) < n;
            const uint32_t d = (uint32_t)(k[r] >> shift) & mask;
            uint64_t peers = __ballot(ok);
            for (int b = 0; b < nbits; ++b) {
                const bool set = (d >> b) & 1u;
                const uint64_t m = __ballot(set);
                peers &= set ? m : ~m;
            }
            const uint32_t below = dev::count_below(peers);
            uint32_t old = 0;
            if (ok) old = s_cnt[w][d];
            // All lanes of the wave read before the lowest peer writes: LDS
            // accesses of one wave execute in program order.
            if (ok && below == 0) s_cnt[w][d] = old + (uint32_t)__popcll(peers);
            rk[r] = old + below;
        }
        __syncthreads();

        const uint32_t c0 = s_cnt[0][tid], c1 = s_cnt[1][tid], c2 = s_cnt[2][tid], c3 = s_cnt[3][tid];
        const uint32_t tot = c0 + c1 + c2 + c3;
        uint32_t all;
        const uint32_t start = dev::block_exclusive_sum(tot, s_tmp, &all);
        s_cnt[0][tid] = start;
        s_cnt[1][tid] = start + c0;
        s_cnt[2][tid] = start + c0 + c1;
        s_cnt[3][tid] = start + c0 + c1 + c2;
        s_start[tid] = start;
        __syncthreads();

#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            if ((wfirst + r * kWave) < n) {
                const uint32_t d = (uint32_t)(k[r] >> shift) & mask;
                const uint32_t lp = s_cnt[w][d] + rk[r];
                s_key[lp] = k[r];
                s_val[lp] = v[r];
            }
        }
        __syncthreads();

        for (uint32_t i = tid; i < nvalid; i += kBlock) {
            const K key = s_key[i];
            const uint32_t d = (uint32_t)(key >> shift) & mask;
            const uint32_t g = s_base[d] + (i - s_start[d]);
            kout[g] = key;
            vout[g] = s_val[i];
        }
        __syncthreads();
        s_base[tid] += tot;
    }
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

uint32_t groups_for(uint32_t n, uint32_t tile, uint32_t *tiles) {
    *tiles = div_up(n, tile);
    return *tiles < kMaxGroups ? (*tiles ? *tiles : 1) : kMaxGroups;
}

template <typename K, int ITEMS>
lor_status radix_pass_items(const K *ki, const uint32_t *vi, uint32_t voff, K *ko, uint32_t *vo, uint32_t n,
                            int shift, int nbits, uint32_t *counts, hipStream_t s) {
    uint32_t tiles;
    const uint32_t groups = groups_for(n, kBlock * ITEMS, &tiles);
    const uint32_t mask = (1u << nbits) - 1u;
    LOR_LAUNCH("k_radix_count", (double)n * sizeof(K), s,
               hipLaunchKernelGGL((k_radix_count<K, ITEMS>), dim3(groups), dim3(kBlock), 0, s, ki, n, tiles, groups,
                                  shift, mask, counts));
    LOR_TRY(scan_exclusive(counts, (uint32_t)kBins * groups, counts + (size_t)kBins * kMaxGroups, nullptr, s));
    LOR_LAUNCH("k_radix_scatter", (double)n * ((vi ? 2.0 : 1.0) * (sizeof(K) + 4) + (vi ? 0.0 : sizeof(K))), s,
               hipLaunchKernelGGL((k_radix_scatter<K, ITEMS>), dim3(groups), dim3(kBlock), 0, s, ki, vi, ko, vo, n,
                                  tiles, groups, shift, nbits, counts, voff));
    return LOR_OK;
}

}  // namespace

size_t radix_counts_words(uint64_t) { return (size_t)kBins * kMaxGroups + kScanTmpWords + 64; }

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
            case 4: return radix_pass_items<K, 4>(ki, vi, voff, ko, vo, n, shift, nbits, counts, s);
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
