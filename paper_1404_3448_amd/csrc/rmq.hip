// Range minimum over the LCP array on gfx950 (Section III: the lcp of two
// suffixes is the minimum LCP between their ranks; RMQ returns the position
// of a smallest element in a range).
//
// The paper answers RMQ through a Cartesian tree, an Euler tour and +-1RMQ.
// Here the structure is a sparse table: level k holds the minimum of every
// window of 2^k LCP entries, and a query reads two overlapping windows that
// cover its range. Levels 1-10 are built in one pass: a workgroup loads a
// tile of the LCP array plus the halo the ten levels reach into, and
// computes and writes those levels from LDS, so the LCP array is read once
// for ten levels. Higher levels (windows wider than a tile) are built three
// (or two) at a time from level k-1 by workgroups that walk columns of
// blocks 2^(k-1) entries apart and keep the blocks they still need in
// registers, so level k-1 is read about once per pass and every level is
// written once. With 288 GB of HBM the table fits next to
// the 1G-suffix arrays, and every query costs four independent gathers
// (two ISA entries, two table entries) instead of a pointer walk.
// Levels hold minima of LCP values, so when the largest LCP is at most
// 65535 (a reduction pass writes it into the table's header first) every
// level is stored as 16-bit entries: half the bytes to write and read. The
// kernels read the header and pick the width themselves, so nothing waits
// on the host.
#include <climits>

#include "lor_internal.hpp"

namespace lor {

namespace {

// One level from the previous one, a tile of kLvTile outputs per workgroup.
// Entry x of the previous level is read twice: by output tile x's workgroup
// and by the one 2^(k-1) entries to its left. When that distance spans H >= 1
// tiles, tiles t and t + H are taken one right after the other (order within
// groups of 2H tiles: 0, H, 1, H + 1, ...), so the second read of the shared
// tile finds it in L2; the sequence is dealt to the XCDs in contiguous
// eighths so that partners run on the same XCD.
constexpr uint32_t kLvItems = 16;
constexpr uint32_t kLvTile = kBlock * kLvItems;

// Level storage of a table: entries from `base` on, 16-bit when the header
// word says every LCP value fits (hdr == nullptr: always 32-bit).
struct TabView {
    int32_t *w32;
    uint16_t *w16;
    bool narrow;
    __device__ __forceinline__ int32_t get(uint64_t i) const { return narrow ? (int32_t)w16[i] : w32[i]; }
    __device__ __forceinline__ void put(uint64_t i, int32_t v) const {
        if (narrow) w16[i] = (uint16_t)v;
        else w32[i] = v;
    }
};

__device__ __forceinline__ TabView tab_view(int32_t *base, const uint32_t *hdr) {
    TabView t;
    t.w32 = base;
    t.w16 = reinterpret_cast<uint16_t *>(base);
    t.narrow = hdr != nullptr && hdr[0] <= 65535u;
    return t;
}

__global__ __launch_bounds__(kBlock) void k_st_level(int32_t *__restrict__ base, const uint32_t *__restrict__ hdr,
                                                     uint64_t prev_off, uint64_t cur_off, uint32_t half,
                                                     uint32_t cnt, uint32_t tiles) {
    const TabView tv = tab_view(base, hdr);
    const uint32_t per = (tiles + kXcds - 1) / kXcds;
    const uint32_t j = (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;   // place in the sequence
    if (blockIdx.x / kXcds >= per || j >= tiles) return;
    const uint32_t H = half / kLvTile;
    uint32_t t = j;
    if (H >= 1) {
        const uint32_t G = 2 * H, g = j / G, k = j % G;
        if ((uint64_t)(g + 1) * G <= tiles) t = g * G + (k >> 1) + (k & 1u) * H;   // a partial last group keeps plain order
    }
    const uint32_t i0 = t * kLvTile + threadIdx.x;
    int32_t a[kLvItems], b[kLvItems];
#pragma unroll
    for (int r = 0; r < (int)kLvItems; ++r) {
        const uint32_t i = i0 + r * kBlock;
        a[r] = i < cnt ? tv.get(prev_off + i) : 0;
        b[r] = i < cnt ? tv.get(prev_off + i + half) : 0;
    }
#pragma unroll
    for (int r = 0; r < (int)kLvItems; ++r) {
        const uint32_t i = i0 + r * kBlock;
        if (i < cnt) tv.put(cur_off + i, min(a[r], b[r]));
    }
}

__device__ __forceinline__ uint64_t level_offset_dev(uint64_t n, int level);

// NL levels k .. k+NL-1 from level k-1 (P) in one pass. With h = 2^(k-1)
// and blocks of B = 256 ITEMS entries (B divides h, H = h / B), output entry
// i of level k+a is the minimum of P[i + u h] over u < 2^(a+1), and
// i + u h lies u blocks of H further along the column of blocks
// b, b + H, b + 2H, ... A workgroup walks `steps` consecutive blocks of one
// column and keeps the last 2^NL blocks of P in registers, so each block of
// P is read from HBM about once for all NL levels (instead of twice per
// level); the writes are the table itself.
template <int NL, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_st_chain(int32_t *__restrict__ table, const uint32_t *__restrict__ hdr,
                                                     uint32_t cnt_p, uint32_t n, int k, uint32_t H, uint32_t nb,
                                                     uint32_t steps) {
    const TabView tv = tab_view(table, hdr);
    const uint64_t p_off = level_offset_dev(n, k - 1);   // level k-1 (k >= 2)
    constexpr int W = 1 << NL;
    constexpr uint32_t B = kBlock * ITEMS;
    const uint32_t c = blockIdx.x % H;
    const uint32_t j0 = (blockIdx.x / H) * steps;
    const uint32_t len = nb > c ? (nb - 1 - c) / H + 1 : 0;   // blocks of this column
    if (j0 >= len) return;
    const uint32_t j1 = min(len, j0 + steps);
    int32_t win[W][ITEMS];
    auto load = [&](uint32_t j, int32_t (&dst)[ITEMS]) {
        const uint64_t base = (uint64_t)(c + (uint64_t)j * H) * B + threadIdx.x;
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            const uint64_t idx = base + (uint64_t)r * kBlock;
            dst[r] = idx < cnt_p ? tv.get(p_off + idx) : INT_MAX;
        }
    };
#pragma unroll
    for (int u = 0; u < W - 1; ++u) load(j0 + u, win[u]);
    for (uint32_t j = j0; j < j1; ++j) {
        load(j + W - 1, win[W - 1]);
        const uint64_t i0 = (uint64_t)(c + (uint64_t)j * H) * B + threadIdx.x;
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            const uint64_t i = i0 + (uint64_t)r * kBlock;
            int32_t m = win[0][r];
#pragma unroll
            for (int a = 0; a < NL; ++a) {
#pragma unroll
                for (int u = 1 << a; u < (2 << a); ++u) m = min(m, win[u][r]);
                const int lv = k + a;
                if (i < (uint64_t)n - (1ull << lv) + 1) tv.put(level_offset_dev(n, lv) + i, m);
            }
        }
#pragma unroll
        for (int u = 0; u < W - 1; ++u)
#pragma unroll
            for (int r = 0; r < ITEMS; ++r) win[u][r] = win[u + 1][r];
    }
}

constexpr uint32_t kChainSteps = 8;         // blocks per workgroup along a column (8 beat 4, 16, 32 and 64)

constexpr uint32_t kStTile = kBlock * 8;    // outputs per workgroup in fused levels
constexpr int kStFuse = 10;                 // levels per fused pass
constexpr int kStFusedTop = 10;             // levels 1..10 are built in LDS (halo < 1024 entries)
constexpr uint32_t kRmqBlock = 64;          // LCP entries per block of the compact table

// Levels k0 .. k0+nl-1 from level k0-1 (`prev`, prev_count entries) for the
// outputs [i0, i0 + kStTile) of this workgroup.
__global__ __launch_bounds__(kBlock) void k_st_fused(const int32_t *__restrict__ prev, uint32_t prev_count,
                                                     uint32_t n, int k0, int nl, int32_t *__restrict__ table,
                                                     const uint32_t *__restrict__ hdr) {
    extern __shared__ int32_t s_buf[];
    const TabView tv = tab_view(table, hdr);
    const uint32_t halo = (1u << (k0 - 1)) * ((1u << nl) - 1u);
    const uint32_t span = kStTile + halo;
    int32_t *b0 = s_buf, *b1 = s_buf + span;
    const uint32_t i0 = blockIdx.x * kStTile;
    for (uint32_t j = threadIdx.x; j < span; j += kBlock) {
        const uint32_t i = i0 + j;
        b0[j] = i < prev_count ? prev[i] : INT_MAX;
    }
    __syncthreads();
    uint32_t valid = span;
    for (int l = 0; l < nl; ++l) {
        const int k = k0 + l;
        const uint32_t half = 1u << (k - 1);
        valid -= half;
        for (uint32_t j = threadIdx.x; j < valid; j += kBlock) b1[j] = min(b0[j], b0[j + half]);
        __syncthreads();
        const uint32_t count = n - (1u << k) + 1u;
        const uint64_t off = level_offset_dev(n, k);
        for (uint32_t j = threadIdx.x; j < kStTile; j += kBlock) {
            const uint32_t i = i0 + j;
            if (i < count) tv.put(off + i, b1[j]);
        }
        int32_t *x = b0; b0 = b1; b1 = x;
        __syncthreads();
    }
}

struct Levels {
    const int32_t *lcp;
    int32_t *table;          // level storage (after the header)
    const uint32_t *hdr;     // the header
    uint32_t n;
    int levels;
};

__device__ __forceinline__ uint64_t level_offset_dev(uint64_t n, int level) {
    // entries of levels 1..level-1: sum over k of (n - 2^k + 1)
    const uint64_t k = (uint64_t)level - 1;
    return k * (n + 1) - ((2ull << k) - 2ull);
}

// Entry i of level k (level 0 is the LCP array).
__device__ __forceinline__ int32_t level_at(const Levels &L, const TabView &tv, int k, uint32_t i) {
    return k == 0 ? L.lcp[i] : tv.get(level_offset_dev(L.n, k) + i);
}

// min of a[lo..hi] (lo <= hi) and, when want_pos, its leftmost position.
__device__ __forceinline__ int32_t range_min(const Levels &L, const TabView &tv, uint32_t lo, uint32_t hi,
                                             bool want_pos, int32_t *pos) {
    const uint32_t len = hi - lo + 1;
    const int k = 31 - __builtin_clz(len);
    const int32_t v = min(level_at(L, tv, k, lo), level_at(L, tv, k, hi + 1 - (1u << k)));
    if (want_pos) {
        uint32_t p = lo;
        for (int kk = k; kk >= 0; --kk) {
            const uint32_t w = 1u << kk;
            if (p + w - 1 <= hi && level_at(L, tv, kk, p) > v) p += w;
        }
        *pos = (int32_t)p;
    }
    return v;
}

__global__ __launch_bounds__(kBlock) void k_query(Levels L, const int32_t *__restrict__ isa, int mode,
                                                  const int32_t *__restrict__ qi, const int32_t *__restrict__ qj,
                                                  uint32_t nq, int32_t *__restrict__ out_min,
                                                  int32_t *__restrict__ out_arg) {
    const TabView tv = tab_view(L.table, L.levels > 0 ? L.hdr : nullptr);
    for (uint32_t q = blockIdx.x * kBlock + threadIdx.x; q < nq; q += gridDim.x * kBlock) {
        const int32_t a = qi[q], b = qj[q];
        int32_t v = -1, pos = -1;
        if (mode == 0) {
            if (a >= 0 && b >= a && (uint32_t)b < L.n)
                v = range_min(L, tv, (uint32_t)a, (uint32_t)b, out_arg != nullptr, &pos);
        } else if (a >= 0 && b >= 0 && (uint32_t)a < L.n && (uint32_t)b < L.n) {
            if (a == b) {
                v = (int32_t)(L.n - (uint32_t)a);
            } else {
                const int32_t ra = isa[a], rb = isa[b];
                if (ra != rb && (uint32_t)ra < L.n && (uint32_t)rb < L.n) {
                    const uint32_t lo = (uint32_t)min(ra, rb) + 1u, hi = (uint32_t)max(ra, rb);
                    v = range_min(L, tv, lo, hi, out_arg != nullptr, &pos);
                }
            }
        }
        out_min[q] = v;
        if (out_arg) out_arg[q] = pos;
    }
}

// Largest LCP value into hdr[0] (zeroed before): a grid of at most
// kMaxGrid workgroups, each reducing in registers and LDS, then one atomic
// per workgroup (skipped when the published value is already as large).
constexpr uint32_t kMaxGrid = 2048;

__global__ __launch_bounds__(kBlock) void k_lcp_max(const int32_t *__restrict__ lcp, uint32_t n,
                                                    uint32_t *__restrict__ hdr) {
    __shared__ uint32_t s_red[kBlock / kWave];
    uint32_t m = 0;
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
        m = max(m, (uint32_t)max(lcp[i], 0));
    for (int o = 32; o > 0; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o, 64));
    if ((threadIdx.x & 63u) == 0) s_red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / kWave; ++w) m = max(m, s_red[w]);
        if (m > __hip_atomic_load(hdr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(hdr, m);
    }
}

__global__ __launch_bounds__(kWave) void k_hdr_zero(uint32_t *hdr) {
    if (threadIdx.x < kRmqHeaderWords) hdr[threadIdx.x] = 0;
}

// ------------------------------------------------------ compact variant
// A sparse table over the minima of kRmqBlock-entry blocks of LCP (level 0 =
// the block minima, levels 1.. over blocks), about 4 n / 64 * log2(n / 64)
// bytes instead of 4 n log2 n. A query scans the partial blocks at its two
// ends in LCP itself and takes the whole blocks between them from the table.

struct Compact {
    const int32_t *lcp;
    const int32_t *table;
    uint32_t n, nb;
    int levels;
};

__device__ __forceinline__ const int32_t *clevel(const Compact &C, int k) {
    return k == 0 ? C.table : C.table + C.nb + level_offset_dev(C.nb, k);
}

// Smallest value of lcp[a..b] (a <= b) and its leftmost position.
__device__ __forceinline__ int32_t scan_min(const int32_t *__restrict__ lcp, uint32_t a, uint32_t b, uint32_t *pos) {
    int32_t best = INT_MAX;
    uint32_t bp = a;
    for (uint32_t x = a; x <= b; ++x) {
        const int32_t y = lcp[x];
        if (y < best) {
            best = y;
            bp = x;
        }
    }
    *pos = bp;
    return best;
}

__device__ int32_t range_min_compact(const Compact &C, uint32_t lo, uint32_t hi, bool want_pos, int32_t *pos) {
    const uint32_t bl = lo / kRmqBlock, bh = hi / kRmqBlock;
    uint32_t p;
    if (bh - bl <= 1) {
        const int32_t v = scan_min(C.lcp, lo, hi, &p);
        *pos = (int32_t)p;
        return v;
    }
    uint32_t pl, pr;
    const int32_t vl = scan_min(C.lcp, lo, (bl + 1) * kRmqBlock - 1, &pl);
    const int32_t vr = scan_min(C.lcp, bh * kRmqBlock, hi, &pr);
    const uint32_t a = bl + 1, c = bh - 1;   // whole blocks in between
    const int k = 31 - __builtin_clz(c - a + 1);
    const int32_t *lv = clevel(C, k);
    const int32_t vm = min(lv[a], lv[c + 1 - (1u << k)]);
    const int32_t v = min(vl, min(vm, vr));
    if (want_pos) {
        if (vl == v) {
            *pos = (int32_t)pl;
        } else if (vm == v) {
            uint32_t b = a;   // leftmost block whose minimum is v
            for (int kk = k; kk >= 0; --kk) {
                const uint32_t w = 1u << kk;
                if (b + w - 1 <= c && clevel(C, kk)[b] > v) b += w;
            }
            uint32_t x = b * kRmqBlock;
            const uint32_t xe = x + kRmqBlock - 1;   // the block holds v; bounded all the same
            while (x < xe && C.lcp[x] != v) ++x;
            *pos = (int32_t)x;
        } else {
            *pos = (int32_t)pr;
        }
    }
    return v;
}

__global__ __launch_bounds__(kBlock) void k_block_min(const int32_t *__restrict__ lcp, uint32_t n, uint32_t nb,
                                                      int32_t *__restrict__ bmin) {
    const uint32_t b = (blockIdx.x * kBlock + threadIdx.x) / kWave, lane = threadIdx.x & 63u;
    if (b >= nb) return;   // whole waves
    const uint32_t i = b * kRmqBlock + lane;
    int32_t v = i < n ? lcp[i] : INT_MAX;
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    if (lane == 0) bmin[b] = v;
}

__global__ __launch_bounds__(kBlock) void k_query_compact(Compact C, const int32_t *__restrict__ isa, int mode,
                                                          const int32_t *__restrict__ qi,
                                                          const int32_t *__restrict__ qj, uint32_t nq,
                                                          int32_t *__restrict__ out_min,
                                                          int32_t *__restrict__ out_arg) {
    for (uint32_t q = blockIdx.x * kBlock + threadIdx.x; q < nq; q += gridDim.x * kBlock) {
        const int32_t a = qi[q], b = qj[q];
        int32_t v = -1, pos = -1;
        if (mode == 0) {
            if (a >= 0 && b >= a && (uint32_t)b < C.n)
                v = range_min_compact(C, (uint32_t)a, (uint32_t)b, out_arg != nullptr, &pos);
        } else if (a >= 0 && b >= 0 && (uint32_t)a < C.n && (uint32_t)b < C.n) {
            if (a == b) {
                v = (int32_t)(C.n - (uint32_t)a);
            } else {
                const int32_t ra = isa[a], rb = isa[b];
                if (ra != rb && (uint32_t)ra < C.n && (uint32_t)rb < C.n) {
                    const uint32_t lo = (uint32_t)min(ra, rb) + 1u, hi = (uint32_t)max(ra, rb);
                    v = range_min_compact(C, lo, hi, out_arg != nullptr, &pos);
                }
            }
        }
        out_min[q] = v;
        if (out_arg) out_arg[q] = pos;
    }
}

}  // namespace

uint64_t rmq_compact_blocks(uint64_t n) { return (n + kRmqBlock - 1) / kRmqBlock; }

uint64_t rmq_compact_entries(uint64_t n, int *levels) {
    const uint64_t nb = rmq_compact_blocks(n);
    const int L = nb >= 2 ? bits_for(nb) - 1 : 0;
    if (levels) *levels = L;
    return nb + (L ? rmq_level_offset(nb, L + 1) : 0);
}

lor_status rmq_build_compact(const int32_t *lcp, uint32_t n, int32_t *table, hipStream_t s) {
    if (n == 0) return LOR_OK;
    int L;
    rmq_compact_entries(n, &L);
    const uint32_t nb = (uint32_t)rmq_compact_blocks(n);
    LOR_LAUNCH("k_block_min", 4.0 * n + 4.0 * nb, s,
               hipLaunchKernelGGL(k_block_min, dim3(div_up((uint64_t)nb * kWave, kBlock)), dim3(kBlock), 0, s, lcp,
                                  n, nb, table));
    return rmq_build_levels(table, nb, table + nb, L, s, nullptr, 4);
}

lor_status rmq_queries_compact(const int32_t *table, uint32_t n, int levels, const int32_t *lcp, const int32_t *isa,
                               int mode, const int32_t *qi, const int32_t *qj, uint32_t nq, int32_t *min_out,
                               int32_t *argmin_out, hipStream_t s) {
    if (nq == 0) return LOR_OK;
    Compact C{lcp, table, n, (uint32_t)rmq_compact_blocks(n), levels};
    LOR_LAUNCH("k_query_compact", (double)nq * (mode ? 28 : 20), s,
               hipLaunchKernelGGL(k_query_compact, dim3(grid_for(nq)), dim3(kBlock), 0, s, C, isa, mode, qi, qj, nq,
                                  min_out, argmin_out));
    return LOR_OK;
}

uint64_t rmq_level_offset(uint64_t n, int level) {
    const uint64_t k = (uint64_t)level - 1;
    return k * (n + 1) - ((2ull << k) - 2ull);
}

lor_status rmq_build_full(const int32_t *lcp, uint32_t n, int32_t *buffer, int levels, hipStream_t s) {
    if (levels <= 0) return LOR_OK;
    uint32_t *hdr = reinterpret_cast<uint32_t *>(buffer);
    LOR_LAUNCH("k_hdr_zero", 4.0 * kRmqHeaderWords, s,
               hipLaunchKernelGGL(k_hdr_zero, dim3(1), dim3(kWave), 0, s, hdr));
    LOR_LAUNCH("k_lcp_max", 4.0 * n, s,
               hipLaunchKernelGGL(k_lcp_max, dim3(min(grid_for(n), kMaxGrid)), dim3(kBlock), 0, s, lcp, n, hdr));
    // The width is the kernels' own decision; only per-kernel byte accounting
    // (timing on) reads it back, to count the entry size the levels really use.
    int eb = 4;
    if (timing_on()) {
        uint32_t mx = 0;
        LOR_HIP(hipMemcpyAsync(&mx, hdr, sizeof(mx), hipMemcpyDeviceToHost, s));
        LOR_HIP(hipStreamSynchronize(s));
        eb = mx <= 65535u ? 2 : 4;
    }
    return rmq_build_levels(lcp, n, buffer + kRmqHeaderWords, levels, s, hdr, eb);
}

lor_status rmq_build_levels(const int32_t *lcp, uint32_t n, int32_t *table, int levels, hipStream_t s,
                            const uint32_t *hdr, int eb) {
    int k = 1;
    while (k <= levels && k <= kStFusedTop) {
        const int nl = min(kStFuse, min(levels, kStFusedTop) - k + 1);
        const int32_t *prev = lcp;   // k == 1: the fused pass starts from level 0
        const uint32_t prev_count = n - (1u << (k - 1)) + 1u;
        const uint32_t count = n - (1u << k) + 1u;
        const uint32_t halo = (1u << (k - 1)) * ((1u << nl) - 1u);
        const size_t lds = 2 * (size_t)(kStTile + halo) * sizeof(int32_t);
        double bytes = 0;
        for (int l = 0; l < nl; ++l) bytes += (double)eb * (n - (1u << (k + l)) + 1u);
        bytes += 4.0 * prev_count;
        LOR_LAUNCH("k_st_fused", bytes, s,
                   hipLaunchKernelGGL(k_st_fused, dim3(div_up(count, kStTile)), dim3(kBlock), lds, s, prev,
                                      prev_count, n, k, nl, table, hdr));
        k += nl;
    }
    while (k <= levels) {
        const uint32_t half = 1u << (k - 1);
        const int nl = min(3, levels - k + 1);
        const uint32_t items = half >= kBlock * 16u && nl < 3 ? 16u : (half >= kBlock * 8u ? 8u : 4u);
        if (nl == 1 || half < kBlock * 4u) {
            const uint32_t cnt = n - (1u << k) + 1u;
            const uint32_t tiles = div_up(cnt, kLvTile);
            LOR_LAUNCH("k_st_level", (double)cnt * 2 * eb, s,
                       hipLaunchKernelGGL(k_st_level, dim3(kXcds * div_up(tiles, kXcds)), dim3(kBlock), 0, s, table,
                                          hdr, rmq_level_offset(n, k - 1), rmq_level_offset(n, k), half, cnt,
                                          tiles));
            ++k;
            continue;
        }
        const uint32_t B = kBlock * items, H = half / B;
        const uint32_t cnt_p = n - half + 1u;
        const uint32_t nb = div_up(n - (1u << k) + 1u, B);   // blocks holding level-k outputs
        const uint32_t segs = div_up(div_up(nb, H), kChainSteps);
        double bytes = (double)eb * cnt_p;
        for (int a = 0; a < nl; ++a) bytes += (double)eb * (n - (1u << (k + a)) + 1u);
        const dim3 grid(H * segs);
#define LOR_CHAIN(NL, IT)                                                                                   \
    LOR_LAUNCH("k_st_chain", bytes, s,                                                                      \
               hipLaunchKernelGGL((k_st_chain<NL, IT>), grid, dim3(kBlock), 0, s, table, hdr, cnt_p, n, k, H, \
                                  nb, kChainSteps))
        if (nl == 3) {
            if (items == 4) LOR_CHAIN(3, 4);
            else LOR_CHAIN(3, 8);
        } else {
            if (items == 4) LOR_CHAIN(2, 4);
            else if (items == 8) LOR_CHAIN(2, 8);
            else LOR_CHAIN(2, 16);
        }
#undef LOR_CHAIN
        k += nl;
    }
    return LOR_OK;
}

lor_status rmq_queries(int32_t *buffer, uint32_t n, int levels, const int32_t *lcp, const int32_t *isa,
                       int mode, const int32_t *qi, const int32_t *qj, uint32_t nq, int32_t *min_out,
                       int32_t *argmin_out, hipStream_t s) {
    if (nq == 0) return LOR_OK;
    Levels L{lcp, levels > 0 ? buffer + kRmqHeaderWords : nullptr, reinterpret_cast<const uint32_t *>(buffer), n,
             levels};
    LOR_LAUNCH("k_query", (double)nq * (mode ? 28 : 20), s,
               hipLaunchKernelGGL(k_query, dim3(grid_for(nq)), dim3(kBlock), 0, s, L, isa, mode, qi, qj, nq,
                                  min_out, argmin_out));
    return LOR_OK;
}

}  // namespace lor
