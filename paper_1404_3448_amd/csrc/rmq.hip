// Range minimum over the LCP array on gfx950 (Section III: the lcp of two
// suffixes is the minimum LCP between their ranks; RMQ returns the position
// of a smallest element in a range).
//
// The paper answers RMQ through a Cartesian tree, an Euler tour and +-1RMQ.
// Here the structure is a sparse table: level k holds the minimum of every
// window of 2^k LCP entries, and a query reads two overlapping windows that
// cover its range. Levels 1-9 are built in one pass: a wave loads a
// segment of the LCP array plus the halo the nine levels reach into, and
// computes and writes those levels in registers (wave shuffles for windows
// narrower than the wave), so the LCP array is read once for nine levels.
// Higher levels are built three (or fewer) at a time from level k-1: entries
// 2^(k-1) apart form columns, each wave loads a window of rows of 512
// neighbouring columns at once and takes the minima down the columns in
// registers, so level k-1 is read about twice per three levels and every
// level is written once. With 288 GB of HBM the table fits next to
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

__device__ __forceinline__ uint64_t level_offset_dev(uint64_t n, int level);

constexpr int kStFusedTop = 9;              // levels 1..9 are built from registers (halo < 512 entries)
constexpr int kStOut = 16;                  // outputs per lane in fused levels (a wave: 64 kStOut entries)
constexpr int kStIn = kStOut + (1 << (kStFusedTop - 6));   // entries loaded per lane: the outputs plus the halo
constexpr uint32_t kStWave = kWave * kStOut;
constexpr uint32_t kRmqBlock = 64;          // LCP entries per block of the compact table

// Levels 1 .. nl (nl <= kStFusedTop) from level 0 (`prev`, prev_count
// entries), one wave per segment of kStWave outputs, with no LDS and no
// barriers. Lane l holds entries i0 + 64 m + l (m < kStIn) of the current
// level in v[m], so the partner of an entry at distance half lies in
// register m + half / 64 of the same lane when half >= 64, and otherwise in
// lane (l + half) mod 64 of register m or m + 1 (a wave shuffle). Each level
// is computed in place in ascending m, which leaves the higher registers,
// still needed, untouched. The 2^kStFusedTop entries loaded past the
// outputs cover the widest window; reads past prev_count load INT_MAX, which
// no minimum keeps. Measured at 1G (16-bit levels): 16 outputs per lane and
// levels 1-9, 5.6 ms; levels 1-10 here 7.6 ms (8 outputs per lane: 7.2 ms,
// 24 or 32: 22-24 ms, fewer waves in flight); levels 1-10 from LDS tiles
// with two barriers per level 9.5 ms.
__global__ __launch_bounds__(kBlock) void k_st_fused(const int32_t *__restrict__ prev, uint32_t prev_count,
                                                     uint32_t n, int nl, int32_t *__restrict__ table,
                                                     const uint32_t *__restrict__ hdr) {
    const bool narrow = hdr != nullptr && hdr[0] <= 65535u;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t w0 = ((uint64_t)blockIdx.x * (kBlock / kWave) + (threadIdx.x >> 6)) * kStWave;
    if (w0 >= n) return;
    const uint64_t i0 = w0 + lane;
    // entries left from this lane's first one: loads and stores test m * 64 against them
    const int64_t have = (int64_t)prev_count - (int64_t)i0;
    const int32_t *src = prev + i0;
    int32_t v[kStIn];
#pragma unroll
    for (int m = 0; m < kStIn; ++m) v[m] = m * (int64_t)kWave < have ? src[m * kWave] : INT_MAX;
#pragma unroll
    for (int k = 1; k <= kStFusedTop; ++k) {
        if (k > nl) break;
        const uint32_t half = 1u << (k - 1);
        if (half >= kWave) {
            const int off = (int)(half / kWave);
#pragma unroll
            for (int m = 0; m < kStIn; ++m)
                if (m + off < kStIn) v[m] = min(v[m], v[m + off]);
        } else {
            const int from = (int)((lane + half) & 63u);
            const bool wrap = lane + half >= kWave;   // the partner is in register m + 1
            int32_t cur = __shfl(v[0], from, kWave);
#pragma unroll
            for (int m = 0; m < kStIn; ++m) {
                const int32_t next = m + 1 < kStIn ? __shfl(v[m + 1], from, kWave) : INT_MAX;
                v[m] = min(v[m], wrap ? next : cur);
                cur = next;
            }
        }
        const int64_t left = (int64_t)n - (int64_t)(1u << k) + 1 - (int64_t)i0;   // outputs of level k from i0 on
        const uint64_t at = level_offset_dev(n, k) + i0;
        if (narrow) {
            uint16_t *dst = reinterpret_cast<uint16_t *>(table) + at;
#pragma unroll
            for (int m = 0; m < kStOut; ++m)
                if (m * (int64_t)kWave < left) dst[m * kWave] = (uint16_t)v[m];
        } else {
            int32_t *dst = table + at;
#pragma unroll
            for (int m = 0; m < kStOut; ++m)
                if (m * (int64_t)kWave < left) dst[m * kWave] = v[m];
        }
    }
}

// Levels k .. k+NL-1 (k > kStFusedTop, so h = 2^(k-1) is a multiple of
// 64 C) from level k-1 (P). Output entry i of level k+a is the minimum of
// P[i + u h] over u < 2^(a+1): entries h apart form a column, and a level
// is a sliding minimum down the columns. A wave takes C groups of 64
// neighbouring columns and S rows: lane l loads P[i0 + 64 c + l + m h] for
// c < C, m < S + 2^NL - 1 into v[c][m], all loads issued at once, then each
// level is computed in place (v[c][m] = min(v[c][m], v[c][m + 2^a]),
// ascending m) and its S rows are stored, each row of a wave a contiguous
// run of 64 C entries. Waves of one row block take neighbouring column
// groups, so their loads and stores meet the same rows together. Rows past
// the level's end load INT_MAX and store nothing. Measured at 1G (levels
// 10-29, 16-bit): 8 groups and 8 rows 14.4 ms; 4 groups and 16 rows 15.0,
// 2 and 16 15.6, 8 and 4 16.6, one group and 8-32 rows 18.8-19.5 ms; four
// levels per pass 21.3 ms; a walk down a column of blocks, one block load
// per step and then its stores, with a single-level pass for level 10,
// 16.4 ms.
template <int NL, int S, int C>
__global__ __launch_bounds__(kBlock) void k_st_cols(int32_t *__restrict__ table, const uint32_t *__restrict__ hdr,
                                                    uint32_t n, int k, uint32_t qcols, uint32_t rblocks) {
    constexpr int M = S + (1 << NL) - 1;
    const bool narrow = hdr != nullptr && hdr[0] <= 65535u;
    const uint64_t wave = (uint64_t)blockIdx.x * (kBlock / kWave) + (threadIdx.x >> 6);
    const uint64_t q = wave % qcols, r = wave / qcols;
    if (r >= rblocks) return;
    const uint64_t h = 1ull << (k - 1);
    const uint64_t i0 = r * (uint64_t)S * h + q * (uint64_t)(kWave * C) + (threadIdx.x & 63u);
    const int64_t have = (int64_t)n - (int64_t)h + 1 - (int64_t)i0;   // entries of level k-1 from i0 on
    const uint64_t p_off = level_offset_dev(n, k - 1) + i0;
    int32_t v[C][M];
    if (narrow) {
        const uint16_t *src = reinterpret_cast<const uint16_t *>(table) + p_off;
#pragma unroll
        for (int m = 0; m < M; ++m)
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int64_t e = (int64_t)(m * h) + c * kWave;
                v[c][m] = e < have ? (int32_t)src[e] : INT_MAX;
            }
    } else {
        const int32_t *src = table + p_off;
#pragma unroll
        for (int m = 0; m < M; ++m)
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int64_t e = (int64_t)(m * h) + c * kWave;
                v[c][m] = e < have ? src[e] : INT_MAX;
            }
    }
#pragma unroll
    for (int a = 0; a < NL; ++a) {
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int m = 0; m + (1 << a) < M; ++m) v[c][m] = min(v[c][m], v[c][m + (1 << a)]);
        const int lv = k + a;
        const int64_t left = (int64_t)n - (int64_t)(1ull << lv) + 1 - (int64_t)i0;   // outputs of level lv from i0 on
        const uint64_t at = level_offset_dev(n, lv) + i0;
        if (narrow) {
            uint16_t *dst = reinterpret_cast<uint16_t *>(table) + at;
#pragma unroll
            for (int m = 0; m < S; ++m)
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const int64_t e = (int64_t)(m * h) + c * kWave;
                    if (e < left) dst[e] = (uint16_t)v[c][m];
                }
        } else {
            int32_t *dst = table + at;
#pragma unroll
            for (int m = 0; m < S; ++m)
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const int64_t e = (int64_t)(m * h) + c * kWave;
                    if (e < left) dst[e] = v[c][m];
                }
        }
    }
}

constexpr int kColLevels = 3;   // levels per column pass
constexpr int kColRows = 8;     // rows per wave in a column pass
constexpr int kColGroups = 8;   // groups of 64 neighbouring columns per wave
static_assert((1 << kStFusedTop) >= kWave * kColGroups, "a column pass needs h >= 64 kColGroups");

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
    if (levels >= 1) {
        // levels 1 .. min(levels, kStFusedTop) in one pass from level 0
        const int nl = min(levels, kStFusedTop);
        double bytes = 4.0 * n;
        for (int l = 1; l <= nl; ++l) bytes += (double)eb * (n - (1u << l) + 1u);
        const uint32_t waves = div_up(n, kStWave);
        LOR_LAUNCH("k_st_fused", bytes, s,
                   hipLaunchKernelGGL(k_st_fused, dim3(div_up(waves, kBlock / kWave)), dim3(kBlock), 0, s, lcp, n,
                                      n, nl, table, hdr));
        k = nl + 1;
    }
    while (k <= levels) {
        // levels k .. k+nl-1 from level k-1, down columns h = 2^(k-1) apart
        const int nl = min(kColLevels, levels - k + 1);
        const uint64_t h = 1ull << (k - 1);
        const uint32_t qcols = (uint32_t)(h / (kWave * kColGroups));
        const uint64_t rows = div_up((uint64_t)n - 2 * h + 1, h);   // rows holding level-k outputs
        const uint32_t rblocks = (uint32_t)div_up(rows, (uint64_t)kColRows);
        const uint64_t waves = (uint64_t)qcols * rblocks;
        const dim3 grid((uint32_t)div_up(waves, (uint64_t)(kBlock / kWave)));
        double bytes = (double)eb * (n - h + 1);
        for (int a = 0; a < nl; ++a) bytes += (double)eb * (n - (1u << (k + a)) + 1u);
#define LOR_COLS(NL)                                                                                     \
    LOR_LAUNCH("k_st_cols", bytes, s,                                                                    \
               hipLaunchKernelGGL((k_st_cols<NL, kColRows, kColGroups>), grid, dim3(kBlock), 0, s, table, hdr, n, \
                                  k, qcols, rblocks))
        static_assert(kColLevels == 3, "one launch form per level count up to kColLevels");
        if (nl == 3) LOR_COLS(3);
        else if (nl == 2) LOR_COLS(2);
        else LOR_COLS(1);
#undef LOR_COLS
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
