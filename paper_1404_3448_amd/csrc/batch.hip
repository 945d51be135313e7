// Batched longest overlap for many independent sequence pairs on gfx950.
//
// All pairs go through one DC3 run. Pair p is written as the tagged text
//   8p+c(A_p) ... 8p+5  8p+c(B_p) ... 8p+6      (c(base) = base + 1)
// with 16-bit symbols. The pair tag is the most significant part of every
// symbol and each pair ends with its own unique separator, so comparing two
// suffixes of one pair never reads past that separator, and suffixes of
// different pairs are ordered by pair. The suffix array of the tagged text
// is therefore the concatenation of every pair's own suffix array, and pair
// p's suffixes hold exactly the ranks [start_p, start_p + |pair p|) -- the
// same range as its positions. LCP over 16-bit symbols is 0 between pairs.
// The overlap scan then runs per pair inside its rank range: one pass for
// every pair's largest cross-sequence LCP (atomicMax per pair), one pass over
// the runs of suffixes sharing that many symbols, where every closed run
// offers (smallest position, smallest position of the other sequence) to its
// pair with an atomicMin on the packed pair of positions -- a minimum does not
// depend on the order of arrival, so the result is deterministic.
#include <algorithm>
#include <climits>
#include <vector>

#include "lor_internal.hpp"

namespace lor {

namespace {

constexpr uint32_t kChunk = 16;                        // ranks per thread in a tile
constexpr uint32_t kTileRanks = kChunk * kBlock;
constexpr uint32_t kTilesPerGroup = 16;
constexpr uint32_t kGroupRanks = kTileRanks * kTilesPerGroup;

// Largest j with start[j] <= x over j in [0, count).
__device__ __forceinline__ uint32_t find_pair(const int32_t *__restrict__ start, uint32_t count, uint32_t x) {
    uint32_t lo = 0, hi = count - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if ((uint32_t)start[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Ranks (and positions) of one workgroup span few pairs. Pairs [lo, lo + k)
// cover the workgroup's range [r0, r1]; with k <= kPairWin their starts (and
// the start after the last) and |A| are kept in LDS, and each thread, whose
// ranks only increase, finds its pair by advancing a cursor there. Larger k
// (very short pairs) falls back to a binary search over all pairs.
constexpr uint32_t kPairWin = 1024;

struct PairWin {
    uint32_t lo, k;
    bool lds;
};

__device__ PairWin pair_window(const int32_t *__restrict__ start, const int32_t *__restrict__ alen, uint32_t P,
                               uint32_t r0, uint32_t r1, int32_t *s_start, int32_t *s_alen, uint32_t *s_sh) {
    if (threadIdx.x == 0) s_sh[0] = find_pair(start, P, r0);
    if (threadIdx.x == 1) s_sh[1] = find_pair(start, P, r1);
    __syncthreads();
    PairWin w;
    w.lo = s_sh[0];
    w.k = s_sh[1] - s_sh[0] + 1;
    w.lds = w.k <= kPairWin;
    if (w.lds) {
        for (uint32_t j = threadIdx.x; j <= w.k; j += kBlock) s_start[j] = start[w.lo + j];   // start[P] = N exists
        for (uint32_t j = threadIdx.x; j < w.k; j += kBlock) s_alen[j] = alen[w.lo + j];
    }
    __syncthreads();
    return w;
}

// Pair of x relative to w.lo; x must not decrease between the calls of one
// thread that share `cur` (which starts at 0).
__device__ __forceinline__ uint32_t pair_at(const PairWin &w, const int32_t *s_start, const int32_t *__restrict__ start,
                                            uint32_t P, uint32_t x, uint32_t &cur) {
    if (w.lds) {
        while (cur + 1 < w.k && (uint32_t)s_start[cur + 1] <= x) ++cur;
        return cur;
    }
    return find_pair(start, P, x) - w.lo;
}

// start[p] = joined start of pair p (start[P] = N); alen[p] = |A_p|;
// src[2p], src[2p+1] = offsets of A_p and B_p in the separator-free input.
constexpr uint32_t kJoinTile = kBlock * 16;   // positions per workgroup

// A thread writes groups of kJoinGroup consecutive positions (groups of
// neighbouring threads are neighbours). A group inside one sequence of a pair
// is its bases shifted: aligned 8-byte loads and a funnel shift, the base
// check on the whole word, one 16-byte store of codes 8p + 1 + base. Other
// groups (a separator, a pair boundary, either end of the input) go position
// by position.
constexpr uint32_t kJoinGroup = 8;

__global__ __launch_bounds__(kBlock) void k_join_pairs(const uint8_t *__restrict__ seqs,
                                                       const int32_t *__restrict__ start,
                                                       const int32_t *__restrict__ alen,
                                                       const int64_t *__restrict__ src, uint32_t P, uint32_t N,
                                                       uint64_t total, uint16_t *__restrict__ out,
                                                       uint32_t *__restrict__ err) {
    __shared__ int32_t s_start[kPairWin + 1];
    __shared__ int32_t s_alen[kPairWin];
    __shared__ uint32_t s_sh[2];
    const uint32_t base = blockIdx.x * kJoinTile;
    if (base >= N) return;
    const uint32_t cnt = min(kJoinTile, N - base);
    const PairWin w = pair_window(start, alen, P, base, base + cnt - 1, s_start, s_alen, s_sh);
    uint32_t bad = 0, cur = 0;
    for (uint32_t g0 = threadIdx.x * kJoinGroup; g0 < cnt; g0 += kBlock * kJoinGroup) {
        const uint32_t i0 = base + g0;
        const uint32_t q0 = pair_at(w, s_start, start, P, i0, cur), p0 = w.lo + q0;
        const uint32_t s0 = w.lds ? (uint32_t)s_start[q0] : (uint32_t)start[p0];
        const uint32_t s1 = w.lds ? (uint32_t)s_start[q0 + 1] : (uint32_t)start[p0 + 1];
        const uint32_t a0 = w.lds ? (uint32_t)s_alen[q0] : (uint32_t)alen[p0];
        const uint32_t o0 = i0 - s0;
        int64_t from = -1;   // input offset of the group's first base, when the group is all bases of one sequence
        if (o0 + kJoinGroup <= a0) from = src[2 * p0] + o0;
        else if (o0 > a0 && o0 + kJoinGroup < s1 - s0) from = src[2 * p0 + 1] + (o0 - a0 - 1);
        if (g0 + kJoinGroup <= cnt && from >= 8 && (uint64_t)from + 16 <= total) {
            const uintptr_t addr = reinterpret_cast<uintptr_t>(seqs + from);
            const uint64_t *wd = reinterpret_cast<const uint64_t *>(addr & ~(uintptr_t)7);
            const uint32_t sh = (uint32_t)(addr & 7u) * 8u;
            const uint64_t v = sh ? (wd[0] >> sh) | (wd[1] << (64u - sh)) : wd[0];
            bad |= (v & 0xfcfcfcfcfcfcfcfcull) != 0;
            const uint32_t tag = 8u * p0 + 1u;
            uint32_t o[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t lo = tag + (uint32_t)((v >> (16 * e)) & 0xffu);
                const uint32_t hi = tag + (uint32_t)((v >> (16 * e + 8)) & 0xffu);
                o[e] = lo | (hi << 16);
            }
            *reinterpret_cast<uint4 *>(out + i0) = make_uint4(o[0], o[1], o[2], o[3]);   // i0 is a multiple of 8
            continue;
        }
        for (uint32_t e = 0; e < kJoinGroup && g0 + e < cnt; ++e) {
            const uint32_t i = i0 + e;
            const uint32_t q = pair_at(w, s_start, start, P, i, cur), p = w.lo + q;
            const uint32_t ps = w.lds ? (uint32_t)s_start[q] : (uint32_t)start[p];
            const uint32_t pe = w.lds ? (uint32_t)s_start[q + 1] : (uint32_t)start[p + 1];
            const uint32_t a = w.lds ? (uint32_t)s_alen[q] : (uint32_t)alen[p];
            const uint32_t o = i - ps, plen = pe - ps;
            uint32_t code;
            if (o < a) {
                code = seqs[src[2 * p] + o];
                bad |= code > 3u;
                code += 1u;
            } else if (o == a) {
                code = 5u;
            } else if (o + 1 < plen) {
                code = seqs[src[2 * p + 1] + (o - a - 1)];
                bad |= code > 3u;
                code += 1u;
            } else {
                code = 6u;
            }
            out[i] = (uint16_t)(8u * p + code);
        }
    }
    if (__any(bad) && dev::lane_id() == 0) atomicOr(err, 1u);
}

__global__ __launch_bounds__(kBlock) void k_pair_init(uint32_t P, uint32_t *__restrict__ lmax,
                                                      unsigned long long *__restrict__ best) {
    for (uint32_t p = blockIdx.x * kBlock + threadIdx.x; p < P; p += gridDim.x * kBlock) {
        lmax[p] = 0;
        best[p] = ~0ull;
    }
}

// Is joined position x (inside pair p) in the pair's second sequence?
__device__ __forceinline__ bool in_b(const int32_t *start, const int32_t *alen, uint32_t p, uint32_t x) {
    return x > (uint32_t)start[p] + (uint32_t)alen[p];
}

// Per pair, the largest LCP between suffixes of its two sequences. A
// workgroup takes one tile of ranks; SA is read only for ranks whose LCP
// exceeds the maximum its pair already has (published by earlier
// workgroups, a lower bound of the result), and maxima meet in LDS before
// one atomicMax per pair and workgroup.
__global__ __launch_bounds__(kBlock) void k_seg_max(const int32_t *__restrict__ sa, const int32_t *__restrict__ lcp,
                                                    uint32_t n, const int32_t *__restrict__ start,
                                                    const int32_t *__restrict__ alen, uint32_t P,
                                                    uint32_t *__restrict__ lmax) {
    __shared__ int32_t s_start[kPairWin + 1];
    __shared__ int32_t s_alen[kPairWin];
    __shared__ uint32_t s_known[kPairWin];
    __shared__ uint32_t s_best[kPairWin];
    __shared__ uint32_t s_sh[2];
    const uint32_t base = blockIdx.x * kTileRanks;
    if (base >= n) return;
    const uint32_t cnt = min(kTileRanks, n - base);
    const PairWin w = pair_window(start, alen, P, base, base + cnt - 1, s_start, s_alen, s_sh);
    if (w.lds) {
        for (uint32_t j = threadIdx.x; j < w.k; j += kBlock) {
            s_known[j] = __hip_atomic_load(&lmax[w.lo + j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_best[j] = 0;
        }
        __syncthreads();
    }
    int32_t v[kChunk];
#pragma unroll
    for (uint32_t i = 0; i < kChunk; ++i) {
        const uint32_t j = i * kBlock + threadIdx.x;
        v[i] = j < cnt ? lcp[base + j] : 0;
    }
    uint32_t cur = 0;
#pragma unroll
    for (uint32_t i = 0; i < kChunk; ++i) {
        const uint32_t j = i * kBlock + threadIdx.x;
        if (j >= cnt || v[i] <= 0) continue;
        const uint32_t r = base + j;
        const uint32_t q = pair_at(w, s_start, start, P, r, cur), p = w.lo + q;
        const uint32_t s0 = w.lds ? (uint32_t)s_start[q] : (uint32_t)start[p];
        if (r <= s0 || (w.lds && (uint32_t)v[i] <= s_known[q])) continue;
        const uint32_t bstart = s0 + (w.lds ? (uint32_t)s_alen[q] : (uint32_t)alen[p]);   // B starts after it
        if (((uint32_t)sa[r - 1] > bstart) == ((uint32_t)sa[r] > bstart)) continue;
        if (w.lds) atomicMax(&s_best[q], (uint32_t)v[i]);
        else atomicMax(&lmax[p], (uint32_t)v[i]);
    }
    if (w.lds) {
        __syncthreads();
        for (uint32_t j = threadIdx.x; j < w.k; j += kBlock)
            if (s_best[j] > s_known[j]) atomicMax(&lmax[w.lo + j], s_best[j]);
    }
}

struct RunSum {
    int32_t m1, s1, m2, s2;
};
struct ChunkSum {
    RunSum head, tail;
    int32_t has_b, pad0, pad1, pad2;
};

__device__ __forceinline__ RunSum run_empty() { return RunSum{INT_MAX, -1, INT_MAX, -1}; }

__device__ __forceinline__ RunSum run_merge(const RunSum &x, const RunSum &y) {
    const bool xf = x.m1 <= y.m1;
    const RunSum &f = xf ? x : y;
    const RunSum &o = xf ? y : x;
    RunSum r{f.m1, f.s1, f.m2, f.s2};
    if (o.m1 != INT_MAX && o.s1 != f.s1 && o.m1 < r.m2) { r.m2 = o.m1; r.s2 = o.s1; }
    if (o.m2 != INT_MAX && o.s2 != f.s1 && o.m2 < r.m2) { r.m2 = o.m2; r.s2 = o.s2; }
    return r;
}

// A closed run offers its pair of positions to the run's pair.
__device__ __forceinline__ void finalize(const RunSum &r, const int32_t *start, uint32_t P,
                                         unsigned long long *best) {
    if (r.m1 == INT_MAX || r.m2 == INT_MAX) return;
    const uint32_t p = find_pair(start, P, (uint32_t)r.m1);
    atomicMin(&best[p], ((unsigned long long)(uint32_t)r.m1 << 32) | (uint32_t)r.m2);
}

__device__ __forceinline__ ChunkSum chunk_empty() {
    ChunkSum c;
    c.head = run_empty();
    c.tail = run_empty();
    c.has_b = 0;
    c.pad0 = c.pad1 = c.pad2 = 0;
    return c;
}

__device__ __forceinline__ ChunkSum chunk_combine(const ChunkSum &x, const ChunkSum &y, const int32_t *start,
                                                  uint32_t P, unsigned long long *best) {
    ChunkSum r = chunk_empty();
    if (!x.has_b) {
        r.head = run_merge(x.head, y.head);
        r.has_b = y.has_b;
        r.tail = y.tail;
    } else {
        r.head = x.head;
        r.has_b = 1;
        if (y.has_b) {
            finalize(run_merge(x.tail, y.head), start, P, best);
            r.tail = y.tail;
        } else {
            r.tail = run_merge(x.tail, y.head);
        }
    }
    return r;
}

__device__ void reduce_chunks(ChunkSum *s, ChunkSum mine, const int32_t *start, uint32_t P,
                              unsigned long long *best) {
    s[threadIdx.x] = mine;
    __syncthreads();
    for (unsigned stride = 1; stride < kBlock; stride <<= 1) {
        if ((threadIdx.x & (2 * stride - 1)) == 0)
            s[threadIdx.x] = chunk_combine(s[threadIdx.x], s[threadIdx.x + stride], start, P, best);
        __syncthreads();
    }
}

// One workgroup per group of kTilesPerGroup tiles. Rank r starts a run
// unless it shares at least its pair's L symbols with r - 1. Every tile is
// first checked for a rank that continues a run, with all its loads in
// flight at once; tiles without one (nearly all) hold only one-suffix runs
// and are summarised by one thread each from their last suffix, the others
// go through the per-rank path. Tile summaries are combined in rank order.
__global__ __launch_bounds__(kBlock) void k_seg_runs(const int32_t *__restrict__ sa, const int32_t *__restrict__ lcp,
                                                     uint32_t n, const int32_t *__restrict__ start,
                                                     const int32_t *__restrict__ alen, uint32_t P,
                                                     const uint32_t *__restrict__ lmax,
                                                     unsigned long long *__restrict__ best,
                                                     ChunkSum *__restrict__ out) {
    __shared__ ChunkSum s_sum[kBlock];
    __shared__ ChunkSum s_tile[kTilesPerGroup];
    __shared__ uint32_t s_any[kTilesPerGroup];
    __shared__ int32_t s_start[kPairWin + 1];
    __shared__ int32_t s_alen[kPairWin];
    __shared__ uint32_t s_L[kPairWin];
    __shared__ uint32_t s_sh[2];
    const uint32_t tiles = (n + kTileRanks - 1) / kTileRanks;
    const uint32_t t0 = blockIdx.x * kTilesPerGroup, t1 = min(tiles, t0 + kTilesPerGroup);
    if (t0 >= t1) return;
    const uint32_t g0 = t0 * kTileRanks, g1 = min(n, t1 * kTileRanks);
    if (threadIdx.x < kTilesPerGroup) s_any[threadIdx.x] = 0;
    const PairWin w = pair_window(start, alen, P, g0, g1 - 1, s_start, s_alen, s_sh);
    if (w.lds) {
        for (uint32_t j = threadIdx.x; j < w.k; j += kBlock) s_L[j] = lmax[w.lo + j];
        __syncthreads();
    }
    auto pstart = [&](uint32_t q) { return w.lds ? (uint32_t)s_start[q] : (uint32_t)start[w.lo + q]; };
    auto pL = [&](uint32_t q) { return w.lds ? s_L[q] : lmax[w.lo + q]; };
    auto pb = [&](uint32_t q) { return pstart(q) + (w.lds ? (uint32_t)s_alen[q] : (uint32_t)alen[w.lo + q]); };

    uint32_t cur = 0;
    for (uint32_t t = t0; t < t1; ++t) {
        const uint32_t base = t * kTileRanks;
        const uint32_t cnt = min(kTileRanks, n - base);
        int32_t v[kChunk];
#pragma unroll
        for (uint32_t i = 0; i < kChunk; ++i) {
            const uint32_t j = i * kBlock + threadIdx.x;
            v[i] = j < cnt ? lcp[base + j] : 0;
        }
        int any = 0;
#pragma unroll
        for (uint32_t i = 0; i < kChunk; ++i) {
            const uint32_t j = i * kBlock + threadIdx.x;
            if (j >= cnt || v[i] <= 0) continue;
            const uint32_t r = base + j;
            const uint32_t q = pair_at(w, s_start, start, P, r, cur);
            const uint32_t L = pL(q);
            any |= r != pstart(q) && L != 0 && (uint32_t)v[i] >= L;
        }
        if (__any(any) && (threadIdx.x & 63u) == 0) s_any[t - t0] = 1;   // LDS store; any wave may set it
    }
    __syncthreads();
    if (threadIdx.x < t1 - t0 && !s_any[threadIdx.x]) {
        // every rank starts a run; only the last run can continue
        const uint32_t base = (t0 + threadIdx.x) * kTileRanks;
        const uint32_t r = base + min(kTileRanks, n - base) - 1;
        const uint32_t p = find_pair(start, P, r);
        const int32_t x = sa[r];
        ChunkSum c = chunk_empty();
        c.has_b = 1;
        c.tail = RunSum{x, in_b(start, alen, p, (uint32_t)x) ? 1 : 0, INT_MAX, -1};
        s_tile[threadIdx.x] = c;
    }
    for (uint32_t t = t0; t < t1; ++t) {
        if (!s_any[t - t0]) continue;   // uniform: s_any is final after the barrier above
        // rare (tiles inside a run of its pair's length): each thread reads its ranks directly
        const uint32_t base = t * kTileRanks;
        const uint32_t cnt = min(kTileRanks, n - base);
        ChunkSum c = chunk_empty();
        const uint32_t j0 = threadIdx.x * kChunk;
        uint32_t c2 = 0;
        for (uint32_t j = j0; j < min(cnt, j0 + kChunk); ++j) {
            const uint32_t r = base + j;
            const int32_t x = sa[r];
            const uint32_t q = w.lds ? pair_at(w, s_start, start, P, r, c2) : find_pair(start, P, r) - w.lo;
            const uint32_t L = pL(q);
            const bool starts = r == pstart(q) || L == 0 || (uint32_t)lcp[r] < L;
            const RunSum e{x, (uint32_t)x > pb(q) ? 1 : 0, INT_MAX, -1};
            if (starts) {
                if (c.has_b) finalize(c.tail, start, P, best);
                c.has_b = 1;
                c.tail = e;
            } else if (c.has_b) {
                c.tail = run_merge(c.tail, e);
            } else {
                c.head = run_merge(c.head, e);
            }
        }
        reduce_chunks(s_sum, c, start, P, best);
        if (threadIdx.x == 0) s_tile[t - t0] = s_sum[0];
        __syncthreads();
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        ChunkSum total = chunk_empty();
        for (uint32_t t = t0; t < t1; ++t) total = chunk_combine(total, s_tile[t - t0], start, P, best);
        out[blockIdx.x] = total;
    }
}

__global__ __launch_bounds__(kBlock) void k_seg_runs_final(const ChunkSum *__restrict__ in, uint32_t count,
                                                           const int32_t *__restrict__ start, uint32_t P,
                                                           unsigned long long *__restrict__ best) {
    __shared__ ChunkSum s_sum[kBlock];
    const uint32_t per = (count + kBlock - 1) / kBlock;
    const uint32_t b = min(count, threadIdx.x * per), e = min(count, b + per);
    ChunkSum c = chunk_empty();
    for (uint32_t i = b; i < e; ++i) c = chunk_combine(c, in[i], start, P, best);
    reduce_chunks(s_sum, c, start, P, best);
    if (threadIdx.x == 0 && s_sum[0].has_b) finalize(s_sum[0].tail, start, P, best);
}

// One lor_overlap record per pair (offsets inside A_p / B_p).
__global__ __launch_bounds__(kBlock) void k_pair_records(const int32_t *__restrict__ start,
                                                         const int32_t *__restrict__ alen, uint32_t P,
                                                         const uint32_t *__restrict__ lmax,
                                                         const unsigned long long *__restrict__ best,
                                                         lor_overlap *__restrict__ out) {
    for (uint32_t p = blockIdx.x * kBlock + threadIdx.x; p < P; p += gridDim.x * kBlock) {
        lor_overlap o;
        o.length = 0;
        o.seq_p = o.seq_q = -1;
        o.off_p = o.off_q = -1;
        const unsigned long long bq = best[p];
        if (lmax[p] > 0 && bq != ~0ull) {
            const uint32_t x = (uint32_t)(bq >> 32), y = (uint32_t)bq;
            const uint32_t s0 = (uint32_t)start[p], a = (uint32_t)alen[p];
            o.length = lmax[p];
            o.seq_p = x > s0 + a ? 1 : 0;
            o.off_p = o.seq_p ? (int64_t)(x - s0 - a - 1) : (int64_t)(x - s0);
            o.seq_q = y > s0 + a ? 1 : 0;
            o.off_q = o.seq_q ? (int64_t)(y - s0 - a - 1) : (int64_t)(y - s0);
        }
        out[p] = o;
    }
}

struct BatchPlan {
    uint64_t N;
    uint32_t P;
};

}  // namespace

size_t batch_workspace(uint64_t total_bases, uint32_t P) {
    const uint64_t N = total_bases + 2ull * P;
    Arena ar;   // measuring
    ar.top = kHeaderBytes;
    ar.take<uint16_t>(N);                       // tagged text
    ar.take<int32_t>(N);                        // SA
    ar.take<int32_t>(N);                        // LCP
    ar.take<int32_t>((size_t)P + 1);            // start
    ar.take<int32_t>(P);                        // alen
    ar.take<int64_t>(2ull * P);                 // src offsets
    ar.take<uint32_t>(P);                       // lmax
    ar.take<unsigned long long>(P);             // best
    const size_t fixed = ar.top;
    const size_t scan = (N + kGroupRanks - 1) / kGroupRanks * sizeof(ChunkSum) + 4096;
    size_t phase = dc3_workspace_bound(N);
    phase = std::max(phase, lcp_workspace(N) + 4096);
    phase = std::max(phase, scan);
    return fixed + phase + 4096;
}

uint64_t batch_tables(const int64_t *offsets, uint32_t P, int32_t *h_start, int32_t *h_alen, int64_t *h_src) {
    uint64_t N = 0;
    for (uint32_t p = 0; p < P; ++p) {
        const int64_t a = offsets[2 * p + 1] - offsets[2 * p], b = offsets[2 * p + 2] - offsets[2 * p + 1];
        h_start[p] = (int32_t)N;
        h_alen[p] = (int32_t)a;
        h_src[2 * p] = offsets[2 * p];
        h_src[2 * p + 1] = offsets[2 * p + 1];
        N += (uint64_t)(a + b + 2);
    }
    h_start[P] = (int32_t)N;
    return N;
}

lor_status batch_overlap_run(const uint8_t *seqs, uint32_t P, uint64_t N, const int32_t *h_start,
                             const int32_t *h_alen, const int64_t *h_src, lor_overlap *out, void *ws,
                             size_t ws_bytes, hipStream_t s, int32_t *lcp_out, int32_t *isa_out) {
    Arena ar;
    ar.base = static_cast<char *>(ws);
    ar.cap = ws_bytes;
    ar.top = kHeaderBytes;
    uint32_t *hdr = static_cast<uint32_t *>(ws);
    uint16_t *text;
    int32_t *sa, *lcp, *start, *alen;
    int64_t *src;
    uint32_t *lmax;
    unsigned long long *best;
    LOR_TAKE(ar, uint16_t, N, text);
    LOR_TAKE(ar, int32_t, N, sa);
    LOR_TAKE(ar, int32_t, N, lcp);
    LOR_TAKE(ar, int32_t, (size_t)P + 1, start);
    LOR_TAKE(ar, int32_t, P, alen);
    LOR_TAKE(ar, int64_t, 2ull * P, src);
    LOR_TAKE(ar, uint32_t, P, lmax);
    LOR_TAKE(ar, unsigned long long, P, best);
    const size_t phase = ar.mark();

    LOR_HIP(hipMemcpyAsync(start, h_start, (P + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    LOR_HIP(hipMemcpyAsync(alen, h_alen, P * sizeof(int32_t), hipMemcpyHostToDevice, s));
    LOR_HIP(hipMemcpyAsync(src, h_src, 2ull * P * sizeof(int64_t), hipMemcpyHostToDevice, s));
    LOR_TRY(zero_words(hdr, 16, s));
    // end of the input bytes the pairs use: the last pair's B ends there
    const uint64_t in_end = P ? (uint64_t)h_src[2 * P - 1] +
                                    (uint64_t)(h_start[P] - h_start[P - 1] - h_alen[P - 1] - 2)
                              : 0;
    LOR_LAUNCH("k_join_pairs", 3.0 * N, s,
               hipLaunchKernelGGL(k_join_pairs, dim3(div_up(N, kJoinTile)), dim3(kBlock), 0, s, seqs, start, alen, src,
                                  P, (uint32_t)N, in_end, text, hdr));
    LOR_TRY(dc3_u16(text, (uint32_t)N, 8u * (P - 1) + 6u, sa, ar, hdr, s));
    ar.release(phase);
    if (lcp_out) lcp = lcp_out;   // the caller keeps the whole batch's LCP (and ISA)
    LOR_TRY(lcp_build_u16(text, (uint32_t)N, sa, lcp, isa_out, ar, s));
    ar.release(phase);

    const uint32_t groups = div_up(N, kGroupRanks);
    ChunkSum *sums;
    LOR_TAKE(ar, ChunkSum, (size_t)groups + 1, sums);
    LOR_LAUNCH("k_pair_init", 8.0 * P, s,
               hipLaunchKernelGGL(k_pair_init, dim3(grid_for(P)), dim3(kBlock), 0, s, P, lmax, best));
    LOR_LAUNCH("k_seg_max", 4.0 * N, s,   // LCP; SA only where an LCP can still raise its pair's maximum
               hipLaunchKernelGGL(k_seg_max, dim3(div_up(N, kTileRanks)), dim3(kBlock), 0, s, sa, lcp, (uint32_t)N,
                                  start, alen, P, lmax));
    LOR_LAUNCH("k_seg_runs", 4.0 * N, s,
               hipLaunchKernelGGL(k_seg_runs, dim3(groups), dim3(kBlock), 0, s, sa, lcp, (uint32_t)N, start, alen, P,
                                  lmax, best, sums));
    LOR_LAUNCH("k_seg_runs_final", (double)groups * sizeof(ChunkSum), s,
               hipLaunchKernelGGL(k_seg_runs_final, dim3(1), dim3(kBlock), 0, s, sums, groups, start, P, best));
    LOR_LAUNCH("k_pair_records", 32.0 * P, s,
               hipLaunchKernelGGL(k_pair_records, dim3(grid_for(P)), dim3(kBlock), 0, s, start, alen, P, lmax, best,
                                  out));
    return LOR_OK;
}

lor_status batch_overlap(const uint8_t *seqs, const int64_t *offsets, uint32_t P, lor_overlap *out, void *ws,
                         size_t ws_bytes, hipStream_t s, int32_t *lcp_out, int32_t *isa_out) {
    std::vector<int32_t> h_start(P + 1), h_alen(P);
    std::vector<int64_t> h_src(2 * (size_t)P);
    const uint64_t N = batch_tables(offsets, P, h_start.data(), h_alen.data(), h_src.data());
    // DC3 reads back one word per level, which also orders the host copies
    LOR_TRY(batch_overlap_run(seqs, P, N, h_start.data(), h_alen.data(), h_src.data(), out, ws, ws_bytes, s, lcp_out,
                              isa_out));
    LOR_HIP(hipStreamSynchronize(s));   // the host tables must outlive their copies
    return LOR_OK;
}

}  // namespace lor
