// Longest overlap region on gfx950 (Section III problem statement: the
// longest common prefix of suffixes of different sequences, with its
// positions).
//
// Pass 1 (max): L = largest LCP[r] over ranks whose two suffixes start in
//   different sequences; coalesced per-rank loads, a workgroup reduction and
//   one atomicMax per workgroup (max is order-independent, so deterministic).
// Pass 2 (positions): the suffixes sharing one L-symbol prefix form a maximal
//   run of ranks whose LCP is >= L. The reported pair is the lexicographically
//   smallest (p, q), p < q, from different sequences inside one run; in a run
//   p is its smallest position and q the smallest position of another
//   sequence. Runs are summarised by (m1, s1, m2, s2): the smallest position
//   and its sequence, and the smallest position whose sequence differs from
//   s1. Merging two summaries keeps this exact, so chunks of ranks are
//   summarised independently (head = part of a run begun earlier, tail =
//   last open run, best = best pair of the runs closed inside) and combined
//   in rank order by an associative rule: a workgroup tree per tile, tiles
//   in order inside a workgroup, then one workgroup over the workgroup
//   results. A tile where no LCP reaches L holds only one-suffix runs; its
//   summary needs the last suffix alone, so such tiles read only LCP.
#include <climits>

#include "lor_internal.hpp"

namespace lor {

namespace {

constexpr uint32_t kChunk = 16;                       // ranks per thread in a tile
constexpr uint32_t kTileRanks = kChunk * kBlock;      // 4096 ranks per tile
constexpr uint32_t kTilesPerGroup = 16;
constexpr uint32_t kGroupRanks = kTileRanks * kTilesPerGroup;

struct RunSum {
    int32_t m1, s1, m2, s2;
};
struct ChunkSum {
    RunSum head, tail;
    int32_t has_b, bp, bq, pad;
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

__device__ __forceinline__ void best_update(int32_t &bp, int32_t &bq, int32_t p, int32_t q) {
    if (p < bp || (p == bp && q < bq)) { bp = p; bq = q; }
}

__device__ __forceinline__ void finalize(const RunSum &r, int32_t &bp, int32_t &bq) {
    if (r.m1 != INT_MAX && r.m2 != INT_MAX) best_update(bp, bq, r.m1, r.m2);
}

__device__ __forceinline__ ChunkSum chunk_empty() {
    ChunkSum c;
    c.head = run_empty();
    c.tail = run_empty();
    c.has_b = 0;
    c.bp = INT_MAX;
    c.bq = INT_MAX;
    c.pad = 0;
    return c;
}

// x precedes y in rank order.
__device__ __forceinline__ ChunkSum chunk_combine(const ChunkSum &x, const ChunkSum &y) {
    ChunkSum r;
    r.pad = 0;
    if (!x.has_b) {
        r.head = run_merge(x.head, y.head);
        r.has_b = y.has_b;
        r.tail = y.tail;
        r.bp = y.bp;
        r.bq = y.bq;
    } else {
        r.head = x.head;
        r.has_b = 1;
        r.bp = x.bp;
        r.bq = x.bq;
        if (y.has_b) {
            finalize(run_merge(x.tail, y.head), r.bp, r.bq);
            best_update(r.bp, r.bq, y.bp, y.bq);
            r.tail = y.tail;
        } else {
            r.tail = run_merge(x.tail, y.head);
        }
    }
    return r;
}

__device__ __forceinline__ int32_t seq_of(const int32_t *s_start, int k, int32_t p) {
    int lo = 0, hi = k - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_start[mid] <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void k_init(uint32_t *w, int count) {
    if (threadIdx.x < (unsigned)count) w[threadIdx.x] = 0;
}

// Largest LCP[r] whose two suffixes start in different sequences. A
// workgroup takes kCrossItems * 256 consecutive ranks; each thread loads its
// LCP entries for all its items first. SA entries are loaded only for ranks
// whose LCP exceeds both the maximum already published by earlier
// workgroups (a lower bound of the result) and the thread's own best, so
// after the first workgroups almost every rank costs its 4-byte LCP alone.
constexpr int kCrossItems = 16;

__global__ __launch_bounds__(kBlock) void k_cross_max(const int32_t *__restrict__ sa, const int32_t *__restrict__ lcp,
                                                      uint32_t n, SeqStarts st, uint32_t *__restrict__ out_max) {
    __shared__ int32_t s_start[kMaxSeqs + 1];
    __shared__ int32_t s_red[kBlock / kWave];
    for (int i = threadIdx.x; i <= st.k; i += kBlock) s_start[i] = st.start[i];
    const int32_t known = (int32_t)__hip_atomic_load(out_max, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const uint32_t r0 = blockIdx.x * (kBlock * kCrossItems) + threadIdx.x + 1;
    int32_t v[kCrossItems];
#pragma unroll
    for (int j = 0; j < kCrossItems; ++j) {
        const uint32_t r = r0 + j * kBlock;
        v[j] = r < n ? lcp[r] : 0;
    }
    int32_t best = 0;
#pragma unroll
    for (int j = 0; j < kCrossItems; ++j) {
        const uint32_t r = r0 + j * kBlock;
        if (v[j] > known && v[j] > best &&
            seq_of(s_start, st.k, sa[r - 1]) != seq_of(s_start, st.k, sa[r]))   // v[j] > 0 implies r < n
            best = v[j];
    }
    for (int o = 32; o > 0; o >>= 1) best = max(best, __shfl_xor(best, o, 64));
    if ((threadIdx.x & 63u) == 0) s_red[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t m = s_red[0];
        for (int i = 1; i < kBlock / kWave; ++i) m = max(m, s_red[i]);
        if (m > known) atomicMax(out_max, (uint32_t)m);
    }
}

__device__ void block_reduce_chunks(ChunkSum *s, ChunkSum mine) {
    s[threadIdx.x] = mine;
    __syncthreads();
    for (unsigned stride = 1; stride < kBlock; stride <<= 1) {
        if ((threadIdx.x & (2 * stride - 1)) == 0) s[threadIdx.x] = chunk_combine(s[threadIdx.x], s[threadIdx.x + stride]);
        __syncthreads();
    }
}

// One workgroup per group of kTilesPerGroup tiles. First every tile is
// checked for an LCP >= L with all its loads in flight at once; tiles
// without one (nearly all) hold only one-suffix runs and are summarised by
// one thread each from their last suffix, the others go through the
// per-rank path. The tile summaries are then combined in rank order.
__global__ __launch_bounds__(kBlock) void k_runs(const int32_t *__restrict__ sa, const int32_t *__restrict__ lcp,
                                                 uint32_t n, SeqStarts st, const uint32_t *__restrict__ Lp,
                                                 ChunkSum *__restrict__ out) {
    __shared__ int32_t s_start[kMaxSeqs + 1];
    __shared__ ChunkSum s_sum[kBlock];
    __shared__ ChunkSum s_tile[kTilesPerGroup];
    __shared__ uint32_t s_any[kTilesPerGroup];
    for (int i = threadIdx.x; i <= st.k; i += kBlock) s_start[i] = st.start[i];
    if (threadIdx.x < kTilesPerGroup) s_any[threadIdx.x] = 0;
    __syncthreads();
    const int32_t L = (int32_t)*Lp;
    const uint32_t tiles = (n + kTileRanks - 1) / kTileRanks;
    const uint32_t t0 = blockIdx.x * kTilesPerGroup, t1 = min(tiles, t0 + kTilesPerGroup);
    for (uint32_t t = t0; t < t1; ++t) {
        const uint32_t base = t * kTileRanks;
        const uint32_t cnt = min(kTileRanks, n - base);
        int any = 0;
#pragma unroll
        for (uint32_t i = 0; i < kChunk; ++i) {
            const uint32_t j = i * kBlock + threadIdx.x;
            any |= j < cnt && (base + j != 0) && lcp[base + j] >= L;
        }
        if (__any(any) && (threadIdx.x & 63u) == 0) s_any[t - t0] = 1;   // LDS store; any wave may set it
    }
    __syncthreads();
    if (threadIdx.x < t1 - t0 && !s_any[threadIdx.x]) {
        // every rank starts a run; only the last run can continue
        const uint32_t base = (t0 + threadIdx.x) * kTileRanks;
        const uint32_t cnt = min(kTileRanks, n - base);
        const int32_t p = sa[base + cnt - 1];
        ChunkSum c = chunk_empty();
        c.has_b = 1;
        c.tail = RunSum{p, seq_of(s_start, st.k, p), INT_MAX, -1};
        s_tile[threadIdx.x] = c;
    }
    for (uint32_t t = t0; t < t1; ++t) {
        if (!s_any[t - t0]) continue;   // uniform: s_any is final after the barrier above
        // rare (tiles inside a longest run): each thread reads its ranks directly
        const uint32_t base = t * kTileRanks;
        const uint32_t cnt = min(kTileRanks, n - base);
        ChunkSum c = chunk_empty();
        const uint32_t j0 = threadIdx.x * kChunk;
        for (uint32_t j = j0; j < min(cnt, j0 + kChunk); ++j) {
            const int32_t p = sa[base + j];
            const RunSum e{p, seq_of(s_start, st.k, p), INT_MAX, -1};
            if (base + j == 0 || lcp[base + j] < L) {    // starts a run
                if (c.has_b) finalize(c.tail, c.bp, c.bq);
                c.has_b = 1;
                c.tail = e;
            } else if (c.has_b) {
                c.tail = run_merge(c.tail, e);
            } else {
                c.head = run_merge(c.head, e);
            }
        }
        block_reduce_chunks(s_sum, c);
        if (threadIdx.x == 0) s_tile[t - t0] = s_sum[0];
        __syncthreads();
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        ChunkSum total = chunk_empty();
        for (uint32_t t = t0; t < t1; ++t) total = chunk_combine(total, s_tile[t - t0]);
        out[blockIdx.x] = total;
    }
}

__global__ __launch_bounds__(kBlock) void k_runs_final(const ChunkSum *__restrict__ in, uint32_t count,
                                                       uint32_t *__restrict__ result) {
    __shared__ ChunkSum s_sum[kBlock];
    const uint32_t per = (count + kBlock - 1) / kBlock;
    const uint32_t b = min(count, threadIdx.x * per), e = min(count, b + per);
    ChunkSum c = chunk_empty();
    for (uint32_t i = b; i < e; ++i) c = chunk_combine(c, in[i]);
    block_reduce_chunks(s_sum, c);
    if (threadIdx.x == 0) {
        ChunkSum g = s_sum[0];
        int32_t bp = g.bp, bq = g.bq;
        if (g.has_b) finalize(g.tail, bp, bq);
        result[0] = (uint32_t)bp;
        result[1] = (uint32_t)bq;
    }
}

}  // namespace

size_t overlap_workspace(uint64_t n) {
    return ((n + kGroupRanks - 1) / kGroupRanks + 1) * sizeof(ChunkSum) + 1024;
}

lor_status overlap_scan(const int32_t *sa, const int32_t *lcp, uint32_t n, const SeqStarts &st, Arena &ar,
                        hipStream_t s, int64_t result[5]) {
    uint32_t *words;
    LOR_TAKE(ar, uint32_t, 64, words);
    const uint32_t groups = div_up(n, kGroupRanks);
    ChunkSum *sums;
    LOR_TAKE(ar, ChunkSum, (size_t)groups + 1, sums);
    for (int x = 0; x < 5; ++x) result[x] = -1;
    result[0] = 0;
    if (n < 2) return LOR_OK;
    LOR_LAUNCH("k_init", 0, s, hipLaunchKernelGGL(k_init, dim3(1), dim3(kBlock), 0, s, words, 4));
    LOR_LAUNCH("k_cross_max", (double)n * 4, s,   // LCP; SA only for the few ranks above the running maximum
               hipLaunchKernelGGL(k_cross_max, dim3(div_up(n - 1, kBlock * kCrossItems)), dim3(kBlock), 0, s, sa, lcp,
                                  n, st, words));
    uint32_t L = 0;
    LOR_HIP(hipMemcpyAsync(&L, words, 4, hipMemcpyDeviceToHost, s));
    LOR_HIP(hipStreamSynchronize(s));
    if (L == 0) return LOR_OK;
    LOR_LAUNCH("k_runs", (double)n * 4, s,
               hipLaunchKernelGGL(k_runs, dim3(groups), dim3(kBlock), 0, s, sa, lcp, n, st, words, sums));
    LOR_LAUNCH("k_runs_final", (double)groups * sizeof(ChunkSum), s,
               hipLaunchKernelGGL(k_runs_final, dim3(1), dim3(kBlock), 0, s, sums, groups, words + 1));
    uint32_t pq[2];
    LOR_HIP(hipMemcpyAsync(pq, words + 1, 8, hipMemcpyDeviceToHost, s));
    LOR_HIP(hipStreamSynchronize(s));
    const int32_t p = (int32_t)pq[0], q = (int32_t)pq[1];
    if (p == INT_MAX || q == INT_MAX || p < 0 || q < 0) {
        set_error("internal: no position pair for overlap length %u", L);
        return LOR_EINVAL;
    }
    auto locate = [&](int32_t pos, int64_t *seq, int64_t *off) {
        int j = 0;
        while (j + 1 < st.k && st.start[j + 1] <= pos) ++j;
        *seq = j;
        *off = pos - st.start[j];
    };
    result[0] = L;
    locate(p, &result[1], &result[2]);
    locate(q, &result[3], &result[4]);
    return LOR_OK;
}

}  // namespace lor
