// Longest common substring of every query sequence with one reference, on
// gfx950: the shape of Section V's experiments (a reference group against
// many query sequences), with one suffix array for the whole set.
//
// Text: reference, then every query, each followed by the same separator
// (symbol 5 after the byte + 1 shift). Repeated separators leave the suffix
// order well defined, but an LCP may run across one; a query suffix x is
// therefore credited min(lcp, d(x)), d(x) = its distance to its separator.
// (If lcp(x, y) > d(y) for a reference suffix y, x reads a separator at
// d(y) too, so d(x) = d(y); hence min(lcp, d(x), d(y)) = min(lcp, d(x)).)
//
// For a query suffix x at rank r, the longest match with any reference
// suffix is the larger of its LCP with the nearest reference suffix above
// and below in rank order (the minimum of the LCP array between them). Two
// segmented scans over the ranks give both: forward, the minimum LCP since
// the last reference rank; backward, up to the next one. A query's answer
// is the largest credited match, the smallest query offset among equals
// (one 64-bit atomicMax per rank), and a reference offset at which that
// match occurs (the neighbour that gave it).
#include <climits>
#include <vector>

#include "lor_internal.hpp"

namespace lor {

namespace {

constexpr uint32_t kRqItems = 16;                      // consecutive ranks per thread
constexpr uint32_t kRqTile = kBlock * kRqItems;
constexpr int kRqScanThreads = 1024;                   // one workgroup scans the tile states

// Largest j in [0, count) with start[j] <= x.
__device__ __forceinline__ uint32_t seq_at(const int32_t *__restrict__ start, uint32_t count, uint32_t x) {
    uint32_t lo = 0, hi = count - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if ((uint32_t)start[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Sequence lookups go through buckets of 2^kRqBucketShift positions:
// tab[b] = the sequence holding position min(b << shift, N - 1), b = 0..nb
// with nb = ceil(N / 2^shift). Sequences only grow with the position, so the
// one holding x lies in [tab[x >> shift], tab[(x >> shift) + 1]]: a search
// of a few starts (queries are at least tens of bases) instead of all of
// them.
constexpr uint32_t kRqBucketShift = 6;

__global__ __launch_bounds__(kBlock) void k_rq_buckets(const int32_t *__restrict__ start, uint32_t S, uint32_t N,
                                                       uint32_t nb, int32_t *__restrict__ tab) {
    for (uint32_t b = blockIdx.x * kBlock + threadIdx.x; b <= nb; b += gridDim.x * kBlock)
        tab[b] = (int32_t)seq_at(start, S, min((uint64_t)b << kRqBucketShift, (uint64_t)N - 1));
}

// Largest j with start[j] <= x, for x < N.
__device__ __forceinline__ uint32_t seq_fast(const int32_t *__restrict__ start, const int32_t *__restrict__ tab,
                                             uint32_t x) {
    const uint32_t b = x >> kRqBucketShift;
    uint32_t lo = (uint32_t)tab[b], hi = (uint32_t)tab[b + 1];
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if ((uint32_t)start[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// start[j] = joined start of sequence j (0 = reference), start[S] = N. A
// thread writes kRqJoinBytes consecutive positions; when they are all bases
// of one sequence they are the input shifted by the sequence index (aligned
// 8-byte loads, a funnel shift, the base check on whole words), otherwise
// they go position by position.
constexpr uint32_t kRqJoinBytes = 16;

__global__ __launch_bounds__(kBlock) void k_rq_join(const uint8_t *__restrict__ seqs, const int32_t *__restrict__ start,
                                                    const int32_t *__restrict__ tab, uint32_t N, uint32_t total,
                                                    uint8_t *__restrict__ out, uint32_t *__restrict__ err) {
    uint32_t bad = 0;
    const uint32_t stride = gridDim.x * kBlock * kRqJoinBytes;
    for (uint32_t p0 = (blockIdx.x * kBlock + threadIdx.x) * kRqJoinBytes; p0 < N; p0 += stride) {
        uint32_t j = seq_fast(start, tab, p0);
        const uint32_t from = p0 - j;
        if (p0 + kRqJoinBytes < (uint32_t)start[j + 1] && from >= 8u && from + 24u <= total) {
            const uintptr_t addr = reinterpret_cast<uintptr_t>(seqs + from);
            const uint64_t *w = reinterpret_cast<const uint64_t *>(addr & ~(uintptr_t)7);
            const uint32_t sh = (uint32_t)(addr & 7u) * 8u;
            const uint64_t w0 = w[0], w1 = w[1], w2 = w[2];
            const uint64_t lo = sh ? (w0 >> sh) | (w1 << (64u - sh)) : w0;
            const uint64_t hi = sh ? (w1 >> sh) | (w2 << (64u - sh)) : w1;
            bad |= ((lo | hi) & 0xfcfcfcfcfcfcfcfcull) != 0;
            *reinterpret_cast<uint4 *>(out + p0) =   // p0 is a multiple of 16; the text buffer is 16-byte aligned
                make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
            continue;
        }
        for (uint32_t u = 0; u < kRqJoinBytes && p0 + u < N; ++u) {
            const uint32_t p = p0 + u;
            while ((uint32_t)start[j + 1] <= p) ++j;
            uint32_t c;
            if (p + 1 == (uint32_t)start[j + 1]) {
                c = 4u;
            } else {
                c = seqs[p - j];
                bad |= c > 3u;
            }
            out[p] = (uint8_t)c;
        }
    }
    if (__any(bad) && dev::lane_id() == 0) atomicOr(err, 1u);
}

// Forward state over a run of ranks: whether it holds a reference rank, the
// minimum LCP after the last one (over the whole run if none), that rank.
struct Fwd {
    int32_t h, m, last;
};
// Backward state: whether the run holds a reference rank, the minimum LCP up
// to and including the first one (over the whole run if none), that rank.
struct Bwd {
    int32_t h, m, first;
};

__device__ __forceinline__ Fwd f_id() { return Fwd{0, INT_MAX, -1}; }
__device__ __forceinline__ Bwd b_id() { return Bwd{0, INT_MAX, -1}; }
// a precedes b
__device__ __forceinline__ Fwd f_comb(const Fwd &a, const Fwd &b) { return b.h ? b : Fwd{a.h, min(a.m, b.m), a.last}; }
// near precedes far
__device__ __forceinline__ Bwd b_comb(const Bwd &nr, const Bwd &fr) {
    return nr.h ? nr : Bwd{fr.h, min(nr.m, fr.m), fr.first};
}

struct RankItem {
    int32_t sa, lcp;
    bool ref;
};

// Target sequence: joined positions [tlo, thi) (its separator at thi).
struct Target {
    uint32_t lo, hi, seq;
};

__device__ __forceinline__ RankItem rank_item(const int32_t *__restrict__ sa, const int32_t *__restrict__ lcp,
                                              uint32_t n, const Target &tg, uint32_t r) {
    RankItem it{-1, 0, false};
    if (r < n) {
        it.sa = sa[r];
        it.lcp = lcp[r];
        it.ref = (uint32_t)it.sa >= tg.lo && (uint32_t)it.sa < tg.hi;
    }
    return it;
}

__device__ __forceinline__ Fwd f_elem(const RankItem &it, uint32_t r) {
    return it.ref ? Fwd{1, INT_MAX, (int32_t)r} : Fwd{0, it.lcp, -1};
}
__device__ __forceinline__ Bwd b_elem(const RankItem &it, uint32_t r) {
    return it.ref ? Bwd{1, it.lcp, (int32_t)r} : Bwd{0, it.lcp, -1};
}

// Exclusive scans of per-thread states across a workgroup of NT threads
// (Hillis-Steele in LDS): forward in thread order, backward from the last
// thread down.
template <int NT>
__device__ Fwd block_fwd_excl(Fwd v, Fwd *s) {
    const unsigned t = threadIdx.x;
    s[t] = v;
    __syncthreads();
    for (unsigned off = 1; off < NT; off <<= 1) {
        const Fwd x = t >= off ? s[t - off] : f_id();
        __syncthreads();
        s[t] = f_comb(x, s[t]);
        __syncthreads();
    }
    const Fwd r = t ? s[t - 1] : f_id();
    __syncthreads();
    return r;
}

template <int NT>
__device__ Bwd block_bwd_excl(Bwd v, Bwd *s) {
    const unsigned u = NT - 1 - threadIdx.x;
    s[u] = v;
    __syncthreads();
    for (unsigned off = 1; off < NT; off <<= 1) {
        const Bwd x = u >= off ? s[u - off] : b_id();
        __syncthreads();
        s[u] = b_comb(s[u], x);
        __syncthreads();
    }
    const Bwd r = u ? s[u - 1] : b_id();
    __syncthreads();
    return r;
}

// Forward and backward states of every tile of kRqTile ranks.
__global__ __launch_bounds__(kBlock) void k_rq_tiles(const int32_t *__restrict__ sa, const int32_t *__restrict__ lcp,
                                                     uint32_t n, Target tg, Fwd *__restrict__ tf,
                                                     Bwd *__restrict__ tb) {
    __shared__ Fwd s_f[kBlock];
    __shared__ Bwd s_b[kBlock];
    const uint32_t c0 = blockIdx.x * kRqTile + threadIdx.x * kRqItems;
    Fwd f = f_id();
    Bwd b = b_id();
#pragma unroll
    for (uint32_t k = 0; k < kRqItems; ++k) {
        const RankItem it = rank_item(sa, lcp, n, tg, c0 + k);
        if (c0 + k < n) f = f_comb(f, f_elem(it, c0 + k));
    }
    for (int k = (int)kRqItems - 1; k >= 0; --k) {
        const RankItem it = rank_item(sa, lcp, n, tg, c0 + k);
        if (c0 + k < n) b = b_comb(b_elem(it, c0 + k), b);
    }
    const Fwd fe = block_fwd_excl<kBlock>(f, s_f);
    const Bwd be = block_bwd_excl<kBlock>(b, s_b);
    if (threadIdx.x == kBlock - 1) tf[blockIdx.x] = f_comb(fe, f);
    if (threadIdx.x == 0) tb[blockIdx.x] = b_comb(b, be);
}

// Tile states -> the state of everything before (forward) and after
// (backward) every tile. One workgroup; thread i folds a contiguous run.
__global__ __launch_bounds__(kRqScanThreads) void k_rq_tile_scan(Fwd *__restrict__ tf, Bwd *__restrict__ tb,
                                                                 uint32_t tiles) {
    __shared__ Fwd s_f[kRqScanThreads];
    __shared__ Bwd s_b[kRqScanThreads];
    const uint32_t per = (tiles + kRqScanThreads - 1) / kRqScanThreads;
    const uint32_t t0 = min(tiles, threadIdx.x * per), t1 = min(tiles, t0 + per);
    Fwd f = f_id();
    Bwd b = b_id();
    for (uint32_t t = t0; t < t1; ++t) f = f_comb(f, tf[t]);
    for (uint32_t t = t1; t > t0; --t) b = b_comb(tb[t - 1], b);
    Fwd run = block_fwd_excl<kRqScanThreads>(f, s_f);
    Bwd back = block_bwd_excl<kRqScanThreads>(b, s_b);
    for (uint32_t t = t0; t < t1; ++t) {
        const Fwd x = tf[t];
        tf[t] = run;
        run = f_comb(run, x);
    }
    for (uint32_t t = t1; t > t0; --t) {
        const Bwd x = tb[t - 1];
        tb[t - 1] = back;
        back = b_comb(x, back);
    }
}

// Per rank: the credited match of every suffix of another sequence j with
// the target. emit == 0: fold it into best[j * stride + base] =
// max(m << 32 | ~offset). emit == 1: the rank that holds its slot's best
// writes the record.
__global__ __launch_bounds__(kBlock) void k_rq_ranks(const int32_t *__restrict__ sa, const int32_t *__restrict__ lcp,
                                                     uint32_t n, Target tg, const int32_t *__restrict__ start,
                                                     const int32_t *__restrict__ tab, uint32_t S,
                                                     const Fwd *__restrict__ pre,
                                                     const Bwd *__restrict__ post, int emit, uint32_t stride,
                                                     int32_t base, unsigned long long *__restrict__ best,
                                                     lor_overlap *__restrict__ out) {
    __shared__ Fwd s_f[kBlock];
    __shared__ Bwd s_b[kBlock];
    const uint32_t c0 = blockIdx.x * kRqTile + threadIdx.x * kRqItems;
    RankItem it[kRqItems];
#pragma unroll
    for (uint32_t k = 0; k < kRqItems; ++k) it[k] = rank_item(sa, lcp, n, tg, c0 + k);
    Fwd f = f_id();
    Bwd b = b_id();
#pragma unroll
    for (uint32_t k = 0; k < kRqItems; ++k)
        if (c0 + k < n) f = f_comb(f, f_elem(it[k], c0 + k));
    for (int k = (int)kRqItems - 1; k >= 0; --k)
        if (c0 + k < n) b = b_comb(b_elem(it[k], c0 + k), b);
    Fwd fs = f_comb(pre[blockIdx.x], block_fwd_excl<kBlock>(f, s_f));
    Bwd bs = b_comb(block_bwd_excl<kBlock>(b, s_b), post[blockIdx.x]);
    int32_t up[kRqItems], up_at[kRqItems];
#pragma unroll
    for (uint32_t k = 0; k < kRqItems; ++k) {
        if (c0 + k < n) fs = f_comb(fs, f_elem(it[k], c0 + k));
        up[k] = fs.h ? fs.m : 0;
        up_at[k] = fs.last;
    }
    for (int k = (int)kRqItems - 1; k >= 0; --k) {
        const uint32_t r = c0 + (uint32_t)k;
        if (r >= n) continue;
        const int32_t down = bs.h ? bs.m : 0;
        const int32_t down_at = bs.first;
        bs = b_comb(b_elem(it[k], r), bs);
        const uint32_t x = (uint32_t)it[k].sa;
        if (x >= tg.lo && x <= tg.hi) continue;   // target suffix or its separator
        const int32_t mx = max(up[k], down);
        if (mx <= 0) continue;
        const uint32_t j = seq_fast(start, tab, x);
        if (j >= S || j == tg.seq) continue;
        const uint32_t d = (uint32_t)start[j + 1] - 1u - x;   // distance to its own separator
        const int32_t m = min(mx, (int32_t)d);
        if (m <= 0) continue;
        const uint32_t off = x - (uint32_t)start[j];
        const unsigned long long key = ((unsigned long long)(uint32_t)m << 32) | (0xffffffffu - off);
        const int64_t slot = (int64_t)j * stride + base;
        if (!emit) {
            // best only grows: a stale read can only let a redundant atomic through
            if (key > __hip_atomic_load(&best[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                atomicMax(&best[slot], key);
        } else if (best[slot] == key) {
            const int32_t at = up[k] >= down ? up_at[k] : down_at;   // the neighbour that gave m
            lor_overlap rec;
            rec.length = m;
            rec.seq_p = (int32_t)j;
            rec.off_p = off;
            rec.seq_q = (int32_t)tg.seq;
            rec.off_q = (at >= 0 && (uint32_t)at < n) ? sa[at] - (int32_t)tg.lo : -1;
            out[slot] = rec;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_rq_init(uint32_t Q, unsigned long long *__restrict__ best,
                                                    lor_overlap *__restrict__ out) {
    for (uint32_t q = blockIdx.x * kBlock + threadIdx.x; q < Q; q += gridDim.x * kBlock) {
        best[q] = 0ull;
        lor_overlap rec;
        rec.length = 0;
        rec.seq_p = -1;
        rec.seq_q = -1;
        rec.off_p = -1;
        rec.off_q = -1;
        out[q] = rec;
    }
}

struct RqLayout {
    uint8_t *text;
    int32_t *sa, *lcp, *start, *tab;
    unsigned long long *best;
    Fwd *tf;
    Bwd *tb;
};

lor_status rq_carve(Arena &ar, uint64_t N, uint32_t S, RqLayout *L) {
    const uint32_t tiles = div_up(N ? N : 1, kRqTile);
    LOR_TAKE(ar, uint8_t, N + 16, L->text);
    LOR_TAKE(ar, int32_t, N, L->sa);
    LOR_TAKE(ar, int32_t, N, L->lcp);
    LOR_TAKE(ar, int32_t, (size_t)S + 1, L->start);
    LOR_TAKE(ar, int32_t, (size_t)div_up(N ? N : 1, 1u << kRqBucketShift) + 1, L->tab);
    LOR_TAKE(ar, unsigned long long, S, L->best);
    LOR_TAKE(ar, Fwd, tiles, L->tf);
    LOR_TAKE(ar, Bwd, tiles, L->tb);
    return LOR_OK;
}

// Matches of every other sequence's suffixes with one target sequence:
// tile states, their scan, then the two per-rank passes.
lor_status target_scan(const int32_t *sa, const int32_t *lcp, uint32_t n, Target tg, const int32_t *start,
                       const int32_t *tab, uint32_t S, uint32_t stride, int32_t base, Fwd *tf, Bwd *tb,
                       unsigned long long *best, lor_overlap *out, hipStream_t s) {
    const uint32_t tiles = div_up(n, kRqTile);
    LOR_LAUNCH("k_rq_tiles", 8.0 * n, s,
               hipLaunchKernelGGL(k_rq_tiles, dim3(tiles), dim3(kBlock), 0, s, sa, lcp, n, tg, tf, tb));
    LOR_LAUNCH("k_rq_tile_scan", 48.0 * tiles, s,
               hipLaunchKernelGGL(k_rq_tile_scan, dim3(1), dim3(kRqScanThreads), 0, s, tf, tb, tiles));
    for (int emit = 0; emit < 2; ++emit)
        LOR_LAUNCH("k_rq_ranks", 8.0 * n, s,
                   hipLaunchKernelGGL(k_rq_ranks, dim3(tiles), dim3(kBlock), 0, s, sa, lcp, n, tg, start, tab, S, tf,
                                      tb, emit, stride, base, best, out));
    return LOR_OK;
}

}  // namespace

size_t refq_workspace(uint64_t total_bases, uint32_t num_queries) {
    const uint32_t S = num_queries + 1;
    const uint64_t N = total_bases + S;
    Arena ar;   // measuring
    ar.top = kHeaderBytes;
    RqLayout L;
    if (rq_carve(ar, N, S, &L) != LOR_OK) return 0;
    size_t phase = dc3_workspace_bound(N);
    phase = phase > lcp_workspace(N) + 4096 ? phase : lcp_workspace(N) + 4096;
    return ar.top + phase + 4096;
}

lor_status refq_overlap(const uint8_t *seqs, const int64_t *offsets, uint32_t Q, lor_overlap *out, void *ws,
                        size_t ws_bytes, hipStream_t s) {
    const uint32_t S = Q + 1;
    std::vector<int32_t> h_start(S + 1);
    uint64_t N = 0;
    for (uint32_t j = 0; j < S; ++j) {
        h_start[j] = (int32_t)N;
        N += (uint64_t)(offsets[j + 1] - offsets[j]) + 1;
    }
    h_start[S] = (int32_t)N;
    const uint32_t ref_len = (uint32_t)(offsets[1] - offsets[0]);

    Arena ar;
    ar.base = static_cast<char *>(ws);
    ar.cap = ws_bytes;
    ar.top = kHeaderBytes;
    uint32_t *hdr = static_cast<uint32_t *>(ws);
    RqLayout L;
    LOR_TRY(rq_carve(ar, N, S, &L));
    const size_t phase = ar.mark();

    LOR_HIP(hipMemcpyAsync(L.start, h_start.data(), (S + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    LOR_TRY(zero_words(hdr, 16, s));
    LOR_LAUNCH("k_rq_init", 40.0 * Q, s,
               hipLaunchKernelGGL(k_rq_init, dim3(grid_for(Q)), dim3(kBlock), 0, s, Q, L.best, out));
    const uint32_t nb = div_up(N, 1u << kRqBucketShift);
    LOR_LAUNCH("k_rq_buckets", 4.0 * (nb + 1), s,
               hipLaunchKernelGGL(k_rq_buckets, dim3(grid_for(nb + 1)), dim3(kBlock), 0, s, L.start, S, (uint32_t)N,
                                  nb, L.tab));
    LOR_LAUNCH("k_rq_join", 2.0 * N, s,
               hipLaunchKernelGGL(k_rq_join, dim3(grid_for(div_up(N, kRqJoinBytes))), dim3(kBlock), 0, s, seqs,
                                  L.start, L.tab, (uint32_t)N, (uint32_t)(N - S), L.text, hdr));
    // symbols byte + 1: bases 1..4, separator 5
    LOR_TRY(dc3_u8(L.text, (uint32_t)N, 5u, L.sa, ar, hdr, s));
    ar.release(phase);
    LOR_TRY(lcp_build(L.text, (uint32_t)N, L.sa, L.lcp, nullptr, ar, s));
    ar.release(phase);
    LOR_TRY(target_scan(L.sa, L.lcp, (uint32_t)N, Target{0u, ref_len, 0u}, L.start, L.tab, S, 1u, -1, L.tf, L.tb,
                        L.best, out, s));
    LOR_HIP(hipStreamSynchronize(s));   // the host table must outlive its copy
    return LOR_OK;
}

}  // namespace lor
