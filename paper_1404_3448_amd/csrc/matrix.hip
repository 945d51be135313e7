// All-pairs longest overlap over one joined text, from its SA and LCP, on
// gfx950 (the pairwise form of the overlap region of Section III, for every
// pair of the k sequences at once).
//
// Record (a, b) is the longest substring sequences a and b share. For a
// suffix x of a at rank r, its longest match with any suffix of b is the
// larger of its LCP with the nearest b-suffix above and below in rank order,
// i.e. the minimum of the LCP array between them. The credited length is
// capped by d(x), x's distance to its own separator: an LCP may run across
// the shared separator symbol (if lcp(x, y) > d(y) for a b-suffix y, x reads
// a separator at d(y) too, so d(x) = d(y)). Record (a, b) keeps the largest
// credited length, the smallest offset in a among equals, and the b-suffix
// that gave it (above wins a tie with below).
//
// Work layout. A workgroup owns a tile of kMxTile consecutive ranks; each
// lane keeps kMxItems consecutive ranks in registers (LCP, sequence, offset,
// distance to its separator), computed once per launch. Targets b are then
// walked one after another over those registers: a lane's fold, a 6-step
// wave scan, the four wave totals through LDS, and the carry of every rank
// before (after) the tile from a two-level scan of tile totals. Per target a
// lane touches no memory but LDS. Candidates are filtered against the
// workgroup's copy of the target's row of best keys in LDS, which meets the
// global table once per workgroup and target.
//
//   k_mx_tiles    forward/backward state of every tile, per target
//   k_mx_chunks   exclusive scan of tile states inside chunks of kMxChunk,
//                 then (a second launch) of the chunk totals
//   k_mx_ranks<0> best key of every (sequence, target) pair
//   k_mx_ranks<1> the rank holding each best key writes its record
#include <climits>
#include <vector>

#include "lor_internal.hpp"

namespace lor {

namespace {

constexpr uint32_t kMxItems = 16;                  // consecutive ranks per lane
constexpr uint32_t kMxTile = kBlock * kMxItems;    // ranks per workgroup
constexpr uint32_t kMxWaves = kBlock / kWave;
constexpr uint32_t kMxChunkThreads = kBlock;
constexpr uint32_t kMxChunkItems = 4;
constexpr uint32_t kMxChunk = kMxChunkThreads * kMxChunkItems;   // tiles per chunk (4M ranks)
constexpr uint32_t kMxChunkWaves = kMxChunkThreads / kWave;
constexpr int32_t kNoSeq = -1;                     // separator or past the end
constexpr uint32_t kMxBatch = 8;                   // candidate keys read from LDS together

// Forward state over a run of ranks for one target: the minimum LCP after
// the run's last target rank (over the whole run if it has none) and that
// rank (-1: none).
struct Up {
    int32_t m, last;
};
// Backward state: the minimum LCP up to and including the run's first
// target rank (over the whole run if none) and that rank (-1: none).
struct Dn {
    int32_t m, first;
};

__device__ __forceinline__ Up up_id() { return Up{INT_MAX, -1}; }
__device__ __forceinline__ Dn dn_id() { return Dn{INT_MAX, -1}; }
// a precedes b
__device__ __forceinline__ Up up_comb(const Up &a, const Up &b) {
    return b.last >= 0 ? b : Up{min(a.m, b.m), a.last};
}
// near precedes far
__device__ __forceinline__ Dn dn_comb(const Dn &nr, const Dn &fr) {
    return nr.first >= 0 ? nr : Dn{min(nr.m, fr.m), fr.first};
}

__device__ __forceinline__ Up shfl_up_state(const Up &v, unsigned d) {
    return Up{__shfl_up(v.m, d, kWave), __shfl_up(v.last, d, kWave)};
}
__device__ __forceinline__ Dn shfl_down_state(const Dn &v, unsigned d) {
    return Dn{__shfl_down(v.m, d, kWave), __shfl_down(v.first, d, kWave)};
}

// Inclusive scans across the 64 lanes of a wave: forward in lane order,
// backward from lane 63 down.
__device__ __forceinline__ Up wave_incl_up(Up v) {
    const unsigned lane = dev::lane_id();
#pragma unroll
    for (unsigned d = 1; d < kWave; d <<= 1) {
        const Up o = shfl_up_state(v, d);
        if (lane >= d) v = up_comb(o, v);
    }
    return v;
}
__device__ __forceinline__ Dn wave_incl_dn(Dn v) {
    const unsigned lane = dev::lane_id();
#pragma unroll
    for (unsigned d = 1; d < kWave; d <<= 1) {
        const Dn o = shfl_down_state(v, d);
        if (lane + d < kWave) v = dn_comb(v, o);
    }
    return v;
}
// Exclusive forms from the inclusive ones.
__device__ __forceinline__ Up wave_excl_up(const Up &incl) {
    const Up o = shfl_up_state(incl, 1);
    return dev::lane_id() ? o : up_id();
}
__device__ __forceinline__ Dn wave_excl_dn(const Dn &incl) {
    const Dn o = shfl_down_state(incl, 1);
    return dev::lane_id() + 1 < kWave ? o : dn_id();
}

// Largest j in [0, k) with start[j] <= x.
__device__ __forceinline__ int32_t seq_of(const int32_t *s_start, uint32_t k, uint32_t x) {
    uint32_t lo = 0, hi = k - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if ((uint32_t)s_start[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return (int32_t)lo;
}

// A lane's ranks, in the forms the per-target loop uses (so that nothing
// derived from them has to be kept beside them): LCP; 8 x the sequence, the
// byte offset of its slot in the LDS row of best keys (-8: a separator or a
// rank past n); ~offset in that sequence, the low word of a candidate key;
// distance to the sequence's separator.
struct Lane {
    int32_t lcp[kMxItems], seq8[kMxItems];
    uint32_t noff[kMxItems];
    int32_t dist[kMxItems];
};
constexpr int32_t kNoSeq8 = 8 * kNoSeq;

// vec: sa and lcp are 16-byte aligned, so a full lane reads them as int4.
__device__ __forceinline__ void load_lane(const int32_t *__restrict__ sa, const int32_t *__restrict__ lcp,
                                          uint32_t n, uint32_t r0, const int32_t *s_start, uint32_t k, bool vec,
                                          Lane &L) {
    int32_t x[kMxItems];
    if (vec && r0 + kMxItems <= n) {
        const int4 *ps = reinterpret_cast<const int4 *>(sa + r0);
        const int4 *pl = reinterpret_cast<const int4 *>(lcp + r0);
#pragma unroll
        for (uint32_t v = 0; v < kMxItems / 4; ++v) {
            const int4 a = ps[v], b = pl[v];
            x[4 * v] = a.x; x[4 * v + 1] = a.y; x[4 * v + 2] = a.z; x[4 * v + 3] = a.w;
            L.lcp[4 * v] = b.x; L.lcp[4 * v + 1] = b.y; L.lcp[4 * v + 2] = b.z; L.lcp[4 * v + 3] = b.w;
        }
    } else {
#pragma unroll
        for (uint32_t i = 0; i < kMxItems; ++i) {
            const bool in = r0 + i < n;
            x[i] = in ? sa[r0 + i] : -1;
            L.lcp[i] = in ? lcp[r0 + i] : INT_MAX;   // past n: the identity of both scans
        }
    }
#pragma unroll
    for (uint32_t i = 0; i < kMxItems; ++i) {
        L.seq8[i] = kNoSeq8;
        L.noff[i] = 0xffffffffu;
        L.dist[i] = 0;
        if (x[i] >= 0) {
            const int32_t j = seq_of(s_start, k, (uint32_t)x[i]);
            const int32_t sep = s_start[j + 1] - 1;
            if (x[i] != sep) {
                L.seq8[i] = 8 * j;
                L.noff[i] = 0xffffffffu - (uint32_t)(x[i] - s_start[j]);
                L.dist[i] = sep - x[i];
            }
        }
    }
}

// Bit i: rank i of the lane belongs to the target (t8 = 8 x its index).
__device__ __forceinline__ uint32_t member_mask(const Lane &L, int32_t t8) {
    uint32_t mask = 0;
#pragma unroll
    for (uint32_t i = 0; i < kMxItems; ++i) mask |= (uint32_t)(L.seq8[i] == t8) << i;
    return mask;
}

// Folds of a lane's ranks for one target (member mask `mem`): the minimum
// LCP after the last member (all of them if none) and that rank; the minimum
// up to and including the first member and that rank.
__device__ __forceinline__ Up lane_up(const Lane &L, uint32_t r0, uint32_t mem) {
    int32_t m = INT_MAX;
#pragma unroll
    for (uint32_t i = 0; i < kMxItems; ++i) m = (mem >> i) & 1u ? INT_MAX : min(m, L.lcp[i]);
    return Up{m, mem ? (int32_t)(r0 + 31u - __clz(mem)) : -1};
}
__device__ __forceinline__ Dn lane_dn(const Lane &L, uint32_t r0, uint32_t mem) {
    int32_t m = INT_MAX;
#pragma unroll
    for (int i = (int)kMxItems - 1; i >= 0; --i) m = (mem >> i) & 1u ? L.lcp[i] : min(m, L.lcp[i]);
    return Dn{m, mem ? (int32_t)(r0 + __ffs(mem) - 1u) : -1};
}

__device__ __forceinline__ void load_starts(const int32_t *__restrict__ start, uint32_t k, int32_t *s_start) {
    for (uint32_t j = threadIdx.x; j <= k; j += kBlock) s_start[j] = start[j];
    __syncthreads();
}

// State of every tile for every target: tu[t * tiles + tile], td[...].
__global__ __launch_bounds__(kBlock) void k_mx_tiles(const int32_t *__restrict__ sa, const int32_t *__restrict__ lcp,
                                                     uint32_t n, const int32_t *__restrict__ start, uint32_t k,
                                                     bool vec, uint32_t tiles, Up *__restrict__ tu,
                                                     Dn *__restrict__ td) {
    __shared__ int32_t s_start[kMaxSeqs + 1];
    __shared__ Up s_wu[2][kMxWaves];
    __shared__ Dn s_wd[2][kMxWaves];
    load_starts(start, k, s_start);
    const uint32_t tile = blockIdx.x, w = threadIdx.x / kWave, lane = dev::lane_id();
    const uint32_t r0 = tile * kMxTile + threadIdx.x * kMxItems;
    Lane L;
    load_lane(sa, lcp, n, r0, s_start, k, vec, L);
    for (uint32_t t = 0; t < k; ++t) {
        const uint32_t buf = t & 1u;   // a wave may write target t + 1 while thread 0 reads target t
        const uint32_t mem = member_mask(L, 8 * (int32_t)t);
        const Up fu = wave_incl_up(lane_up(L, r0, mem));
        const Dn fd = wave_incl_dn(lane_dn(L, r0, mem));
        if (lane == kWave - 1) s_wu[buf][w] = fu;
        if (lane == 0) s_wd[buf][w] = fd;
        __syncthreads();
        if (threadIdx.x == 0) {
            Up u = up_id();
            Dn d = dn_id();
            for (uint32_t v = 0; v < kMxWaves; ++v) u = up_comb(u, s_wu[buf][v]);
            for (int v = (int)kMxWaves - 1; v >= 0; --v) d = dn_comb(s_wd[buf][v], d);
            tu[(size_t)t * tiles + tile] = u;
            td[(size_t)t * tiles + tile] = d;
        }
    }
}

// Exclusive scans across a workgroup of kMxChunkThreads threads: wave scans,
// then the wave totals through LDS. Returns the exclusive state and the
// workgroup total.
__device__ __forceinline__ void chunk_scan(Up &u, Dn &d, Up *s_u, Dn *s_d, Up *tot_u, Dn *tot_d) {
    const uint32_t w = threadIdx.x / kWave, lane = dev::lane_id();
    const Up iu = wave_incl_up(u);
    const Dn id = wave_incl_dn(d);
    if (lane == kWave - 1) s_u[w] = iu;
    if (lane == 0) s_d[w] = id;
    __syncthreads();
    Up cu = up_id();
    for (uint32_t v = 0; v < w; ++v) cu = up_comb(cu, s_u[v]);
    Dn cd = dn_id();
    for (uint32_t v = kMxChunkWaves - 1; v > w; --v) cd = dn_comb(s_d[v], cd);
    Up all_u = up_id();
    Dn all_d = dn_id();
    for (uint32_t v = 0; v < kMxChunkWaves; ++v) all_u = up_comb(all_u, s_u[v]);
    for (int v = (int)kMxChunkWaves - 1; v >= 0; --v) all_d = dn_comb(s_d[v], all_d);
    u = up_comb(cu, wave_excl_up(iu));
    d = dn_comb(wave_excl_dn(id), cd);
    *tot_u = all_u;
    *tot_d = all_d;
}

// Tile states -> inside each chunk of kMxChunk tiles, the state of the
// chunk's tiles before (tu) and after (td) each tile; chunk totals to cu/cd.
// Grid: (chunks, k). Run again over the chunk totals (one chunk, at most
// kMxChunk of them), it turns those into the state before and after each
// chunk; its own totals then go to a scratch pair.
__global__ __launch_bounds__(kMxChunkThreads) void k_mx_chunks(Up *__restrict__ tu_all, Dn *__restrict__ td_all,
                                                               uint32_t tiles, uint32_t chunks,
                                                               Up *__restrict__ cu, Dn *__restrict__ cd) {
    __shared__ Up s_u[kMxChunkWaves];
    __shared__ Dn s_d[kMxChunkWaves];
    const uint32_t t = blockIdx.y, c = blockIdx.x;
    Up *tu = tu_all + (size_t)t * tiles;
    Dn *td = td_all + (size_t)t * tiles;
    const uint32_t b0 = c * kMxChunk + threadIdx.x * kMxChunkItems;
    Up u = up_id();
    Dn d = dn_id();
    for (uint32_t i = 0; i < kMxChunkItems; ++i)
        if (b0 + i < tiles) u = up_comb(u, tu[b0 + i]);
    for (int i = (int)kMxChunkItems - 1; i >= 0; --i)
        if (b0 + i < tiles) d = dn_comb(td[b0 + i], d);
    Up tot_u;
    Dn tot_d;
    chunk_scan(u, d, s_u, s_d, &tot_u, &tot_d);
    for (uint32_t i = 0; i < kMxChunkItems; ++i)
        if (b0 + i < tiles) {
            const Up x = tu[b0 + i];
            tu[b0 + i] = u;
            u = up_comb(u, x);
        }
    for (int i = (int)kMxChunkItems - 1; i >= 0; --i)
        if (b0 + i < tiles) {
            const Dn x = td[b0 + i];
            td[b0 + i] = d;
            d = dn_comb(x, d);
        }
    if (threadIdx.x == 0) {
        cu[(size_t)t * chunks + c] = tot_u;
        cd[(size_t)t * chunks + c] = tot_d;
    }
}

// EMIT 0: fold every credited match of a rank of sequence j != t with target
// t into best[j * k + t] = max(m << 32 | ~offset). EMIT 1: the rank holding
// its pair's best key writes the record.
// (at most 256 VGPRs: 2 waves per SIMD without spills)
template <int EMIT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_mx_ranks(
    const int32_t *__restrict__ sa, const int32_t *__restrict__ lcp, uint32_t n, const int32_t *__restrict__ start,
    uint32_t k, bool vec, uint32_t tiles, uint32_t chunks, const Up *__restrict__ tu, const Dn *__restrict__ td,
    const Up *__restrict__ cu, const Dn *__restrict__ cd, unsigned long long *__restrict__ best,
    lor_overlap *__restrict__ out) {
    __shared__ int32_t s_start[kMaxSeqs + 1];
    __shared__ unsigned long long s_best[kMaxSeqs];   // column t of best, this workgroup's copy
    __shared__ Up s_wu[kMxWaves];
    __shared__ Dn s_wd[kMxWaves];
    // EMIT 1: the ranks holding a best key queue {j, neighbour, m, offset};
    // the records are written after the target's walk. A key belongs to one
    // rank, so a target queues at most k entries. Indexed by target parity,
    // so a queue is cleared only when no thread can still be reading it.
    __shared__ int4 s_q[2][kMaxSeqs];
    __shared__ uint32_t s_nq[2];
    if (threadIdx.x < 2) s_nq[threadIdx.x] = 0;
    load_starts(start, k, s_start);
    const uint32_t tile = blockIdx.x, w = threadIdx.x / kWave, lane = dev::lane_id();
    const uint32_t r0 = tile * kMxTile + threadIdx.x * kMxItems;
    const uint32_t c = tile / kMxChunk;
    Lane L;
    load_lane(sa, lcp, n, r0, s_start, k, vec, L);
    for (uint32_t t = 0; t < k; ++t) {
        const int32_t ti = (int32_t)t;
        const uint32_t buf = t & 1u;
        // this target's queue was last read for target t - 2, by every thread
        // before the barrier that ended target t - 1; it is filled only after
        // the next barrier
        if (EMIT == 1 && threadIdx.x == 0 && t >= 2) s_nq[buf] = 0;
        // carries of everything before and after the tile (two-level scan)
        const Up carry_u = up_comb(cu[(size_t)t * chunks + c], tu[(size_t)t * tiles + tile]);
        const Dn carry_d = dn_comb(td[(size_t)t * tiles + tile], cd[(size_t)t * chunks + c]);
        for (uint32_t j = threadIdx.x; j < k; j += kBlock) s_best[j] = j == t ? 0ull : best[(size_t)j * k + t];
        const int32_t t8 = 8 * ti;
        const uint32_t members = member_mask(L, t8);
        const Up iu = wave_incl_up(lane_up(L, r0, members));
        const Dn id = wave_incl_dn(lane_dn(L, r0, members));
        if (lane == kWave - 1) s_wu[w] = iu;
        if (lane == 0) s_wd[w] = id;
        __syncthreads();
        Up fs = carry_u;
        for (uint32_t v = 0; v < w; ++v) fs = up_comb(fs, s_wu[v]);
        fs = up_comb(fs, wave_excl_up(iu));
        Dn bs = carry_d;
        for (uint32_t v = kMxWaves - 1; v > w; --v) bs = dn_comb(s_wd[v], bs);
        bs = dn_comb(wave_excl_dn(id), bs);
        // Walks. With no target rank yet seen the running minimum starts at 0
        // (the match is 0 then) and a member resets it, so the running value
        // is the match itself. Forward: the match above every rank.
        const int32_t in_last = fs.last, in_first = bs.first;
        int32_t fm = fs.last >= 0 ? fs.m : 0;
        int32_t up_m[kMxItems];
#pragma unroll
        for (uint32_t i = 0; i < kMxItems; ++i) {
            fm = (members >> i) & 1u ? INT_MAX : min(fm, L.lcp[i]);
            up_m[i] = fm;
        }
        // backward: the match below; the credited length replaces the match
        // above in up_m, and bit i of from_up says the rank above gave it (it
        // wins a tie)
        int32_t bm = bs.first >= 0 ? bs.m : 0;
        uint32_t from_up = 0;
#pragma unroll
        for (int i = (int)kMxItems - 1; i >= 0; --i) {
            const int32_t down = bm;
            bm = (members >> i) & 1u ? L.lcp[i] : min(bm, L.lcp[i]);
            const bool other = L.seq8[i] != kNoSeq8 && L.seq8[i] != t8;
            from_up |= (uint32_t)(up_m[i] >= down) << i;
            up_m[i] = other ? min(max(up_m[i], down), L.dist[i]) : 0;
        }
        // candidates, kMxBatch at a time: the best keys are read before any
        // compare, so their LDS latency overlaps; only the rare insert (or
        // queue) is a branch
        const char *s_row = reinterpret_cast<const char *>(s_best);
        uint32_t hit = 0;
#pragma unroll
        for (uint32_t c0 = 0; c0 < kMxItems; c0 += kMxBatch) {
            unsigned long long cur[kMxBatch];
#pragma unroll
            for (uint32_t u = 0; u < kMxBatch; ++u)
                cur[u] = *reinterpret_cast<const unsigned long long *>(s_row + (up_m[c0 + u] > 0 ? L.seq8[c0 + u] : 0));
#pragma unroll
            for (uint32_t u = 0; u < kMxBatch; ++u) {
                const uint32_t i = c0 + u;
                const int32_t m = up_m[i];
                const unsigned long long key = ((unsigned long long)(uint32_t)m << 32) | L.noff[i];
                if (EMIT == 0) {
                    if (m > 0 && key > cur[u])
                        atomicMax(reinterpret_cast<unsigned long long *>(reinterpret_cast<char *>(s_best) + L.seq8[i]),
                                  key);
                } else {
                    hit |= (uint32_t)(m > 0 && key == cur[u]) << i;
                }
            }
        }
        // EMIT 1: ranks holding their pair's best key (rare). The key gives
        // m and the offset, the rank's suffix its sequence; the neighbour is
        // the lane's last member at or before it (else the one carried in)
        // or its first member after it (else the one carried in).
        while (EMIT == 1 && hit) {
            const uint32_t i = __ffs(hit) - 1u;
            hit &= hit - 1u;
            const int32_t j = seq_of(s_start, k, (uint32_t)sa[r0 + i]);
            const unsigned long long key = s_best[j];
            const uint32_t upto = members & ((2u << i) - 1u), after = members & ~((2u << i) - 1u);
            const int32_t up_at = upto ? (int32_t)(r0 + 31u - __clz(upto)) : in_last;
            const int32_t down_at = after ? (int32_t)(r0 + __ffs(after) - 1u) : in_first;
            const int32_t at = (from_up >> i) & 1u ? up_at : down_at;   // the neighbour that gave m
            const uint32_t q = atomicAdd(&s_nq[buf], 1u);
            if (q < kMaxSeqs)
                s_q[buf][q] = make_int4(j, at, (int32_t)(key >> 32), (int32_t)(0xffffffffu - (uint32_t)key));
        }
        __syncthreads();
        if (EMIT == 1) {
            const uint32_t nq = min(s_nq[buf], (uint32_t)kMaxSeqs);
            for (uint32_t e = threadIdx.x; e < nq; e += kBlock) {
                const int4 q = s_q[buf][e];
                lor_overlap rec;
                rec.length = q.z;
                rec.seq_p = q.x;
                rec.off_p = q.w;
                rec.seq_q = ti;
                rec.off_q = (q.y >= 0 && (uint32_t)q.y < n) ? sa[q.y] - s_start[t] : -1;
                out[(size_t)q.x * k + t] = rec;
            }
        }
        if (EMIT == 0)
            // same thread-to-slot map as the copy-in above, so the next
            // target's copy-in needs no barrier of its own
            for (uint32_t j = threadIdx.x; j < k; j += kBlock) {
                const unsigned long long key = s_best[j];
                unsigned long long *g = &best[(size_t)j * k + t];
                if (j != t && key && key > __hip_atomic_load(g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                    atomicMax(g, key);
            }
    }
}

__global__ __launch_bounds__(kBlock) void k_mx_init(uint32_t count, unsigned long long *__restrict__ best,
                                                    lor_overlap *__restrict__ out) {
    for (uint32_t q = blockIdx.x * kBlock + threadIdx.x; q < count; q += gridDim.x * kBlock) {
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

struct MxLayout {
    int32_t *start;
    unsigned long long *best;
    Up *tu, *cu, *su;
    Dn *td, *cd, *sd;
};

lor_status mx_carve(Arena &ar, uint64_t n, uint32_t k, MxLayout *L) {
    const uint32_t tiles = div_up(n ? n : 1, kMxTile);
    const uint32_t chunks = div_up(tiles, kMxChunk);
    LOR_TAKE(ar, int32_t, (size_t)k + 1, L->start);
    LOR_TAKE(ar, unsigned long long, (size_t)k * k, L->best);
    LOR_TAKE(ar, Up, (size_t)tiles * k, L->tu);
    LOR_TAKE(ar, Dn, (size_t)tiles * k, L->td);
    LOR_TAKE(ar, Up, (size_t)chunks * k, L->cu);
    LOR_TAKE(ar, Dn, (size_t)chunks * k, L->cd);
    LOR_TAKE(ar, Up, k, L->su);
    LOR_TAKE(ar, Dn, k, L->sd);
    if (chunks > kMxChunk) return LOR_EINVAL;   // n < 2^31 keeps chunks <= 512
    return LOR_OK;
}

}  // namespace

size_t matrix_workspace(uint64_t n, uint32_t k) {
    Arena ar;   // measuring
    ar.top = kHeaderBytes;
    MxLayout L;
    if (mx_carve(ar, n, k, &L) != LOR_OK) return 0;
    return ar.top + 1024;
}

lor_status overlap_matrix(const int32_t *sa, const int32_t *lcp, uint32_t n, const int64_t *offsets, uint32_t k,
                          lor_overlap *out, void *ws, size_t ws_bytes, hipStream_t s) {
    if (k > (uint32_t)kMaxSeqs) {
        set_error("%u sequences: at most %d", k, kMaxSeqs);
        return LOR_EINVAL;
    }
    std::vector<int32_t> h_start(k + 1);
    for (uint32_t j = 0; j <= k; ++j) h_start[j] = (int32_t)(offsets[j] + j);
    Arena ar;
    ar.base = static_cast<char *>(ws);
    ar.cap = ws_bytes;
    ar.top = kHeaderBytes;
    MxLayout L;
    LOR_TRY(mx_carve(ar, n, k, &L));
    const uint32_t tiles = div_up(n ? n : 1, kMxTile);
    const uint32_t chunks = div_up(tiles, kMxChunk);
    LOR_HIP(hipMemcpyAsync(L.start, h_start.data(), (k + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    LOR_LAUNCH("k_mx_init", 40.0 * k * k, s,
               hipLaunchKernelGGL(k_mx_init, dim3(grid_for((uint64_t)k * k)), dim3(kBlock), 0, s, k * k, L.best, out));
    if (n > 0 && k > 1) {
        const bool vec = ((reinterpret_cast<uintptr_t>(sa) | reinterpret_cast<uintptr_t>(lcp)) & 15u) == 0;
        LOR_LAUNCH("k_mx_tiles", 8.0 * n, s,
                   hipLaunchKernelGGL(k_mx_tiles, dim3(tiles), dim3(kBlock), 0, s, sa, lcp, n, L.start, k, vec,
                                      tiles, L.tu, L.td));
        LOR_LAUNCH("k_mx_chunks", 32.0 * tiles * k, s,
                   hipLaunchKernelGGL(k_mx_chunks, dim3(chunks, k), dim3(kMxChunkThreads), 0, s, L.tu, L.td, tiles,
                                      chunks, L.cu, L.cd));
        LOR_LAUNCH("k_mx_chunks", 32.0 * chunks * k, s,
                   hipLaunchKernelGGL(k_mx_chunks, dim3(1, k), dim3(kMxChunkThreads), 0, s, L.cu, L.cd, chunks, 1u,
                                      L.su, L.sd));
        LOR_LAUNCH("k_mx_ranks", 8.0 * n, s,
                   hipLaunchKernelGGL(k_mx_ranks<0>, dim3(tiles), dim3(kBlock), 0, s, sa, lcp, n, L.start, k, vec,
                                      tiles, chunks, L.tu, L.td, L.cu, L.cd, L.best, out));
        LOR_LAUNCH("k_mx_emit", 8.0 * n, s,
                   hipLaunchKernelGGL(k_mx_ranks<1>, dim3(tiles), dim3(kBlock), 0, s, sa, lcp, n, L.start, k, vec,
                                      tiles, chunks, L.tu, L.td, L.cu, L.cd, L.best, out));
    }
    LOR_HIP(hipStreamSynchronize(s));   // the host table must outlive its copy
    return LOR_OK;
}

}  // namespace lor
