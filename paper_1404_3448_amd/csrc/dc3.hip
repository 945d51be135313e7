// DC3 (skew) suffix sorting on gfx950, Section III Steps 1-3.
//
// One level on a text t[0..n) whose symbols are >= 1 (positions >= n read 0):
//   Step 1  sample positions are i mod 3 in {1, 2}; when n mod 3 == 1 the
//           padding-only position n joins the mod-1 class so that the last
//           mod-1 triple is unique and the suffixes of R stop before R2.
//           Each sample position gets the key of its triple
//           (t_i, t_{i+1}, t_{i+2}); the keys are radix sorted, named in
//           sorted order (a flag where a key differs from its predecessor,
//           prefix-summed into 1-based names, as in Table II), and the names
//           form the text R = R1 R2 (mod-1 block, then mod-2 block, each in
//           position order). If a name repeats, DC3 recurses on R.
//           "R-index" below is a position in R.
//   Step 2  non-sample suffixes S_i (i mod 3 == 0) in order of
//           (t_i, rank(S_{i+1})): take the sample order, keep mod-1 entries
//           (whose predecessors are the mod-0 positions), stable-sort by t_i.
//   Step 3  merge: a mod-1 suffix S_i against a mod-0 suffix S_j compares
//           (t_i, rank(S_{i+1})) with (t_j, rank(S_{j+1})); a mod-2 suffix
//           compares (t_i, t_{i+1}, rank(S_{i+2})) with
//           (t_j, t_{j+1}, rank(S_{j+2})). rank() of a position >= n is 0.
//
// MI355X design notes: every step streams or gathers whole arrays in HBM;
// the merge needs, per element, two symbols and one or two ranks from
// random places. A streaming pass first builds one record per position
// triple q = (t_3q..t_3q+3, rank(3q+1), rank(3q+2), rank(3q+4)); every merge
// element (mod 0, 1 or 2) then needs exactly one record gather, and the
// merge-path partitioning keeps each workgroup on a fixed output tile.
#include <stdio.h>

#include "lor_internal.hpp"

namespace lor {

namespace {

constexpr int kScanItems = 4;                         // consecutive items per thread in scan-emit kernels
static_assert(kScanItems % 4 == 0, "k_ns_write reads a thread's items as 16-byte LDS groups");
constexpr uint32_t kScanTile = kBlock * kScanItems;
constexpr uint32_t kMaxScanGroups = 4096;

struct Dims {
    uint32_t n, n0, n1, n2, m, dummy;
    __host__ __device__ uint32_t pos_of(uint32_t idx) const {
        return idx < n0 ? 3u * idx + 1u : 3u * (idx - n0) + 2u;
    }
};

Dims make_dims(uint32_t n) {
    Dims d;
    d.n = n;
    d.n0 = (n + 2) / 3;
    d.n1 = (n + 1) / 3;
    d.n2 = n / 3;
    d.m = d.n0 + d.n2;
    d.dummy = d.n0 - d.n1;
    return d;
}

template <typename CH> __device__ __forceinline__ uint32_t sym(const CH *t, uint32_t n, uint32_t i);
template <> __device__ __forceinline__ uint32_t sym<uint8_t>(const uint8_t *t, uint32_t n, uint32_t i) {
    return i < n ? (uint32_t)t[i] + 1u : 0u;
}
template <> __device__ __forceinline__ uint32_t sym<int32_t>(const int32_t *t, uint32_t n, uint32_t i) {
    return i < n ? (uint32_t)t[i] : 0u;
}
// Pair-tagged texts of the batched path: symbol = 8 * pair + code, code 1..6.
template <> __device__ __forceinline__ uint32_t sym<uint16_t>(const uint16_t *t, uint32_t n, uint32_t i) {
    return i < n ? (uint32_t)t[i] : 0u;
}

// Packed key of the triple at sample position p.
// Byte and int32 texts: the three symbols, b bits each.
// Pair-tagged texts: the pair tag, then the three codes (3 bits each), a code
// of the next pair reading 0. Such a code only follows the pair's last or
// second-to-last symbol, whose own prefix (ending in the pair's unique final
// separator) already decides every comparison, so names keep the order and
// equality of the full tagged triples while the key stays tag + 9 bits.
template <typename CH> struct Triple {
    static int key_bits(int b) { return 3 * b; }
    template <typename K>
    __device__ static K pack(const CH *t, const Dims &d, int b, uint32_t p) {
        return ((K)sym(t, d.n, p) << (2 * b)) | ((K)sym(t, d.n, p + 1) << b) | (K)sym(t, d.n, p + 2);
    }
};
template <> struct Triple<uint16_t> {
    static int key_bits(int b) { return b + 6; }   // b = 3 + tag bits
    template <typename K>
    __device__ static K pack(const uint16_t *t, const Dims &d, int, uint32_t p) {
        const uint32_t s0 = sym(t, d.n, p), s1 = sym(t, d.n, p + 1), s2 = sym(t, d.n, p + 2);
        const uint32_t tag = s0 >> 3;
        const uint32_t c1 = (s1 >> 3) == tag ? (s1 & 7u) : 0u;
        const uint32_t c2 = (s2 >> 3) == tag && c1 ? (s2 & 7u) : 0u;
        return (K)((tag << 9) | ((s0 & 7u) << 6) | (c1 << 3) | c2);
    }
};

__device__ __forceinline__ void group_tiles(uint32_t items, uint32_t groups, uint32_t g, uint32_t *t0,
                                            uint32_t *t1) {
    const uint32_t tiles = (items + kScanTile - 1) / kScanTile;
    *t0 = (uint32_t)((uint64_t)tiles * g / groups);
    *t1 = (uint32_t)((uint64_t)tiles * (g + 1) / groups);
}

uint32_t scan_groups(uint32_t items) {
    uint32_t tiles = div_up(items, kScanTile);
    if (tiles == 0) tiles = 1;
    return tiles < kMaxScanGroups ? tiles : kMaxScanGroups;
}

// ---------------------------------------------------------------- join

// A thread writes kJoinBytes consecutive output bytes. When they are all
// bases of one sequence (almost always), they are the input shifted by the
// sequence index: three aligned 8-byte loads and a funnel shift, the base
// check on whole words. Windows that hold a separator, or sit near either
// end of the input, go byte by byte.
constexpr uint32_t kJoinBytes = 16;

__global__ __launch_bounds__(kBlock) void k_join(const uint8_t *__restrict__ seqs, SeqStarts st,
                                                 uint32_t N, uint32_t total, uint8_t *__restrict__ out,
                                                 uint32_t *__restrict__ err) {
    __shared__ int32_t s_start[kMaxSeqs + 1];
    for (int i = threadIdx.x; i <= st.k; i += kBlock) s_start[i] = st.start[i];
    __syncthreads();
    const int k = st.k;
    uint32_t bad = 0;
    const uint32_t stride = gridDim.x * kBlock * kJoinBytes;
    for (uint32_t p0 = (blockIdx.x * kBlock + threadIdx.x) * kJoinBytes; p0 < N; p0 += stride) {
        int j = 0;
        {   // sequence containing p0: largest j with start[j] <= p0
            int lo = 0, hi = k - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if ((uint32_t)s_start[mid] <= p0) lo = mid; else hi = mid - 1;
            }
            j = lo;
        }
        uint32_t *o = reinterpret_cast<uint32_t *>(out + p0);   // p0 is a multiple of 16, out of 4
        const uint32_t src = p0 - (uint32_t)j;
        if (p0 + kJoinBytes < (uint32_t)s_start[j + 1] && src >= 8u && src + 24u <= total) {
            const uintptr_t addr = reinterpret_cast<uintptr_t>(seqs + src);
            const uint64_t *w = reinterpret_cast<const uint64_t *>(addr & ~(uintptr_t)7);
            const uint32_t sh = (uint32_t)(addr & 7u) * 8u;
            const uint64_t w0 = w[0], w1 = w[1], w2 = w[2];
            const uint64_t lo = sh ? (w0 >> sh) | (w1 << (64u - sh)) : w0;
            const uint64_t hi = sh ? (w1 >> sh) | (w2 << (64u - sh)) : w1;
            bad |= ((lo | hi) & 0xfcfcfcfcfcfcfcfcull) != 0;
            o[0] = (uint32_t)lo;
            o[1] = (uint32_t)(lo >> 32);
            o[2] = (uint32_t)hi;
            o[3] = (uint32_t)(hi >> 32);
            continue;
        }
        for (uint32_t q = 0; q < kJoinBytes / 4; ++q) {
            uint32_t word = 0;
            for (uint32_t u = 0; u < 4; ++u) {
                const uint32_t p = p0 + 4 * q + u;
                if (p >= N) break;
                while ((uint32_t)s_start[j + 1] <= p) ++j;
                uint32_t byte;
                if (p == (uint32_t)s_start[j + 1] - 1u) {
                    byte = 4u + (uint32_t)j;
                } else {
                    byte = seqs[p - (uint32_t)j];
                    bad |= byte > 3u;
                }
                word |= byte << (8 * u);
            }
            const uint32_t pw = p0 + 4 * q;
            if (pw >= N) break;
            if (pw + 4 <= N) {
                o[q] = word;
            } else {
                for (uint32_t u = 0; pw + u < N; ++u) out[pw + u] = (uint8_t)(word >> (8 * u));
            }
        }
    }
    if (__any(bad) && dev::lane_id() == 0) atomicOr(err, 1u);
}

// ------------------------------------------------------- Step 1: keys

// mode 0: triple key (t_i, t_{i+1}, t_{i+2}), b-bit fields or mixed radix
// mixA (nonzero);
// mode 1: packed pair (t_{i+1}, t_{i+2}) of b-bit symbols, the first stage of
// wide triples.
template <typename CH, typename K>
__global__ __launch_bounds__(kBlock) void k_sample_keys(const CH *__restrict__ t, Dims d, int b, int mode,
                                                        uint64_t mixA, K *__restrict__ keys,
                                                        uint32_t *__restrict__ vals) {
    for (uint32_t idx = blockIdx.x * kBlock + threadIdx.x; idx < d.m; idx += gridDim.x * kBlock) {
        const uint32_t p = d.pos_of(idx);
        K key;
        if (mode == 0 && mixA) {   // mixed radix; A^3 fits K
            key = ((K)sym(t, d.n, p) * (K)mixA + (K)sym(t, d.n, p + 1)) * (K)mixA + (K)sym(t, d.n, p + 2);
        } else if (mode == 0) {
            key = Triple<CH>::template pack<K>(t, d, b, p);
        } else {
            key = ((K)sym(t, d.n, p + 1) << b) | (K)sym(t, d.n, p + 2);
        }
        keys[idx] = key;
        vals[idx] = idx;
    }
}

// Second stage of wide triples: keys[r] = (t_i << 32) | rank of the pair
// (t_{i+1}, t_{i+2}) of sorted entry r.
template <typename CH>
__global__ __launch_bounds__(kBlock) void k_pair_rekey(const CH *__restrict__ t, Dims d,
                                                       const uint32_t *__restrict__ vals,
                                                       const uint32_t *__restrict__ pair_rank,
                                                       uint64_t *__restrict__ keys) {
    for (uint32_t r = blockIdx.x * kBlock + threadIdx.x; r < d.m; r += gridDim.x * kBlock)
        keys[r] = ((uint64_t)sym(t, d.n, d.pos_of(vals[r])) << 32) | pair_rank[r];
}

// ------------------------------------------------------ Step 1: naming

// A sorted entry starts a new name when its key differs from its
// predecessor's (the keys hold whole triples, or a triple's first symbol and
// the rank of its last two).
template <typename K>
__global__ __launch_bounds__(kBlock) void k_name_count(const K *__restrict__ keys, uint32_t m, uint32_t groups,
                                                       uint32_t *__restrict__ counts) {
    __shared__ uint32_t s_tmp[kBlock / kWave];
    uint32_t t0, t1;
    group_tiles(m, groups, blockIdx.x, &t0, &t1);
    uint32_t c = 0;
    for (uint32_t r = t0 * kScanTile + threadIdx.x; r < min(m, t1 * kScanTile); r += kBlock)
        c += (r == 0) || keys[r] != keys[r - 1];
    uint32_t tot;
    dev::block_exclusive_sum(c, s_tmp, &tot);
    if (threadIdx.x == 0) counts[blockIdx.x] = tot;
}

// names[r] = 1-based name of sorted entry r (written in sorted order; a
// bucketed scatter then moves each name to its R-index). Tiles go through
// LDS so that the per-thread runs of consecutive entries cost coalesced
// loads and stores.
template <typename K>
__global__ __launch_bounds__(kBlock) void k_name_write(const K *__restrict__ keys, uint32_t m, uint32_t groups,
                                                       const uint32_t *__restrict__ counts,
                                                       uint32_t *__restrict__ names) {
    __shared__ uint32_t s_tmp[kBlock / kWave];
    __shared__ K s_key[kScanTile + 1];      // s_key[1 + l] = keys[g0 + l]; s_key[0] = its predecessor
    __shared__ uint32_t s_name[kScanTile];
    uint32_t t0, t1;
    group_tiles(m, groups, blockIdx.x, &t0, &t1);
    uint32_t base = counts[blockIdx.x];
    for (uint32_t tile = t0; tile < t1; ++tile) {
        const uint32_t g0 = tile * kScanTile;
        for (uint32_t l = threadIdx.x; l <= kScanTile; l += kBlock) {
            const uint32_t r = g0 + l;   // keys[r - 1] lands in s_key[l]
            s_key[l] = (r >= 1 && r - 1 < m) ? keys[r - 1] : K(0);
        }
        __syncthreads();
        const uint32_t l0 = threadIdx.x * kScanItems;
        bool f[kScanItems];
        uint32_t c = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            const uint32_t r = g0 + l0 + i;
            f[i] = r < m && (r == 0 || s_key[l0 + i + 1] != s_key[l0 + i]);
            c += f[i];
        }
        uint32_t tot;
        uint32_t name = base + dev::block_exclusive_sum(c, s_tmp, &tot);
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            name += f[i];
            s_name[l0 + i] = name;
        }
        __syncthreads();
        for (uint32_t l = threadIdx.x; l < kScanTile; l += kBlock)
            if (g0 + l < m) names[g0 + l] = s_name[l];
        base += tot;
        __syncthreads();   // the next tile reuses the LDS
    }
}

// ------------------------------------ Step 1: naming by a key bitmap

// When the packed triple keys span at most 2^24 values and that span is not
// much larger than the number of sample positions, lexicographic names need no
// sort: mark every key present in a bitmap, prefix-count the marks, and the
// name of a key is 1 + the number of present keys below it. Names are then
// written in R-index order (streaming) instead of scattered from sorted order.
template <typename CH>
__device__ __forceinline__ uint32_t triple_key(const CH *t, const Dims &d, int b, uint32_t idx) {
    return Triple<CH>::template pack<uint32_t>(t, d, b, d.pos_of(idx));
}

template <typename CH>
__global__ __launch_bounds__(kBlock) void k_presence(const CH *__restrict__ t, Dims d, int b,
                                                     uint32_t *__restrict__ bitmap, uint32_t words, int in_lds) {
    extern __shared__ uint32_t s_bits[];
    if (in_lds) {
        for (uint32_t w = threadIdx.x; w < words; w += kBlock) s_bits[w] = 0;
        __syncthreads();
    }
    for (uint32_t idx = blockIdx.x * kBlock + threadIdx.x; idx < d.m; idx += gridDim.x * kBlock) {
        const uint32_t key = triple_key(t, d, b, idx);
        const uint32_t w = key >> 5, bit = 1u << (key & 31u);
        if (w >= words) continue;
        if (in_lds) {
            if (!(s_bits[w] & bit)) atomicOr(&s_bits[w], bit);
        } else if (!(bitmap[w] & bit)) {
            atomicOr(&bitmap[w], bit);   // a stale read only costs a redundant atomic
        }
    }
    if (in_lds) {
        __syncthreads();
        for (uint32_t w = threadIdx.x; w < words; w += kBlock)
            if (s_bits[w]) atomicOr(&bitmap[w], s_bits[w]);
    }
}

// Pair-tagged texts: the key is tag * 512 + codes and tags only grow along
// the text, so the sample positions of one workgroup (q in [q0, q0 + kTagQ))
// reach a short slice of bitmap words. The slice is marked in LDS and merged
// into the bitmap once; a key outside it (the padding triple) goes to the
// bitmap directly, as does everything when the slice is too wide.
constexpr uint32_t kTagQ = kBlock * 16;
constexpr uint32_t kTagWords = 4096;

__global__ __launch_bounds__(kBlock) void k_presence_tagged(const uint16_t *__restrict__ t, Dims d, int b,
                                                            uint32_t *__restrict__ bitmap, uint32_t words) {
    __shared__ uint32_t s_bits[kTagWords];
    const uint32_t q0 = blockIdx.x * kTagQ;
    if (q0 >= d.n0) return;
    const uint32_t q1 = min(d.n0, q0 + kTagQ);
    const uint32_t w_lo = (sym(t, d.n, min(3u * q0 + 1u, d.n - 1u)) >> 3) * 16u;
    const uint32_t w_hi = ((sym(t, d.n, min(3u * q1 + 1u, d.n - 1u)) >> 3) + 1u) * 16u;   // exclusive
    const bool local = w_hi > w_lo && w_hi - w_lo <= kTagWords;
    if (local) {
        for (uint32_t w = threadIdx.x; w < w_hi - w_lo; w += kBlock) s_bits[w] = 0;
        __syncthreads();
    }
    for (uint32_t q = q0 + threadIdx.x; q < q1; q += kBlock) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            if (c == 1 && q >= d.n2) break;
            const uint32_t key = Triple<uint16_t>::template pack<uint32_t>(t, d, b, 3u * q + 1u + c);
            const uint32_t w = key >> 5, bit = 1u << (key & 31u);
            if (w >= words) continue;
            if (local && w >= w_lo && w < w_hi) {
                if (!(s_bits[w - w_lo] & bit)) atomicOr(&s_bits[w - w_lo], bit);
            } else if (!(bitmap[w] & bit)) {
                atomicOr(&bitmap[w], bit);
            }
        }
    }
    if (local) {
        __syncthreads();
        for (uint32_t w = threadIdx.x; w < w_hi - w_lo; w += kBlock)
            if (s_bits[w]) atomicOr(&bitmap[w_lo + w], s_bits[w]);
    }
}

__global__ __launch_bounds__(kBlock) void k_popc(const uint32_t *__restrict__ bitmap, uint32_t words,
                                                 uint32_t *__restrict__ cnt) {
    for (uint32_t w = blockIdx.x * kBlock + threadIdx.x; w < words; w += gridDim.x * kBlock)
        cnt[w] = (uint32_t)__popc(bitmap[w]);
}

template <typename CH>
__global__ __launch_bounds__(kBlock) void k_name_table(const CH *__restrict__ t, Dims d, int b,
                                                       const uint32_t *__restrict__ bitmap,
                                                       const uint32_t *__restrict__ below, uint32_t words,
                                                       int32_t *__restrict__ R) {
    for (uint32_t idx = blockIdx.x * kBlock + threadIdx.x; idx < d.m; idx += gridDim.x * kBlock) {
        const uint32_t key = triple_key(t, d, b, idx);
        const uint32_t w = min(key >> 5, words - 1);
        R[idx] = (int32_t)(below[w] + (uint32_t)__popc(bitmap[w] & ((1u << (key & 31u)) - 1u)) + 1u);
    }
}

// Byte and int32 texts: the code of a triple is mixed-radix in A = alphabet
// + 1 (symbols are 0..alphabet), (s0 A + s1) A + s2, which keeps the order
// and equality of the triples in a code space of A^3 instead of 2^(3b); at
// the second level (97 symbols) the bitmap then fits in LDS. Each thread
// takes four consecutive q: sample positions 3q+1 (R-index q) and 3q+2
// (R-index n0 + q) for q in [q0, q0 + 4) need the 16 symbols from 3 q0,
// read as whole words while the window lies inside the text.
constexpr uint32_t kWinQ = 4;
constexpr int kTblBlock = 1024;

template <typename CH>
__device__ __forceinline__ void sym_window(const CH *t, uint32_t n, uint32_t p0, uint32_t s[16]) {
    if (p0 + 16u <= n) {
        if constexpr (sizeof(CH) == 1) {
            const uint32_t *w = reinterpret_cast<const uint32_t *>(t + p0);   // p0 = 12 g: 4-byte aligned
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t x = w[i];
#pragma unroll
                for (int j = 0; j < 4; ++j) s[4 * i + j] = ((x >> (8 * j)) & 255u) + 1u;
            }
        } else {
            const uint4 *w = reinterpret_cast<const uint4 *>(t + p0);        // p0 = 12 g words: 16-byte aligned
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint4 x = w[i];
                s[4 * i] = x.x; s[4 * i + 1] = x.y; s[4 * i + 2] = x.z; s[4 * i + 3] = x.w;
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < 16; ++i) s[i] = sym(t, n, p0 + i);
    }
}

__device__ __forceinline__ uint32_t mixed_code(uint32_t a, uint32_t b, uint32_t c, uint32_t A) {
    return (a * A + b) * A + c;
}

// Codes of the (up to) eight sample triples of group g; ok bits say which exist.
template <typename CH>
__device__ __forceinline__ void group_codes(const CH *t, const Dims &d, uint32_t A, uint32_t g, uint32_t c1[kWinQ],
                                            uint32_t c2[kWinQ]) {
    uint32_t s[16];
    sym_window<CH>(t, d.n, 3u * kWinQ * g, s);
#pragma unroll
    for (int j = 0; j < (int)kWinQ; ++j) {
        c1[j] = mixed_code(s[3 * j + 1], s[3 * j + 2], s[3 * j + 3], A);
        c2[j] = mixed_code(s[3 * j + 2], s[3 * j + 3], s[3 * j + 4], A);
    }
}

__device__ __forceinline__ void mark_present(uint32_t *bits, uint32_t words, uint32_t code) {
    const uint32_t w = code >> 5, bit = 1u << (code & 31u);
    if (w < words && !(bits[w] & bit)) atomicOr(&bits[w], bit);   // a stale read only costs a redundant atomic
}

template <typename CH, bool IN_LDS>
__global__ __launch_bounds__(kTblBlock) void k_presence_w(const CH *__restrict__ t, Dims d, uint32_t A,
                                                          uint32_t *__restrict__ bitmap, uint32_t words) {
    extern __shared__ uint32_t s_bits[];
    if (IN_LDS) {
        for (uint32_t w = threadIdx.x; w < words; w += kTblBlock) s_bits[w] = 0;
        __syncthreads();
    }
    uint32_t *bits = IN_LDS ? s_bits : bitmap;
    const uint32_t groups = (d.n0 + kWinQ - 1) / kWinQ;   // n0 >= n2
    for (uint32_t g = blockIdx.x * kTblBlock + threadIdx.x; g < groups; g += gridDim.x * kTblBlock) {
        uint32_t c1[kWinQ], c2[kWinQ];
        group_codes<CH>(t, d, A, g, c1, c2);
#pragma unroll
        for (int j = 0; j < (int)kWinQ; ++j) {
            const uint32_t q = kWinQ * g + j;
            if (q < d.n0) mark_present(bits, words, c1[j]);
            if (q < d.n2) mark_present(bits, words, c2[j]);
        }
    }
    if (IN_LDS) {
        __syncthreads();
        for (uint32_t w = threadIdx.x; w < words; w += kTblBlock)
            if (s_bits[w]) atomicOr(&bitmap[w], s_bits[w]);
    }
}

// name = 1 + number of present codes below the code. In LDS the table keeps
// the bitmap and the exclusive count at every fourth word.
__device__ __forceinline__ uint32_t table_name(const uint32_t *bits, const uint32_t *below4, uint32_t words,
                                               uint32_t code) {
    const uint32_t w = min(code >> 5, words - 1);
    uint32_t c = below4[w >> 2];
    for (uint32_t u = w & ~3u; u < w; ++u) c += (uint32_t)__popc(bits[u]);
    return c + (uint32_t)__popc(bits[w] & ((1u << (code & 31u)) - 1u)) + 1u;
}

template <typename CH>
__global__ __launch_bounds__(kTblBlock) void k_name_table_w(const CH *__restrict__ t, Dims d, uint32_t A,
                                                            const uint32_t *__restrict__ bitmap,
                                                            const uint32_t *__restrict__ below, uint32_t words,
                                                            int in_lds, int32_t *__restrict__ R) {
    extern __shared__ uint32_t s_tab[];
    const uint32_t quads = (words + 3u) / 4u;
    if (in_lds) {
        for (uint32_t w = threadIdx.x; w < words; w += kTblBlock) s_tab[w] = bitmap[w];
        for (uint32_t g = threadIdx.x; g < quads; g += kTblBlock) s_tab[words + g] = below[4u * g];
        __syncthreads();
    }
    const uint32_t groups = (d.n0 + kWinQ - 1) / kWinQ;
    for (uint32_t g = blockIdx.x * kTblBlock + threadIdx.x; g < groups; g += gridDim.x * kTblBlock) {
        uint32_t c1[kWinQ], c2[kWinQ];
        group_codes<CH>(t, d, A, g, c1, c2);
#pragma unroll
        for (int j = 0; j < (int)kWinQ; ++j) {
            const uint32_t q = kWinQ * g + j;
            uint32_t n1, n2;
            if (in_lds) {
                n1 = table_name(s_tab, s_tab + words, words, c1[j]);
                n2 = table_name(s_tab, s_tab + words, words, c2[j]);
            } else {
                const uint32_t w1 = min(c1[j] >> 5, words - 1), w2 = min(c2[j] >> 5, words - 1);
                n1 = below[w1] + (uint32_t)__popc(bitmap[w1] & ((1u << (c1[j] & 31u)) - 1u)) + 1u;
                n2 = below[w2] + (uint32_t)__popc(bitmap[w2] & ((1u << (c2[j] & 31u)) - 1u)) + 1u;
            }
            if (q < d.n0) R[q] = (int32_t)n1;
            if (q < d.n2) R[d.n0 + q] = (int32_t)n2;
        }
    }
}

// Unique names are ranks: sa12[name - 1] = R-index.
__global__ __launch_bounds__(kBlock) void k_sa12_from_names(const int32_t *__restrict__ R, uint32_t m,
                                                            int32_t *__restrict__ sa12) {
    for (uint32_t idx = blockIdx.x * kBlock + threadIdx.x; idx < m; idx += gridDim.x * kBlock) {
        const uint32_t r = (uint32_t)R[idx] - 1u;
        if (r < m) sa12[r] = (int32_t)idx;
    }
}

// ----------------------------------------------- comparison records

__device__ __forceinline__ uint32_t rank_at(const int32_t *rank12, const Dims &d, uint32_t p) {
    if (p >= d.n) return 0u;
    const uint32_t ri = (p % 3u == 1u) ? p / 3u : d.n0 + p / 3u;
    return (uint32_t)rank12[ri];
}

// Record of triple q: symbols t_{3q..3q+3}, ranks of 3q+1, 3q+2, 3q+4.
// u8 texts: one uint4 {c0|c1<<8|c2<<16|c3<<24, r1, r2, r4}; symbols are
// byte + 1 <= 255 so each fits a byte (0 = past the end).
// i32 texts: two uint4 {c0, c1, c2, c3}, {r1, r2, r4, 0}.
template <typename CH> struct Rec;
template <> struct Rec<uint8_t> { uint4 a; };
template <> struct Rec<int32_t> { uint4 a, b; };
template <> struct Rec<uint16_t> { uint4 a, b; };

// RT picks the layout: Rec<uint8_t> (one uint4) for any text whose symbols
// fit a byte (byte texts, and int32 texts of at most 255 symbols such as the
// level over the byte text's triple names), the two-uint4 form otherwise.
// For q < n0 it also writes Step 2's pair of the mod-0 suffix 3q: slot[q] =
// rank of suffix 3q+1 minus one (read from rank12 itself: when n mod 3 = 1
// the last one is the padding-only position n) and sym0[q] = t_{3q}.
template <typename CH, typename RT>
__global__ __launch_bounds__(kBlock) void k_records(const CH *__restrict__ t, Dims d,
                                                    const int32_t *__restrict__ rank12,
                                                    Rec<RT> *__restrict__ rec, uint32_t *__restrict__ slot,
                                                    uint32_t *__restrict__ sym0) {
    const uint32_t nq = d.n0 + 1;
    for (uint32_t q = blockIdx.x * kBlock + threadIdx.x; q < nq; q += gridDim.x * kBlock) {
        const uint32_t p = 3u * q;
        const uint32_t c0 = sym(t, d.n, p), c1 = sym(t, d.n, p + 1), c2 = sym(t, d.n, p + 2),
                       c3 = sym(t, d.n, p + 3);
        const uint32_t r1 = rank_at(rank12, d, p + 1), r2 = rank_at(rank12, d, p + 2),
                       r4 = rank_at(rank12, d, p + 4);
        Rec<RT> x;
        if constexpr (sizeof(RT) == 1) {
            x.a = make_uint4(c0 | (c1 << 8) | (c2 << 16) | (c3 << 24), r1, r2, r4);
        } else {
            x.a = make_uint4(c0, c1, c2, c3);
            x.b = make_uint4(r1, r2, r4, 0u);
        }
        rec[q] = x;
        if (slot && q < d.n0) {
            slot[q] = (uint32_t)rank12[q] - 1u;
            sym0[q] = c0;
        }
    }
}

// Comparison view of one merge element: c0, c1 symbols, r = rank used
// against mod-0 elements (mod 1: rank(i+1); mod 2: rank(i+2)); for mod-0
// elements r = rank(j+1) and r2 = rank(j+2). cls = position mod 3.
struct Key4 {
    uint32_t c0, c1, r, r2cls;   // r2cls: mod-0 elements hold rank(j+2); others hold their class
};

template <typename CH> __device__ __forceinline__ Key4 key_of(const Rec<CH> *rec, uint32_t pos);

__device__ __forceinline__ Key4 make_key(uint32_t cls, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         uint32_t r1, uint32_t r2, uint32_t r4) {
    Key4 k;
    if (cls == 0) { k.c0 = c0; k.c1 = c1; k.r = r1; k.r2cls = r2; }
    else if (cls == 1) { k.c0 = c1; k.c1 = c2; k.r = r2; k.r2cls = 1; }
    else { k.c0 = c2; k.c1 = c3; k.r = r4; k.r2cls = 2; }
    return k;
}

// Positions always come from a permutation of 0..n-1; pos is clamped to n-1
// by the callers so that a broken permutation cannot read past the records.
template <> __device__ __forceinline__ Key4 key_of<uint8_t>(const Rec<uint8_t> *rec, uint32_t pos) {
    const uint4 a = rec[pos / 3u].a;
    return make_key(pos % 3u, a.x & 255u, (a.x >> 8) & 255u, (a.x >> 16) & 255u, a.x >> 24, a.y, a.z, a.w);
}
template <> __device__ __forceinline__ Key4 key_of<int32_t>(const Rec<int32_t> *rec, uint32_t pos) {
    const Rec<int32_t> x = rec[pos / 3u];
    return make_key(pos % 3u, x.a.x, x.a.y, x.a.z, x.a.w, x.b.x, x.b.y, x.b.z);
}
template <> __device__ __forceinline__ Key4 key_of<uint16_t>(const Rec<uint16_t> *rec, uint32_t pos) {
    const Rec<uint16_t> x = rec[pos / 3u];
    return make_key(pos % 3u, x.a.x, x.a.y, x.a.z, x.a.w, x.b.x, x.b.y, x.b.z);
}

// Is sample suffix b smaller than mod-0 suffix a? (Step 3 rules.)
__device__ __forceinline__ bool sample_less(const Key4 &b, const Key4 &a) {
    if (b.c0 != a.c0) return b.c0 < a.c0;
    if (b.r2cls == 1) return b.r < a.r;
    if (b.c1 != a.c1) return b.c1 < a.c1;
    return b.r < a.r2cls;
}

// --------------------------------------------- Step 2: non-sample order

// Count sample-order entries that are mod-1 positions (R-index < n0).
__global__ __launch_bounds__(kBlock) void k_ns_count(const int32_t *__restrict__ sa12, Dims d, uint32_t groups,
                                                     uint32_t *__restrict__ counts) {
    __shared__ uint32_t s_tmp[kBlock / kWave];
    uint32_t t0, t1;
    group_tiles(d.m, groups, blockIdx.x, &t0, &t1);
    uint32_t c = 0;
    for (uint32_t r = t0 * kScanTile + threadIdx.x; r < min(d.m, t1 * kScanTile); r += kBlock)
        c += (uint32_t)sa12[r] < d.n0;
    uint32_t tot;
    dev::block_exclusive_sum(c, s_tmp, &tot);
    if (threadIdx.x == 0) counts[blockIdx.x] = tot;
}

// The first symbol of every mod-0 suffix, laid out by the rank of the
// mod-1 suffix that follows it: for R-index q < n0 (position 3q+1), the pair
// (rank(3q+1) - 1, t_{3q}). A bucketed scatter of these pairs puts t_{3q}
// at sample-order slot rank(3q+1) - 1, so Step 2 then reads its keys in
// order instead of gathering one text symbol per mod-0 suffix.

// Emit mod-0 position 3*idx (predecessor of mod-1 entry idx) with key
// t_{3 idx}, which first[r] holds for sample-order slot r. A tile is staged
// in LDS: coalesced loads, the order-keeping compaction per thread reads
// LDS, and the compacted pairs leave as coalesced stores.
__global__ __launch_bounds__(kBlock) void k_ns_write(const int32_t *__restrict__ first, const int32_t *__restrict__ sa12,
                                                     Dims d, uint32_t groups,
                                                     const uint32_t *__restrict__ counts,
                                                     uint32_t *__restrict__ keys0,
                                                     uint32_t *__restrict__ vals0) {
    __shared__ uint32_t s_tmp[kBlock / kWave];
    __shared__ __align__(16) uint32_t s_idx[kScanTile];
    __shared__ __align__(16) uint32_t s_first[kScanTile];
    __shared__ uint32_t s_k[kScanTile];
    __shared__ uint32_t s_v[kScanTile];
    uint32_t t0, t1;
    group_tiles(d.m, groups, blockIdx.x, &t0, &t1);
    uint32_t base = counts[blockIdx.x];
    for (uint32_t tile = t0; tile < t1; ++tile) {
        const uint32_t g0 = tile * kScanTile;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            const uint32_t l = i * kBlock + threadIdx.x, r = g0 + l;
            const uint32_t x = r < d.m ? (uint32_t)sa12[r] : 0xffffffffu;
            s_idx[l] = x;
            s_first[l] = x < d.n0 ? (uint32_t)first[r] : 0u;
        }
        __syncthreads();
        const uint32_t l0 = threadIdx.x * kScanItems;
        uint32_t idx[kScanItems], fs[kScanItems];
#pragma unroll
        for (int h = 0; h < kScanItems / 4; ++h) {
            const uint4 a = *reinterpret_cast<const uint4 *>(&s_idx[l0 + 4 * h]);
            const uint4 f = *reinterpret_cast<const uint4 *>(&s_first[l0 + 4 * h]);
            idx[4 * h] = a.x; idx[4 * h + 1] = a.y; idx[4 * h + 2] = a.z; idx[4 * h + 3] = a.w;
            fs[4 * h] = f.x; fs[4 * h + 1] = f.y; fs[4 * h + 2] = f.z; fs[4 * h + 3] = f.w;
        }
        uint32_t c = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) c += idx[i] < d.n0;
        uint32_t tot;
        uint32_t jl = dev::block_exclusive_sum(c, s_tmp, &tot);
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            if (idx[i] < d.n0) {
                s_k[jl] = fs[i];
                s_v[jl] = 3u * idx[i];
                ++jl;
            }
        }
        __syncthreads();
        for (uint32_t x = threadIdx.x; x < tot; x += kBlock) {
            const uint32_t j = base + x;
            if (j < d.n0) {
                keys0[j] = s_k[x];
                vals0[j] = s_v[x];
            }
        }
        base += tot;
        __syncthreads();   // the next tile reuses the LDS
    }
}

// ------------------- Step 1 at deep levels: order from the parent level
//
// A level's text is the name array R of its parent, and the parent sorted
// its triples before naming them: its sample order (kept in this level's SA
// buffer until the merge writes it) lists this level's text positions by
// symbol value, and its names in that order are this level's symbols in that
// order. Keeping the positions i mod 3 != 0 gives the sample positions
// sorted by their first symbol s0 with no sort at all (the padding-only
// position, triple (0, 0, 0), goes first). When the parent's names are
// nearly all distinct (the texts of deep levels), only the runs of equal s0
// still need an order, by (s1, s2): that subset is sorted on its own and put
// back into its runs' slots.

// Sample positions in P (text positions sorted by symbol), per group of tiles.
__global__ __launch_bounds__(kBlock) void k_po_count(const int32_t *__restrict__ P, uint32_t n, uint32_t groups,
                                                     uint32_t *__restrict__ counts) {
    __shared__ uint32_t s_tmp[kBlock / kWave];
    uint32_t t0, t1;
    group_tiles(n, groups, blockIdx.x, &t0, &t1);
    uint32_t c = 0;
    for (uint32_t r = t0 * kScanTile + threadIdx.x; r < min(n, t1 * kScanTile); r += kBlock)
        c += ((uint32_t)P[r] % 3u) != 0u;
    uint32_t tot;
    dev::block_exclusive_sum(c, s_tmp, &tot);
    if (threadIdx.x == 0) counts[blockIdx.x] = tot;
}

// ord[k] = R-index of the k-th sample position in s0 order, s0v[k] = its s0
// (from the parent's names in the same order). Tiles are staged in LDS.
__global__ __launch_bounds__(kBlock) void k_po_write(const int32_t *__restrict__ P, const uint32_t *__restrict__ NS,
                                                     Dims d, uint32_t groups, const uint32_t *__restrict__ counts,
                                                     int32_t *__restrict__ ord, uint32_t *__restrict__ s0v) {
    __shared__ uint32_t s_tmp[kBlock / kWave];
    __shared__ __align__(16) uint32_t s_p[kScanTile];
    __shared__ __align__(16) uint32_t s_ns[kScanTile];
    __shared__ uint32_t s_k[kScanTile];
    __shared__ uint32_t s_v[kScanTile];
    if (blockIdx.x == 0 && threadIdx.x == 0 && d.dummy) {
        ord[0] = (int32_t)(d.n0 - 1);   // position n: triple (0, 0, 0), below every other
        s0v[0] = 0;
    }
    uint32_t t0, t1;
    group_tiles(d.n, groups, blockIdx.x, &t0, &t1);
    uint32_t base = d.dummy + counts[blockIdx.x];
    for (uint32_t tile = t0; tile < t1; ++tile) {
        const uint32_t g0 = tile * kScanTile;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            const uint32_t l = i * kBlock + threadIdx.x, r = g0 + l;
            const bool ok = r < d.n;
            s_p[l] = ok ? (uint32_t)P[r] : 0u;   // position 0 is not a sample position: padding drops out
            s_ns[l] = ok ? NS[r] : 0u;
        }
        __syncthreads();
        const uint32_t l0 = threadIdx.x * kScanItems;
        uint32_t p[kScanItems], ns[kScanItems];
#pragma unroll
        for (int h = 0; h < kScanItems / 4; ++h) {
            const uint4 a = *reinterpret_cast<const uint4 *>(&s_p[l0 + 4 * h]);
            const uint4 f = *reinterpret_cast<const uint4 *>(&s_ns[l0 + 4 * h]);
            p[4 * h] = a.x; p[4 * h + 1] = a.y; p[4 * h + 2] = a.z; p[4 * h + 3] = a.w;
            ns[4 * h] = f.x; ns[4 * h + 1] = f.y; ns[4 * h + 2] = f.z; ns[4 * h + 3] = f.w;
        }
        uint32_t c = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) c += (p[i] % 3u) != 0u;
        uint32_t tot;
        uint32_t jl = dev::block_exclusive_sum(c, s_tmp, &tot);
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            const uint32_t cls = p[i] % 3u;
            if (cls != 0u) {
                s_k[jl] = cls == 1u ? p[i] / 3u : d.n0 + p[i] / 3u;
                s_v[jl] = ns[i];
                ++jl;
            }
        }
        __syncthreads();
        for (uint32_t x = threadIdx.x; x < tot; x += kBlock) {
            const uint32_t j = base + x;
            if (j < d.m) {
                ord[j] = (int32_t)s_k[x];
                s0v[j] = s_v[x];
            }
        }
        base += tot;
        __syncthreads();   // the next tile reuses the LDS
    }
}

// Entry k of the s0 order shares its s0 with a neighbour.
__device__ __forceinline__ bool po_in_run(const uint32_t *s0v, uint32_t m, uint32_t k) {
    const uint32_t x = s0v[k];
    return (k > 0 && s0v[k - 1] == x) || (k + 1 < m && s0v[k + 1] == x);
}

__global__ __launch_bounds__(kBlock) void k_po_runs_count(const uint32_t *__restrict__ s0v, uint32_t m,
                                                          uint32_t groups, uint32_t *__restrict__ counts) {
    __shared__ uint32_t s_tmp[kBlock / kWave];
    uint32_t t0, t1;
    group_tiles(m, groups, blockIdx.x, &t0, &t1);
    uint32_t c = 0;
    for (uint32_t k = t0 * kScanTile + threadIdx.x; k < min(m, t1 * kScanTile); k += kBlock) c += po_in_run(s0v, m, k);
    uint32_t tot;
    dev::block_exclusive_sum(c, s_tmp, &tot);
    if (threadIdx.x == 0) counts[blockIdx.x] = tot;
}

// The subset (entries in runs of equal s0), in order: its slot k and ord[k];
// flag[k] (nullable) = 1 (a new name) for every entry outside the subset, 0
// inside (set later from the subset's order).
__global__ __launch_bounds__(kBlock) void k_po_runs_write(const uint32_t *__restrict__ s0v,
                                                          const int32_t *__restrict__ ord, uint32_t m,
                                                          uint32_t groups, const uint32_t *__restrict__ counts,
                                                          uint32_t cap, uint32_t *__restrict__ sub_slot,
                                                          uint32_t *__restrict__ sub_idx,
                                                          uint32_t *__restrict__ flag) {
    __shared__ uint32_t s_tmp[kBlock / kWave];
    uint32_t t0, t1;
    group_tiles(m, groups, blockIdx.x, &t0, &t1);
    uint32_t base = counts[blockIdx.x];
    for (uint32_t tile = t0; tile < t1; ++tile) {
        const uint32_t k0 = tile * kScanTile + threadIdx.x * kScanItems;
        bool in[kScanItems];
        uint32_t c = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            const uint32_t k = k0 + i;
            in[i] = k < m && po_in_run(s0v, m, k);
            c += in[i];
            if (flag && k < m) flag[k] = in[i] ? 0u : 1u;
        }
        uint32_t tot;
        uint32_t j = base + dev::block_exclusive_sum(c, s_tmp, &tot);
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            if (in[i]) {
                if (j < cap) {   // the host checks the count against cap before using the subset
                    sub_slot[j] = k0 + i;
                    sub_idx[j] = (uint32_t)ord[k0 + i];
                }
                ++j;
            }
        }
        base += tot;
    }
}

// First stage of the subset's sort: keys (t_{i+1}, t_{i+2}) of its positions.
template <typename CH>
__global__ __launch_bounds__(kBlock) void k_po_keys(const CH *__restrict__ t, Dims d, int b,
                                                    const uint32_t *__restrict__ sub_idx, uint32_t ms,
                                                    uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    for (uint32_t j = blockIdx.x * kBlock + threadIdx.x; j < ms; j += gridDim.x * kBlock) {
        const uint32_t idx = min(sub_idx[j], d.m - 1);
        const uint32_t p = d.pos_of(idx);
        keys[j] = ((uint64_t)sym(t, d.n, p + 1) << b) | (uint64_t)sym(t, d.n, p + 2);
        vals[j] = idx;
    }
}

// The subset, sorted by whole triples (keys: s0 << 32 | rank of (s1, s2)),
// goes back into its slots in order; an entry starts a new name when its
// triple differs from the subset entry before it.
__global__ __launch_bounds__(kBlock) void k_po_place(const uint64_t *__restrict__ keys,
                                                     const uint32_t *__restrict__ vals,
                                                     const uint32_t *__restrict__ sub_slot, uint32_t ms, uint32_t m,
                                                     int32_t *__restrict__ sa12, uint32_t *__restrict__ flag) {
    for (uint32_t j = blockIdx.x * kBlock + threadIdx.x; j < ms; j += gridDim.x * kBlock) {
        const uint32_t k = sub_slot[j];
        if (k < m) {
            sa12[k] = (int32_t)vals[j];
            flag[k] = (j == 0 || keys[j] != keys[j - 1]) ? 1u : 0u;
        }
    }
}

// names[k] = 1-based name of sorted entry k from the new-name flags (tiles
// staged in LDS, as k_name_write).
__global__ __launch_bounds__(kBlock) void k_flag_count(const uint32_t *__restrict__ flag, uint32_t m, uint32_t groups,
                                                       uint32_t *__restrict__ counts) {
    __shared__ uint32_t s_tmp[kBlock / kWave];
    uint32_t t0, t1;
    group_tiles(m, groups, blockIdx.x, &t0, &t1);
    uint32_t c = 0;
    for (uint32_t k = t0 * kScanTile + threadIdx.x; k < min(m, t1 * kScanTile); k += kBlock) c += flag[k];
    uint32_t tot;
    dev::block_exclusive_sum(c, s_tmp, &tot);
    if (threadIdx.x == 0) counts[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_flag_write(const uint32_t *__restrict__ flag, uint32_t m, uint32_t groups,
                                                       const uint32_t *__restrict__ counts,
                                                       uint32_t *__restrict__ names) {
    __shared__ uint32_t s_tmp[kBlock / kWave];
    __shared__ __align__(16) uint32_t s_f[kScanTile];
    uint32_t t0, t1;
    group_tiles(m, groups, blockIdx.x, &t0, &t1);
    uint32_t base = counts[blockIdx.x];
    for (uint32_t tile = t0; tile < t1; ++tile) {
        const uint32_t g0 = tile * kScanTile;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            const uint32_t l = i * kBlock + threadIdx.x;
            s_f[l] = g0 + l < m ? flag[g0 + l] : 0u;
        }
        __syncthreads();
        const uint32_t l0 = threadIdx.x * kScanItems;
        uint32_t f[kScanItems], c = 0;
#pragma unroll
        for (int h = 0; h < kScanItems / 4; ++h) {
            const uint4 a = *reinterpret_cast<const uint4 *>(&s_f[l0 + 4 * h]);
            f[4 * h] = a.x; f[4 * h + 1] = a.y; f[4 * h + 2] = a.z; f[4 * h + 3] = a.w;
        }
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) c += f[i];
        uint32_t tot;
        uint32_t name = base + dev::block_exclusive_sum(c, s_tmp, &tot);
        __syncthreads();   // every thread has read its flags: the tile is rewritten with names
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            name += f[i];
            s_f[l0 + i] = name;
        }
        __syncthreads();
        for (uint32_t l = threadIdx.x; l < kScanTile; l += kBlock)
            if (g0 + l < m) names[g0 + l] = s_f[l];
        base += tot;
        __syncthreads();   // the next tile reuses the LDS
    }
}

// Bit 31 set when symbol x = NS[r] of P's entry r occurs more than once in
// the text (a neighbour in P has it too); symbols stay below 2^31.
__device__ __forceinline__ uint32_t repeat_flag(const uint32_t *__restrict__ NS, uint32_t n, uint32_t r,
                                                uint32_t x) {
    return ((r > 0 && NS[r - 1] == x) || (r + 1 < n && NS[r + 1] == x)) ? 0x80000000u : 0u;
}

// Step 2 from the parent's order: the mod-0 positions of P, in order, with
// their symbols (ties of the symbol then need the rank of the next suffix),
// flagged by repeat_flag for the merge.
__global__ __launch_bounds__(kBlock) void k_po0_count(const int32_t *__restrict__ P, uint32_t n, uint32_t groups,
                                                      uint32_t *__restrict__ counts) {
    __shared__ uint32_t s_tmp[kBlock / kWave];
    uint32_t t0, t1;
    group_tiles(n, groups, blockIdx.x, &t0, &t1);
    uint32_t c = 0;
    for (uint32_t r = t0 * kScanTile + threadIdx.x; r < min(n, t1 * kScanTile); r += kBlock)
        c += ((uint32_t)P[r] % 3u) == 0u;
    uint32_t tot;
    dev::block_exclusive_sum(c, s_tmp, &tot);
    if (threadIdx.x == 0) counts[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_po0_write(const int32_t *__restrict__ P, const uint32_t *__restrict__ NS,
                                                      Dims d, uint32_t groups, const uint32_t *__restrict__ counts,
                                                      uint32_t *__restrict__ pos0, uint32_t *__restrict__ sym0) {
    __shared__ uint32_t s_tmp[kBlock / kWave];
    uint32_t t0, t1;
    group_tiles(d.n, groups, blockIdx.x, &t0, &t1);
    uint32_t base = counts[blockIdx.x];
    for (uint32_t tile = t0; tile < t1; ++tile) {
        const uint32_t r0 = tile * kScanTile + threadIdx.x * kScanItems;
        uint32_t p[kScanItems];
        bool keep[kScanItems];
        uint32_t c = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            p[i] = r0 + i < d.n ? (uint32_t)P[r0 + i] : 1u;
            keep[i] = (p[i] % 3u) == 0u;
            c += keep[i];
        }
        uint32_t tot;
        uint32_t j = base + dev::block_exclusive_sum(c, s_tmp, &tot);
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            if (keep[i]) {
                if (j < d.n0) {
                    const uint32_t x = NS[r0 + i];
                    pos0[j] = p[i];
                    sym0[j] = x | repeat_flag(NS, d.n, r0 + i, x);   // the flag only matters to the merge
                }
                ++j;
            }
        }
        base += tot;
    }
}

// Keys of the Step 2 subset: (t_j, rank of suffix j + 1) for mod-0 position j.
__global__ __launch_bounds__(kBlock) void k_po0_keys(const uint32_t *__restrict__ sym0,
                                                     const uint32_t *__restrict__ sub_slot,
                                                     const uint32_t *__restrict__ sub_pos, uint32_t ms,
                                                     const int32_t *__restrict__ rank12, Dims d,
                                                     uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    for (uint32_t j = blockIdx.x * kBlock + threadIdx.x; j < ms; j += gridDim.x * kBlock) {
        const uint32_t p = sub_pos[j];
        const uint32_t q = min(p / 3u, d.n0 - 1u);   // R-index of position p + 1 (the padding position when p + 1 = n)
        keys[j] = ((uint64_t)sym0[min(sub_slot[j], d.n0 - 1u)] << 32) | (uint32_t)rank12[q];
        vals[j] = p;
    }
}

__global__ __launch_bounds__(kBlock) void k_po0_place(const uint32_t *__restrict__ vals,
                                                      const uint32_t *__restrict__ sub_slot, uint32_t ms, uint32_t n0,
                                                      uint32_t *__restrict__ pos0) {
    for (uint32_t j = blockIdx.x * kBlock + threadIdx.x; j < ms; j += gridDim.x * kBlock) {
        const uint32_t k = sub_slot[j];
        if (k < n0) pos0[k] = vals[j];
    }
}

// Step 3 from the parent's order. Both merge inputs list their suffixes by
// first symbol (A by Step 2, B as the sample order), in the same order of
// symbols as the mod-0 and the sample entries of P. A suffix whose symbol
// occurs once in the text differs in its first symbol from every other
// suffix, so the merge places it by that symbol alone and needs its record
// only when the symbol repeats. symA[j] / symB[k]: the symbol of A[j] /
// B[k], with bit 31 set when the symbol occurs more than once in the text.
// symB[k] = symbol of the k-th sample entry of P, flagged (counts: the
// per-group sample counts of k_po_count, scanned). Tiles of P and NS (with
// one entry of halo on each side) are staged in LDS.
__global__ __launch_bounds__(kBlock) void k_msym_write(const int32_t *__restrict__ P, const uint32_t *__restrict__ NS,
                                                       Dims d, uint32_t groups, const uint32_t *__restrict__ counts,
                                                       uint32_t *__restrict__ symB) {
    __shared__ uint32_t s_tmp[kBlock / kWave];
    __shared__ __align__(16) uint32_t s_p[kScanTile];
    __shared__ uint32_t s_ns[kScanTile + 2];
    uint32_t t0, t1;
    group_tiles(d.n, groups, blockIdx.x, &t0, &t1);
    uint32_t base = counts[blockIdx.x];
    const uint32_t nB = d.m - d.dummy;
    for (uint32_t tile = t0; tile < t1; ++tile) {
        const uint32_t g0 = tile * kScanTile;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            const uint32_t l = i * kBlock + threadIdx.x, r = g0 + l;
            s_p[l] = r < d.n ? (uint32_t)P[r] : 0u;   // 0: a mod-0 position, dropped
            s_ns[l + 1] = r < d.n ? NS[r] : 0xffffffffu;
        }
        if (threadIdx.x == 0) s_ns[0] = g0 > 0 ? NS[g0 - 1] : 0xffffffffu;
        if (threadIdx.x == 1) s_ns[kScanTile + 1] = g0 + kScanTile < d.n ? NS[g0 + kScanTile] : 0xffffffffu;
        __syncthreads();
        const uint32_t l0 = threadIdx.x * kScanItems;
        uint32_t p[kScanItems], x[kScanItems];
#pragma unroll
        for (int h = 0; h < kScanItems / 4; ++h) {
            const uint4 a = *reinterpret_cast<const uint4 *>(&s_p[l0 + 4 * h]);
            p[4 * h] = a.x; p[4 * h + 1] = a.y; p[4 * h + 2] = a.z; p[4 * h + 3] = a.w;
        }
        uint32_t c = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            const uint32_t l = l0 + i, v = s_ns[l + 1];
            x[i] = v | ((s_ns[l] == v || s_ns[l + 2] == v) ? 0x80000000u : 0u);   // halo 0xffffffff matches no symbol
            c += (p[i] % 3u) != 0u;
        }
        uint32_t tot;
        uint32_t j = base + dev::block_exclusive_sum(c, s_tmp, &tot);
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            if ((p[i] % 3u) != 0u) {
                if (j < nB) symB[j] = x[i];
                ++j;
            }
        }
        base += tot;
        __syncthreads();   // the next tile reuses the LDS
    }
}

// ------------------------------------------------------ Step 3: merge

// A = mod-0 positions sorted (Step 2), B = sample order without the padding
// position (R-indices). Merge path: the number of A elements among the first
// `diag` outputs, by binary search inside [lo, hi] (which must hold it).
// Key of merge input element j (symbols as above; sym == nullptr: always
// from the record). pos() gives the element's text position.
template <typename RT, typename POS>
__device__ __forceinline__ Key4 merge_key(const Rec<RT> *rec, const uint32_t *sym, uint32_t j, POS pos) {
    if (sym) {
        const uint32_t x = sym[j];
        if (!(x >> 31)) {
            Key4 k;
            k.c0 = x;   // unique first symbol: every comparison ends on it
            k.c1 = k.r = k.r2cls = 0;
            return k;
        }
    }
    return key_of<RT>(rec, pos());
}

template <typename RT>
__device__ __forceinline__ uint32_t merge_split(const Rec<RT> *rec, const uint32_t *A, const int32_t *B,
                                                const uint32_t *symA, const uint32_t *symB, const Dims &d,
                                                uint32_t diag, uint32_t lo, uint32_t hi) {
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1, bj = diag - 1 - mid;
        const Key4 a = merge_key<RT>(rec, symA, mid, [&] { return min(A[mid], d.n - 1); });
        const Key4 b = merge_key<RT>(rec, symB, bj,
                                     [&] { return min(d.pos_of(min((uint32_t)B[bj], d.m - 1)), d.n - 1); });
        if (!sample_less(b, a)) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Splits at diagonals p * tile for p = 0..parts. The split is monotone in the
// diagonal, so a first launch over every kCoarse-th diagonal (coarse ==
// nullptr) bounds the searches of the second launch to one coarse interval:
// about 16 steps instead of about 30, and the coarse searches share the top
// of every later search.
constexpr uint32_t kCoarse = 64;

template <typename RT>
__global__ __launch_bounds__(kBlock) void k_merge_partition(const Rec<RT> *__restrict__ rec,
                                                            const uint32_t *__restrict__ A, uint32_t nA,
                                                            const int32_t *__restrict__ B, uint32_t nB,
                                                            Dims d, uint32_t parts, uint64_t tile,
                                                            const uint32_t *__restrict__ coarse, uint32_t cparts,
                                                            const uint32_t *__restrict__ symA,
                                                            const uint32_t *__restrict__ symB,
                                                            uint32_t *__restrict__ split) {
    const uint32_t p = blockIdx.x * kBlock + threadIdx.x;
    if (p > parts) return;
    const uint32_t diag = (uint32_t)min<uint64_t>((uint64_t)p * tile, (uint64_t)nA + nB);
    const uint32_t lo0 = diag > nB ? diag - nB : 0u, hi0 = min(diag, nA);
    uint32_t lo = lo0, hi = hi0;
    if (coarse) {
        const uint32_t c = p / kCoarse;
        lo = min(max(lo0, coarse[c]), hi0);
        hi = max(min(hi0, coarse[min(c + 1, cparts)]), lo);
    }
    split[p] = merge_split<RT>(rec, A, B, symA, symB, d, diag, lo, hi);
}

template <typename RT, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_merge(const Rec<RT> *__restrict__ rec,
                                                  const uint32_t *__restrict__ A, uint32_t nA,
                                                  const int32_t *__restrict__ B, uint32_t nB, Dims d,
                                                  const uint32_t *__restrict__ split,
                                                  const uint32_t *__restrict__ symA,
                                                  const uint32_t *__restrict__ symB, int32_t *__restrict__ sa) {
    constexpr uint32_t kMergeTile = kBlock * ITEMS;
    __shared__ Key4 s_key[kMergeTile];
    __shared__ uint32_t s_pos[kMergeTile];
    __shared__ int32_t s_out[kMergeTile];
    const uint32_t total = nA + nB;
    const uint32_t d0 = blockIdx.x * kMergeTile;
    const uint32_t d1 = min(total, d0 + kMergeTile);
    const uint32_t a0 = split[blockIdx.x], a1 = split[blockIdx.x + 1];
    // A consistent comparator gives monotone splits; anything else stops the
    // workgroup before it can index outside A or B (block-uniform exit).
    if (a0 > a1 || a1 > nA || a0 > d0 || a1 > d1 || d0 - a0 > nB || d1 - a1 > nB || d1 - a1 < d0 - a0) return;
    const uint32_t b0 = d0 - a0, b1 = d1 - a1;
    const uint32_t na = a1 - a0, nb = b1 - b0, cnt = d1 - d0;
    for (uint32_t i = threadIdx.x; i < cnt; i += kBlock) {
        uint32_t pos;
        if (i < na) pos = A[a0 + i];
        else pos = d.pos_of(min((uint32_t)B[b0 + (i - na)], d.m - 1));
        pos = min(pos, d.n - 1);
        s_pos[i] = pos;
        s_key[i] = i < na ? merge_key<RT>(rec, symA, a0 + i, [&] { return pos; })
                          : merge_key<RT>(rec, symB, b0 + (i - na), [&] { return pos; });
    }
    __syncthreads();
    const Key4 *sA = s_key;
    const Key4 *sB = s_key + na;
    const uint32_t diag = min(cnt, threadIdx.x * (uint32_t)ITEMS);
    const uint32_t dend = min(cnt, diag + (uint32_t)ITEMS);
    uint32_t lo = diag > nb ? diag - nb : 0u, hi = min(diag, na);
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (!sample_less(sB[diag - 1 - mid], sA[mid])) lo = mid + 1; else hi = mid;
    }
    uint32_t ia = lo, ib = diag - lo;
    for (uint32_t o = diag; o < dend; ++o) {
        bool take_a;
        if (ia >= na) take_a = false;
        else if (ib >= nb) take_a = true;
        else take_a = !sample_less(sB[ib], sA[ia]);
        if (take_a) { s_out[o] = (int32_t)s_pos[ia]; ++ia; }
        else { s_out[o] = (int32_t)s_pos[na + ib]; ++ib; }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < cnt; i += kBlock) sa[d0 + i] = s_out[i];
}

// ------------------------------------------------------------- driver

struct HostHdr {
    uint32_t error;
    uint32_t maxname;
};

// Replayed launch sequences: flag the header when a count the host decided
// on (header word `word`) differs from the recorded one (lane 0 stores;
// vector memory only).
__global__ __launch_bounds__(kWave) void k_expect_names(uint32_t *hdr, int word, uint32_t expected) {
    if (threadIdx.x == 0 && hdr[word] != expected) hdr[kStaleWord] = 1u;
}

thread_local DecisionTape *t_tape = nullptr;

// A count the host needs to size launches (header word `word`): read back,
// or under a replayed launch sequence taken from the tape and checked on the
// device.
lor_status decided_count(uint32_t *hdr, int word, uint32_t *out, hipStream_t s) {
    DecisionTape *tape = t_tape;
    if (tape && tape->replay) {
        if (tape->next >= tape->names.size()) {
            set_error("internal: launch sequence longer than the recorded one");
            return LOR_EINVAL;
        }
        *out = tape->names[tape->next++];
        LOR_LAUNCH("k_expect_names", 8.0, s,
                   hipLaunchKernelGGL(k_expect_names, dim3(1), dim3(kWave), 0, s, hdr, word, *out));
        return LOR_OK;
    }
    LOR_HIP(hipMemcpyAsync(out, hdr + word, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    LOR_HIP(hipStreamSynchronize(s));
    if (tape) tape->names.push_back(*out);
    return LOR_OK;
}

enum KeyMode { KM_U32, KM_U64, KM_STAGED };

// Step 3 launches: coarse then fine merge-path splits, then the merge.
struct MergeArgs {
    const uint32_t *A;
    uint32_t nA;
    const int32_t *B;
    uint32_t nB;
    Dims d;
    uint32_t parts, cparts, mtile;
    int mitems;
    uint32_t *csplit, *split;
    const uint32_t *symA, *symB;
    int32_t *sa;
};

template <typename RT>
lor_status launch_merge(const Rec<RT> *rec, const MergeArgs &m, hipStream_t s) {
    LOR_LAUNCH("k_merge_partition", (double)(m.cparts + 1) * 4, s,
               hipLaunchKernelGGL(k_merge_partition<RT>, dim3(div_up(m.cparts + 1, kBlock)), dim3(kBlock), 0, s, rec,
                                  m.A, m.nA, m.B, m.nB, m.d, m.cparts, (uint64_t)m.mtile * kCoarse, nullptr, 0u, m.symA,
                                  m.symB, m.csplit));
    LOR_LAUNCH("k_merge_partition", (double)(m.parts + 1) * 4, s,
               hipLaunchKernelGGL(k_merge_partition<RT>, dim3(div_up(m.parts + 1, kBlock)), dim3(kBlock), 0, s, rec,
                                  m.A, m.nA, m.B, m.nB, m.d, m.parts, (uint64_t)m.mtile, m.csplit, m.cparts, m.symA,
                                  m.symB, m.split));
    const double mbytes = (double)m.d.n * (4 + 4 + sizeof(Rec<RT>));
    switch (m.mitems) {
        case 4:
            LOR_LAUNCH("k_merge", mbytes, s,
                       hipLaunchKernelGGL((k_merge<RT, 4>), dim3(m.parts), dim3(kBlock), 0, s, rec, m.A, m.nA, m.B,
                                          m.nB, m.d, m.split, m.symA, m.symB, m.sa));
            break;
        case 12:
            LOR_LAUNCH("k_merge", mbytes, s,
                       hipLaunchKernelGGL((k_merge<RT, 12>), dim3(m.parts), dim3(kBlock), 0, s, rec, m.A, m.nA, m.B,
                                          m.nB, m.d, m.split, m.symA, m.symB, m.sa));
            break;
        default:
            LOR_LAUNCH("k_merge", mbytes, s,
                       hipLaunchKernelGGL((k_merge<RT, 8>), dim3(m.parts), dim3(kBlock), 0, s, rec, m.A, m.nA, m.B,
                                          m.nB, m.d, m.split, m.symA, m.symB, m.sa));
            break;
    }
    return LOR_OK;
}

template <typename CH>
lor_status dc3_level(const CH *t, uint32_t n, uint32_t alphabet, int32_t *sa, Arena &ar, uint32_t *hdr,
                     hipStream_t s, int depth, const uint32_t *pnames) {
    if (n == 0) return LOR_OK;
    if (depth > 64) {
        set_error("DC3 recursion deeper than 64 levels");
        return LOR_EINVAL;
    }
    const bool run = !ar.measuring();
    const Dims d = make_dims(n);
    const int b = bits_for(alphabet);
    const size_t mark_level = ar.mark();

    int32_t *R;        // names of the sample triples; later rank12 (rank by R-index)
    int32_t *sa12;     // sample order as R-indices
    LOR_TAKE(ar, int32_t, d.m, R);
    LOR_TAKE(ar, int32_t, d.m, sa12);

    // ---- Step 1: sort the sample triples
    const int kb = Triple<CH>::key_bits(b);
    // Sort keys of byte and int32 texts are mixed-radix, (s0 A + s1) A + s2
    // with A = alphabet + 1, when that takes fewer bits than three b-bit
    // fields (level 2 of the 1G text: 54 bits instead of 57, one radix pass
    // fewer).
    const uint64_t mixA = (uint64_t)alphabet + 1;
    int kbs = kb;
    bool mixed = false;
    if (sizeof(CH) != 2 && mixA <= (1ull << 21)) {   // A^3 < 2^63
        const int mb = bits_for(mixA * mixA * mixA - 1);
        if (mb < kb) {
            kbs = mb;
            mixed = true;
        }
    }
    KeyMode km = (kbs <= 32) ? KM_U32 : (kbs <= 64 ? KM_U64 : KM_STAGED);
    if (!run) km = KM_U64;   // measuring: the largest footprint

    // Byte and int32 texts name through mixed-radix codes (A^3 of them) with
    // word-window reads when the text is aligned for them; the pair-tagged
    // texts of the batched path keep their b-bit packed keys.
    const uint64_t A = (uint64_t)alphabet + 1;
    const bool windowed = sizeof(CH) != 2 && A <= 1625 &&   // A^3 < 2^32
                          ((uintptr_t)t % (sizeof(CH) == 1 ? 4 : 16)) == 0;
    const uint64_t code_space = windowed ? A * A * A : (kb <= 24 ? (1ull << kb) : ~0ull);
    const bool use_table = run && code_space <= (1ull << 24) && code_space <= 2ull * d.m + 65536ull;
    // Order from the parent (see k_po_write): this level's text is the
    // parent's names, so when at least 7/8 of the n symbols are distinct,
    // at most 2 (n - alphabet) <= n / 4 positions share their first symbol
    // with another and go through the sort.
    const bool parent_order = run && sizeof(CH) == 4 && pnames != nullptr && !use_table && d.m >= 2 &&
                              (uint64_t)alphabet * 8 >= (uint64_t)n * 7;
    // Names of the sorted triples in sorted order, kept through the recursion
    // for the child level's order (levels that sort keep them).
    uint32_t *keep = nullptr;
    if (!use_table) LOR_TAKE(ar, uint32_t, d.m, keep);
    const size_t mark_tmp = ar.mark();

    uint32_t *counts;
    LOR_TAKE(ar, uint32_t, radix_counts_words(d.m) + kMaxScanGroups + 64, counts);
    uint32_t *gcount = counts + radix_counts_words(d.m);
    uint32_t *tmpv;
    LOR_TAKE(ar, uint32_t, d.m, tmpv);
    const int passes = d.m <= 1 ? 0
                       : (km == KM_STAGED ? radix_passes(0, 2 * b) + radix_passes(32, 32 + b) : radix_passes(0, kbs));
    uint32_t *v0 = (passes % 2 == 0) ? (uint32_t *)sa12 : tmpv;
    uint32_t *v1 = (passes % 2 == 0) ? tmpv : (uint32_t *)sa12;
    const uint32_t g_el = grid_for(d.m);
    uint32_t hmax = 0;

    // Subset of the parent-order path: at most n / 4 entries (see above).
    const uint32_t ms_cap = min(d.m, d.n / 4u + 2u);
    if (parent_order || !run) {
        const size_t mk = ar.mark();
        uint32_t *s0v, *flag, *x4, *sub_slot, *sub_idx;
        LOR_TAKE(ar, uint32_t, d.m, s0v);
        LOR_TAKE(ar, uint32_t, d.m, flag);
        LOR_TAKE(ar, uint32_t, d.m, x4);
        LOR_TAKE(ar, uint32_t, ms_cap, sub_slot);
        LOR_TAKE(ar, uint32_t, ms_cap, sub_idx);
        const uint32_t Gn = scan_groups(d.n), Gm = scan_groups(d.m);
        if (run) {
            LOR_LAUNCH("k_po_count", 4.0 * d.n, s,
                       hipLaunchKernelGGL(k_po_count, dim3(Gn), dim3(kBlock), 0, s, sa, d.n, Gn, gcount));
            LOR_TRY(scan_block_totals(gcount, Gn, nullptr, s));
            LOR_LAUNCH("k_po_write", 8.0 * d.n + 8.0 * d.m, s,
                       hipLaunchKernelGGL(k_po_write, dim3(Gn), dim3(kBlock), 0, s, sa, pnames, d, Gn, gcount, sa12,
                                          s0v));
            LOR_LAUNCH("k_po_runs_count", 4.0 * d.m, s,
                       hipLaunchKernelGGL(k_po_runs_count, dim3(Gm), dim3(kBlock), 0, s, s0v, d.m, Gm, gcount));
            LOR_TRY(scan_block_totals(gcount, Gm, hdr + 3, s));
            LOR_LAUNCH("k_po_runs_write", 8.0 * d.m, s,
                       hipLaunchKernelGGL(k_po_runs_write, dim3(Gm), dim3(kBlock), 0, s, s0v, sa12, d.m, Gm, gcount,
                                          ms_cap, sub_slot, sub_idx, flag));
        }
        uint32_t ms = ms_cap;
        if (run) {
            LOR_TRY(decided_count(hdr, 3, &ms, s));
            if (ms > ms_cap) {
                set_error("internal: %u of %u sample triples share a first symbol (at most %u expected)", ms, d.m,
                          ms_cap);
                return LOR_EINVAL;
            }
        }
        if (ms > 0) {
            uint64_t *sk0, *sk1;
            uint32_t *sv0, *sv1, *saux, *scnt;
            LOR_TAKE(ar, uint64_t, ms, sk0);
            LOR_TAKE(ar, uint64_t, ms, sk1);
            LOR_TAKE(ar, uint32_t, ms, sv0);
            LOR_TAKE(ar, uint32_t, ms, sv1);
            LOR_TAKE(ar, uint32_t, ms, saux);
            LOR_TAKE(ar, uint32_t, radix_counts_words(ms) + kMaxScanGroups + 64, scnt);
            if (run) {
                uint32_t *sg = scnt + radix_counts_words(ms);
                uint64_t *kc = sk0, *ka = sk1;
                uint32_t *vc = sv0, *va = sv1;
                bool alt = false;
                auto swap_if = [&](bool x) {
                    if (x) {
                        uint64_t *y = kc; kc = ka; ka = y;
                        uint32_t *z = vc; vc = va; va = z;
                    }
                };
                LOR_LAUNCH("k_po_keys", 12.0 * ms, s,
                           hipLaunchKernelGGL(k_po_keys<CH>, dim3(grid_for(ms)), dim3(kBlock), 0, s, t, d, b, sub_idx,
                                              ms, kc, vc));
                LOR_TRY(radix_sort<uint64_t>(kc, vc, ka, va, ms, 0, 2 * b, scnt, s, &alt));
                swap_if(alt);
                const uint32_t Gs = scan_groups(ms);
                LOR_LAUNCH("k_name_count", (double)ms * 8, s,
                           hipLaunchKernelGGL(k_name_count<uint64_t>, dim3(Gs), dim3(kBlock), 0, s, kc, ms, Gs, sg));
                LOR_TRY(scan_block_totals(sg, Gs, nullptr, s));
                LOR_LAUNCH("k_name_write", (double)ms * 12, s,
                           hipLaunchKernelGGL(k_name_write<uint64_t>, dim3(Gs), dim3(kBlock), 0, s, kc, ms, Gs, sg,
                                              saux));
                Dims ds = d;
                ds.m = ms;   // k_pair_rekey walks the subset
                LOR_LAUNCH("k_pair_rekey", (double)ms * 16 + (double)ms * sizeof(CH), s,
                           hipLaunchKernelGGL(k_pair_rekey<CH>, dim3(grid_for(ms)), dim3(kBlock), 0, s, t, ds, vc, saux,
                                              kc));
                LOR_TRY(radix_sort<uint64_t>(kc, vc, ka, va, ms, 32, 32 + b, scnt, s, &alt));
                swap_if(alt);
                LOR_LAUNCH("k_po_place", 20.0 * ms, s,
                           hipLaunchKernelGGL(k_po_place, dim3(grid_for(ms)), dim3(kBlock), 0, s, kc, vc, sub_slot, ms,
                                              d.m, sa12, flag));
            }
        }
        if (run) {
            LOR_LAUNCH("k_flag_count", 4.0 * d.m, s,
                       hipLaunchKernelGGL(k_flag_count, dim3(Gm), dim3(kBlock), 0, s, flag, d.m, Gm, gcount));
            LOR_TRY(scan_block_totals(gcount, Gm, hdr + 1, s));
            LOR_LAUNCH("k_flag_write", 8.0 * d.m, s,
                       hipLaunchKernelGGL(k_flag_write, dim3(Gm), dim3(kBlock), 0, s, flag, d.m, Gm, gcount, keep));
            uint32_t *const tmp4[4] = {s0v, flag, tmpv, x4};
            LOR_TRY(bucketed_scatter(R, d.m, (const uint32_t *)sa12, keep, 0, d.m, tmp4, counts, s, true));
        } else {
            ar.release(mk);   // measuring: the sort branch below is measured too
        }
    }
    if (parent_order) {
        // named above
    } else if (use_table) {
        const uint32_t words = max(1u, (uint32_t)div_up(code_space, 32));
        uint32_t *bitmap, *below, *stmp;
        LOR_TAKE(ar, uint32_t, words, bitmap);
        LOR_TAKE(ar, uint32_t, words, below);
        LOR_TAKE(ar, uint32_t, kScanTmpWords, stmp);
        LOR_TRY(zero_words(bitmap, words, s));
        if constexpr (sizeof(CH) != 2) if (windowed) {
            const size_t lds_max = max_lds_per_block();
            const size_t pres_lds = (size_t)words * 4, name_lds = 4 * ((size_t)words + div_up(words, 4));
            const int pres_in = pres_lds <= lds_max, name_in = name_lds <= lds_max;
            const uint32_t groups = div_up(d.n0, kWinQ);
            const uint32_t full = max(1u, div_up(groups, (uint32_t)kTblBlock));
            const uint32_t gp = pres_in ? min(full, pres_lds <= 32768 ? 1024u : 256u) : full;
            const uint32_t gn = name_in ? min(full, name_lds <= 32768 ? 1024u : 256u) : full;
            if (pres_in)
                LOR_LAUNCH("k_presence", (double)n * sizeof(CH), s,
                           hipLaunchKernelGGL((k_presence_w<CH, true>), dim3(gp), dim3(kTblBlock), pres_lds, s, t, d,
                                              (uint32_t)A, bitmap, words));
            else
                LOR_LAUNCH("k_presence", (double)n * sizeof(CH), s,
                           hipLaunchKernelGGL((k_presence_w<CH, false>), dim3(gp), dim3(kTblBlock), 0, s, t, d,
                                              (uint32_t)A, bitmap, words));
            LOR_LAUNCH("k_popc", 8.0 * words, s,
                       hipLaunchKernelGGL(k_popc, dim3(grid_for(words)), dim3(kBlock), 0, s, bitmap, words, below));
            LOR_TRY(scan_exclusive(below, words, stmp, hdr + 1, s));
            LOR_LAUNCH("k_name_table", (double)n * sizeof(CH) + 4.0 * d.m, s,
                       hipLaunchKernelGGL(k_name_table_w<CH>, dim3(gn), dim3(kTblBlock), name_in ? name_lds : 0, s,
                                          t, d, (uint32_t)A, bitmap, below, words, name_in, R));
        }
        if (!windowed) {
            const int in_lds = words <= 8192;
            if (sizeof(CH) == 2 && !in_lds)
                LOR_LAUNCH("k_presence", (double)n * sizeof(CH), s,
                           hipLaunchKernelGGL(k_presence_tagged, dim3(div_up(d.n0, kTagQ)), dim3(kBlock), 0, s,
                                              reinterpret_cast<const uint16_t *>(t), d, b, bitmap, words));
            else
                LOR_LAUNCH("k_presence", (double)n * sizeof(CH), s,
                           hipLaunchKernelGGL(k_presence<CH>, dim3(in_lds ? min(grid_for(d.m), 2048u) : grid_for(d.m)),
                                              dim3(kBlock), in_lds ? words * 4 : 0, s, t, d, b, bitmap, words, in_lds));
            LOR_LAUNCH("k_popc", 8.0 * words, s,
                       hipLaunchKernelGGL(k_popc, dim3(grid_for(words)), dim3(kBlock), 0, s, bitmap, words, below));
            LOR_TRY(scan_exclusive(below, words, stmp, hdr + 1, s));
            LOR_LAUNCH("k_name_table", (double)n * sizeof(CH) + 4.0 * d.m, s,
                       hipLaunchKernelGGL(k_name_table<CH>, dim3(g_el), dim3(kBlock), 0, s, t, d, b, bitmap, below,
                                          words, R));
        }
    } else if (km != KM_U32) {
        // 64-bit keys: whole triples, or (for wide symbols) two stages.
        uint64_t *k0, *k1;
        uint32_t *aux;
        LOR_TAKE(ar, uint64_t, d.m, k0);
        LOR_TAKE(ar, uint64_t, d.m, k1);
        LOR_TAKE(ar, uint32_t, d.m, aux);
        if (!run) {
            // the bitmap path may take up to 2 x (2m + 65536) / 32 words plus scan space
            uint8_t *extra;
            LOR_TAKE(ar, uint8_t, (size_t)d.m / 2 + 16384 + kScanTmpWords * 4 + 1024, extra);
        }
        if (run) {
            uint64_t *kc = k0, *ka = k1;
            uint32_t *vc = v0, *va = v1;
            bool alt = false;
            auto swap_if = [&](bool x) {
                if (x) {
                    uint64_t *y = kc; kc = ka; ka = y;
                    uint32_t *z = vc; vc = va; va = z;
                }
            };
            const uint32_t G = scan_groups(d.m);
            if (km == KM_U64) {
                LOR_LAUNCH("k_sample_keys", (double)d.m * 12 + (double)n * sizeof(CH), s,
                           hipLaunchKernelGGL((k_sample_keys<CH, uint64_t>), dim3(g_el), dim3(kBlock), 0, s, t, d, b,
                                              0, mixed ? mixA : 0ull, kc, vc));
                LOR_TRY(radix_sort<uint64_t>(kc, vc, ka, va, d.m, 0, kbs, counts, s, &alt));
                swap_if(alt);
            } else {
                // stage A: sort the pairs (t_{i+1}, t_{i+2}) and rank them
                LOR_LAUNCH("k_sample_keys", (double)d.m * 12 + (double)n * sizeof(CH), s,
                           hipLaunchKernelGGL((k_sample_keys<CH, uint64_t>), dim3(g_el), dim3(kBlock), 0, s, t, d, b,
                                              1, 0ull, kc, vc));
                LOR_TRY(radix_sort<uint64_t>(kc, vc, ka, va, d.m, 0, 2 * b, counts, s, &alt));
                swap_if(alt);
                LOR_LAUNCH("k_name_count", (double)d.m * 8, s,
                           hipLaunchKernelGGL(k_name_count<uint64_t>, dim3(G), dim3(kBlock), 0, s, kc, d.m, G,
                                              gcount));
                LOR_TRY(scan_block_totals(gcount, G, nullptr, s));
                LOR_LAUNCH("k_name_write", (double)d.m * 12, s,
                           hipLaunchKernelGGL(k_name_write<uint64_t>, dim3(G), dim3(kBlock), 0, s, kc, d.m, G, gcount,
                                              aux));
                // stage B: (t_i, pair rank), sorted on t_i (stable)
                LOR_LAUNCH("k_pair_rekey", (double)d.m * 16 + (double)d.m * sizeof(CH), s,
                           hipLaunchKernelGGL(k_pair_rekey<CH>, dim3(g_el), dim3(kBlock), 0, s, t, d, vc, aux, kc));
                LOR_TRY(radix_sort<uint64_t>(kc, vc, ka, va, d.m, 32, 32 + b, counts, s, &alt));
                swap_if(alt);
            }
            if (vc != (uint32_t *)sa12) {
                set_error("internal: sorted sample order not in its buffer");
                return LOR_EINVAL;
            }
            // names go to `keep`; scatter buffers: ka (2 x m words), va, and kc once the names are out
            uint32_t *names = keep;
            uint32_t *const tmp4[4] = {reinterpret_cast<uint32_t *>(ka), va, reinterpret_cast<uint32_t *>(kc),
                                       reinterpret_cast<uint32_t *>(kc) + d.m};
            LOR_LAUNCH("k_name_count", (double)d.m * 8, s,
                       hipLaunchKernelGGL(k_name_count<uint64_t>, dim3(G), dim3(kBlock), 0, s, kc, d.m, G, gcount));
            LOR_TRY(scan_block_totals(gcount, G, hdr + 1, s));
            LOR_LAUNCH("k_name_write", (double)d.m * 12, s,
                       hipLaunchKernelGGL(k_name_write<uint64_t>, dim3(G), dim3(kBlock), 0, s, kc, d.m, G, gcount,
                                          names));
            LOR_TRY(bucketed_scatter(R, d.m, (const uint32_t *)sa12, names, 0, d.m, tmp4, counts, s, true));
        }
    } else {
        uint32_t *k0, *k1, *aux, *aux2;
        LOR_TAKE(ar, uint32_t, d.m, k0);
        LOR_TAKE(ar, uint32_t, d.m, k1);
        LOR_TAKE(ar, uint32_t, d.m, aux);
        LOR_TAKE(ar, uint32_t, d.m, aux2);
        if (run) {
            bool alt = false;
            uint32_t *kc = k0, *ka = k1, *vc = v0, *va = v1;
            LOR_LAUNCH("k_sample_keys", (double)d.m * 8 + (double)n * sizeof(CH), s,
                       hipLaunchKernelGGL((k_sample_keys<CH, uint32_t>), dim3(g_el), dim3(kBlock), 0, s, t, d, b, 0,
                                          mixed ? mixA : 0ull, kc, vc));
            LOR_TRY(radix_sort<uint32_t>(kc, vc, ka, va, d.m, 0, kbs, counts, s, &alt));
            if (alt) {
                uint32_t *x = kc; kc = ka; ka = x;
                x = vc; vc = va; va = x;
            }
            if (vc != (uint32_t *)sa12) {
                set_error("internal: sorted sample order not in its buffer");
                return LOR_EINVAL;
            }
            uint32_t *names = keep;
            uint32_t *const tmp4[4] = {va, aux, aux2, kc};   // kc is free once the names are out
            const uint32_t G = scan_groups(d.m);
            LOR_LAUNCH("k_name_count", (double)d.m * 4, s,
                       hipLaunchKernelGGL(k_name_count<uint32_t>, dim3(G), dim3(kBlock), 0, s, kc, d.m, G, gcount));
            LOR_TRY(scan_block_totals(gcount, G, hdr + 1, s));
            LOR_LAUNCH("k_name_write", (double)d.m * 8, s,
                       hipLaunchKernelGGL(k_name_write<uint32_t>, dim3(G), dim3(kBlock), 0, s, kc, d.m, G, gcount,
                                          names));
            LOR_TRY(bucketed_scatter(R, d.m, (const uint32_t *)sa12, names, 0, d.m, tmp4, counts, s, true));
        }
    }

    bool unique = true;
    if (run) {
        HostHdr h;
        DecisionTape *tape = decision_tape();
        if (tape && tape->replay) {
            if (tape->next >= tape->names.size()) {
                set_error("internal: launch sequence longer than the recorded one");
                return LOR_EINVAL;
            }
            h.error = 0;
            h.maxname = tape->names[tape->next++];
            LOR_LAUNCH("k_expect_names", 8.0, s,
                       hipLaunchKernelGGL(k_expect_names, dim3(1), dim3(kWave), 0, s, hdr, 1, h.maxname));
        } else {
            LOR_HIP(hipMemcpyAsync(&h, hdr, sizeof(h), hipMemcpyDeviceToHost, s));
            LOR_HIP(hipStreamSynchronize(s));
            if (tape) tape->names.push_back(h.maxname);
        }
        if (h.error) {
            set_error("input base outside 0..3");
            return LOR_EALPHABET;
        }
        hmax = h.maxname;
        if (hmax > d.m || hmax == 0) {
            set_error("internal: %u names for %u sample triples", hmax, d.m);
            return LOR_EINVAL;
        }
        unique = (hmax == d.m);
        if (trace_on())
            fprintf(stderr, "[lor] dc3 level %d: n=%u m=%u bits/sym=%d %s passes=%d names=%u%s\n", depth, n, d.m, b,
                    use_table      ? "bitmap-naming"
                    : parent_order ? "parent-order"
                    : (km == KM_U32 ? "sort-u32" : km == KM_U64 ? "sort-u64" : "sort-2stage"),
                    use_table || parent_order ? 0 : passes, hmax, unique ? " unique" : "");
        if (unique && use_table)
            LOR_LAUNCH("k_sa12_from_names", 12.0 * d.m, s,
                       hipLaunchKernelGGL(k_sa12_from_names, dim3(g_el), dim3(kBlock), 0, s, R, d.m, sa12));
    } else {
        unique = d.m < 2;
        hmax = d.m;
    }
    ar.release(mark_tmp);

    if (!unique) {
        // the child reads this level's sorted order (sa12) and names (keep) before its merge writes sa12
        LOR_TRY(dc3_level<int32_t>(R, d.m, hmax, sa12, ar, hdr, s, depth + 1, keep));
        // rank12[sa12[r]] = r + 1, as a bucketed scatter
        const size_t mk = ar.mark();
        uint32_t *tb[4], *cr;
        for (int i = 0; i < 4; ++i) LOR_TAKE(ar, uint32_t, d.m, tb[i]);
        LOR_TAKE(ar, uint32_t, radix_counts_words(d.m), cr);
        if (run) LOR_TRY(bucketed_scatter(R, d.m, (const uint32_t *)sa12, nullptr, 1, d.m, tb, cr, s, true));
        ar.release(mk);
    }
    const int32_t *rank12 = R;

    // ---- records for the merge, and Step 2's (slot, first symbol) pairs
    Rec<CH> *rec;
    LOR_TAKE(ar, Rec<CH>, (size_t)d.n0 + 1, rec);
    uint32_t *keys0, *vals0, *keys1, *vals1, *sc0, *sc1, *counts2;
    LOR_TAKE(ar, uint32_t, d.n0, keys0);
    LOR_TAKE(ar, uint32_t, d.n0, vals0);
    // records in one uint4 when every symbol fits a byte (sized above for the wide form)
    const bool narrow_rec = sizeof(CH) == 1 || (sizeof(CH) == 4 && alphabet <= 255u);
    Rec<uint8_t> *rec8 = reinterpret_cast<Rec<uint8_t> *>(rec);
    if (run) {
        const double rbytes = (double)(d.n0 + 1) * ((narrow_rec ? sizeof(Rec<uint8_t>) : sizeof(Rec<CH>)) + 12) +
                              (double)n * sizeof(CH) + (parent_order ? 0.0 : 8.0 * d.n0);
        if (narrow_rec)
            LOR_LAUNCH("k_records", rbytes, s,
                       hipLaunchKernelGGL((k_records<CH, uint8_t>), dim3(grid_for(d.n0 + 1)), dim3(kBlock), 0, s, t,
                                          d, rank12, rec8, parent_order ? nullptr : keys0,
                                          parent_order ? nullptr : vals0));
        else
            LOR_LAUNCH("k_records", rbytes, s,
                       hipLaunchKernelGGL((k_records<CH, CH>), dim3(grid_for(d.n0 + 1)), dim3(kBlock), 0, s, t, d,
                                          rank12, rec, parent_order ? nullptr : keys0, parent_order ? nullptr : vals0));
    }

    // ---- Step 2: mod-0 suffixes
    LOR_TAKE(ar, uint32_t, d.n0, keys1);
    LOR_TAKE(ar, uint32_t, d.n0, vals1);
    LOR_TAKE(ar, uint32_t, d.n0, sc0);
    LOR_TAKE(ar, uint32_t, d.n0, sc1);
    LOR_TAKE(ar, uint32_t, radix_counts_words(d.n0) + kMaxScanGroups + 64, counts2);
    uint32_t *gcount2 = counts2 + radix_counts_words(d.n0);
    const int mitems = plan().merge_items;
    const uint32_t mtile = kBlock * (uint32_t)mitems;
    const uint32_t parts = div_up(n, mtile);
    uint32_t *split, *csplit;   // sized for the smallest merge tile, so the workspace does not depend on the plan
    LOR_TAKE(ar, uint32_t, (size_t)div_up(n, kBlock * 4) + 2, split);
    LOR_TAKE(ar, uint32_t, (size_t)div_up(n, kBlock * 4 * kCoarse) + 2, csplit);
    // Step 2 from the parent's order (see k_po0_write): the subset of mod-0
    // positions whose symbol repeats among them is sorted by (symbol, rank of
    // the next suffix) and put back into its slots.
    const uint32_t ms0_cap = min(d.n0, d.n / 4u + 2u);
    uint32_t *sub0_slot = nullptr, *sub0_pos = nullptr;
    uint32_t *symA = nullptr, *symB = nullptr;   // merge symbols (see k_msym_write); symA is Step 2's vals0
    if (parent_order || !run) {
        LOR_TAKE(ar, uint32_t, ms0_cap, sub0_slot);
        LOR_TAKE(ar, uint32_t, ms0_cap, sub0_pos);
        LOR_TAKE(ar, uint32_t, d.m, symB);
    }
    if (parent_order) {
        const uint32_t Gn = scan_groups(d.n), G0 = scan_groups(d.n0);
        LOR_LAUNCH("k_po_count", 4.0 * d.n, s,
                   hipLaunchKernelGGL(k_po0_count, dim3(Gn), dim3(kBlock), 0, s, sa, d.n, Gn, gcount2));
        LOR_TRY(scan_block_totals(gcount2, Gn, nullptr, s));
        LOR_LAUNCH("k_po_write", 4.0 * d.n + 8.0 * d.n0, s,   // NS read for the kept third only
                   hipLaunchKernelGGL(k_po0_write, dim3(Gn), dim3(kBlock), 0, s, sa, pnames, d, Gn, gcount2, keys0,
                                      vals0));
        LOR_LAUNCH("k_po_runs_count", 4.0 * d.n0, s,
                   hipLaunchKernelGGL(k_po_runs_count, dim3(G0), dim3(kBlock), 0, s, vals0, d.n0, G0, gcount2));
        LOR_TRY(scan_block_totals(gcount2, G0, hdr + 2, s));
        LOR_LAUNCH("k_po_runs_write", 8.0 * d.n0, s,
                   hipLaunchKernelGGL(k_po_runs_write, dim3(G0), dim3(kBlock), 0, s, vals0,
                                      reinterpret_cast<const int32_t *>(keys0), d.n0, G0, gcount2, ms0_cap, sub0_slot,
                                      sub0_pos, (uint32_t *)nullptr));
    }
    uint32_t ms0 = 0;
    if (parent_order) {
        LOR_TRY(decided_count(hdr, 2, &ms0, s));
        if (ms0 > ms0_cap) {
            set_error("internal: %u of %u mod-0 suffixes share a first symbol (at most %u expected)", ms0, d.n0,
                      ms0_cap);
            return LOR_EINVAL;
        }
    } else if (!run) {
        ms0 = ms0_cap;
    }
    if (ms0 > 0) {
        uint64_t *zk0, *zk1;
        uint32_t *zv0, *zv1, *zcnt;
        LOR_TAKE(ar, uint64_t, ms0, zk0);
        LOR_TAKE(ar, uint64_t, ms0, zk1);
        LOR_TAKE(ar, uint32_t, ms0, zv0);
        LOR_TAKE(ar, uint32_t, ms0, zv1);
        LOR_TAKE(ar, uint32_t, radix_counts_words(ms0), zcnt);
        if (run) {
            LOR_LAUNCH("k_po_keys", 20.0 * ms0, s,
                       hipLaunchKernelGGL(k_po0_keys, dim3(grid_for(ms0)), dim3(kBlock), 0, s, vals0, sub0_slot,
                                          sub0_pos, ms0, rank12, d, zk0, zv0));
            bool zalt;
            LOR_TRY(radix_sort<uint64_t>(zk0, zv0, zk1, zv1, ms0, 0, 32 + b, zcnt, s, &zalt));
            LOR_LAUNCH("k_po_place", 12.0 * ms0, s,
                       hipLaunchKernelGGL(k_po0_place, dim3(grid_for(ms0)), dim3(kBlock), 0, s, zalt ? zv1 : zv0,
                                          sub0_slot, ms0, d.n0, keys0));
        }
    }
    if (run) {
        const uint32_t *A;
        if (parent_order) {
            A = keys0;
        } else {
            // first symbols of the mod-0 suffixes in sample order, into R (its
            // ranks were consumed by k_records, which also wrote these pairs)
            uint32_t *const tmp4[4] = {keys1, vals1, sc0, sc1};
            LOR_TRY(bucketed_scatter(R, d.m, keys0, vals0, 0, d.n0, tmp4, counts2, s, false));
            const uint32_t G = scan_groups(d.m);
            LOR_LAUNCH("k_ns_count", (double)d.m * 4, s,
                       hipLaunchKernelGGL(k_ns_count, dim3(G), dim3(kBlock), 0, s, sa12, d, G, gcount2));
            LOR_TRY(scan_block_totals(gcount2, G, hdr + 2, s));
            LOR_LAUNCH("k_ns_write", (double)d.m * 4 + (double)d.n0 * 12, s,
                       hipLaunchKernelGGL(k_ns_write, dim3(G), dim3(kBlock), 0, s, R, sa12, d, G, gcount2, keys0,
                                          vals0));
            bool alt;
            LOR_TRY(radix_sort<uint32_t>(keys0, vals0, keys1, vals1, d.n0, 0, b, counts2, s, &alt));
            A = alt ? vals1 : vals0;
        }
        const int32_t *B = sa12 + d.dummy;
        const uint32_t nB = d.m - d.dummy;
        if (parent_order) {
            // A's flagged symbols came with Step 2; B's from P (this level's
            // SA buffer, still the parent's order here)
            symA = vals0;
            const uint32_t Gn = scan_groups(d.n);
            LOR_LAUNCH("k_po_count", 4.0 * d.n, s,
                       hipLaunchKernelGGL(k_po_count, dim3(Gn), dim3(kBlock), 0, s, sa, d.n, Gn, gcount2));
            LOR_TRY(scan_block_totals(gcount2, Gn, nullptr, s));
            LOR_LAUNCH("k_msym_write", 8.0 * d.n + 4.0 * d.m, s,
                       hipLaunchKernelGGL(k_msym_write, dim3(Gn), dim3(kBlock), 0, s, sa, pnames, d, Gn, gcount2,
                                          symB));
        }
        const MergeArgs ma{A, d.n0, B, nB, d, parts, div_up(parts, kCoarse), mtile, mitems, csplit, split, symA,
                           symB, sa};
        if (narrow_rec) LOR_TRY(launch_merge<uint8_t>(rec8, ma, s));
        else LOR_TRY(launch_merge<CH>(rec, ma, s));
    }
    ar.release(mark_level);
    return LOR_OK;
}

}  // namespace

lor_status dc3_u8(const uint8_t *text, uint32_t n, uint32_t alphabet, int32_t *sa, Arena &ar, uint32_t *hdr,
                  hipStream_t s) {
    return dc3_level<uint8_t>(text, n, alphabet, sa, ar, hdr, s, 0, nullptr);
}

lor_status dc3_i32(const int32_t *text, uint32_t n, uint32_t alphabet, int32_t *sa, Arena &ar, uint32_t *hdr,
                   hipStream_t s) {
    return dc3_level<int32_t>(text, n, alphabet, sa, ar, hdr, s, 0, nullptr);
}

lor_status dc3_u16(const uint16_t *text, uint32_t n, uint32_t alphabet, int32_t *sa, Arena &ar, uint32_t *hdr,
                   hipStream_t s) {
    return dc3_level<uint16_t>(text, n, alphabet, sa, ar, hdr, s, 0, nullptr);
}

void set_decision_tape(DecisionTape *tape) { t_tape = tape; }
DecisionTape *decision_tape() { return t_tape; }

size_t dc3_workspace_bound(uint64_t n) {
    Arena ar;   // measuring
    if (n == 0) return 0;
    dc3_level<int32_t>(nullptr, (uint32_t)n, 0x7fffffffu, nullptr, ar, nullptr, nullptr, 0, nullptr);
    return ar.high + 4096;
}

__global__ __launch_bounds__(kBlock) void k_zero_words(uint32_t *p, uint32_t count) {
    for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < count; i += gridDim.x * kBlock) p[i] = 0;
}

lor_status zero_words(uint32_t *p, uint32_t count, hipStream_t s) {
    if (!count) return LOR_OK;
    LOR_LAUNCH("k_zero_words", 4.0 * count, s,
               hipLaunchKernelGGL(k_zero_words, dim3(grid_for(count)), dim3(kBlock), 0, s, p, count));
    return LOR_OK;
}

lor_status join_text(const uint8_t *seqs, const int64_t *offsets, int32_t k, uint8_t *out, uint32_t *err_word,
                     hipStream_t s) {
    SeqStarts st;
    st.k = k;
    for (int j = 0; j <= k; ++j) st.start[j] = (int32_t)(offsets[j] + j);
    const uint32_t N = (uint32_t)(offsets[k] + k);
    if (N == 0) return LOR_OK;
    LOR_LAUNCH("k_join", 2.0 * N, s,
               hipLaunchKernelGGL(k_join, dim3(grid_for(div_up(N, kJoinBytes))), dim3(kBlock), 0, s, seqs, st, N,
                                  (uint32_t)offsets[k], out, err_word));
    return LOR_OK;
}

}  // namespace lor
