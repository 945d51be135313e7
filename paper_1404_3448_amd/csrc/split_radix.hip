// The radix sort of Section IV as the paper designs it (its Alg. 1 kernel and
// the chunk merge described after it), built for gfx950 so that its design
// can be measured against this library's digit sort (radix.hip).
//
// The paper's design, in two phases:
//   1. every thread block sorts one chunk of the input in shared memory with
//      one split per key bit, from the least significant bit up. A split of
//      the chunk by bit b is: L = the bit of every key, E = L xor 1 (keys
//      whose bit is 0), F = exclusive prefix sum of E, totalFalse =
//      E[n-1] + F[n-1] (the number of zero bits), and the destination of
//      key i is F[i] when its bit is 0 and i - F[i] + totalFalse when it is
//      1. Keys with a 0 bit keep their order at the front, keys with a 1 bit
//      keep theirs behind them, so each split is stable and the chunk ends
//      sorted by all its bits;
//   2. sorted chunks are merged pairwise into longer sorted runs until one
//      run holds everything.
//
// On a 64-lane wavefront the prefix sum of a 0/1 array needs no scan tree:
// one ballot gives the wave's E bits and a masked bit count (mbcnt) gives
// every lane the number of set bits below it. Element e of a chunk is item
// e / 256 of thread e % 256, so one LDS access of a wave covers 64
// consecutive words; the per-(item, wave) counts of E meet in LDS once per
// split. The merge of phase 2 takes the merge path: each workgroup finds
// where its output tile starts and ends in the two runs by binary search,
// stages both slices in LDS and merges them there; ties take the left run
// first, so the whole sort is stable.
#include "lor_internal.hpp"

namespace lor {

namespace {

constexpr int kSplitItems = 8;
constexpr uint32_t kChunk = kBlock * kSplitItems;   // keys per chunk (one workgroup)
constexpr int kMergeItems = 8;
constexpr uint32_t kMergeTile = kBlock * kMergeItems;
static_assert(kMergeTile == kChunk, "merge tiles must not straddle two pairs of runs");

__global__ __launch_bounds__(kBlock) void k_split_chunks(const uint32_t *__restrict__ kin,
                                                         const uint32_t *__restrict__ vin,
                                                         uint32_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                         uint32_t n, int bit_lo, int bit_hi) {
    constexpr int W = kBlock / kWave;
    __shared__ uint32_t s_k[2][kChunk];
    __shared__ uint32_t s_v[2][kChunk];
    __shared__ uint32_t s_zero[kSplitItems][W];   // E count of every (item, wave)
    const uint32_t c0 = blockIdx.x * kChunk;
    if (c0 >= n) return;
    const uint32_t cnt = min(kChunk, n - c0);
    const unsigned tid = threadIdx.x, w = tid >> 6;
#pragma unroll
    for (int r = 0; r < kSplitItems; ++r) {
        const uint32_t e = r * kBlock + tid;
        if (e < cnt) {
            s_k[0][e] = kin[c0 + e];
            s_v[0][e] = vin[c0 + e];
        }
    }
    __syncthreads();
    int cur = 0;
    for (int bit = bit_lo; bit < bit_hi; ++bit) {
        uint32_t k[kSplitItems], v[kSplitItems];
        uint64_t emask[kSplitItems];
#pragma unroll
        for (int r = 0; r < kSplitItems; ++r) {
            const uint32_t e = r * kBlock + tid;
            const bool ok = e < cnt;
            k[r] = ok ? s_k[cur][e] : 0u;
            v[r] = ok ? s_v[cur][e] : 0u;
            const bool ebit = ok && ((k[r] >> bit) & 1u) == 0u;   // E = L xor 1
            emask[r] = __ballot(ebit);
            if ((tid & 63u) == 0) s_zero[r][w] = (uint32_t)__popcll(emask[r]);
        }
        __syncthreads();
        // F[e] = E count of earlier items (all waves) plus earlier waves of
        // this item plus lower lanes of this wave; totalFalse = all of them.
        uint32_t before[kSplitItems], total = 0;
#pragma unroll
        for (int r = 0; r < kSplitItems; ++r) {
            uint32_t in_item = 0, below = 0;
#pragma unroll
            for (int x = 0; x < W; ++x) {
                const uint32_t c = s_zero[r][x];
                in_item += c;
                below += (x < (int)w) ? c : 0u;
            }
            before[r] = total + below;
            total += in_item;
        }
#pragma unroll
        for (int r = 0; r < kSplitItems; ++r) {
            const uint32_t e = r * kBlock + tid;
            if (e < cnt) {
                const uint32_t f = before[r] + dev::count_below(emask[r]);
                const bool one = (k[r] >> bit) & 1u;
                const uint32_t dest = one ? e - f + total : f;
                s_k[cur ^ 1][dest] = k[r];
                s_v[cur ^ 1][dest] = v[r];
            }
        }
        __syncthreads();   // the next split reads the other buffer; s_zero is rewritten
        cur ^= 1;
    }
#pragma unroll
    for (int r = 0; r < kSplitItems; ++r) {
        const uint32_t e = r * kBlock + tid;
        if (e < cnt) {
            kout[c0 + e] = s_k[cur][e];
            vout[c0 + e] = s_v[cur][e];
        }
    }
}

__device__ __forceinline__ uint32_t digit_of(uint32_t k, int bit_lo, uint32_t mask) { return (k >> bit_lo) & mask; }

// Elements of run A among the first `diag` outputs of the stable merge of A
// (na keys) and B (nb keys): A's key is taken while it is not greater.
__device__ __forceinline__ uint32_t path_split(const uint32_t *A, uint32_t na, const uint32_t *B, uint32_t nb,
                                               uint32_t diag, int bit_lo, uint32_t mask) {
    uint32_t lo = diag > nb ? diag - nb : 0u, hi = min(diag, na);
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (digit_of(B[diag - 1 - mid], bit_lo, mask) < digit_of(A[mid], bit_lo, mask)) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// Runs of `width` keys (width a multiple of the tile) are merged pairwise:
// output tile g lies inside the pair of runs that starts at its multiple of
// 2 * width.
__global__ __launch_bounds__(kBlock) void k_merge_runs(const uint32_t *__restrict__ kin,
                                                       const uint32_t *__restrict__ vin,
                                                       uint32_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                       uint32_t n, uint32_t width, int bit_lo, uint32_t mask) {
    __shared__ uint32_t s_k[kMergeTile];
    __shared__ uint32_t s_v[kMergeTile];
    __shared__ uint32_t s_ok[kMergeTile];
    __shared__ uint32_t s_ov[kMergeTile];
    __shared__ uint32_t s_split[2];
    const uint64_t d0g = (uint64_t)blockIdx.x * kMergeTile;
    if (d0g >= n) return;
    const uint64_t ps = d0g / (2ull * width) * (2ull * width);   // start of this pair of runs
    const uint32_t na = (uint32_t)min<uint64_t>(width, n - ps);
    const uint32_t nb = (uint32_t)min<uint64_t>(width, n - min<uint64_t>(n, ps + width));
    const uint32_t *A = kin + ps, *B = kin + ps + na;
    const uint32_t d0 = (uint32_t)(d0g - ps), d1 = (uint32_t)min<uint64_t>(d0 + kMergeTile, (uint64_t)na + nb);
    if (threadIdx.x < 2) s_split[threadIdx.x] = path_split(A, na, B, nb, threadIdx.x ? d1 : d0, bit_lo, mask);
    __syncthreads();
    const uint32_t a0 = s_split[0], a1 = s_split[1];
    const uint32_t b0 = d0 - a0, b1 = d1 - a1;
    const uint32_t la = a1 - a0, lb = b1 - b0, cnt = d1 - d0;
    for (uint32_t i = threadIdx.x; i < cnt; i += kBlock) {   // A slice, then B slice
        const uint64_t g = i < la ? ps + a0 + i : ps + na + b0 + (i - la);
        s_k[i] = kin[g];
        s_v[i] = vin[g];
    }
    __syncthreads();
    const uint32_t *sA = s_k, *sB = s_k + la;
    const uint32_t diag = min(cnt, threadIdx.x * (uint32_t)kMergeItems);
    const uint32_t dend = min(cnt, diag + (uint32_t)kMergeItems);
    uint32_t ia = path_split(sA, la, sB, lb, diag, bit_lo, mask), ib = diag - ia;
    for (uint32_t o = diag; o < dend; ++o) {
        const bool take_a = ia < la && (ib >= lb || digit_of(sB[ib], bit_lo, mask) >= digit_of(sA[ia], bit_lo, mask));
        const uint32_t src = take_a ? ia++ : la + ib++;
        s_ok[o] = s_k[src];
        s_ov[o] = s_v[src];
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < cnt; i += kBlock) {
        kout[ps + d0 + i] = s_ok[i];
        vout[ps + d0 + i] = s_ov[i];
    }
}

}  // namespace

lor_status split_radix_sort(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, uint32_t n, int bit_lo,
                            int bit_hi, hipStream_t s, bool *in_alt) {
    *in_alt = false;
    if (n <= 1 || bit_hi <= bit_lo) return LOR_OK;
    const uint32_t chunks = div_up(n, kChunk);
    LOR_LAUNCH("k_split_chunks", 16.0 * n, s,
               hipLaunchKernelGGL(k_split_chunks, dim3(chunks), dim3(kBlock), 0, s, k0, v0, k1, v1, n, bit_lo,
                                  bit_hi));
    uint32_t *ki = k1, *vi = v1, *ko = k0, *vo = v0;
    bool alt = true;
    const uint32_t mask = bit_hi - bit_lo >= 32 ? 0xffffffffu : ((1u << (bit_hi - bit_lo)) - 1u);
    for (uint64_t width = kChunk; width < n; width *= 2) {
        LOR_LAUNCH("k_merge_runs", 16.0 * n, s,
                   hipLaunchKernelGGL(k_merge_runs, dim3(div_up(n, kMergeTile)), dim3(kBlock), 0, s, ki, vi, ko, vo,
                                      n, (uint32_t)width, bit_lo, mask));
        uint32_t *t = ki; ki = ko; ko = t;
        t = vi; vi = vo; vo = t;
        alt = !alt;
    }
    *in_alt = alt;
    return LOR_OK;
}

}  // namespace lor
