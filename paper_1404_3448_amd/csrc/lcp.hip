// LCP array on gfx950 (Section III, Table IV: LCP[r] = lcp of the suffixes
// at ranks r-1 and r; the paper cites Kasai et al. for its construction).
//
// Permuted-LCP method:
//   phi    : for every rank r, the pair (r, SA[r-1]) goes to text position
//            SA[r] -- the inverse permutation and Phi together. The pairs
//            travel as 64-bit keys (SA[r] << 32 | SA[r-1]) through radix
//            passes on the top 16 bits of SA[r], then are stored bucket by
//            bucket (see scatter.hip for why bucketing beats a random
//            scatter);
//   plcp   : PLCP[i] = lcp(suffix i, suffix Phi[i]). Kasai's bound
//            PLCP[i+1] >= PLCP[i] - 1 iterates to PLCP[i+d] >= PLCP[i] - d.
//            A wave owns a run of 64*K consecutive positions; lane l takes
//            positions l, l+64, l+128, ... and resumes each comparison from
//            its previous result minus 64. Loads of neighbouring lanes are
//            contiguous, and inside long repeats (where the bound pays off)
//            every lane does the same short extension, so no lane stalls
//            its wave. The comparison reads 8 symbols at a time. ISA is
//            written out here, sequentially;
//   place  : LCP[ISA[i]] = PLCP[i], a bucketed scatter.
#include "lor_internal.hpp"

namespace lor {

namespace {


__global__ __launch_bounds__(kBlock) void k_phi_keys(const int32_t *__restrict__ sa, uint32_t n,
                                                     uint64_t *__restrict__ keys) {
    for (uint32_t r = blockIdx.x * kBlock + threadIdx.x; r < n; r += gridDim.x * kBlock) {
        const uint32_t p = (uint32_t)sa[r];
        const uint32_t prev = r ? (uint32_t)sa[r - 1] : 0xffffffffu;
        keys[r] = ((uint64_t)(p < n ? p : 0xffffffffu) << 32) | prev;
    }
}

// isa_phi[SA[r]] = (r, SA[r-1]) from the bucketed (key, r) pairs.
__global__ __launch_bounds__(kBlock) void k_phi_place(const uint64_t *__restrict__ keys,
                                                      const uint32_t *__restrict__ ranks, uint32_t n,
                                                      int2 *__restrict__ isa_phi) {
    const uint32_t i = dev::xcd_block() * kBlock + threadIdx.x;   // one pair per thread, in bucket order
    if (i >= n) return;
    const uint64_t k = keys[i];
    const uint32_t p = (uint32_t)(k >> 32);
    if (p < n) isa_phi[p] = make_int2((int32_t)ranks[i], (int32_t)(uint32_t)k);
}

// 8 text bytes starting at byte offset a; requires a + 16 <= text bytes and
// an 8-byte aligned text (two aligned loads, then a funnel shift).
__device__ __forceinline__ uint64_t load8(const uint8_t *__restrict__ t, uint32_t a) {
    const uint64_t *w = reinterpret_cast<const uint64_t *>(t + (a & ~7u));
    const uint32_t sh = (a & 7u) * 8u;
    const uint64_t lo = w[0], hi = w[1];
    return sh ? (lo >> sh) | (hi << (64u - sh)) : lo;
}

// Common-prefix length of suffixes i and j (in symbols), knowing the first h
// symbols agree. Wide mode compares 8 bytes (8 / sizeof(CH) symbols) a step.
template <typename CH>
__device__ __forceinline__ uint32_t extend(const CH *__restrict__ t, uint32_t n, uint32_t i, uint32_t j, uint32_t h,
                                           bool wide) {
    constexpr uint32_t per = 8 / sizeof(CH);
    const uint32_t lim = n - max(i, j);   // symbols available in both
    if (wide) {
        const uint8_t *tb = reinterpret_cast<const uint8_t *>(t);
        while (h + 2 * per <= lim) {
            const uint64_t x = load8(tb, (i + h) * (uint32_t)sizeof(CH)) ^ load8(tb, (j + h) * (uint32_t)sizeof(CH));
            if (x) return h + (uint32_t)(__builtin_ctzll(x) / (8 * sizeof(CH)));
            h += per;
        }
    }
    while (h < lim && t[i + h] == t[j + h]) ++h;
    return h;
}

// A step of a wave takes 64 consecutive positions, one per lane. When
// Phi[i] = Phi[i-1] + 1 and PLCP[i-1] >= 1, then PLCP[i] = PLCP[i-1] - 1
// exactly (both suffixes lose the same first symbol), so a run of such
// positions follows from the PLCP at its head with no text read: only heads
// compare text (Kasai's bound, from the lane's previous step), then every
// lane of a run takes head - distance by a wave-wide segmented propagation
// (the run may continue from the previous step's last lane). A run whose head
// value drops to 0 before its end leaves the rest to compare for themselves.
template <typename CH>
__global__ __launch_bounds__(kBlock) void k_plcp(const CH *__restrict__ t, uint32_t n,
                                                 const int2 *__restrict__ isa_phi, int32_t *__restrict__ plcp,
                                                 int32_t *__restrict__ isa_out, int wide, uint32_t steps) {
    const uint32_t span = kWave * steps;
    const uint32_t waves = (n + span - 1) / span;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t below = lane ? (~0ull >> (64u - lane)) : 0ull;   // lanes under this one
    for (uint32_t w = (blockIdx.x * kBlock + threadIdx.x) / kWave; w < waves; w += gridDim.x * (kBlock / kWave)) {
        uint32_t h = 0;                                    // Kasai bound from this lane's previous step
        uint32_t prev_j = 0xffffffffu, prev_p = 0;         // Phi and PLCP of the position before lane 0
        for (uint32_t k = 0, i0 = w * span; k < steps && i0 < n; ++k, i0 += kWave) {
            const uint32_t i = i0 + lane;
            const bool valid = i < n;
            uint32_t j = 0xffffffffu;
            if (valid) {
                const int2 q = isa_phi[i];
                isa_out[i] = q.x;
                j = (uint32_t)q.y;                           // n or more: no predecessor (rank 0)
            }
            const bool has = valid && j < n;
            uint32_t jl = (uint32_t)__shfl_up((int)j, 1, kWave);
            if (lane == 0) jl = prev_j;
            const bool chained = has && j > 0 && jl < n && jl == j - 1;
            uint32_t p = 0;
            if (has && !chained) p = extend(t, n, i, j, h, wide != 0);
            // segment heads: every lane not chained to the one before it
            const uint64_t starts = __ballot(!chained);
            const uint64_t mine = starts & (below | (1ull << lane));
            const int head = mine ? 63 - __builtin_clzll(mine) : -1;
            const uint32_t hv = (uint32_t)__shfl((int)p, head < 0 ? 0 : head, kWave);
            const uint32_t H = head < 0 ? prev_p : hv;
            const uint32_t d = head < 0 ? lane + 1u : lane - (uint32_t)head;
            if (chained) {
                if (H >= d) p = H - d;
                else p = extend(t, n, i, j, h, wide != 0);   // the run reached 0 before this lane
            }
            if (valid) plcp[i] = (int32_t)p;
            h = p > kWave ? p - kWave : 0;
            prev_j = (uint32_t)__shfl((int)j, 63, kWave);
            prev_p = (uint32_t)__shfl((int)p, 63, kWave);
        }
    }
}

}  // namespace

size_t lcp_workspace(uint64_t n) { return (size_t)n * 28 + radix_counts_words(n) * 4 + 4096; }

template <typename CH>
lor_status lcp_build_t(const CH *text, uint32_t n, const int32_t *sa, int32_t *lcp, int32_t *isa, Arena &ar,
                       hipStream_t s) {
    uint64_t *keys, *keys2;       // keys later holds the (ISA, Phi) pairs
    uint32_t *vals2, *plcp, *isa_tmp, *counts;
    LOR_TAKE(ar, uint64_t, n, keys);
    LOR_TAKE(ar, uint64_t, n, keys2);
    LOR_TAKE(ar, uint32_t, n, vals2);
    LOR_TAKE(ar, uint32_t, n, plcp);
    LOR_TAKE(ar, uint32_t, n, isa_tmp);
    LOR_TAKE(ar, uint32_t, radix_counts_words(n), counts);
    if (n == 0) return LOR_OK;
    int32_t *isa_w = isa ? isa : reinterpret_cast<int32_t *>(isa_tmp);
    const int wide = ((uintptr_t)text % 8) == 0;
    LOR_LAUNCH("k_phi_keys", (double)n * 12, s,
               hipLaunchKernelGGL(k_phi_keys, dim3(grid_for(n)), dim3(kBlock), 0, s, sa, n, keys));
    // Bucket the pairs by the top bits of SA[r] (two passes for large n);
    // the (ISA, Phi) pairs then go to whichever 8-byte buffer is free.
    const BucketDigits g = bucket_digits(n);
    const uint64_t *bk;
    const uint32_t *bv;
    int2 *isa_phi;
    if (g.lo_bits > 0) {
        LOR_TRY(radix_pass<uint64_t>(keys, nullptr, 0, keys2, vals2, n, 32 + g.lo_shift, g.lo_bits, counts, s));
        LOR_TRY(radix_pass<uint64_t>(keys2, vals2, 0, keys, plcp, n, 32 + g.hi_shift, g.hi_bits, counts, s));
        bk = keys;
        bv = plcp;
        isa_phi = reinterpret_cast<int2 *>(keys2);
    } else {
        LOR_TRY(radix_pass<uint64_t>(keys, nullptr, 0, keys2, vals2, n, 32 + g.hi_shift, g.hi_bits, counts, s));
        bk = keys2;
        bv = vals2;
        isa_phi = reinterpret_cast<int2 *>(keys);
    }
    LOR_LAUNCH("k_phi_place", (double)n * 20, s,
               hipLaunchKernelGGL(k_phi_place, dim3(xcd_grid(n)), dim3(kBlock), 0, s, bk, bv, n, isa_phi));
    const uint32_t steps = (uint32_t)plan().plcp_steps;
    const uint32_t waves = div_up(n, kWave * steps);
    LOR_LAUNCH("k_plcp", (double)n * (16 + sizeof(CH)), s,
               hipLaunchKernelGGL(k_plcp<CH>, dim3(grid_for((uint64_t)waves * kWave)), dim3(kBlock), 0, s, text, n,
                                  isa_phi, reinterpret_cast<int32_t *>(plcp), isa_w, wide, steps));
    // both 8-byte buffers are free again: four n-word scatter buffers
    uint32_t *k32 = reinterpret_cast<uint32_t *>(keys), *k232 = reinterpret_cast<uint32_t *>(keys2);
    uint32_t *const tmp4[4] = {k32, k32 + n, k232, k232 + n};
    return bucketed_scatter(lcp, n, reinterpret_cast<const uint32_t *>(isa_w), plcp, 0, n, tmp4, counts, s, true);
}

lor_status lcp_build(const uint8_t *text, uint32_t n, const int32_t *sa, int32_t *lcp, int32_t *isa, Arena &ar,
                     hipStream_t s) {
    return lcp_build_t<uint8_t>(text, n, sa, lcp, isa, ar, s);
}

lor_status lcp_build_u16(const uint16_t *text, uint32_t n, const int32_t *sa, int32_t *lcp, int32_t *isa, Arena &ar,
                         hipStream_t s) {
    return lcp_build_t<uint16_t>(text, n, sa, lcp, isa, ar, s);
}

}  // namespace lor
