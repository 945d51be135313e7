// Bucketed scatter on gfx950.
//
// A plain scatter dst[idx[i]] = val[i] with a random permutation idx puts
// every 4-byte store on its own cache line; on MI355X such stores cost about
// a full line of HBM traffic each. Here stable radix passes first group the
// (idx, val) pairs by the top 16 bits of idx (two 8-bit passes, LDS-staged,
// coalesced stores), and a last kernel stores them in that order: the stores
// an XCD has in flight then fall into one 1/65536 slice of dst (64 KB at a
// billion entries), which stays resident in that XCD's L2 until its lines are
// complete, so lines leave L2 whole instead of part-written.
#include <atomic>

#include "lor_internal.hpp"

namespace lor {

namespace {

// One element per thread, in array order. Workgroups are dealt to the 8 XCDs
// round-robin by index, so workgroup b works on the (b mod 8)-th eighth of the
// array: each XCD then walks its own run of buckets and its L2 sees stores to
// one slice of dst at a time.
__global__ __launch_bounds__(kBlock) void k_scatter_local(const uint32_t *__restrict__ idx,
                                                          const uint32_t *__restrict__ val, uint32_t n,
                                                          uint32_t dst_n, int32_t *__restrict__ dst) {
    const uint32_t i = dev::xcd_block() * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t d = idx[i];
    if (d < dst_n) dst[d] = (int32_t)val[i];
}

// Permutations (idx holds every value of 0..n-1 once and dst_n == n): once
// the pairs are grouped by the top bits of idx, positions [w*T, (w+1)*T) of
// the grouped arrays hold exactly the indices [w*T, (w+1)*T) whenever T is a
// multiple of the group width. A workgroup then places its window's values
// in LDS and writes the window out as contiguous stores.
constexpr int kWinBlock = 1024;   // threads per window workgroup (16 waves share one LDS window)
constexpr int kWinBatch = 8;      // pairs each thread loads before placing them

__global__ __launch_bounds__(kWinBlock) void k_scatter_window(const uint32_t *__restrict__ idx,
                                                              const uint32_t *__restrict__ val, uint32_t n,
                                                              uint32_t T, int32_t *__restrict__ dst) {
    extern __shared__ int32_t s_win[];
    const uint64_t base = (uint64_t)dev::xcd_block() * T;
    if (base >= n) return;
    const uint32_t cnt = (uint32_t)min((uint64_t)T, (uint64_t)n - base);
    const uint32_t *wi = idx + base, *wv = val + base;
    for (uint32_t i0 = threadIdx.x; i0 < cnt; i0 += kWinBlock * kWinBatch) {
        uint32_t d[kWinBatch], v[kWinBatch];
#pragma unroll
        for (int j = 0; j < kWinBatch; ++j) {
            const uint32_t i = i0 + j * kWinBlock;
            d[j] = i < cnt ? wi[i] - (uint32_t)base : 0xffffffffu;
            v[j] = i < cnt ? wv[i] : 0u;
        }
#pragma unroll
        for (int j = 0; j < kWinBatch; ++j)
            if (d[j] < cnt) s_win[d[j]] = (int32_t)v[j];
    }
    __syncthreads();
    for (uint32_t i0 = threadIdx.x; i0 < cnt; i0 += kWinBlock * kWinBatch) {
#pragma unroll
        for (int j = 0; j < kWinBatch; ++j) {
            const uint32_t i = i0 + j * kWinBlock;
            if (i < cnt) dst[base + i] = s_win[i];
        }
    }
}

}  // namespace

size_t max_lds_per_block() {
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 65536;
    int v = cache[dev].load(std::memory_order_relaxed);
    if (v == 0) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = 65536;
        cache[dev].store(v, std::memory_order_relaxed);
    }
    return (size_t)v;
}

// Entries per window of k_scatter_window for a destination of dst_n entries:
// a multiple of the width of one group of the bucketing (at least 4096).
uint32_t scatter_window(uint32_t dst_n) {
    const BucketDigits g = bucket_digits(dst_n);
    const int low = g.lo_bits > 0 ? g.lo_shift : g.hi_shift;
    return (1u << low) > 4096u ? (1u << low) : 4096u;
}

// Digits that split 0..dst_n-1 into contiguous slices by the top (at most
// 16) bits of an index: the high digit (top 8 bits) and the low digit (the
// next up to 8 bits; lo_bits = 0 when dst_n needs 8 bits or fewer).
BucketDigits bucket_digits(uint32_t dst_n) {
    const int b = dst_n > 1 ? bits_for(dst_n - 1) : 1;
    BucketDigits g;
    g.hi_shift = b > 8 ? b - 8 : 0;
    g.hi_bits = b - g.hi_shift;
    g.lo_shift = g.hi_shift > 8 ? g.hi_shift - 8 : 0;
    g.lo_bits = g.hi_shift - g.lo_shift;
    return g;
}

lor_status bucketed_scatter(int32_t *dst, uint32_t dst_n, const uint32_t *idx, const uint32_t *val, uint32_t voff,
                            uint32_t n, uint32_t *const tmp[4], uint32_t *counts, hipStream_t s, bool permutation) {
    if (n == 0) return LOR_OK;
    const BucketDigits g = bucket_digits(dst_n);
    const uint32_t *bi = tmp[0], *bv = tmp[1];
    if (g.lo_bits > 0) {
        LOR_TRY(radix_pass<uint32_t>(idx, val, voff, tmp[2], tmp[3], n, g.lo_shift, g.lo_bits, counts, s));
        LOR_TRY(radix_pass<uint32_t>(tmp[2], tmp[3], 0, tmp[0], tmp[1], n, g.hi_shift, g.hi_bits, counts, s));
    } else {
        LOR_TRY(radix_pass<uint32_t>(idx, val, voff, tmp[0], tmp[1], n, g.hi_shift, g.hi_bits, counts, s));
    }
    const uint32_t T = scatter_window(dst_n);
    if (permutation && n == dst_n && (size_t)T * sizeof(int32_t) <= max_lds_per_block()) {
        LOR_LAUNCH("k_scatter_window", 12.0 * n, s,
                   hipLaunchKernelGGL(k_scatter_window, dim3(kXcds * div_up(div_up(n, T), kXcds)), dim3(kWinBlock),
                                      (size_t)T * sizeof(int32_t), s, bi, bv, n, T, dst));
    } else {
        LOR_LAUNCH("k_scatter_local", 12.0 * n, s,
                   hipLaunchKernelGGL(k_scatter_local, dim3(xcd_grid(n)), dim3(kBlock), 0, s, bi, bv, n, dst_n, dst));
    }
    return LOR_OK;
}

}  // namespace lor
