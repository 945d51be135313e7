// Bucketed scatter on gfx950.
//
// A plain scatter dst[idx[i]] = val[i] with a random permutation idx puts
// every 4-byte store on its own cache line; on MI355X such stores cost about
// a full line of HBM traffic each. Here one stable radix pass first groups the
// (idx, val) pairs by the top 8 bits of idx (LDS-staged, coalesced stores),
// and a second kernel stores them in that order: the stores in flight then
// fall into one or two 1/256 slices of dst, which stay resident in L2 and
// the Infinity Cache, so lines are completed there before they are written
// back.
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

}  // namespace

// Digit that splits 0..dst_n-1 into at most 256 contiguous slices.
void bucket_digit(uint32_t dst_n, int *shift, int *nbits) {
    const int b = dst_n > 1 ? bits_for(dst_n - 1) : 1;
    *shift = b > 8 ? b - 8 : 0;
    *nbits = b - *shift;
}

lor_status bucketed_scatter(int32_t *dst, uint32_t dst_n, const uint32_t *idx, const uint32_t *val, uint32_t voff,
                            uint32_t n, uint32_t *tmp_idx, uint32_t *tmp_val, uint32_t *counts, hipStream_t s) {
    if (n == 0) return LOR_OK;
    int shift, nbits;
    bucket_digit(dst_n, &shift, &nbits);
    LOR_TRY(radix_pass<uint32_t>(idx, val, voff, tmp_idx, tmp_val, n, shift, nbits, counts, s));
    LOR_LAUNCH("k_scatter_local", 12.0 * n, s,
               hipLaunchKernelGGL(k_scatter_local, dim3(xcd_grid(n)), dim3(kBlock), 0, s, tmp_idx, tmp_val, n, dst_n,
                                  dst));
    return LOR_OK;
}

}  // namespace lor
