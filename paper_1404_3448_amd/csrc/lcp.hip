// LCP array on gfx950 (Section III, Table IV: LCP[r] = lcp of the suffixes
// at ranks r-1 and r; the paper cites Kasai et al. for its construction).
//
// Permuted-LCP method in three passes:
//   phi    : Phi[SA[r]] = SA[r-1] (Phi[SA[0]] = -1), optionally ISA[SA[r]] = r;
//   plcp   : PLCP[i] = lcp(suffix i, suffix Phi[i]) walking the text in
//            position order, so PLCP[i+1] >= PLCP[i] - 1 (Kasai's bound)
//            lets each step resume the comparison; the text is cut into
//            chunks of consecutive positions, one per thread, and each chunk
//            starts its first comparison from zero. PLCP overwrites Phi.
//   permute: LCP[r] = PLCP[SA[r]].
#include "lor_internal.hpp"

namespace lor {

namespace {

constexpr uint32_t kPlcpChunk = 64;   // consecutive text positions per thread

__global__ __launch_bounds__(kBlock) void k_phi(const int32_t *__restrict__ sa, uint32_t n,
                                                int32_t *__restrict__ phi, int32_t *__restrict__ isa) {
    for (uint32_t r = blockIdx.x * kBlock + threadIdx.x; r < n; r += gridDim.x * kBlock) {
        const int32_t p = sa[r];
        if ((uint32_t)p >= n) continue;   // not a permutation of 0..n-1: skip
        phi[p] = r ? sa[r - 1] : -1;
        if (isa) isa[p] = (int32_t)r;
    }
}

// Common-prefix length of suffixes i and j, knowing the first h symbols agree.
__device__ __forceinline__ uint32_t extend(const uint8_t *__restrict__ t, uint32_t n, uint32_t i, uint32_t j,
                                           uint32_t h) {
    const uint32_t lim = n - max(i, j);   // symbols available in both
    while (h < lim && t[i + h] == t[j + h]) ++h;
    return h;
}

__global__ __launch_bounds__(kBlock) void k_plcp(const uint8_t *__restrict__ t, uint32_t n,
                                                 int32_t *__restrict__ phi_plcp) {
    const uint32_t chunks = (n + kPlcpChunk - 1) / kPlcpChunk;
    for (uint32_t c = blockIdx.x * kBlock + threadIdx.x; c < chunks; c += gridDim.x * kBlock) {
        const uint32_t i0 = c * kPlcpChunk, i1 = min(n, i0 + kPlcpChunk);
        uint32_t h = 0;
        for (uint32_t i = i0; i < i1; ++i) {
            const int32_t j = phi_plcp[i];
            if (j < 0 || (uint32_t)j >= n) {
                phi_plcp[i] = 0;
                h = 0;
                continue;
            }
            h = extend(t, n, i, (uint32_t)j, h);
            phi_plcp[i] = (int32_t)h;
            h = h ? h - 1 : 0;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_permute(const int32_t *__restrict__ sa,
                                                    const int32_t *__restrict__ plcp, uint32_t n,
                                                    int32_t *__restrict__ lcp) {
    for (uint32_t r = blockIdx.x * kBlock + threadIdx.x; r < n; r += gridDim.x * kBlock) {
        const uint32_t p = (uint32_t)sa[r];
        lcp[r] = p < n ? plcp[p] : -1;
    }
}

}  // namespace

size_t lcp_workspace(uint64_t n) { return (size_t)n * 4 + 512; }

lor_status lcp_build(const uint8_t *text, uint32_t n, const int32_t *sa, int32_t *lcp, int32_t *isa, Arena &ar,
                     hipStream_t s) {
    int32_t *phi;
    LOR_TAKE(ar, int32_t, n, phi);
    if (n == 0) return LOR_OK;
    LOR_LAUNCH(F_PHI, (double)n * (isa ? 12 : 8), s,
               hipLaunchKernelGGL(k_phi, dim3(grid_for(n)), dim3(kBlock), 0, s, sa, n, phi, isa));
    const uint32_t chunks = div_up(n, kPlcpChunk);
    LOR_LAUNCH(F_PLCP, (double)n * 11, s,
               hipLaunchKernelGGL(k_plcp, dim3(grid_for(chunks)), dim3(kBlock), 0, s, text, n, phi));
    LOR_LAUNCH(F_PERMUTE, (double)n * 12, s,
               hipLaunchKernelGGL(k_permute, dim3(grid_for(n)), dim3(kBlock), 0, s, sa, phi, n, lcp));
    return LOR_OK;
}

}  // namespace lor
