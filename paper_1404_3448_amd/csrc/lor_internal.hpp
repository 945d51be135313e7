// Internal declarations shared by the liblor.so translation units:
// error reporting, the workspace arena, kernel-family timing, and wave64
// device primitives for gfx950.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "lor.h"

namespace lor {

constexpr int kWave = 64;     // CDNA wavefront width
constexpr int kBlock = 256;   // threads per workgroup for every kernel (4 waves)

// ------------------------------------------------------------------ errors
void set_error(const char *fmt, ...);

#define LOR_TRY(expr)                        \
    do {                                     \
        lor_status st_ = (expr);             \
        if (st_ != LOR_OK) return st_;       \
    } while (0)

#define LOR_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) {                                                         \
            ::lor::set_error("%s:%d: %s failed: %s", __FILE__, __LINE__, #call,          \
                             hipGetErrorString(e_));                                    \
            return LOR_EHIP;                                                            \
        }                                                                               \
    } while (0)

#define LOR_CHECK_LAUNCH() LOR_HIP(hipGetLastError())

// ------------------------------------------------------------------ arena
// Bump allocator over the caller's workspace. With base == nullptr it only
// measures (the size queries run the same carving code as the real calls).
struct Arena {
    char *base = nullptr;
    size_t cap = 0;
    size_t top = 0;
    size_t high = 0;
    bool overflow = false;

    template <class T>
    T *take(size_t count) {
        size_t a = (top + 255) & ~size_t(255);
        size_t need = a + count * sizeof(T);
        if (base && need > cap) {
            overflow = true;
            return nullptr;
        }
        top = need;
        if (top > high) high = top;
        return base ? reinterpret_cast<T *>(base + a) : reinterpret_cast<T *>(uintptr_t(256));
    }
    size_t mark() const { return top; }
    void release(size_t m) { top = m; }
    bool measuring() const { return base == nullptr; }
};

#define LOR_TAKE(arena, T, count, ptr)                                                  \
    do {                                                                                \
        (ptr) = (arena).template take<T>(count);                                        \
        if (!(ptr)) {                                                                   \
            ::lor::set_error("workspace too small (%s:%d)", __FILE__, __LINE__);        \
            return LOR_EWORKSPACE;                                                      \
        }                                                                               \
    } while (0)

// Small device header at the start of every workspace: an error word and a
// few result words read back by the host.
struct WsHeader {
    uint32_t error;        // bit 0: input base outside 0..3
    uint32_t word[15];
};
constexpr size_t kHeaderBytes = 256;
constexpr int kStaleWord = 15;   // header word set when a replayed launch sequence no longer fits the data

// ------------------------------------------------ captured launch sequences
// The only data-dependent host decision of DC3 is the name count of every
// level (it decides recursion and the key width of the next level). An eager
// run records the counts; a run under stream capture replays them and, in
// place of each read-back, launches a device check that sets header word
// kStaleWord when the data give a different count. Every kernel bounds its
// memory accesses by sizes the host passes, so a replay whose check fails
// still stays inside its buffers; its results are then discarded.
struct DecisionTape {
    std::vector<uint32_t> names;   // name count per DC3 level, in call order
    size_t next = 0;
    bool replay = false;           // under capture: take recorded counts, emit checks
};
void set_decision_tape(DecisionTape *tape);   // for the calling thread; nullptr turns it off
DecisionTape *decision_tape();
void set_capturing(bool on);                  // no event timing while a stream is captured

// Largest LDS allocation one workgroup may take on the current device
// (queried once per device).
size_t max_lds_per_block();

// ------------------------------------------------------------------ plan
// Tuning knobs chosen by the autotuner. A plan changes speed, never results.
struct Plan {
    int digit_bits;     // radix digit width, 4..8
    int items_u32;      // radix items per thread, 32-bit keys: 8, 12, 16, 24
    int items_u64;      // radix items per thread, 64-bit keys: 4, 8, 12, 16
    int merge_items;    // merge outputs per thread: 4, 8, 12
    int plcp_steps;     // PLCP positions per lane: 32..512
};
const Plan &plan();                 // the calling thread's plan
bool plan_valid(const Plan &p);
void plan_set_global(const Plan &p);
// Per-call override for the calling thread (nullptr clears it).
void plan_set_thread(const Plan *p);

// -------------------------------------------------------- kernel timing
// Timing is keyed by kernel name, so the figures line up with a profiler's.
bool timing_on();
int timing_begin(hipStream_t s, const char *kernel, double bytes);
void timing_end(int token, hipStream_t s);
bool trace_on();   // LOR_TRACE set in the environment: per-level notes on stderr

// Launch helper: records events around the launch when timing is enabled.
// `kernel` is the kernel's name; `bytes` its algorithmic bytes for this launch.
#define LOR_LAUNCH(kernel, bytes, stream, ...)                                          \
    do {                                                                                \
        int tk_ = ::lor::timing_on() ? ::lor::timing_begin((stream), (kernel), (bytes)) : -1; \
        __VA_ARGS__;                                                                    \
        LOR_CHECK_LAUNCH();                                                             \
        if (tk_ >= 0) ::lor::timing_end(tk_, (stream));                                 \
    } while (0)

inline uint32_t div_up(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// Grid size for elementwise kernels: one thread per item, capped; kernels
// stride over the rest.
inline uint32_t grid_for(uint64_t items, uint32_t per_block = kBlock) {
    uint64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 65536u * 8u) g = 65536u * 8u;
    return (uint32_t)g;
}

// MI355X: 8 XCDs (each with its own L2); workgroups are dealt to them
// round-robin by workgroup index.
constexpr uint32_t kXcds = 8;

// Grid of one thread per item for kernels that remap workgroups per XCD:
// a multiple of kXcds workgroups.
inline uint32_t xcd_grid(uint64_t items) {
    uint64_t g = (items + kBlock - 1) / kBlock;
    g = (g + kXcds - 1) / kXcds * kXcds;
    return (uint32_t)(g ? g : kXcds);
}

inline int bits_for(uint64_t maxval) {   // bits needed to hold 0..maxval
    int b = 0;
    while (b < 64 && (maxval >> b) != 0) ++b;
    return b;
}

// ------------------------------------------------------------ radix sort
// Stable LSD sort of (key, u32 value) by key bits [bit_lo, bit_hi).
// (k0, v0) hold the input; (k1, v1) are same-sized alternates. On return
// *in_alt says whether the sorted data ended in (k1, v1).
size_t radix_counts_words(uint64_t n);
// One stable pass on digit bits [shift, shift + nbits) (nbits <= 8) from
// (ki, vi) to (ko, vo); vi == nullptr stands for values e + voff.
template <typename K>
lor_status radix_pass(const K *ki, const uint32_t *vi, uint32_t voff, K *ko, uint32_t *vo, uint32_t n, int shift,
                      int nbits, uint32_t *counts, hipStream_t s);
template <typename K>
lor_status radix_sort(K *k0, uint32_t *v0, K *k1, uint32_t *v1, uint32_t n, int bit_lo,
                      int bit_hi, uint32_t *counts, hipStream_t s, bool *in_alt);
int radix_passes(int bit_lo, int bit_hi);
// The paper's radix-sort design (one split per key bit inside every chunk,
// then pairwise merges of sorted chunks), u32 keys and values; the sorted
// data end in (k1, v1) when *in_alt is set.
lor_status split_radix_sort(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, uint32_t n, int bit_lo,
                            int bit_hi, hipStream_t s, bool *in_alt);

// ------------------------------------------------------ bucketed scatter
// dst[idx[i]] = val[i] for i < n (idx a permutation into dst[0..dst_n) or a
// subset of it): stable radix passes partition the pairs by the top (up to
// 16) bits of idx, then a last kernel stores them bucket by bucket, so stores
// to one range of dst are close in time and combine in L2 instead of each
// costing a line of HBM traffic. val == nullptr stands for values i + voff.
// tmp: four buffers of n words (the last two are unused when dst_n needs at
// most 8 index bits); counts: radix_counts_words(n).
struct BucketDigits {
    int hi_shift, hi_bits;   // top digit of an index
    int lo_shift, lo_bits;   // the digit below it (lo_bits == 0: none)
};
BucketDigits bucket_digits(uint32_t dst_n);
// permutation: idx holds every value of 0..dst_n-1 exactly once (n == dst_n);
// the last kernel then writes whole windows of dst from LDS.
lor_status bucketed_scatter(int32_t *dst, uint32_t dst_n, const uint32_t *idx, const uint32_t *val, uint32_t voff,
                            uint32_t n, uint32_t *const tmp[4], uint32_t *counts, hipStream_t s, bool permutation);
// Window (entries) of the permutation store for a destination of dst_n entries.
uint32_t scatter_window(uint32_t dst_n);

// ------------------------------------------------------------- device scan
// Exclusive scan of `count` u32 block totals in place (one workgroup);
// writes the grand total to *total (nullable).
lor_status scan_block_totals(uint32_t *vals, uint32_t count, uint32_t *total, hipStream_t s);
// Exclusive scan of `count` words in place across the device (reduce, scan
// of partials, downsweep). tmp: scan_tmp_words() words.
constexpr size_t kScanTmpWords = 1024 + 64;
lor_status scan_exclusive(uint32_t *data, uint32_t count, uint32_t *tmp, uint32_t *total, hipStream_t s);

// ----------------------------------------------------------------- DC3
// Suffix array of a text with symbols in 1..alphabet (u8 texts are read as
// byte + 1). Carves its buffers from `ar`; with a measuring arena it only
// records the worst-case footprint.
lor_status dc3_u8(const uint8_t *text, uint32_t n, uint32_t alphabet, int32_t *sa, Arena &ar,
                  uint32_t *hdr_dev, hipStream_t s);
lor_status dc3_i32(const int32_t *text, uint32_t n, uint32_t alphabet, int32_t *sa, Arena &ar,
                   uint32_t *hdr_dev, hipStream_t s);
// Pair-tagged 16-bit text of the batched path (symbol = 8 * pair + code).
lor_status dc3_u16(const uint16_t *text, uint32_t n, uint32_t alphabet, int32_t *sa, Arena &ar,
                   uint32_t *hdr_dev, hipStream_t s);
size_t dc3_workspace_bound(uint64_t n);

// Zero `count` words on the stream with a kernel (no memset nodes).
lor_status zero_words(uint32_t *p, uint32_t count, hipStream_t s);

// Join: seqs + offsets -> joined text (separator 4+j after sequence j);
// sets bit 0 of *err_word on a base outside 0..3.
lor_status join_text(const uint8_t *seqs, const int64_t *offsets, int32_t k, uint8_t *out,
                     uint32_t *err_word, hipStream_t s);

// ------------------------------------------------------------------ LCP
size_t lcp_workspace(uint64_t n);
lor_status lcp_build(const uint8_t *text, uint32_t n, const int32_t *sa, int32_t *lcp, int32_t *isa,
                     Arena &ar, hipStream_t s);
lor_status lcp_build_u16(const uint16_t *text, uint32_t n, const int32_t *sa, int32_t *lcp, int32_t *isa,
                         Arena &ar, hipStream_t s);

// ------------------------------------------------------------------ RMQ
// A full table is a header of kRmqHeaderWords words (word 0: the largest LCP
// value) followed by the levels: 16-bit entries when that value is at most
// 65535, else 32-bit; the buffer is sized for 32-bit entries.
constexpr uint32_t kRmqHeaderWords = 64;
uint64_t rmq_level_offset(uint64_t n, int level);   // entries before `level` (levels from 1)
// Levels 1..levels of a sparse table over lcp[0..n) into `table` (level
// storage); hdr: the header that sets the width, or nullptr for 32-bit; eb:
// entry bytes, for the per-kernel byte accounting only.
lor_status rmq_build_levels(const int32_t *lcp, uint32_t n, int32_t *table, int levels, hipStream_t s,
                            const uint32_t *hdr, int eb);
// The full table with its header: largest LCP, then the levels.
lor_status rmq_build_full(const int32_t *lcp, uint32_t n, int32_t *buffer, int levels, hipStream_t s);
// Compact table: block minima of 64-entry blocks, then levels 1..levels
// over the blocks. Entries in total (and the level count via *levels).
uint64_t rmq_compact_blocks(uint64_t n);
uint64_t rmq_compact_entries(uint64_t n, int *levels);
lor_status rmq_build_compact(const int32_t *lcp, uint32_t n, int32_t *table, hipStream_t s);
lor_status rmq_queries_compact(const int32_t *table, uint32_t n, int levels, const int32_t *lcp, const int32_t *isa,
                               int mode, const int32_t *qi, const int32_t *qj, uint32_t nq, int32_t *min_out,
                               int32_t *argmin_out, hipStream_t s);
lor_status rmq_queries(int32_t *buffer, uint32_t n, int levels, const int32_t *lcp,
                       const int32_t *isa, int mode, const int32_t *qi, const int32_t *qj,
                       uint32_t nq, int32_t *min_out, int32_t *argmin_out, hipStream_t s);

// -------------------------------------------------------------- overlap
constexpr int kMaxSeqs = 251;   // separators 4..254, so byte + 1 fits a byte
struct SeqStarts {           // joined start of every sequence, plus N
    int32_t start[kMaxSeqs + 1];
    int32_t k;
};
size_t overlap_workspace(uint64_t n);

// ------------------------------------------------------------ batched
constexpr uint32_t kMaxPairs = 8191;   // tags 0..8190: 8 * tag + 6 fits 16 bits
size_t batch_workspace(uint64_t total_bases, uint32_t num_pairs);
// lcp_out / isa_out (nullable): the whole batch's LCP and ISA over the tagged
// text instead of workspace scratch.
lor_status batch_overlap(const uint8_t *seqs, const int64_t *offsets, uint32_t num_pairs, lor_overlap *out,
                         void *ws, size_t ws_bytes, hipStream_t s, int32_t *lcp_out = nullptr,
                         int32_t *isa_out = nullptr);
// The two halves of batch_overlap, for launch-sequence capture: host tables
// of the pairs (returns the tagged length N), and the device work without
// any final synchronisation (the host tables must outlive the copies).
uint64_t batch_tables(const int64_t *offsets, uint32_t num_pairs, int32_t *h_start, int32_t *h_alen, int64_t *h_src);
lor_status batch_overlap_run(const uint8_t *seqs, uint32_t num_pairs, uint64_t N, const int32_t *h_start,
                             const int32_t *h_alen, const int64_t *h_src, lor_overlap *out, void *ws,
                             size_t ws_bytes, hipStream_t s, int32_t *lcp_out = nullptr,
                             int32_t *isa_out = nullptr);
// ---------------------------------------------- reference against queries
size_t refq_workspace(uint64_t total_bases, uint32_t num_queries);
lor_status refq_overlap(const uint8_t *seqs, const int64_t *offsets, uint32_t num_queries, lor_overlap *out,
                        void *ws, size_t ws_bytes, hipStream_t s);
// All-pairs matrix over an existing SA/LCP of the joined text of k sequences.
size_t matrix_workspace(uint64_t n, uint32_t k);
lor_status overlap_matrix(const int32_t *sa, const int32_t *lcp, uint32_t n, const int64_t *offsets, uint32_t k,
                          lor_overlap *out, void *ws, size_t ws_bytes, hipStream_t s);

lor_status overlap_scan(const int32_t *sa, const int32_t *lcp, uint32_t n, const SeqStarts &st,
                        Arena &ar, hipStream_t s, int64_t result[5]);

}  // namespace lor

// ------------------------------------------------------- device helpers
namespace lor {
namespace dev {

// Workgroup b is placed on XCD b mod kXcds; this maps it to the
// (b mod kXcds)-th contiguous share of a one-thread-per-item grid.
__device__ __forceinline__ uint32_t xcd_block() {
    const uint32_t per = gridDim.x / kXcds;
    return (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
}

__device__ __forceinline__ unsigned lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Number of set bits of m in lanes below the calling lane.
__device__ __forceinline__ unsigned count_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t x) {
    const unsigned lane = threadIdx.x & 63u;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= (unsigned)o) x += y;
    }
    return x;
}

// Exclusive sum over the 256 threads of the block. tmp: 4 words of LDS.
// Contains barriers; every thread of the block must call it.
__device__ __forceinline__ uint32_t block_exclusive_sum(uint32_t v, uint32_t *tmp, uint32_t *total) {
    const unsigned lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    uint32_t inc = wave_inclusive_sum(v);
    if (lane == 63) tmp[w] = inc;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kBlock / kWave; ++i) {
        uint32_t t = tmp[i];
        base += (i < (int)w) ? t : 0u;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return base + inc - v;
}

}  // namespace dev
}  // namespace lor
