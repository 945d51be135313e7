// C-ABI entry points of liblor.so: argument checks, workspace carving, the
// per-thread error text and the optional kernel-family timing registry.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <initializer_list>
#include <mutex>
#include <string>
#include <vector>

#include "lor_internal.hpp"

namespace lor {

namespace {
thread_local char g_err[512] = "";

struct Pending {
    hipEvent_t a, b;
    int family;
    double bytes;
};
struct FamilyStat {
    const char *name = nullptr;
    int64_t launches = 0;
    double ms = 0;
    double bytes = 0;
};
constexpr int kMaxFamilies = 96;
bool g_timing = false;
std::string g_timing_only;   // empty: every family
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_event_pool;
FamilyStat g_stats[kMaxFamilies];
int g_nfam = 0;

int family_of(const char *name) {
    for (int i = 0; i < g_nfam; ++i)
        if (g_stats[i].name == name || strcmp(g_stats[i].name, name) == 0) return i;
    if (g_nfam == kMaxFamilies) return kMaxFamilies - 1;
    g_stats[g_nfam].name = name;
    return g_nfam++;
}

hipEvent_t take_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void drain_pending() {
    for (Pending &p : g_pending) {
        float ms = 0;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            g_stats[p.family].launches += 1;
            g_stats[p.family].ms += ms;
            g_stats[p.family].bytes += p.bytes;
        }
        g_event_pool.push_back(p.a);
        g_event_pool.push_back(p.b);
    }
    g_pending.clear();
}
}  // namespace

namespace {
Plan g_plan = {8, 16, 8, 8, 128};
thread_local const Plan *t_plan = nullptr;
}  // namespace

const Plan &plan() { return t_plan ? *t_plan : g_plan; }

bool plan_valid(const Plan &p) {
    auto in = [](int v, std::initializer_list<int> ok) {
        for (int x : ok)
            if (v == x) return true;
        return false;
    };
    return p.digit_bits >= 1 && p.digit_bits <= 8 && in(p.items_u32, {8, 12, 16, 24}) &&
           in(p.items_u64, {8, 12, 16}) && in(p.merge_items, {4, 8, 12}) && p.plcp_steps >= 16 &&
           p.plcp_steps <= 1024;
}

void plan_set_global(const Plan &p) { g_plan = p; }
void plan_set_thread(const Plan *p) { t_plan = p; }

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

thread_local bool t_capturing = false;
bool timing_on() { return g_timing && !t_capturing; }
void set_capturing(bool on) { t_capturing = on; }

bool trace_on() {
    static const bool on = getenv("LOR_TRACE") != nullptr;
    return on;
}

int timing_begin(hipStream_t s, const char *kernel, double bytes) {
    if (!g_timing_only.empty() && g_timing_only != kernel) return -1;
    const int f = family_of(kernel);
    if (g_pending.size() > 100000) drain_pending();
    Pending p;
    p.a = take_event();
    p.b = take_event();
    p.family = f;
    p.bytes = bytes;
    if (!p.a || !p.b) return -1;
    (void)hipEventRecord(p.a, s);
    g_pending.push_back(p);
    return (int)g_pending.size() - 1;
}

void timing_end(int token, hipStream_t s) {
    if (token >= 0 && token < (int)g_pending.size()) (void)hipEventRecord(g_pending[token].b, s);
}

}  // namespace lor

using namespace lor;

namespace {

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

Plan to_plan(const lor_plan *p) {
    return Plan{p->digit_bits, p->radix_items_u32, p->radix_items_u64, p->merge_items, p->plcp_steps};
}

lor_status check_ws(void *ws, size_t ws_bytes, size_t need) {
    if (need && !ws) {
        set_error("workspace pointer is NULL");
        return LOR_EINVAL;
    }
    if (ws && !aligned(ws, 256)) {
        set_error("workspace must be 256-byte aligned");
        return LOR_EINVAL;
    }
    if (ws_bytes < need) {
        set_error("workspace of %zu bytes, %zu needed", ws_bytes, need);
        return LOR_EWORKSPACE;
    }
    return LOR_OK;
}

lor_status check_offsets(const int64_t *offsets, int32_t num_seqs, int64_t *N) {
    if (!offsets) {
        set_error("offsets is NULL");
        return LOR_EINVAL;
    }
    if (num_seqs < 1 || num_seqs > kMaxSeqs) {
        set_error("num_seqs %d outside 1..%d", num_seqs, kMaxSeqs);
        return LOR_EINVAL;
    }
    if (offsets[0] != 0) {
        set_error("offsets[0] must be 0");
        return LOR_EINVAL;
    }
    for (int j = 0; j < num_seqs; ++j) {
        if (offsets[j + 1] < offsets[j]) {
            set_error("offsets decrease at %d", j);
            return LOR_EINVAL;
        }
    }
    const int64_t total = offsets[num_seqs];
    if (total > (int64_t)INT32_MAX - num_seqs) {
        set_error("joined length %lld exceeds 2^31-1", (long long)(total + num_seqs));
        return LOR_ETOOLARGE;
    }
    *N = total + num_seqs;
    return LOR_OK;
}

Arena arena_after_header(void *ws, size_t ws_bytes) {
    Arena ar;
    ar.base = static_cast<char *>(ws);
    ar.cap = ws_bytes;
    ar.top = kHeaderBytes;
    ar.high = ar.top;
    return ar;
}

size_t sa_bytes(int64_t N, bool need_joined) {
    size_t b = kHeaderBytes + 256;
    if (need_joined) b += ((size_t)N + 255) & ~size_t(255);
    return b + dc3_workspace_bound((uint64_t)N);
}

// Workspace of lor_build_sa_static: one fixed array per GPU, shared by every
// call on that GPU. In host code `scratch` only names the array; its device
// address comes from hipGetSymbolAddress, once per device.
constexpr size_t kStaticScratchBytes = LOR_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`.
lor_status static_scratch(void **out) {
    int dev = -1;
    LOR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device %d outside 0..%d", dev, kMaxDevices - 1);
        return LOR_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress of the static workspace on device %d: %s", dev, hipGetErrorString(e));
            return LOR_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LOR_OK;
}

}  // namespace

namespace {
template <typename K>
lor_status sort_pairs(K *keys, uint32_t *vals, int64_t n, int32_t bit_lo, int32_t bit_hi, void *ws,
                             size_t ws_bytes, void *hip_stream) {
    const int kb = (int)sizeof(K) * 8;
    if (n < 0 || n > INT32_MAX || bit_lo < 0 || bit_hi > kb || bit_lo >= bit_hi || (n > 0 && (!keys || !vals))) {
        set_error("invalid sort arguments");
        return LOR_EINVAL;
    }
    LOR_TRY(check_ws(ws, ws_bytes, lor_sort_pairs_workspace(n, (int32_t)sizeof(K))));
    hipStream_t s = (hipStream_t)hip_stream;
    Arena ar = arena_after_header(ws, ws_bytes);
    K *k1;
    uint32_t *v1, *counts;
    LOR_TAKE(ar, K, (size_t)n, k1);
    LOR_TAKE(ar, uint32_t, (size_t)n, v1);
    LOR_TAKE(ar, uint32_t, radix_counts_words((uint64_t)n), counts);
    bool alt = false;
    LOR_TRY(radix_sort<K>(keys, vals, k1, v1, (uint32_t)n, bit_lo, bit_hi, counts, s, &alt));
    if (alt) {
        LOR_HIP(hipMemcpyAsync(keys, k1, (size_t)n * sizeof(K), hipMemcpyDeviceToDevice, s));
        LOR_HIP(hipMemcpyAsync(vals, v1, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
    }
    return LOR_OK;
}

}  // namespace

extern "C" {

const char *lor_status_string(lor_status s) {
    switch (s) {
        case LOR_OK: return "ok";
        case LOR_EINVAL: return "invalid argument";
        case LOR_EALPHABET: return "base outside A,C,G,T (0..3)";
        case LOR_ETOOLARGE: return "joined text longer than 2^31-1";
        case LOR_EWORKSPACE: return "workspace too small";
        case LOR_EHIP: return "HIP runtime error";
        case LOR_ESTALE: return "stale state: an RMQ handle or a replayed graph no longer fits the data";
        default: return "unknown status";
    }
}

const char *lor_last_error(void) { return g_err; }

int32_t lor_version(void) { return 1; }

size_t lor_build_sa_workspace(int64_t total_bases, int32_t num_seqs) {
    if (total_bases < 0 || num_seqs < 1 || total_bases + num_seqs > INT32_MAX) return 0;
    return sa_bytes(total_bases + num_seqs, true);
}

lor_status lor_build_sa(const uint8_t *seqs, const int64_t *offsets, int32_t num_seqs, uint8_t *joined_out,
                        int32_t *sa_out, void *ws, size_t ws_bytes, void *hip_stream) {
    int64_t N = 0;
    LOR_TRY(check_offsets(offsets, num_seqs, &N));
    if (!sa_out || (!seqs && offsets[num_seqs] > 0)) {
        set_error("NULL seqs or sa_out");
        return LOR_EINVAL;
    }
    if (joined_out && !aligned(joined_out, 4)) {
        set_error("joined_out must be 4-byte aligned");
        return LOR_EINVAL;
    }
    LOR_TRY(check_ws(ws, ws_bytes, sa_bytes(N, joined_out == nullptr)));
    hipStream_t s = (hipStream_t)hip_stream;
    Arena ar = arena_after_header(ws, ws_bytes);
    uint32_t *hdr = static_cast<uint32_t *>(ws);
    uint8_t *joined = joined_out;
    if (!joined) LOR_TAKE(ar, uint8_t, (size_t)N, joined);
    LOR_TRY(zero_words(hdr, 16, s));
    LOR_TRY(join_text(seqs, offsets, num_seqs, joined, hdr, s));
    // symbols are byte + 1: bases 1..4, separators 5..4+num_seqs
    return dc3_u8(joined, (uint32_t)N, 4u + (uint32_t)num_seqs, sa_out, ar, hdr, s);
}

lor_status lor_build_sa_static(const uint8_t *seqs, const int64_t *offsets, int32_t num_seqs, uint8_t *joined_out,
                               int32_t *sa_out, void *hip_stream) {
    int64_t N = 0;
    LOR_TRY(check_offsets(offsets, num_seqs, &N));
    const size_t need = sa_bytes(N, joined_out == nullptr);
    if (need > kStaticScratchBytes) {
        set_error("joined length %lld needs %zu workspace bytes; the static workspace holds %zu", (long long)N, need,
                  kStaticScratchBytes);
        return LOR_ETOOLARGE;
    }
    void *ws = nullptr;
    LOR_TRY(static_scratch(&ws));
    // no event timing inside: its events would be created on demand
    const bool was = t_capturing;
    set_capturing(true);
    const lor_status st = lor_build_sa(seqs, offsets, num_seqs, joined_out, sa_out, ws, kStaticScratchBytes, hip_stream);
    set_capturing(was);
    return st;
}

size_t lor_suffix_array_workspace(int64_t n) {
    if (n < 0 || n > INT32_MAX) return 0;
    return sa_bytes(n, false);
}

lor_status lor_suffix_array_i32(const int32_t *text, int64_t n, int32_t alphabet_max, int32_t *sa_out, void *ws,
                                size_t ws_bytes, void *hip_stream) {
    if (n < 0 || n > INT32_MAX) {
        set_error("n = %lld outside 0..2^31-1", (long long)n);
        return n < 0 ? LOR_EINVAL : LOR_ETOOLARGE;
    }
    if (n > 0 && (!text || !sa_out)) {
        set_error("NULL text or sa_out");
        return LOR_EINVAL;
    }
    if (alphabet_max < 1 || alphabet_max > INT32_MAX - 1) {
        set_error("alphabet_max %d outside 1..2^31-2", alphabet_max);
        return LOR_EINVAL;
    }
    LOR_TRY(check_ws(ws, ws_bytes, sa_bytes(n, false)));
    hipStream_t s = (hipStream_t)hip_stream;
    Arena ar = arena_after_header(ws, ws_bytes);
    uint32_t *hdr = static_cast<uint32_t *>(ws);
    LOR_TRY(zero_words(hdr, 16, s));
    return dc3_i32(text, (uint32_t)n, (uint32_t)alphabet_max, sa_out, ar, hdr, s);
}

size_t lor_build_lcp_workspace(int64_t n) {
    if (n < 0 || n > INT32_MAX) return 0;
    return kHeaderBytes + 256 + lcp_workspace((uint64_t)n);
}

lor_status lor_build_lcp(const uint8_t *text, int64_t n, const int32_t *sa, int32_t *lcp_out, int32_t *isa_out,
                         void *ws, size_t ws_bytes, void *hip_stream) {
    if (n < 0 || n > INT32_MAX) {
        set_error("n = %lld outside 0..2^31-1", (long long)n);
        return n < 0 ? LOR_EINVAL : LOR_ETOOLARGE;
    }
    if (n > 0 && (!text || !sa || !lcp_out)) {
        set_error("NULL text, sa or lcp_out");
        return LOR_EINVAL;
    }
    LOR_TRY(check_ws(ws, ws_bytes, lor_build_lcp_workspace(n)));
    Arena ar = arena_after_header(ws, ws_bytes);
    return lcp_build(text, (uint32_t)n, sa, lcp_out, isa_out, ar, (hipStream_t)hip_stream);
}

size_t lor_rmq_bytes(int64_t n) {
    if (n < 2 || n > INT32_MAX) return 0;
    const int levels = bits_for((uint64_t)n) - 1;
    return ((size_t)kRmqHeaderWords + (size_t)rmq_level_offset((uint64_t)n, levels + 1)) * sizeof(int32_t);
}

lor_status lor_rmq_build(const int32_t *lcp, int64_t n, void *table, size_t table_bytes, lor_rmq *out,
                         void *hip_stream) {
    if (!out || n < 0 || n > INT32_MAX || (n > 0 && !lcp)) {
        set_error("invalid RMQ build arguments");
        return LOR_EINVAL;
    }
    const size_t need = lor_rmq_bytes(n);
    if (need && (!table || !aligned(table, 4))) {
        set_error("RMQ table NULL or misaligned");
        return LOR_EINVAL;
    }
    if (table_bytes < need) {
        set_error("RMQ table of %zu bytes, %zu needed", table_bytes, need);
        return LOR_EWORKSPACE;
    }
    const int levels = n >= 2 ? bits_for((uint64_t)n) - 1 : 0;
    LOR_TRY(rmq_build_full(lcp, (uint32_t)n, static_cast<int32_t *>(table), levels, (hipStream_t)hip_stream));
    out->table = static_cast<int32_t *>(table);
    out->n = n;
    out->levels = levels;
    out->kind = 0;
    return LOR_OK;
}

size_t lor_rmq_compact_bytes(int64_t n) {
    if (n < 1 || n > INT32_MAX) return 0;
    return (size_t)rmq_compact_entries((uint64_t)n, nullptr) * sizeof(int32_t);
}

lor_status lor_rmq_compact_build(const int32_t *lcp, int64_t n, void *table, size_t table_bytes, lor_rmq *out,
                                 void *hip_stream) {
    if (!out || n < 0 || n > INT32_MAX || (n > 0 && !lcp)) {
        set_error("invalid RMQ build arguments");
        return LOR_EINVAL;
    }
    const size_t need = lor_rmq_compact_bytes(n);
    if (need && (!table || !aligned(table, 4))) {
        set_error("RMQ table NULL or misaligned");
        return LOR_EINVAL;
    }
    if (table_bytes < need) {
        set_error("RMQ table of %zu bytes, %zu needed", table_bytes, need);
        return LOR_EWORKSPACE;
    }
    int levels = 0;
    if (n > 0) rmq_compact_entries((uint64_t)n, &levels);
    LOR_TRY(rmq_build_compact(lcp, (uint32_t)n, static_cast<int32_t *>(table), (hipStream_t)hip_stream));
    out->table = static_cast<int32_t *>(table);
    out->n = n;
    out->levels = levels;
    out->kind = 1;
    return LOR_OK;
}

lor_status lor_rmq_query(const lor_rmq *rmq, const int32_t *lcp, const int32_t *isa, int32_t mode,
                         const int32_t *qi, const int32_t *qj, int64_t nq, int32_t *min_out, int32_t *argmin_out,
                         void *hip_stream) {
    if (!rmq || mode < 0 || mode > 1 || nq < 0 || nq > INT32_MAX) {
        set_error("invalid RMQ query arguments");
        return LOR_EINVAL;
    }
    if (nq == 0) return LOR_OK;
    if (!lcp || !qi || !qj || !min_out || (mode == 1 && !isa)) {
        set_error("NULL query array");
        return LOR_EINVAL;
    }
    if (rmq->n < 1 || rmq->n > INT32_MAX || (rmq->kind != 0 && rmq->kind != 1)) {
        set_error("RMQ handle does not describe a built table");
        return LOR_ESTALE;
    }
    if (rmq->kind == 1) {
        int expect = 0;
        rmq_compact_entries((uint64_t)rmq->n, &expect);
        if (rmq->levels != expect || !rmq->table) {
            set_error("RMQ handle does not describe a built table");
            return LOR_ESTALE;
        }
        return rmq_queries_compact(rmq->table, (uint32_t)rmq->n, rmq->levels, lcp, isa, mode, qi, qj, (uint32_t)nq,
                                   min_out, argmin_out, (hipStream_t)hip_stream);
    }
    const int expect = rmq->n >= 2 ? bits_for((uint64_t)rmq->n) - 1 : 0;
    if (rmq->levels != expect || (expect > 0 && !rmq->table)) {
        set_error("RMQ handle does not describe a built table");
        return LOR_ESTALE;
    }
    return rmq_queries(rmq->table, (uint32_t)rmq->n, rmq->levels, lcp, isa, mode, qi, qj, (uint32_t)nq, min_out,
                       argmin_out, (hipStream_t)hip_stream);
}

size_t lor_longest_overlap_workspace(int64_t n, int32_t num_seqs) {
    (void)num_seqs;
    if (n < 0 || n > INT32_MAX) return 0;
    return kHeaderBytes + 512 + overlap_workspace((uint64_t)n);
}

lor_status lor_longest_overlap(const int32_t *sa, const int32_t *lcp, int64_t n, const int64_t *offsets,
                               int32_t num_seqs, lor_overlap *out_host, void *ws, size_t ws_bytes,
                               void *hip_stream) {
    int64_t N = 0;
    LOR_TRY(check_offsets(offsets, num_seqs, &N));
    if (!out_host || N != n || (n > 0 && (!sa || !lcp))) {
        set_error("overlap: NULL array/result or n != joined length of offsets");
        return LOR_EINVAL;
    }
    LOR_TRY(check_ws(ws, ws_bytes, lor_longest_overlap_workspace(n, num_seqs)));
    SeqStarts st;
    st.k = num_seqs;
    for (int j = 0; j <= num_seqs; ++j) st.start[j] = (int32_t)(offsets[j] + j);
    Arena ar = arena_after_header(ws, ws_bytes);
    int64_t r[5];
    LOR_TRY(overlap_scan(sa, lcp, (uint32_t)n, st, ar, (hipStream_t)hip_stream, r));
    out_host->length = r[0];
    out_host->seq_p = (int32_t)r[1];
    out_host->off_p = r[2];
    out_host->seq_q = (int32_t)r[3];
    out_host->off_q = r[4];
    return LOR_OK;
}

size_t lor_longest_overlap_batched_workspace(int64_t total_bases, int32_t num_pairs) {
    if (total_bases < 0 || num_pairs < 1 || num_pairs > (int32_t)kMaxPairs ||
        total_bases + 2ll * num_pairs > INT32_MAX)
        return 0;
    return batch_workspace((uint64_t)total_bases, (uint32_t)num_pairs);
}

}  // extern "C"

namespace {

// Argument checks shared by the batched entry points; fills *call_plan when
// a plan is given.
lor_status check_batched(const uint8_t *seqs, const int64_t *offsets, int32_t num_pairs, const void *plan,
                         const lor_overlap *out_device, void *ws, size_t ws_bytes, Plan *call_plan) {
    if (num_pairs < 1 || num_pairs > (int32_t)kMaxPairs) {
        set_error("num_pairs %d outside 1..%u", num_pairs, kMaxPairs);
        return LOR_EINVAL;
    }
    if (!offsets || !out_device) {
        set_error("NULL offsets or out_device");
        return LOR_EINVAL;
    }
    if (plan) {
        const lor_plan *lp = static_cast<const lor_plan *>(plan);
        *call_plan = to_plan(lp);
        if (lp->version != 1 || !plan_valid(*call_plan)) {
            set_error("invalid plan");
            return LOR_EINVAL;
        }
    }
    if (offsets[0] != 0) {
        set_error("offsets[0] must be 0");
        return LOR_EINVAL;
    }
    for (int64_t j = 0; j < 2ll * num_pairs; ++j) {
        if (offsets[j + 1] < offsets[j]) {
            set_error("offsets decrease at %lld", (long long)j);
            return LOR_EINVAL;
        }
    }
    const int64_t total = offsets[2ll * num_pairs];
    if (total + 2ll * num_pairs > INT32_MAX) {
        set_error("batched joined length exceeds 2^31-1");
        return LOR_ETOOLARGE;
    }
    if (total > 0 && !seqs) {
        set_error("seqs is NULL");
        return LOR_EINVAL;
    }
    return check_ws(ws, ws_bytes, lor_longest_overlap_batched_workspace(total, num_pairs));
}

}  // namespace

// A captured batched call: the graph, the pinned host tables its copy nodes
// read, and the workspace header its device checks write.
struct lor_batched_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t *h_start = nullptr;
    int32_t *h_alen = nullptr;
    int64_t *h_src = nullptr;
    uint32_t *hdr = nullptr;
    uint32_t levels = 0;
};

namespace {
void free_graph(lor_batched_graph *g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->h_start) (void)hipHostFree(g->h_start);
    if (g->h_alen) (void)hipHostFree(g->h_alen);
    if (g->h_src) (void)hipHostFree(g->h_src);
    delete g;
}
}  // namespace

extern "C" {

lor_status lor_longest_overlap_batched(const uint8_t *seqs, const int64_t *offsets, int32_t num_pairs,
                                       const void *plan, lor_overlap *out_device, void *ws, size_t ws_bytes,
                                       void *hip_stream) {
    Plan call_plan{};
    LOR_TRY(check_batched(seqs, offsets, num_pairs, plan, out_device, ws, ws_bytes, &call_plan));
    if (plan) plan_set_thread(&call_plan);
    const lor_status st =
        batch_overlap(seqs, offsets, (uint32_t)num_pairs, out_device, ws, ws_bytes, (hipStream_t)hip_stream);
    plan_set_thread(nullptr);
    return st;
}

lor_status lor_longest_overlap_batched_state(const uint8_t *seqs, const int64_t *offsets, int32_t num_pairs,
                                             const void *plan, lor_overlap *out_device, int32_t *lcp_out,
                                             int32_t *isa_out, void *ws, size_t ws_bytes, void *hip_stream) {
    Plan call_plan{};
    LOR_TRY(check_batched(seqs, offsets, num_pairs, plan, out_device, ws, ws_bytes, &call_plan));
    if (!lcp_out || !isa_out) {
        set_error("NULL lcp_out or isa_out");
        return LOR_EINVAL;
    }
    if (plan) plan_set_thread(&call_plan);
    const lor_status st = batch_overlap(seqs, offsets, (uint32_t)num_pairs, out_device, ws, ws_bytes,
                                        (hipStream_t)hip_stream, lcp_out, isa_out);
    plan_set_thread(nullptr);
    return st;
}

lor_status lor_longest_overlap_batched_graph_create(const uint8_t *seqs, const int64_t *offsets, int32_t num_pairs,
                                                    const void *plan, lor_overlap *out_device, void *ws,
                                                    size_t ws_bytes, void *hip_stream, lor_batched_graph **graph) {
    if (!graph) {
        set_error("NULL graph");
        return LOR_EINVAL;
    }
    *graph = nullptr;
    if (!hip_stream) {
        set_error("graph capture needs a stream other than the null stream");
        return LOR_EINVAL;
    }
    Plan call_plan{};
    LOR_TRY(check_batched(seqs, offsets, num_pairs, plan, out_device, ws, ws_bytes, &call_plan));
    const uint32_t P = (uint32_t)num_pairs;
    hipStream_t s = (hipStream_t)hip_stream;
    lor_batched_graph *g = new lor_batched_graph;
    g->hdr = static_cast<uint32_t *>(ws);
    lor_status st = LOR_OK;
    if (hipHostMalloc((void **)&g->h_start, ((size_t)P + 1) * sizeof(int32_t), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&g->h_alen, (size_t)P * sizeof(int32_t), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&g->h_src, 2ull * P * sizeof(int64_t), hipHostMallocDefault) != hipSuccess) {
        set_error("pinned host allocation failed");
        free_graph(g);
        return LOR_EHIP;
    }
    const uint64_t N = batch_tables(offsets, P, g->h_start, g->h_alen, g->h_src);
    if (plan) plan_set_thread(&call_plan);
    DecisionTape tape;
    set_decision_tape(&tape);
    // 1. eager run: results, and the name count of every DC3 level
    st = batch_overlap_run(seqs, P, N, g->h_start, g->h_alen, g->h_src, out_device, ws, ws_bytes, s);
    if (st == LOR_OK && hipStreamSynchronize(s) != hipSuccess) {
        set_error("hipStreamSynchronize failed");
        st = LOR_EHIP;
    }
    // 2. the same launch sequence under capture, checks in place of read-backs
    if (st == LOR_OK) {
        tape.replay = true;
        tape.next = 0;
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            set_error("hipStreamBeginCapture failed");
            st = LOR_EHIP;
        } else {
            set_capturing(true);
            st = batch_overlap_run(seqs, P, N, g->h_start, g->h_alen, g->h_src, out_device, ws, ws_bytes, s);
            set_capturing(false);
            hipGraph_t graph_obj = nullptr;
            const hipError_t e = hipStreamEndCapture(s, &graph_obj);
            g->graph = graph_obj;
            if (st == LOR_OK && (e != hipSuccess || !graph_obj)) {
                set_error("hipStreamEndCapture failed: %s", hipGetErrorString(e));
                st = LOR_EHIP;
            }
            if (st == LOR_OK && tape.next != tape.names.size()) {
                set_error("internal: captured %zu of %zu DC3 levels", tape.next, tape.names.size());
                st = LOR_EINVAL;
            }
            if (st == LOR_OK && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) {
                set_error("hipGraphInstantiate failed");
                st = LOR_EHIP;
            }
        }
    }
    g->levels = (uint32_t)tape.names.size();
    set_decision_tape(nullptr);
    plan_set_thread(nullptr);
    if (st != LOR_OK) {
        free_graph(g);
        return st;
    }
    *graph = g;
    return LOR_OK;
}

lor_status lor_longest_overlap_batched_graph_launch(lor_batched_graph *graph, void *hip_stream) {
    if (!graph || !graph->exec) {
        set_error("NULL graph");
        return LOR_EINVAL;
    }
    LOR_HIP(hipGraphLaunch(graph->exec, (hipStream_t)hip_stream));
    return LOR_OK;
}

lor_status lor_check(const void *ws, void *hip_stream) {
    if (!ws || !aligned(ws, 256)) {
        set_error("workspace pointer is NULL or not 256-byte aligned");
        return LOR_EINVAL;
    }
    uint32_t words[16];
    LOR_HIP(hipMemcpyAsync(words, ws, sizeof(words), hipMemcpyDeviceToHost, (hipStream_t)hip_stream));
    LOR_HIP(hipStreamSynchronize((hipStream_t)hip_stream));
    if (words[0]) {
        set_error("input base outside 0..3");
        return LOR_EALPHABET;
    }
    if (words[kStaleWord]) {
        set_error("the data changed the DC3 name counts the graph was captured with; results are invalid");
        return LOR_ESTALE;
    }
    return LOR_OK;
}

lor_status lor_longest_overlap_batched_graph_status(lor_batched_graph *graph, void *hip_stream) {
    if (!graph) {
        set_error("NULL graph");
        return LOR_EINVAL;
    }
    return lor_check(graph->hdr, hip_stream);
}

int32_t lor_longest_overlap_batched_graph_levels(const lor_batched_graph *graph) {
    return graph ? (int32_t)graph->levels : -1;
}

void lor_longest_overlap_batched_graph_destroy(lor_batched_graph *graph) { free_graph(graph); }

size_t lor_longest_overlap_ref_workspace(int64_t total_bases, int32_t num_queries) {
    if (total_bases < 0 || num_queries < 1 || total_bases + (int64_t)num_queries + 1 > INT32_MAX) return 0;
    return refq_workspace((uint64_t)total_bases, (uint32_t)num_queries);
}

lor_status lor_longest_overlap_ref(const uint8_t *seqs, const int64_t *offsets, int32_t num_queries,
                                   lor_overlap *out_device, void *ws, size_t ws_bytes, void *hip_stream) {
    if (num_queries < 1) {
        set_error("num_queries %d < 1", num_queries);
        return LOR_EINVAL;
    }
    if (!offsets || !out_device) {
        set_error("NULL offsets or out_device");
        return LOR_EINVAL;
    }
    if (offsets[0] != 0) {
        set_error("offsets[0] must be 0");
        return LOR_EINVAL;
    }
    for (int64_t j = 0; j <= (int64_t)num_queries; ++j) {
        if (offsets[j + 1] < offsets[j]) {
            set_error("offsets decrease at %lld", (long long)j);
            return LOR_EINVAL;
        }
    }
    const int64_t total = offsets[num_queries + 1];
    if (total + (int64_t)num_queries + 1 > INT32_MAX) {
        set_error("joined length exceeds 2^31-1");
        return LOR_ETOOLARGE;
    }
    if (total > 0 && !seqs) {
        set_error("seqs is NULL");
        return LOR_EINVAL;
    }
    LOR_TRY(check_ws(ws, ws_bytes, lor_longest_overlap_ref_workspace(total, num_queries)));
    return refq_overlap(seqs, offsets, (uint32_t)num_queries, out_device, ws, ws_bytes, (hipStream_t)hip_stream);
}

size_t lor_overlap_matrix_workspace(int64_t n, int32_t num_seqs) {
    if (n < 0 || n > INT32_MAX || num_seqs < 1 || num_seqs > kMaxSeqs) return 0;
    return matrix_workspace((uint64_t)n, (uint32_t)num_seqs);
}

lor_status lor_overlap_matrix(const int32_t *sa, const int32_t *lcp, int64_t n, const int64_t *offsets,
                              int32_t num_seqs, lor_overlap *out_device, void *ws, size_t ws_bytes,
                              void *hip_stream) {
    int64_t N = 0;
    LOR_TRY(check_offsets(offsets, num_seqs, &N));
    if (N != n) {
        set_error("n = %lld does not match the joined length %lld", (long long)n,
                  (long long)(offsets[num_seqs] + num_seqs));
        return LOR_EINVAL;
    }
    if (n > 0 && (!sa || !lcp)) {
        set_error("NULL sa or lcp");
        return LOR_EINVAL;
    }
    if (!out_device) {
        set_error("NULL out_device");
        return LOR_EINVAL;
    }
    LOR_TRY(check_ws(ws, ws_bytes, lor_overlap_matrix_workspace(n, num_seqs)));
    return overlap_matrix(sa, lcp, (uint32_t)n, offsets, (uint32_t)num_seqs, out_device, ws, ws_bytes,
                          (hipStream_t)hip_stream);
}

size_t lor_sort_pairs_workspace(int64_t n, int32_t key_bytes) {
    if (n < 0 || n > INT32_MAX || (key_bytes != 4 && key_bytes != 8)) return 0;
    return kHeaderBytes + 1024 + (size_t)n * (size_t)(key_bytes + 4) + radix_counts_words((uint64_t)n) * 4;
}

lor_status lor_sort_pairs_u32(uint32_t *keys, uint32_t *vals, int64_t n, int32_t bit_lo, int32_t bit_hi, void *ws,
                              size_t ws_bytes, void *hip_stream) {
    return sort_pairs<uint32_t>(keys, vals, n, bit_lo, bit_hi, ws, ws_bytes, hip_stream);
}

lor_status lor_sort_pairs_u64(uint64_t *keys, uint32_t *vals, int64_t n, int32_t bit_lo, int32_t bit_hi, void *ws,
                              size_t ws_bytes, void *hip_stream) {
    return sort_pairs<uint64_t>(keys, vals, n, bit_lo, bit_hi, ws, ws_bytes, hip_stream);
}

lor_status lor_sort_pairs_split_u32(uint32_t *keys, uint32_t *vals, int64_t n, int32_t bit_lo, int32_t bit_hi,
                                    void *ws, size_t ws_bytes, void *hip_stream) {
    if (n < 0 || n > INT32_MAX || bit_lo < 0 || bit_hi > 32 || bit_lo >= bit_hi || (n > 0 && (!keys || !vals))) {
        set_error("invalid sort arguments");
        return LOR_EINVAL;
    }
    LOR_TRY(check_ws(ws, ws_bytes, lor_sort_pairs_workspace(n, 4)));
    hipStream_t s = (hipStream_t)hip_stream;
    Arena ar = arena_after_header(ws, ws_bytes);
    uint32_t *k1, *v1;
    LOR_TAKE(ar, uint32_t, (size_t)n, k1);
    LOR_TAKE(ar, uint32_t, (size_t)n, v1);
    bool alt = false;
    LOR_TRY(split_radix_sort(keys, vals, k1, v1, (uint32_t)n, bit_lo, bit_hi, s, &alt));
    if (alt) {
        LOR_HIP(hipMemcpyAsync(keys, k1, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
        LOR_HIP(hipMemcpyAsync(vals, v1, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
    }
    return LOR_OK;
}

void lor_plan_default(lor_plan *out) {
    if (!out) return;
    *out = lor_plan{1, 8, 16, 8, 8, 128};
}

void lor_plan_get(lor_plan *out) {
    if (!out) return;
    const Plan &p = plan();
    *out = lor_plan{1, p.digit_bits, p.items_u32, p.items_u64, p.merge_items, p.plcp_steps};
}

lor_status lor_plan_set(const lor_plan *p) {
    if (!p) {
        lor_plan d;
        lor_plan_default(&d);
        plan_set_global(to_plan(&d));
        return LOR_OK;
    }
    const Plan q = to_plan(p);
    if (p->version != 1 || !plan_valid(q)) {
        set_error("invalid plan");
        return LOR_EINVAL;
    }
    plan_set_global(q);
    return LOR_OK;
}

void lor_timing_enable(int32_t on) { g_timing = on != 0; }

void lor_timing_only(const char *family) { g_timing_only = family ? family : ""; }

void lor_timing_reset(void) {
    drain_pending();
    for (int i = 0; i < g_nfam; ++i) {
        const char *nm = g_stats[i].name;
        g_stats[i] = FamilyStat();
        g_stats[i].name = nm;
    }
}

int32_t lor_timing_read(lor_timing *out, int32_t cap) {
    drain_pending();
    int32_t w = 0;
    for (int f = 0; f < g_nfam; ++f) {
        if (!g_stats[f].launches) continue;
        if (out && w < cap) {
            memset(&out[w], 0, sizeof(lor_timing));
            strncpy(out[w].name, g_stats[f].name, sizeof(out[w].name) - 1);
            out[w].launches = g_stats[f].launches;
            out[w].ms = g_stats[f].ms;
            out[w].bytes = g_stats[f].bytes;
        }
        ++w;
    }
    return w;
}

}  // extern "C"
