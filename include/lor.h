/*
 * lor.h -- C-ABI of liblor.so: longest overlap region between DNA sequences
 * on MI355X (gfx950).
 *
 * The library builds the suffix array (SA) of a separator-joined DNA text with
 * DC3 (Section III, Steps 1-3), its LCP array (Section III, Table IV), a range
 * minimum structure over the LCP (Section III, RMQ), and scans the LCP for the
 * longest region shared by two different sequences (Section III, problem
 * statement). Every stage runs as hand-written HIP kernels.
 *
 * Conventions for every entry point:
 *  - Device pointers point to memory of the current HIP device. The library
 *    never allocates device memory: the caller owns every buffer, including a
 *    workspace whose size the matching *_workspace() query returns (the one
 *    exception is the fixed per-GPU array of lor_build_sa_static).
 *  - `hip_stream` is a hipStream_t (NULL = the null stream). Work is enqueued
 *    on it in order. Entry points whose result is a host value synchronise the
 *    stream before returning; the others return once work is enqueued, except
 *    lor_build_sa and lor_suffix_array_i32, which read one word back per DC3
 *    level (recursion depth depends on the text) and so return after the work.
 *  - Argument errors are detected on the host before any work is enqueued and
 *    leave outputs untouched. No function throws across the ABI.
 *  - Sizes: joined length N = total bases + number of sequences must satisfy
 *    N <= 2^31 - 1 (int32 SA/LCP).
 *  - Calls that share a workspace must not overlap; calls with distinct
 *    workspaces may run concurrently on distinct streams.
 */
#ifndef LOR_H
#define LOR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lor_status;
enum {
    LOR_OK = 0,
    LOR_EINVAL = 1,      /* bad pointer, size, offsets or mode */
    LOR_EALPHABET = 2,   /* an input base is not in 0..3 */
    LOR_ETOOLARGE = 3,   /* joined length would exceed 2^31 - 1 */
    LOR_EWORKSPACE = 4,  /* workspace smaller than the size query returned */
    LOR_EHIP = 5,        /* a HIP runtime call failed (see lor_last_error) */
    LOR_ESTALE = 6       /* an RMQ handle does not match the arrays passed, or a replayed
                            graph's data no longer fit its launch sequence */
};

/* Static description of a status code. */
const char *lor_status_string(lor_status s);
/* Detail of the last error raised on the calling thread (thread-local, static storage). */
const char *lor_last_error(void);
/* ABI version, currently 1. */
int32_t lor_version(void);

/* ------------------------------------------------------------ suffix array
 * Suffix array of the joined text (Section III, Table I; DC3 Steps 1-3).
 *
 * seqs    : device uint8, the sequences concatenated without separators, each
 *           base coded A=0, C=1, G=2, T=3 (the order of Table I).
 * offsets : HOST int64[num_seqs + 1]; sequence j is seqs[offsets[j] ..
 *           offsets[j+1]); offsets[0] = 0 and non-decreasing. Empty sequences
 *           are allowed.
 * num_seqs: 1 .. 251 (separators 4..254).
 * The joined text places after sequence j its own separator symbol 4 + j, so
 * every separator is unique and sorts after every base; its length is
 * N = offsets[num_seqs] + num_seqs and position p of the joined text is a
 * "joined position". Because the last symbol is unique, no suffix is a prefix
 * of another and the SA is unique.
 * joined_out: device uint8[N] or NULL; receives the joined text.
 * sa_out  : device int32[N]; receives SA, sa_out[r] = joined position of the
 *           suffix of rank r (0-based).
 * ws      : device workspace of at least lor_build_sa_workspace() bytes,
 *           256-byte aligned.
 * A base outside 0..3 returns LOR_EALPHABET (detected on the device; sa_out
 * is then unspecified).
 */
size_t lor_build_sa_workspace(int64_t total_bases, int32_t num_seqs);
lor_status lor_build_sa(const uint8_t *seqs, const int64_t *offsets, int32_t num_seqs,
                        uint8_t *joined_out, int32_t *sa_out,
                        void *ws, size_t ws_bytes, void *hip_stream);

/* Allocation-free form of lor_build_sa, for callers that cannot allocate
 * device memory or pass a workspace (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc). Same inputs, outputs and
 * results as lor_build_sa; the workspace is a fixed device array inside the
 * library, LOR_STATIC_SCRATCH_BYTES (64 MiB) on every GPU the library runs
 * on, held from the first call on that GPU until the process ends. The call
 * itself allocates nothing (no hipMalloc, no events).
 * joined_out may be NULL (the joined text then also lives in the array).
 * Returns LOR_ETOOLARGE, before any GPU work, when lor_build_sa_workspace
 * (or, with joined_out given, that less the joined text) exceeds
 * LOR_STATIC_SCRATCH_BYTES: beyond about 1.8M joined symbols.
 * hip_stream must belong to the current device. Every call on one GPU
 * shares that GPU's array and leaves its contents behind: calls that overlap
 * on one GPU (from other streams or threads) race and must be serialised. */
#define LOR_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
lor_status lor_build_sa_static(const uint8_t *seqs, const int64_t *offsets, int32_t num_seqs,
                               uint8_t *joined_out, int32_t *sa_out, void *hip_stream);

/* DC3 core on an integer text (Section III, Steps 1-3, recursion on the
 * text of triple names). text: device int32[n] with every symbol in
 * 1 .. alphabet_max; positions at or past n read as 0, below every symbol
 * (the paper's zero padding of the last triples, e.g. "C00"), so a suffix
 * that is a prefix of another sorts first. sa_out: device int32[n].
 * 1 <= n <= 2^31 - 1, 1 <= alphabet_max <= 2^31 - 2. Symbols outside the
 * range give an unspecified order (not detected). */
size_t lor_suffix_array_workspace(int64_t n);
lor_status lor_suffix_array_i32(const int32_t *text, int64_t n, int32_t alphabet_max,
                                int32_t *sa_out, void *ws, size_t ws_bytes, void *hip_stream);

/* ------------------------------------------------------------------- LCP
 * LCP array (Section III, Table IV): lcp_out[0] = 0 and lcp_out[r] = length
 * of the longest common prefix of the suffixes sa[r-1] and sa[r] of
 * text[0..n). Computed with the permuted-LCP method: Phi[sa[r]] = sa[r-1],
 * PLCP[i] = lcp(i, Phi[i]) using PLCP[i] >= PLCP[i-1] - 1 (Kasai et al.),
 * LCP[r] = PLCP[sa[r]].
 * text: device uint8[n] (any byte values; the joined text of lor_build_sa);
 * sa: device int32[n], a permutation of 0..n-1 (the suffix array of text);
 * lcp_out: device int32[n]; isa_out: device int32[n] or NULL, receives the
 * inverse permutation isa_out[sa[r]] = r (Table III, 0-based).
 * ws: at least lor_build_lcp_workspace(n) bytes. */
size_t lor_build_lcp_workspace(int64_t n);
lor_status lor_build_lcp(const uint8_t *text, int64_t n, const int32_t *sa,
                         int32_t *lcp_out, int32_t *isa_out,
                         void *ws, size_t ws_bytes, void *hip_stream);

/* ------------------------------------------------------------------- RMQ
 * Range minimum over the LCP array (Section III, RMQ definition; the lcp of
 * two suffixes is the minimum of the LCP between their ranks). Built as a
 * sparse table: level k (1 <= k <= levels = floor(log2 n)) holds, for every
 * i with i + 2^k <= n, the minimum of LCP[i .. i + 2^k). Level 0 is the LCP
 * array itself and is not copied. The table memory is caller-owned; the
 * handle is plain data that records where the levels are. The buffer starts
 * with a 256-byte header that the build fills (the largest LCP value);
 * when that value is at most 65535 the levels are stored as 16-bit entries,
 * otherwise as 32-bit ones. The kernels read the header themselves (no host
 * round trip), so answers do not depend on the width. */
typedef struct {
    int32_t *table;      /* device memory holding the levels */
    int64_t n;           /* length of the LCP array */
    int32_t levels;      /* full: floor(log2 n), 0 when n < 2; compact: see below */
    int32_t kind;        /* 0: full sparse table, 1: compact block table */
} lor_rmq;

/* Bytes of the header plus levels 1..floor(log2 n) at 32 bits per entry
 * (0 when n < 2: queries then need no table). */
size_t lor_rmq_bytes(int64_t n);
lor_status lor_rmq_build(const int32_t *lcp, int64_t n, void *table, size_t table_bytes,
                         lor_rmq *out, void *hip_stream);

/* Low-memory variant: the same structure over the minima of 64-entry blocks
 * of LCP. Level 0 holds the nb = ceil(n / 64) block minima and level k
 * (1 <= k <= levels = floor(log2 nb)) the minimum of every run of 2^k
 * blocks: about 4 (n / 64) log2(n / 64) bytes instead of 4 n log2 n (1.6 GB
 * instead of 120 GB at n = 2^30). A query scans the partial blocks at the
 * ends of its range in LCP and reads the whole blocks between them from
 * the table. lor_rmq_query answers through such a handle with the same
 * values and the same leftmost positions as through a full table. */
size_t lor_rmq_compact_bytes(int64_t n);
lor_status lor_rmq_compact_build(const int32_t *lcp, int64_t n, void *table, size_t table_bytes,
                                 lor_rmq *out, void *hip_stream);

/* Batched queries, one result per query k < nq:
 *  mode 0 (rank ranges): lo = qi[k], hi = qj[k], 0 <= lo <= hi < n;
 *         min_out[k] = min LCP[lo..hi]; argmin_out[k] (nullable) = leftmost
 *         position of that minimum (the RMQ of Section III returns a position).
 *  mode 1 (suffix pairs): i = qi[k], j = qj[k] are text positions in 0..n-1;
 *         min_out[k] = lcp of suffixes i and j, i.e. n - i when i == j and
 *         otherwise min LCP over ranks (min(isa[i],isa[j]), max(isa[i],isa[j])]
 *         (Section III, lcp as a range minimum). isa is required;
 *         argmin_out (nullable) receives the rank of that minimum.
 * A query whose indices fall outside 0..n-1 (or lo > hi in mode 0) yields
 * -1 in both outputs and is otherwise ignored.
 * lcp must be the array the handle was built from; a handle whose n, kind
 * or level count do not match a built table returns LOR_ESTALE. */
lor_status lor_rmq_query(const lor_rmq *rmq, const int32_t *lcp, const int32_t *isa, int32_t mode,
                         const int32_t *qi, const int32_t *qj, int64_t nq,
                         int32_t *min_out, int32_t *argmin_out, void *hip_stream);

/* ------------------------------------------------------- longest overlap
 * Longest overlap region (Section III problem statement): the longest
 * substring that occurs in two different sequences, found as the largest
 * LCP between rank-adjacent suffixes that start in different sequences
 * (unique separators stop every such common prefix inside both sequences).
 * Among all pairs of joined positions (p, q), p < q, in different
 * sequences whose suffixes share that many symbols, the lexicographically
 * smallest is reported (for two sequences: smallest offset in the first,
 * then smallest offset in the second).
 * sa, lcp: device int32[n] of the joined text built from `offsets`
 * (host int64[num_seqs+1], as in lor_build_sa). Result on the host.
 * length == 0 reports -1 for the sequences and offsets.
 * ws: at least lor_longest_overlap_workspace(n, num_seqs) bytes.
 * Synchronises hip_stream. */
typedef struct {
    int64_t length;
    int32_t seq_p, seq_q;     /* sequence indices, seq_p < seq_q not implied */
    int64_t off_p, off_q;     /* offsets inside their own sequences */
} lor_overlap;

size_t lor_longest_overlap_workspace(int64_t n, int32_t num_seqs);
lor_status lor_longest_overlap(const int32_t *sa, const int32_t *lcp, int64_t n,
                               const int64_t *offsets, int32_t num_seqs,
                               lor_overlap *out_host, void *ws, size_t ws_bytes, void *hip_stream);

/* ------------------------------------------------- batched longest overlap
 * The longest overlap region (as lor_longest_overlap) of every pair in a
 * batch of independent sequence pairs, from one DC3 run over all pairs.
 * seqs: device uint8 bases (0..3) of all sequences concatenated without
 * separators; offsets: HOST int64[2 * num_pairs + 1], pair p being sequences
 * 2p (A) and 2p+1 (B), offsets[0] = 0 and non-decreasing; empty sequences
 * are allowed. 1 <= num_pairs <= 8191 and sum of (|A_p| + |B_p| + 2) must
 * not exceed 2^31 - 1. out_device: device lor_overlap[num_pairs]; record p
 * has seq_p/seq_q in {0 (A), 1 (B)} and offsets inside those sequences, and
 * equals what lor_longest_overlap reports for the pair alone (length 0 gives
 * -1 for the rest). plan: NULL (use the process-wide plan) or a lor_plan
 * for this call only. A base outside 0..3 returns LOR_EALPHABET.
 * Synchronises hip_stream before returning. */
size_t lor_longest_overlap_batched_workspace(int64_t total_bases, int32_t num_pairs);
lor_status lor_longest_overlap_batched(const uint8_t *seqs, const int64_t *offsets, int32_t num_pairs,
                                       const void *plan, lor_overlap *out_device,
                                       void *ws, size_t ws_bytes, void *hip_stream);

/* The batched call that also keeps every pair's LCP and ISA, so that
 * follow-up suffix-pair lcp queries (Section III: the lcp of two suffixes is
 * the minimum LCP between their ranks) can be answered per pair. In the
 * batch's tagged text pair p occupies positions, and its suffixes ranks,
 * [s_p, s_p + n_p) with n_p = |A_p| + |B_p| + 2 and s_p the sum of n_q over
 * q < p, in the pair's own order. lcp_out, isa_out: device int32[sum of n_p];
 * lcp_out[s_p + r] is pair p's own LCP[r] (lor_build_lcp of its joined text
 * A 4 B 5) and isa_out[s_p + x] - s_p its own ISA[x]. Workspace, arguments,
 * records and synchronisation as lor_longest_overlap_batched. */
lor_status lor_longest_overlap_batched_state(const uint8_t *seqs, const int64_t *offsets, int32_t num_pairs,
                                             const void *plan, lor_overlap *out_device, int32_t *lcp_out,
                                             int32_t *isa_out, void *ws, size_t ws_bytes, void *hip_stream);

/* --------------------------------------------------- all-pairs overlap
 * The longest overlap region of every pair of different sequences of one
 * joined text (lor_build_sa's layout), from its SA and LCP: a num_seqs x
 * num_seqs matrix of records. Record a * num_seqs + b (a != b) holds the
 * length L of the longest substring sequences a and b share, seq_p = a with
 * off_p the smallest offset in a where such a substring starts, and
 * seq_q = b with off_q an offset in b where it occurs; L = 0 and the
 * diagonal give -1 for the sequences and offsets. The maximum over the
 * matrix is the length lor_longest_overlap reports.
 * sa, lcp: device int32[n]; offsets: host int64[num_seqs + 1] as in
 * lor_build_sa (n must equal offsets[num_seqs] + num_seqs); out_device:
 * device lor_overlap[num_seqs * num_seqs]. Synchronises hip_stream. */
size_t lor_overlap_matrix_workspace(int64_t n, int32_t num_seqs);
lor_status lor_overlap_matrix(const int32_t *sa, const int32_t *lcp, int64_t n, const int64_t *offsets,
                              int32_t num_seqs, lor_overlap *out_device, void *ws, size_t ws_bytes,
                              void *hip_stream);

/* ------------------------------------- one reference, many query sequences
 * The shape of the experiments of Section V (a reference group against many
 * query sequences): for every query, the longest substring it shares with
 * the reference, from one suffix array over the reference and all queries.
 * seqs: device uint8 bases (0..3), the reference (sequence 0) and then the
 * queries 1..num_queries, concatenated; offsets: HOST
 * int64[num_queries + 2], offsets[0] = 0, non-decreasing (empty sequences
 * are allowed). The sum of the lengths plus num_queries + 1 must not exceed
 * 2^31 - 1. out_device: device lor_overlap[num_queries]; record q - 1 holds
 * the length L of the longest common substring of query q and the
 * reference, seq_p = q with off_p the smallest offset in the query where a
 * common substring of length L starts, and seq_q = 0 with off_q an offset
 * in the reference where that substring occurs. L = 0 gives -1 for the
 * sequences and offsets. A base outside 0..3 returns LOR_EALPHABET.
 * Synchronises hip_stream before returning. */
size_t lor_longest_overlap_ref_workspace(int64_t total_bases, int32_t num_queries);
lor_status lor_longest_overlap_ref(const uint8_t *seqs, const int64_t *offsets, int32_t num_queries,
                                   lor_overlap *out_device, void *ws, size_t ws_bytes, void *hip_stream);

/* ----------------------------------- batched longest overlap, HIP graph
 * The batched call captured once as a HIP graph and replayed. The graph is
 * bound to seqs, offsets (copied into pinned host memory it owns), plan,
 * out_device and ws: a replay reads the bases currently in seqs and
 * rewrites out_device, and nothing else may use ws while the graph exists.
 * DC3's recursion depends on the data through the name count of every
 * level. _create runs the batch once eagerly (out_device then holds valid
 * records), records those counts, and captures the same launch sequence
 * with a device check per level in place of the read-back. A replay over
 * different bases whose counts differ still stays inside its buffers, but
 * its records are invalid: _status then returns LOR_ESTALE, and the caller
 * runs lor_longest_overlap_batched (or creates a new graph) instead.
 * hip_stream must not be the null stream for _create (capture needs a
 * created stream); _launch may use any stream. Arguments and errors of
 * _create are those of lor_longest_overlap_batched.
 *   _launch   enqueues one replay (asynchronous)
 *   _status   waits for hip_stream, then LOR_OK, LOR_EALPHABET (a base
 *             outside 0..3) or LOR_ESTALE (the replay does not fit the data)
 *   _levels   number of DC3 levels the graph holds
 *   _destroy  frees the graph and its host memory (NULL is allowed) */
typedef struct lor_batched_graph lor_batched_graph;
lor_status lor_longest_overlap_batched_graph_create(const uint8_t *seqs, const int64_t *offsets,
                                                    int32_t num_pairs, const void *plan,
                                                    lor_overlap *out_device, void *ws, size_t ws_bytes,
                                                    void *hip_stream, lor_batched_graph **graph);
lor_status lor_longest_overlap_batched_graph_launch(lor_batched_graph *graph, void *hip_stream);
lor_status lor_longest_overlap_batched_graph_status(lor_batched_graph *graph, void *hip_stream);
int32_t lor_longest_overlap_batched_graph_levels(const lor_batched_graph *graph);
void lor_longest_overlap_batched_graph_destroy(lor_batched_graph *graph);

/* ------------------------------------------------------------ radix sort
 * Stable LSD radix sort of (key, value) pairs by key bits [bit_lo, bit_hi)
 * (Section IV: radix sort from the least to the most significant digit, the
 * sort DC3 uses for sample and non-sample suffixes). Digits of up to 8 bits
 * are ranked per tile from per-wave lane masks built in LDS and scattered
 * through LDS.
 * keys/vals: device arrays of n entries, sorted in place (the workspace holds
 * the second buffers). 0 <= bit_lo < bit_hi <= 32 (u32) or 64 (u64).
 * ws: at least lor_sort_pairs_workspace(n, key_bytes) bytes (key_bytes 4|8). */
size_t lor_sort_pairs_workspace(int64_t n, int32_t key_bytes);
lor_status lor_sort_pairs_u32(uint32_t *keys, uint32_t *vals, int64_t n, int32_t bit_lo, int32_t bit_hi,
                              void *ws, size_t ws_bytes, void *hip_stream);
lor_status lor_sort_pairs_u64(uint64_t *keys, uint32_t *vals, int64_t n, int32_t bit_lo, int32_t bit_hi,
                              void *ws, size_t ws_bytes, void *hip_stream);

/* The same stable sort (u32 keys) with the design of Section IV's kernel
 * (Alg. 1) and the chunk merge described after it, kept to measure that
 * design on this GPU: each workgroup sorts a chunk of 2048 keys in LDS with
 * one split per key bit (E = bit xor 1, F = exclusive prefix sum of E,
 * totalFalse = E[n-1] + F[n-1], destination F[i] for a 0 bit and
 * i - F[i] + totalFalse for a 1 bit; the prefix sum of the split example of
 * Section IV is read as F = {0,0,1,1,1}), then runs of sorted chunks are
 * merged pairwise (ties from the left run) until one run remains. Same
 * arguments, workspace size and result as lor_sort_pairs_u32. */
lor_status lor_sort_pairs_split_u32(uint32_t *keys, uint32_t *vals, int64_t n, int32_t bit_lo, int32_t bit_hi,
                                    void *ws, size_t ws_bytes, void *hip_stream);

/* --------------------------------------------------------------- tuning
 * Tuning knobs of the kernels, chosen by the autotuner
 * (paper_1404_3448_amd/autotune.py). A plan changes speed, never results.
 *   digit_bits       radix digit width, 1..8 (Section IV's radix sort takes
 *                    one bit per pass; wider digits mean fewer passes)
 *   radix_items_u32  radix tile = 256 threads x items, 32-bit keys: 8|12|16|24
 *   radix_items_u64  same for 64-bit keys: 8|12|16
 *   merge_items      Step 3 merge-path tile = 256 x items outputs: 4|8|12
 *   plcp_steps       PLCP positions per lane, 16..1024
 * lor_plan_set(NULL) restores the defaults. The process-wide plan is not
 * synchronised: set it before launching work from several threads. */
typedef struct {
    int32_t version;          /* 1 */
    int32_t digit_bits;
    int32_t radix_items_u32;
    int32_t radix_items_u64;
    int32_t merge_items;
    int32_t plcp_steps;
} lor_plan;

void lor_plan_default(lor_plan *out);
void lor_plan_get(lor_plan *out);
lor_status lor_plan_set(const lor_plan *plan);

/* ------------------------------------------------------- deferred errors
 * A condition found on the device (a base outside 0..3; under a replayed
 * HIP graph, data that no longer fit the captured launch sequence) is
 * written into the first words of the call's workspace. The next
 * synchronous step of the call returns it; lor_check returns it for the
 * workspace of any lor_build_sa, lor_suffix_array_i32,
 * lor_longest_overlap_batched(_state) or lor_longest_overlap_ref call once
 * the stream has run it: synchronises hip_stream, then LOR_OK,
 * LOR_EALPHABET or LOR_ESTALE (a graph's data changed). Other workspaces
 * have no such header. */
lor_status lor_check(const void *ws, void *hip_stream);

/* --------------------------------------------------------- kernel timing
 * Optional per-kernel timing with HIP events recorded on the launch stream
 * around every launch of the named kernel families. Disabled by default.
 * lor_timing_only(family) limits the events to one family (NULL or "": all
 * families); the string is copied. lor_timing_read fills up to `cap` records
 * and returns how many families were timed; it synchronises each pending
 * event. Not thread-safe. */
typedef struct {
    char name[32];          /* kernel family */
    int64_t launches;
    double ms;              /* summed event-measured duration */
    double bytes;           /* summed algorithmic bytes (model in the design notes) */
} lor_timing;

void lor_timing_enable(int32_t on);
void lor_timing_only(const char *family);
void lor_timing_reset(void);
int32_t lor_timing_read(lor_timing *out, int32_t cap);

#ifdef __cplusplus
}
#endif
#endif /* LOR_H */
