/*
 * CPU oracle for the longest-overlap-region path (suffix array, LCP, RMQ,
 * longest overlap between DNA sequences).
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load or call this library. It shares no
 * code, header, table or helper with the GPU path and includes none of its
 * files. Every function computes its result straight from the definition the
 * paper gives (Section III), written for a reader to check by eye:
 *
 *   - suffix array: the permutation that lists the suffixes in increasing
 *     lexicographic order (Section III, Table I); a suffix that is a proper
 *     prefix of another is the smaller one;
 *   - LCP: LCP[0] = 0 and LCP[r] = length of the longest common prefix of the
 *     suffixes at ranks r-1 and r (Section III, Table IV);
 *   - lcp of two suffixes: direct character comparison;
 *   - range minimum: the smallest value of LCP[lo..hi] and its leftmost
 *     position (Section III, RMQ definition);
 *   - longest overlap region: the longest substring common to two different
 *     sequences, found as the largest LCP between adjacent suffixes of
 *     different sequences (Section III), and independently by the O(nm)
 *     longest-common-substring dynamic programme.
 *
 * Multi-threading (pthreads) only splits independent work: each thread sorts
 * a slice of the suffixes with the same comparison, the sorted slices are
 * merged with the same comparison, and per-rank LCP values are independent.
 */
#define _GNU_SOURCE
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ join */

/* Joined text: sequence j followed by its own separator 4+j.
   Returns the joined length, or -1 if a base is not in 0..3. */
int64_t orc_join(const uint8_t *seqs, const int64_t *offsets, int32_t k, uint8_t *out)
{
    int64_t w = 0;
    for (int32_t j = 0; j < k; ++j) {
        for (int64_t x = offsets[j]; x < offsets[j + 1]; ++x) {
            if (seqs[x] > 3) return -1;
            out[w++] = seqs[x];
        }
        out[w++] = (uint8_t)(4 + j);
    }
    return w;
}

/* ------------------------------------------------- suffix comparison */

/* <0, 0, >0 as suffix i of t[0..n) is smaller, equal, larger than suffix j. */
static int cmp_suffix_u8(const uint8_t *t, int64_t n, int64_t i, int64_t j)
{
    int64_t li = n - i, lj = n - j;
    int64_t l = li < lj ? li : lj;
    int c = memcmp(t + i, t + j, (size_t)l);
    if (c) return c;
    return (li < lj) ? -1 : (li > lj ? 1 : 0);
}

static int cmp_suffix_i32(const int32_t *t, int64_t n, int64_t i, int64_t j)
{
    int64_t li = n - i, lj = n - j;
    int64_t l = li < lj ? li : lj;
    for (int64_t x = 0; x < l; ++x) {
        if (t[i + x] != t[j + x]) return t[i + x] < t[j + x] ? -1 : 1;
    }
    return (li < lj) ? -1 : (li > lj ? 1 : 0);
}

typedef struct {
    const void *t;
    int64_t n;
    int is_u8;
} text_ref;

static int cmp_text(const text_ref *r, int64_t i, int64_t j)
{
    return r->is_u8 ? cmp_suffix_u8((const uint8_t *)r->t, r->n, i, j)
                    : cmp_suffix_i32((const int32_t *)r->t, r->n, i, j);
}

static int qsort_cmp(const void *a, const void *b, void *arg)
{
    return cmp_text((const text_ref *)arg, *(const int32_t *)a, *(const int32_t *)b);
}

/* --------------------------------------------- parallel sort + merge */

typedef struct {
    const text_ref *r;
    int32_t *base;
    int64_t len;
} sort_job;

static void *sort_worker(void *p)
{
    sort_job *j = (sort_job *)p;
    qsort_r(j->base, (size_t)j->len, sizeof(int32_t), qsort_cmp, (void *)j->r);
    return NULL;
}

typedef struct {
    const text_ref *r;
    const int32_t *a;
    int64_t na;
    const int32_t *b;
    int64_t nb;
    int32_t *out;
} merge_job;

static void *merge_worker(void *p)
{
    merge_job *m = (merge_job *)p;
    int64_t i = 0, j = 0, w = 0;
    while (i < m->na && j < m->nb) {
        if (cmp_text(m->r, m->a[i], m->b[j]) < 0) m->out[w++] = m->a[i++];
        else m->out[w++] = m->b[j++];
    }
    while (i < m->na) m->out[w++] = m->a[i++];
    while (j < m->nb) m->out[w++] = m->b[j++];
    return NULL;
}

static int sort_suffixes(const text_ref *r, int32_t *sa, int nthreads)
{
    int64_t n = r->n;
    for (int64_t i = 0; i < n; ++i) sa[i] = (int32_t)i;
    if (n < 2) return 0;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if ((int64_t)nthreads > n) nthreads = (int)n;

    int64_t bounds[257];
    for (int c = 0; c <= nthreads; ++c) bounds[c] = n * c / nthreads;

    pthread_t th[256];
    sort_job sj[256];
    for (int c = 0; c < nthreads; ++c) {
        sj[c].r = r;
        sj[c].base = sa + bounds[c];
        sj[c].len = bounds[c + 1] - bounds[c];
        if (pthread_create(&th[c], NULL, sort_worker, &sj[c])) sort_worker(&sj[c]), th[c] = 0;
    }
    for (int c = 0; c < nthreads; ++c) if (th[c]) pthread_join(th[c], NULL);
    if (nthreads == 1) return 0;

    int32_t *tmp = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!tmp) return -1;
    int32_t *src = sa, *dst = tmp;
    int runs = nthreads;
    while (runs > 1) {
        merge_job mj[128];
        pthread_t mt[128];
        int nm = 0;
        int newruns = 0;
        int64_t nb[257];
        for (int c = 0; c < runs; c += 2) {
            if (c + 1 < runs) {
                mj[nm].r = r;
                mj[nm].a = src + bounds[c];
                mj[nm].na = bounds[c + 1] - bounds[c];
                mj[nm].b = src + bounds[c + 1];
                mj[nm].nb = bounds[c + 2] - bounds[c + 1];
                mj[nm].out = dst + bounds[c];
                ++nm;
            } else {
                memcpy(dst + bounds[c], src + bounds[c],
                       (size_t)(bounds[c + 1] - bounds[c]) * sizeof(int32_t));
            }
            nb[newruns++] = bounds[c];
        }
        nb[newruns] = n;
        for (int x = 0; x < nm; ++x)
            if (pthread_create(&mt[x], NULL, merge_worker, &mj[x])) merge_worker(&mj[x]), mt[x] = 0;
        for (int x = 0; x < nm; ++x) if (mt[x]) pthread_join(mt[x], NULL);
        for (int c = 0; c <= newruns; ++c) bounds[c] = nb[c];
        runs = newruns;
        int32_t *s = src; src = dst; dst = s;
    }
    if (src != sa) memcpy(sa, src, (size_t)n * sizeof(int32_t));
    free(tmp);
    return 0;
}

/* Suffix array of a byte text by comparison sort. 0 on success. */
int orc_sa_u8(const uint8_t *t, int64_t n, int32_t *sa, int nthreads)
{
    text_ref r = {t, n, 1};
    return sort_suffixes(&r, sa, nthreads);
}

/* Suffix array of an int32 text by comparison sort. 0 on success. */
int orc_sa_i32(const int32_t *t, int64_t n, int32_t *sa, int nthreads)
{
    text_ref r = {t, n, 0};
    return sort_suffixes(&r, sa, nthreads);
}

/* -------------------------------------------------------------- LCP */

/* Common-prefix length of suffixes i and j of t[0..n) (i == j gives n - i). */
int64_t orc_pair_lcp_u8(const uint8_t *t, int64_t n, int64_t i, int64_t j)
{
    int64_t h = 0;
    while (i + h < n && j + h < n && t[i + h] == t[j + h]) ++h;
    return h;
}

static int64_t pair_lcp_i32(const int32_t *t, int64_t n, int64_t i, int64_t j)
{
    int64_t h = 0;
    while (i + h < n && j + h < n && t[i + h] == t[j + h]) ++h;
    return h;
}

typedef struct {
    const void *t;
    int is_u8;
    int64_t n;
    const int32_t *sa;
    int32_t *lcp;
    int64_t r0, r1;
} lcp_job;

static void *lcp_worker(void *p)
{
    lcp_job *j = (lcp_job *)p;
    for (int64_t r = j->r0; r < j->r1; ++r) {
        if (r == 0) { j->lcp[0] = 0; continue; }
        j->lcp[r] = (int32_t)(j->is_u8
            ? orc_pair_lcp_u8((const uint8_t *)j->t, j->n, j->sa[r - 1], j->sa[r])
            : pair_lcp_i32((const int32_t *)j->t, j->n, j->sa[r - 1], j->sa[r]));
    }
    return NULL;
}

static void lcp_by_definition(const void *t, int is_u8, int64_t n, const int32_t *sa,
                              int32_t *lcp, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    lcp_job jb[256];
    for (int c = 0; c < nthreads; ++c) {
        jb[c] = (lcp_job){t, is_u8, n, sa, lcp, n * c / nthreads, n * (c + 1) / nthreads};
        if (pthread_create(&th[c], NULL, lcp_worker, &jb[c])) lcp_worker(&jb[c]), th[c] = 0;
    }
    for (int c = 0; c < nthreads; ++c) if (th[c]) pthread_join(th[c], NULL);
}

/* LCP[r] = lcp(suffix SA[r-1], suffix SA[r]) by direct comparison, LCP[0] = 0. */
void orc_lcp_u8(const uint8_t *t, int64_t n, const int32_t *sa, int32_t *lcp, int nthreads)
{
    lcp_by_definition(t, 1, n, sa, lcp, nthreads);
}

void orc_lcp_i32(const int32_t *t, int64_t n, const int32_t *sa, int32_t *lcp, int nthreads)
{
    lcp_by_definition(t, 0, n, sa, lcp, nthreads);
}

/* ISA[SA[r]] = r. */
void orc_isa(const int32_t *sa, int64_t n, int32_t *isa)
{
    for (int64_t r = 0; r < n; ++r) isa[sa[r]] = (int32_t)r;
}

/* ------------------------------------------------------------- RMQ */

/* min LCP[lo..hi] (inclusive) and its leftmost position. */
int32_t orc_range_min(const int32_t *a, int64_t lo, int64_t hi, int64_t *argmin)
{
    int64_t best = lo;
    for (int64_t k = lo + 1; k <= hi; ++k)
        if (a[k] < a[best]) best = k;
    if (argmin) *argmin = best;
    return a[best];
}

/* Suffix-pair lcp queries answered by direct comparison of the two suffixes. */
void orc_pair_queries_u8(const uint8_t *t, int64_t n, const int32_t *qi, const int32_t *qj,
                         int64_t nq, int32_t *out)
{
    for (int64_t q = 0; q < nq; ++q) out[q] = (int32_t)orc_pair_lcp_u8(t, n, qi[q], qj[q]);
}

/* ------------------------------------------------- longest overlap */

/* Sequence index of every joined position (separator 4+j belongs to j). */
static int32_t *seq_of_positions(const int64_t *offsets, int32_t k, int64_t n)
{
    int32_t *s = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!s) return NULL;
    int64_t w = 0;
    for (int32_t j = 0; j < k; ++j) {
        int64_t len = offsets[j + 1] - offsets[j] + 1;
        for (int64_t x = 0; x < len && w < n; ++x) s[w++] = j;
    }
    return s;
}

/*
 * Longest overlap region from SA and LCP of the joined text.
 * out[0] = length L; out[1] = seq_p; out[2] = offset of p in seq_p;
 * out[3] = seq_q; out[4] = offset of q in seq_q. L == 0 gives -1 for the rest.
 *
 * L is the largest LCP[r] over ranks whose two suffixes start in different
 * sequences. Among all position pairs (p, q), p < q, in different sequences
 * whose suffixes share L symbols, the lexicographically smallest is reported:
 * the suffixes sharing one L-symbol prefix form a maximal run of ranks with
 * LCP >= L; in such a run p is the smallest position and q the smallest
 * position of another sequence.
 * Returns 0, or -1 on allocation failure.
 */
int orc_overlap(const int32_t *sa, const int32_t *lcp, int64_t n, const int64_t *offsets,
                int32_t k, int64_t out[5])
{
    for (int x = 0; x < 5; ++x) out[x] = -1;
    out[0] = 0;
    int32_t *seq = seq_of_positions(offsets, k, n);
    if (!seq) return -1;
    int64_t L = 0;
    for (int64_t r = 1; r < n; ++r)
        if (seq[sa[r - 1]] != seq[sa[r]] && lcp[r] > L) L = lcp[r];
    if (L == 0) { free(seq); return 0; }

    int64_t best_p = -1, best_q = -1;
    int64_t r = 0;
    while (r < n) {
        int64_t e = r + 1;                       /* run is ranks [r, e) */
        while (e < n && lcp[e] >= L) ++e;
        if (e - r >= 2) {
            int64_t p = -1;
            for (int64_t x = r; x < e; ++x) if (p < 0 || sa[x] < p) p = sa[x];
            int64_t q = -1;
            for (int64_t x = r; x < e; ++x)
                if (seq[sa[x]] != seq[p] && (q < 0 || sa[x] < q)) q = sa[x];
            if (q >= 0 && (best_p < 0 || p < best_p || (p == best_p && q < best_q))) {
                best_p = p;
                best_q = q;
            }
        }
        r = e;
    }
    out[0] = L;
    out[1] = seq[best_p];
    out[2] = best_p - (offsets[seq[best_p]] + seq[best_p]);
    out[3] = seq[best_q];
    out[4] = best_q - (offsets[seq[best_q]] + seq[best_q]);
    free(seq);
    return 0;
}

/*
 * Longest common substring of a and b by dynamic programming:
 * D[i][j] = (a[i-1] == b[j-1]) ? D[i-1][j-1] + 1 : 0, rows i then columns j in
 * increasing order, keeping the first strict maximum met.
 * out = {length, start in a, start in b}; length 0 gives -1 for the starts.
 */
int orc_lcs_dp(const uint8_t *a, int64_t na, const uint8_t *b, int64_t nb, int64_t out[3])
{
    int32_t *prev = (int32_t *)calloc((size_t)nb + 1, sizeof(int32_t));
    int32_t *cur = (int32_t *)calloc((size_t)nb + 1, sizeof(int32_t));
    if (!prev || !cur) { free(prev); free(cur); return -1; }
    int64_t best = 0, bi = 0, bj = 0;
    for (int64_t i = 1; i <= na; ++i) {
        cur[0] = 0;
        for (int64_t j = 1; j <= nb; ++j) {
            int32_t v = (a[i - 1] == b[j - 1]) ? prev[j - 1] + 1 : 0;
            cur[j] = v;
            if (v > best) { best = v; bi = i; bj = j; }
        }
        int32_t *s = prev; prev = cur; cur = s;
    }
    free(prev);
    free(cur);
    out[0] = best;
    out[1] = best ? bi - best : -1;
    out[2] = best ? bj - best : -1;
    return 0;
}

/* ------------------------------------------------------ certificate */

typedef struct {
    const uint8_t *t;
    int64_t n;
    const int32_t *sa;
    const int32_t *lcp;
    int64_t r0, r1;
    int64_t bad;
} cert_job;

static void *cert_worker(void *p)
{
    cert_job *c = (cert_job *)p;
    c->bad = -1;
    for (int64_t r = c->r0; r < c->r1; ++r) {
        if (r == 0) {
            if (c->lcp && c->lcp[0] != 0) { c->bad = 0; return NULL; }
            continue;
        }
        int64_t a = c->sa[r - 1], b = c->sa[r];
        int64_t h = c->lcp ? c->lcp[r] : orc_pair_lcp_u8(c->t, c->n, a, b);
        if (h < 0 || a + h > c->n || b + h > c->n) { c->bad = r; return NULL; }
        if (memcmp(c->t + a, c->t + b, (size_t)h) != 0) { c->bad = r; return NULL; }
        if (b + h == c->n) { c->bad = r; return NULL; }          /* b ended: b < a */
        if (a + h < c->n && c->t[a + h] >= c->t[b + h]) { c->bad = r; return NULL; }
    }
    return NULL;
}

/*
 * Certificate for a suffix array (and optionally its LCP) of t[0..n):
 *   I1: sa is a permutation of [0, n);
 *   I2: for every r >= 1 with h = lcp[r], the suffixes at ranks r-1 and r agree
 *       on h symbols and then the one at rank r-1 is smaller (it ends, or its
 *       next symbol is smaller); with lcp == NULL, h is measured directly.
 * Together these prove sa is the suffix array and lcp is exact.
 * Returns -1 if both hold, -2 if I1 fails, or the first rank where I2 fails.
 */
int64_t orc_certify_u8(const uint8_t *t, int64_t n, const int32_t *sa, const int32_t *lcp,
                       int nthreads)
{
    uint8_t *seen = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    if (!seen) return -3;
    for (int64_t r = 0; r < n; ++r) {
        int64_t v = sa[r];
        if (v < 0 || v >= n || seen[v]) { free(seen); return -2; }
        seen[v] = 1;
    }
    free(seen);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    cert_job cj[256];
    for (int c = 0; c < nthreads; ++c) {
        cj[c] = (cert_job){t, n, sa, lcp, n * c / nthreads, n * (c + 1) / nthreads, -1};
        if (pthread_create(&th[c], NULL, cert_worker, &cj[c])) cert_worker(&cj[c]), th[c] = 0;
    }
    int64_t bad = -1;
    for (int c = 0; c < nthreads; ++c) {
        if (th[c]) pthread_join(th[c], NULL);
        if (cj[c].bad >= 0 && (bad < 0 || cj[c].bad < bad)) bad = cj[c].bad;
    }
    return bad;
}
