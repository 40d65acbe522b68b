/*
 * ggo.c -- ORACLE for the indexed similar-sequence search of Genoogle
 * (F. F. Albrecht, arXiv 1507.02987).
 *
 * TEST INFRASTRUCTURE ONLY: plain, slow, obviously-correct CPU code.  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares nothing with the GPU library.  Each function names the part of the
 * paper it follows; a reading taken where the paper is silent is marked [R].
 */
#include "ggo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NEG_INF (-(1 << 30)) /* stands for minus infinity in the alignment DP */

void ggo_free(void *ptr) { free(ptr); }

static int32_t imin(int32_t a, int32_t b) { return a < b ? a : b; }
static int32_t imax(int32_t a, int32_t b) { return a > b ? a : b; }

/* floor(x / 2) for any sign */
static int32_t floor_half(int32_t x) { return (x >= 0) ? x / 2 : -((-x + 1) / 2); }

/* ------------------------------------------------------------------ O0: coding
 * Section 2: bases of {A,C,G,T} (DNA) or {A,C,G,U} (RNA) are coded in 2 bits.
 * The paper fixes the width, not the mapping: A=0, C=1, G=2, T=U=3, either
 * case [R].  Any other byte is an input error [R]. */
int32_t ggo_base_code(int32_t ch)
{
    switch (ch) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': case 'U': case 'u': return 3;
    default: return -1;
    }
}

int32_t ggo_encode(const char *s, int64_t n, uint8_t *out)
{
    for (int64_t i = 0; i < n; i++) {
        int32_t c = ggo_base_code((unsigned char)s[i]);
        if (c < 0) return GGO_EINVAL;
        out[i] = (uint8_t)c;
    }
    return GGO_OK;
}

/* Section 2: a sub-sequence of k <= 16 bases is a bit vector in a 32-bit
 * integer; the first base takes the most significant bits [R]. */
uint32_t ggo_kmer_code(const uint8_t *b, int32_t k)
{
    uint32_t c = 0;
    for (int32_t t = 0; t < k; t++) c = c * 4u + (uint32_t)b[t];
    return c;
}

/* Section 2.1: a mask marks which bases of a window are kept ('1') or removed
 * ('0'); the kept bases, in window order, form the code (first most significant). */
uint32_t ggo_masked_code(const uint8_t *b, int32_t span, uint32_t mask)
{
    uint32_t c = 0;
    for (int32_t t = 0; t < span; t++)
        if ((mask >> t) & 1u) c = c * 4u + (uint32_t)b[t];
    return c;
}

/* ------------------------------------------------------------------ O1: index
 * Section 2: the data bank is cut into NON-overlapping windows of k bases; a tail
 * shorter than k is not indexed [R].  Section 2.1: the main vector has 4^k
 * entries, one per possible sub-sequence, and each entry lists every occurrence
 * as (sequence id, position), two 4-byte integers.  No occurrence is dropped: the
 * paper has no repeat cutoff [R].  The lists are built by a stable sort of the
 * windows, taken in (sequence, position) order, on their code (a counting sort),
 * so each list is in ascending (sequence, position) order, as the sort-based
 * inversion the paper cites produces. */
static int32_t index_build(const char *seqs, const int64_t *seq_off, int64_t n_seqs,
                           int32_t span, uint32_t mask, int32_t k, ggo_index **out);

int32_t ggo_index_build(const char *seqs, const int64_t *seq_off, int64_t n_seqs, int32_t k,
                        ggo_index **out)
{
    if (k < 1 || k > 16) return GGO_EINVAL;
    return index_build(seqs, seq_off, n_seqs, k, (1u << k) - 1u, k, out);
}

/* Section 2.1 with a mask: the bank is cut into non-overlapping windows of the
 * mask's length m; each window's code keeps the bases under the mask's '1's, so
 * the main vector has 4^s entries for a mask of weight s.  A tail shorter than m
 * is not indexed [R]. */
int32_t ggo_index_build_masked(const char *seqs, const int64_t *seq_off, int64_t n_seqs,
                               const char *mask, ggo_index **out)
{
    if (!mask) return GGO_EINVAL;
    int32_t span = 0, weight = 0;
    uint32_t bits = 0;
    for (; mask[span]; span++) {
        if (span >= 32) return GGO_EINVAL;
        if (mask[span] == '1') {
            bits |= 1u << span;
            weight++;
        } else if (mask[span] != '0') {
            return GGO_EINVAL;
        }
    }
    if (weight < 1 || weight > 16) return GGO_EINVAL;
    return index_build(seqs, seq_off, n_seqs, span, bits, weight, out);
}

/* Both strands [R]: the paper indexes one strand only.  The option adds, after the
 * n given sequences, the reverse complement of each (sequence n + s is sequence s
 * read backwards with every base replaced by its pair: A-T, C-G; U pairs with A),
 * and indexes all 2n in the same way, so a query is compared with both strands of
 * every bank sequence and its hits on the reverse strand are reported on the
 * reverse complement's own coordinates.  A byte that is not a base is copied as
 * it is, so the coding step rejects it on either strand.
 *
 * Repeat cutoff [R]: the paper keeps every occurrence.  With max_posting > 0 a
 * list holding more than max_posting occurrences is dropped whole, so its
 * windows give no hits; the other lists are unchanged. */
static char complement_base(char ch)
{
    switch (ch) {
    case 'A': case 'a': return 'T';
    case 'C': case 'c': return 'G';
    case 'G': case 'g': return 'C';
    case 'T': case 't': case 'U': case 'u': return 'A';
    default: return ch;
    }
}

static int32_t drop_long_lists(ggo_index *ix, int64_t max_posting)
{
    int64_t *keep_off = (int64_t *)calloc((size_t)(ix->n_lists + 1), sizeof(int64_t));
    if (!keep_off) return GGO_ENOMEM;
    for (int64_t c = 0; c < ix->n_lists; c++) {
        int64_t len = ix->list_off[c + 1] - ix->list_off[c];
        keep_off[c + 1] = keep_off[c] + (len > max_posting ? 0 : len);
    }
    /* move each kept list down to its new start (never past its old start) */
    for (int64_t c = 0; c < ix->n_lists; c++) {
        if (keep_off[c + 1] == keep_off[c]) continue;
        for (int64_t j = 0; j < keep_off[c + 1] - keep_off[c]; j++) {
            ix->post_seq[keep_off[c] + j] = ix->post_seq[ix->list_off[c] + j];
            ix->post_pos[keep_off[c] + j] = ix->post_pos[ix->list_off[c] + j];
        }
    }
    free(ix->list_off);
    ix->list_off = keep_off;
    ix->n_post = keep_off[ix->n_lists];
    return GGO_OK;
}

int32_t ggo_index_build_opts(const char *seqs, const int64_t *seq_off, int64_t n_seqs,
                             int32_t k, const char *mask, int32_t strands, int64_t max_posting,
                             ggo_index **out)
{
    if (!out) return GGO_EINVAL;
    *out = NULL;
    if ((strands != 1 && strands != 2) || max_posting < 0 || n_seqs < 0 ||
        (n_seqs > 0 && (!seqs || !seq_off)))
        return GGO_EINVAL;
    int32_t rc;
    if (strands == 1) {
        rc = mask ? ggo_index_build_masked(seqs, seq_off, n_seqs, mask, out)
                  : ggo_index_build(seqs, seq_off, n_seqs, k, out);
    } else {
        int64_t base0 = n_seqs > 0 ? seq_off[0] : 0;
        int64_t total = n_seqs > 0 ? seq_off[n_seqs] - base0 : 0;
        for (int64_t s = 0; s < n_seqs; s++)
            if (seq_off[s + 1] < seq_off[s]) return GGO_EINVAL;
        char *both = (char *)malloc((size_t)(2 * total + 1));
        int64_t *both_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * n_seqs + 1));
        if (!both || !both_off) {
            free(both);
            free(both_off);
            return GGO_ENOMEM;
        }
        if (total > 0) memcpy(both, seqs + base0, (size_t)total);
        both_off[0] = 0;
        for (int64_t s = 0; s < n_seqs; s++) both_off[s + 1] = seq_off[s + 1] - base0;
        for (int64_t s = 0; s < n_seqs; s++) {
            int64_t lo = seq_off[s] - base0, n_s = seq_off[s + 1] - seq_off[s];
            int64_t at = both_off[n_seqs + s];
            for (int64_t i = 0; i < n_s; i++)
                both[at + i] = complement_base(seqs[base0 + lo + n_s - 1 - i]);
            both_off[n_seqs + s + 1] = at + n_s;
        }
        rc = mask ? ggo_index_build_masked(both, both_off, 2 * n_seqs, mask, out)
                  : ggo_index_build(both, both_off, 2 * n_seqs, k, out);
        free(both);
        free(both_off);
    }
    if (rc != GGO_OK) return rc;
    (*out)->strands = strands;
    if (max_posting > 0) {
        rc = drop_long_lists(*out, max_posting);
        if (rc != GGO_OK) {
            ggo_index_free(*out);
            *out = NULL;
        }
    }
    return rc;
}

static int32_t index_build(const char *seqs, const int64_t *seq_off, int64_t n_seqs,
                           int32_t span, uint32_t mask, int32_t k, ggo_index **out)
{
    if (!out || n_seqs < 0 || (n_seqs > 0 && (!seqs || !seq_off))) return GGO_EINVAL;
    *out = NULL;
    for (int64_t s = 0; s < n_seqs; s++)
        if (seq_off[s + 1] < seq_off[s] || seq_off[s + 1] - seq_off[s] > INT32_MAX)
            return GGO_EINVAL;
    if (n_seqs > INT32_MAX) return GGO_EINVAL;

    ggo_index *ix = (ggo_index *)calloc(1, sizeof(ggo_index));
    if (!ix) return GGO_ENOMEM;
    ix->k = k;
    ix->span = span;
    ix->mask = mask;
    ix->strands = 1;
    ix->n_seqs = n_seqs;
    ix->n_lists = (int64_t)1 << (2 * k);
    ix->seq_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_seqs + 1));
    int64_t base0 = n_seqs > 0 ? seq_off[0] : 0;
    int64_t total = n_seqs > 0 ? seq_off[n_seqs] - base0 : 0;
    ix->base = (uint8_t *)malloc((size_t)(total > 0 ? total : 1));
    ix->list_off = (int64_t *)calloc((size_t)(ix->n_lists + 1), sizeof(int64_t));
    if (!ix->seq_off || !ix->base || !ix->list_off) { ggo_index_free(ix); return GGO_ENOMEM; }
    for (int64_t s = 0; s <= n_seqs; s++) ix->seq_off[s] = (n_seqs > 0 ? seq_off[s] : 0) - base0;
    if (ggo_encode(seqs ? seqs + base0 : "", total, ix->base) != GGO_OK) {
        ggo_index_free(ix);
        return GGO_EINVAL;
    }

    /* count the windows of each code */
    for (int64_t s = 0; s < n_seqs; s++) {
        const uint8_t *b = ix->base + ix->seq_off[s];
        int64_t n_s = ix->seq_off[s + 1] - ix->seq_off[s];
        for (int64_t w = 0; (w + 1) * span <= n_s; w++)
            ix->list_off[ggo_masked_code(b + w * span, span, mask) + 1] += 1;
    }
    for (int64_t c = 0; c < ix->n_lists; c++) ix->list_off[c + 1] += ix->list_off[c];
    ix->n_post = ix->list_off[ix->n_lists];
    ix->post_seq = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ix->n_post + 1));
    ix->post_pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ix->n_post + 1));
    if (!ix->post_seq || !ix->post_pos) { ggo_index_free(ix); return GGO_ENOMEM; }

    /* place each window, in (sequence, position) order, at its list's cursor;
     * list_off[c] is used as the cursor of list c and restored afterwards */
    for (int64_t s = 0; s < n_seqs; s++) {
        const uint8_t *b = ix->base + ix->seq_off[s];
        int64_t n_s = ix->seq_off[s + 1] - ix->seq_off[s];
        for (int64_t w = 0; (w + 1) * span <= n_s; w++) {
            uint32_t c = ggo_masked_code(b + w * span, span, mask);
            int64_t j = ix->list_off[c]++;
            ix->post_seq[j] = (int32_t)s;
            ix->post_pos[j] = (int32_t)(w * span);
        }
    }
    for (int64_t c = ix->n_lists; c > 0; c--) ix->list_off[c] = ix->list_off[c - 1];
    ix->list_off[0] = 0;
    *out = ix;
    return GGO_OK;
}

void ggo_index_free(ggo_index *ix)
{
    if (!ix) return;
    free(ix->seq_off);
    free(ix->base);
    free(ix->list_off);
    free(ix->post_seq);
    free(ix->post_pos);
    free(ix);
}

/* ------------------------------------------------------------------ O2 + O3
 * Section 2 and 2.2: the query is read with OVERLAPPING windows, one at every
 * offset qpos in [0, L-m] (m = k, or the mask's length, the window read masked);
 * each code is its own slot in the main vector, and every occurrence (s, dpos)
 * stored there is retrieved.  Repeated query sub-sequences are not deduplicated
 * [R].  A hit is kept as (s, diag = dpos - qpos, qpos). */
int32_t ggo_hits(const ggo_index *ix, const uint8_t *q, int32_t L, ggo_hitrec **out, int64_t *n)
{
    const int32_t m = ix->span;  /* with a mask, the window is read masked too */
    *out = NULL;
    *n = 0;
    if (L < m) return GGO_OK;
    int64_t count = 0;
    for (int32_t qpos = 0; qpos + m <= L; qpos++) {
        uint32_t c = ggo_masked_code(q + qpos, m, ix->mask);
        count += ix->list_off[c + 1] - ix->list_off[c];
    }
    ggo_hitrec *h = (ggo_hitrec *)malloc(sizeof(ggo_hitrec) * (size_t)(count > 0 ? count : 1));
    if (!h) return GGO_ENOMEM;
    int64_t nh = 0;
    for (int32_t qpos = 0; qpos + m <= L; qpos++) {
        uint32_t c = ggo_masked_code(q + qpos, m, ix->mask);
        for (int64_t j = ix->list_off[c]; j < ix->list_off[c + 1]; j++) {
            h[nh].seq = ix->post_seq[j];
            h[nh].diag = ix->post_pos[j] - qpos;
            h[nh].qpos = qpos;
            nh++;
        }
    }
    *out = h;
    *n = nh;
    return GGO_OK;
}

/* ------------------------------------------------------------------ O4
 * Section 2.2 gathers the retrieved occurrences "by data bank sequence"; hits
 * are further grouped by diagonal so that only hits on one diagonal are chained
 * [R].  Order: (seq, diag, qpos) ascending. */
static int cmp_hit(const void *a, const void *b)
{
    const ggo_hitrec *x = (const ggo_hitrec *)a, *y = (const ggo_hitrec *)b;
    if (x->seq != y->seq) return x->seq < y->seq ? -1 : 1;
    if (x->diag != y->diag) return x->diag < y->diag ? -1 : 1;
    if (x->qpos != y->qpos) return x->qpos < y->qpos ? -1 : 1;
    return 0;
}

void ggo_group(ggo_hitrec *h, int64_t n)
{
    if (n > 1) qsort(h, (size_t)n, sizeof(ggo_hitrec), cmp_hit);
}

/* ------------------------------------------------------------------ O5
 * Section 2.2 with the run-time parameters of Section 2: retrieved occurrences
 * "closer than" the maximum-distance parameter G are merged into one, and the
 * result is filtered by the minimum-HSP-length parameter M.  Within one
 * (seq, diag) group, in qpos order, the next hit joins the open run when
 * qpos_next - (qpos_last + k) <= G [R: "closer than" read as <=]; a run covers
 * [qpos_first, qpos_last + k) and is kept when that length is >= M. */
int32_t ggo_chain(const ggo_hitrec *h, int64_t n, int32_t k, int32_t max_gap, int32_t min_len,
                  ggo_cand **out, int64_t *n_out)
{
    ggo_cand *c = (ggo_cand *)malloc(sizeof(ggo_cand) * (size_t)(n > 0 ? n : 1));
    if (!c) return GGO_ENOMEM;
    int64_t m = 0;
    int64_t i = 0;
    while (i < n) {
        int64_t first = i, last = i, j = i + 1;
        while (j < n && h[j].seq == h[first].seq && h[j].diag == h[first].diag &&
               h[j].qpos - (h[last].qpos + k) <= max_gap) {
            last = j;
            j++;
        }
        int32_t qs = h[first].qpos, qe = h[last].qpos + k;
        if (qe - qs >= min_len) {
            c[m].seq = h[first].seq;
            c[m].diag = h[first].diag;
            c[m].qs = qs;
            c[m].qe = qe;
            m++;
        }
        i = j;
    }
    *out = c;
    *n_out = m;
    return GGO_OK;
}

/* ------------------------------------------------------------------ O6
 * Section 2.2 (phase 3) with the drop-off parameter of Section 2: each HSP is
 * extended in both directions.  The extension is ungapped along the run's
 * diagonal [R], scoring +match / -mismatch.  Each side walks away from the run
 * keeping the running sum; the extension is the step count at the first strict
 * maximum of the running sum [R], and the walk stops when the sum is more than X
 * below that maximum [R] or at a sequence end.  Sides are independent and the
 * run's interior is not rescored. */
void ggo_extend(const uint8_t *q, int32_t L, const uint8_t *s, int32_t n_s, const ggo_cand *c,
                const ggo_params *p, ggo_box *out)
{
    const int32_t d = c->diag;
    int32_t run, best, bl, t;

    /* right side: query positions qe, qe+1, ... against database qe+d, ... */
    run = 0, best = 0, bl = 0, t = 0;
    while (c->qe + t < L && c->qe + d + t < n_s) {
        run += (q[c->qe + t] == s[c->qe + d + t]) ? p->match : -p->mismatch;
        t++;
        if (run > best) { best = run; bl = t; }
        if (best - run > p->xdrop) break;
    }
    int32_t qe = c->qe + bl;

    /* left side: query positions qs-1, qs-2, ... against database qs-1+d, ... */
    run = 0, best = 0, bl = 0, t = 0;
    while (c->qs - 1 - t >= 0 && c->qs - 1 - t + d >= 0) {
        run += (q[c->qs - 1 - t] == s[c->qs - 1 - t + d]) ? p->match : -p->mismatch;
        t++;
        if (run > best) { best = run; bl = t; }
        if (best - run > p->xdrop) break;
    }
    int32_t qs = c->qs - bl;

    out->seq = c->seq;
    out->qs = qs;
    out->qe = qe;
    out->ds = qs + d;
    out->de = qe + d;
    out->dmin = d;
    out->dmax = d;
}

/* ------------------------------------------------------------------ O7
 * Section 2.2 (phase 4): extended HSPs whose regions overlap are merged into one.
 * Per data-bank sequence, boxes are taken in (qs, ds, qe, de) order and swept
 * once [R: single pass]: the next box merges into the open one when their query
 * intervals and their database intervals both intersect (half-open); the merged
 * box is the bounding box and keeps the extreme diagonals. */
static int cmp_box_pos(const void *a, const void *b)
{
    const ggo_box *x = (const ggo_box *)a, *y = (const ggo_box *)b;
    if (x->seq != y->seq) return x->seq < y->seq ? -1 : 1;
    if (x->qs != y->qs) return x->qs < y->qs ? -1 : 1;
    if (x->ds != y->ds) return x->ds < y->ds ? -1 : 1;
    if (x->qe != y->qe) return x->qe < y->qe ? -1 : 1;
    if (x->de != y->de) return x->de < y->de ? -1 : 1;
    if (x->dmin != y->dmin) return x->dmin < y->dmin ? -1 : 1;
    if (x->dmax != y->dmax) return x->dmax < y->dmax ? -1 : 1;
    return 0;
}

int32_t ggo_merge(const ggo_box *in, int64_t n, ggo_box **out, int64_t *n_out)
{
    ggo_box *a = (ggo_box *)malloc(sizeof(ggo_box) * (size_t)(n > 0 ? n : 1));
    ggo_box *o = (ggo_box *)malloc(sizeof(ggo_box) * (size_t)(n > 0 ? n : 1));
    if (!a || !o) { free(a); free(o); return GGO_ENOMEM; }
    memcpy(a, in, sizeof(ggo_box) * (size_t)n);
    if (n > 1) qsort(a, (size_t)n, sizeof(ggo_box), cmp_box_pos);
    int64_t m = 0;
    if (n > 0) {
        ggo_box cur = a[0];
        for (int64_t i = 1; i < n; i++) {
            const ggo_box *h = &a[i];
            if (h->seq == cur.seq && h->qs < cur.qe && h->ds < cur.de && cur.ds < h->de) {
                cur.qs = imin(cur.qs, h->qs);
                cur.qe = imax(cur.qe, h->qe);
                cur.ds = imin(cur.ds, h->ds);
                cur.de = imax(cur.de, h->de);
                cur.dmin = imin(cur.dmin, h->dmin);
                cur.dmax = imax(cur.dmax, h->dmax);
            } else {
                o[m++] = cur;
                cur = *h;
            }
        }
        o[m++] = cur;
    }
    free(a);
    *out = o;
    *n_out = m;
    return GGO_OK;
}

/* ------------------------------------------------------------------ O8
 * Section 2.2: an HSP's length is the smaller of its query span and its database
 * span.  Phase 5 sorts HSPs by length, decreasing, and keeps as many as the
 * maximum-alignments parameter asks (all when it is <= 0).  Equal lengths are
 * ordered by (seq, qs, ds, qe, de) [R].  Extension and merging come before this
 * selection, as in the paper's list of seven phases [R]. */
static int32_t box_len(const ggo_box *b) { return imin(b->qe - b->qs, b->de - b->ds); }

static int cmp_box_len(const void *a, const void *b)
{
    const ggo_box *x = (const ggo_box *)a, *y = (const ggo_box *)b;
    int32_t lx = box_len(x), ly = box_len(y);
    if (lx != ly) return lx > ly ? -1 : 1;
    return cmp_box_pos(a, b);
}

int32_t ggo_select(const ggo_box *in, int64_t n, int32_t max_hits, ggo_box **out, int64_t *n_out)
{
    ggo_box *a = (ggo_box *)malloc(sizeof(ggo_box) * (size_t)(n > 0 ? n : 1));
    if (!a) return GGO_ENOMEM;
    memcpy(a, in, sizeof(ggo_box) * (size_t)n);
    if (n > 1) qsort(a, (size_t)n, sizeof(ggo_box), cmp_box_len);
    *out = a;
    *n_out = (max_hits > 0 && n > max_hits) ? max_hits : n;
    return GGO_OK;
}

/* ------------------------------------------------------------------ O9
 * Section 2.2 (phase 6): local alignment by Smith-Waterman restricted to the
 * cells near the main diagonal.
 *   rows i = 0..R-1 are query bases qs+i, columns j = 0..C-1 database bases ds+j;
 *   cell (i, j) is in the band iff |(ds+j) - (qs+i) - d0| <= W, with
 *   d0 = floor((dmin + dmax) / 2), the middle of the merged diagonals [R];
 *   row -1 and column -1 are borders with H = 0 and E = F = -inf; every other
 *   out-of-band cell has H = E = F = -inf;
 *   a gap of length g costs open + g * extend [R];
 *   E(i,j) = max(H(i,j-1) - open - extend, E(i,j-1) - extend)   (left)
 *   F(i,j) = max(H(i-1,j) - open - extend, F(i-1,j) - extend)   (up)
 *   G(i,j) = H(i-1,j-1) + (q == s ? match : -mismatch)
 *   H(i,j) = max(0, G, E, F).
 * Start tracking [R]: E and F take the start of the cell they open from when the
 * open term is >= the extend term; for H > 0 the start comes from G if G == H
 * (the diagonal predecessor's start if its H > 0, else this cell), else from E
 * if E == H, else from F.  The best cell is the first maximum of H in row-major
 * order [R].  The exact band is computed; the paper's segmentation is a memory
 * device and is not applied to scores [R]. */
typedef struct { int32_t h, e, f, shi, shj, sei, sej, sfi, sfj; } ggo_cell;

int64_t ggo_bsw(const uint8_t *q, const uint8_t *s, const ggo_box *b, const ggo_params *p,
                ggo_hit *out)
{
    const int32_t R = b->qe - b->qs, C = b->de - b->ds, W = p->band;
    const int32_t d0 = floor_half(b->dmin + b->dmax);
    const int32_t c0 = d0 - (b->ds - b->qs); /* in band iff |j - i - c0| <= W */
    const int32_t open1 = p->gap_open + p->gap_extend, ext = p->gap_extend;
    const int32_t width = 2 * W + 1;
    ggo_cell *prev = (ggo_cell *)malloc(sizeof(ggo_cell) * (size_t)width);
    ggo_cell *cur = (ggo_cell *)malloc(sizeof(ggo_cell) * (size_t)width);
    int64_t cells = 0;
    int32_t best = 0, bi = -1, bj = -1, bsi = -1, bsj = -1;

    for (int32_t i = 0; i < R && prev && cur; i++) {
        /* row i holds columns j = i + c0 - W + t for band index t in [0, 2W] */
        const int32_t jfirst = i + c0 - W;
        const int32_t jlo = imax(0, jfirst), jhi = imin(C - 1, i + c0 + W);
        for (int32_t t = 0; t < width; t++) {
            cur[t].h = cur[t].e = cur[t].f = NEG_INF;
            cur[t].shi = cur[t].shj = cur[t].sei = cur[t].sej = cur[t].sfi = cur[t].sfj = -1;
        }
        for (int32_t j = jlo; j <= jhi; j++) {
            const int32_t t = j - jfirst;
            int32_t hd, sdi, sdj, hl, el, shli, shlj, seli, selj, hu, fu, shui, shuj, sfui, sfuj;
            /* diagonal predecessor (i-1, j-1): same band index in the previous row */
            if (i == 0 || j == 0) { hd = 0; sdi = sdj = -1; }
            else { hd = prev[t].h; sdi = prev[t].shi; sdj = prev[t].shj; }
            /* left predecessor (i, j-1): band index t-1 of this row */
            if (j == 0) { hl = 0; el = NEG_INF; shli = shlj = seli = selj = -1; }
            else if (t == 0) { hl = NEG_INF; el = NEG_INF; shli = shlj = seli = selj = -1; }
            else {
                hl = cur[t - 1].h; el = cur[t - 1].e;
                shli = cur[t - 1].shi; shlj = cur[t - 1].shj;
                seli = cur[t - 1].sei; selj = cur[t - 1].sej;
            }
            /* up predecessor (i-1, j): band index t+1 of the previous row */
            if (i == 0) { hu = 0; fu = NEG_INF; shui = shuj = sfui = sfuj = -1; }
            else if (t == width - 1) { hu = NEG_INF; fu = NEG_INF; shui = shuj = sfui = sfuj = -1; }
            else {
                hu = prev[t + 1].h; fu = prev[t + 1].f;
                shui = prev[t + 1].shi; shuj = prev[t + 1].shj;
                sfui = prev[t + 1].sfi; sfuj = prev[t + 1].sfj;
            }
            ggo_cell x;
            /* E: open from the left cell, or extend its gap; open wins ties */
            if (hl - open1 >= el - ext) { x.e = hl - open1; x.sei = shli; x.sej = shlj; }
            else { x.e = el - ext; x.sei = seli; x.sej = selj; }
            /* F: open from the cell above, or extend its gap; open wins ties */
            if (hu - open1 >= fu - ext) { x.f = hu - open1; x.sfi = shui; x.sfj = shuj; }
            else { x.f = fu - ext; x.sfi = sfui; x.sfj = sfuj; }
            const int32_t g = hd + ((q[b->qs + i] == s[b->ds + j]) ? p->match : -p->mismatch);
            x.h = imax(imax(0, g), imax(x.e, x.f));
            if (x.h > 0 && g == x.h) {
                if (hd > 0) { x.shi = sdi; x.shj = sdj; }
                else { x.shi = i; x.shj = j; }
            } else if (x.h > 0 && x.e == x.h) { x.shi = x.sei; x.shj = x.sej; }
            else if (x.h > 0) { x.shi = x.sfi; x.shj = x.sfj; }
            else { x.shi = i; x.shj = j; }
            cur[t] = x;
            if (x.h > best) { best = x.h; bi = i; bj = j; bsi = x.shi; bsj = x.shj; }
            cells++;
        }
        ggo_cell *tmp = prev; prev = cur; cur = tmp;
    }
    free(prev);
    free(cur);

    out->seq_id = b->seq;
    out->score = best;
    if (best > 0) {
        out->q_start = b->qs + bsi;
        out->q_end = b->qs + bi + 1;
        out->d_start = b->ds + bsj;
        out->d_end = b->ds + bj + 1;
    } else {
        out->q_start = out->q_end = out->d_start = out->d_end = -1;
    }
    out->box_q_start = b->qs;
    out->box_q_end = b->qe;
    out->box_d_start = b->ds;
    out->box_d_end = b->de;
    out->box_len = box_len(b);
    out->band_d0 = d0;
    return cells;
}

/* ------------------------------------------------------------------ O10
 * Section 2.2 (phase 7): alignments are sorted by score and returned with their
 * positions.  Score <= 0 means no local alignment and is dropped [R]; equal
 * scores are ordered by (seq, q_start, d_start, q_end, d_end) and then by the
 * box [R]; equal alignments from distinct boxes are all kept [R]. */
static int cmp_report(const void *a, const void *b)
{
    const ggo_hit *x = (const ggo_hit *)a, *y = (const ggo_hit *)b;
    if (x->score != y->score) return x->score > y->score ? -1 : 1;
    if (x->seq_id != y->seq_id) return x->seq_id < y->seq_id ? -1 : 1;
    if (x->q_start != y->q_start) return x->q_start < y->q_start ? -1 : 1;
    if (x->d_start != y->d_start) return x->d_start < y->d_start ? -1 : 1;
    if (x->q_end != y->q_end) return x->q_end < y->q_end ? -1 : 1;
    if (x->d_end != y->d_end) return x->d_end < y->d_end ? -1 : 1;
    if (x->box_q_start != y->box_q_start) return x->box_q_start < y->box_q_start ? -1 : 1;
    if (x->box_d_start != y->box_d_start) return x->box_d_start < y->box_d_start ? -1 : 1;
    if (x->box_q_end != y->box_q_end) return x->box_q_end < y->box_q_end ? -1 : 1;
    if (x->box_d_end != y->box_d_end) return x->box_d_end < y->box_d_end ? -1 : 1;
    if (x->band_d0 != y->band_d0) return x->band_d0 < y->band_d0 ? -1 : 1;
    return 0;
}

int64_t ggo_report(ggo_hit *h, int64_t n)
{
    int64_t m = 0;
    for (int64_t i = 0; i < n; i++)
        if (h[i].score > 0) h[m++] = h[i];
    if (m > 1) qsort(h, (size_t)m, sizeof(ggo_hit), cmp_report);
    return m;
}

/* ------------------------------------------------------------------ O0..O10
 * Section 2.2: one query against the data bank, phases in the paper's order.
 * Only the forward strand is searched [R]. */
int32_t ggo_search(const ggo_index *ix, const char *query, int64_t qlen, const ggo_params *p,
                   ggo_hit *out, int32_t cap, int32_t *n_out, ggo_stats *st)
{
    ggo_stats local;
    if (!st) st = &local;
    memset(st, 0, sizeof(*st));
    if (!ix || !p || !n_out || qlen < 0 || qlen > INT32_MAX || cap < 0 || (cap > 0 && !out) ||
        (qlen > 0 && !query))
        return GGO_EINVAL;
    *n_out = 0;
    const int32_t L = (int32_t)qlen;
    uint8_t *q = (uint8_t *)malloc((size_t)(L > 0 ? L : 1));
    if (!q) return GGO_ENOMEM;
    if (ggo_encode(query, L, q) != GGO_OK) { free(q); return GGO_EINVAL; }
    if (L < ix->span) { free(q); return GGO_OK; }
    st->n_kmers = L - ix->span + 1;

    int32_t rc = GGO_OK;
    ggo_hitrec *hits = NULL;
    ggo_cand *cands = NULL;
    ggo_box *boxes = NULL, *merged = NULL, *sel = NULL;
    ggo_hit *res = NULL;
    int64_t nh = 0, nc = 0, nm = 0, ns = 0;

    if ((rc = ggo_hits(ix, q, L, &hits, &nh)) != GGO_OK) goto done;
    st->n_hits = nh;
    ggo_group(hits, nh);
    /* a hit covers its window's whole span: runs and gaps are measured with it [R] */
    if ((rc = ggo_chain(hits, nh, ix->span, p->max_gap, p->min_hsp_len, &cands, &nc)) != GGO_OK)
        goto done;
    st->n_cands = nc;
    boxes = (ggo_box *)malloc(sizeof(ggo_box) * (size_t)(nc > 0 ? nc : 1));
    if (!boxes) { rc = GGO_ENOMEM; goto done; }
    for (int64_t i = 0; i < nc; i++) {
        const int32_t s = cands[i].seq;
        const uint8_t *sb = ix->base + ix->seq_off[s];
        const int32_t n_s = (int32_t)(ix->seq_off[s + 1] - ix->seq_off[s]);
        ggo_extend(q, L, sb, n_s, &cands[i], p, &boxes[i]);
    }
    if ((rc = ggo_merge(boxes, nc, &merged, &nm)) != GGO_OK) goto done;
    st->n_merged = nm;
    if ((rc = ggo_select(merged, nm, p->max_hits, &sel, &ns)) != GGO_OK) goto done;
    st->n_selected = ns;
    res = (ggo_hit *)malloc(sizeof(ggo_hit) * (size_t)(ns > 0 ? ns : 1));
    if (!res) { rc = GGO_ENOMEM; goto done; }
    for (int64_t i = 0; i < ns; i++) {
        const int32_t s = sel[i].seq;
        st->n_cells += ggo_bsw(q, ix->base + ix->seq_off[s], &sel[i], p, &res[i]);
    }
    int64_t nr = ggo_report(res, ns);
    st->n_out = nr;
    *n_out = (int32_t)nr;
    for (int64_t i = 0; i < nr && i < cap; i++) out[i] = res[i];
    if (nr > cap) rc = GGO_ETRUNC;
done:
    free(q);
    free(hits);
    free(cands);
    free(boxes);
    free(merged);
    free(sel);
    free(res);
    return rc;
}


/* ------------------------------------------------------------------ significance
 * Section 2.2 returns an e-value and a normalized score with each alignment but
 * does not say how they are computed.  Reading [R]: Karlin-Altschul statistics of
 * ungapped local alignment (Karlin and Altschul 1990) for the scoring scheme on
 * uniform, independent bases, so one aligned pair scores +match with probability
 * 1/4 and -mismatch with probability 3/4.
 *   lambda: the positive root of E[exp(lambda X)] = 1;
 *   H = lambda E[X exp(lambda X)] (relative entropy of the target pairs);
 *   K, lattice case with span d = gcd(match, mismatch):
 *     K = exp(-2 sigma) lambda d / (H (1 - exp(-lambda d))),
 *     sigma = sum over k >= 1 of (1/k) (E[exp(lambda S_k); S_k < 0] + P(S_k >= 0)),
 *   S_k the sum of k independent pair scores: with j matches out of k,
 *   S_k = j match - (k - j) mismatch and j is binomial(k, 1/4). */
static int32_t gcd32(int32_t a, int32_t b)
{
    while (b) {
        int32_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

int32_t ggo_karlin_altschul(int32_t match, int32_t mismatch, double *lambda, double *K, double *H)
{
    if (match <= 0 || mismatch <= 0 || !lambda || !K || !H) return GGO_EINVAL;
    const double p = 0.25, q = 0.75;
    /* E[exp(l X)] - 1 is negative just above 0 (negative drift) and grows without
     * bound: bisect on it */
    double lo = 0.0, hi = 1.0;
    while (p * exp(hi * match) + q * exp(-hi * mismatch) - 1.0 < 0.0) hi *= 2.0;
    for (int it = 0; it < 200; it++) {
        double mid = 0.5 * (lo + hi);
        if (p * exp(mid * match) + q * exp(-mid * mismatch) - 1.0 > 0.0) hi = mid;
        else lo = mid;
    }
    const double l = 0.5 * (lo + hi);
    const double h = l * (p * match * exp(l * match) - q * mismatch * exp(-l * mismatch));
    double sigma = 0.0;
    for (int32_t k = 1; k <= 5000; k++) {
        double term = 0.0;
        for (int32_t j = 0; j <= k; j++) {
            double logpr = lgamma(k + 1.0) - lgamma(j + 1.0) - lgamma(k - j + 1.0) + j * log(p) +
                           (k - j) * log(q);
            double s = (double)j * match - (double)(k - j) * mismatch;
            term += s < 0 ? exp(logpr + l * s) : exp(logpr);
        }
        sigma += term / k;
        if (term / k < 1e-18) break;
    }
    const double d = (double)gcd32(match, mismatch);
    *lambda = l;
    *H = h;
    *K = exp(-2.0 * sigma) * l * d / (h * (1.0 - exp(-l * d)));
    return GGO_OK;
}

void ggo_significance(int32_t score, int64_t m, int64_t n, double lambda, double K, double *bits,
                      double *evalue)
{
    *bits = (lambda * score - log(K)) / log(2.0);
    *evalue = K * (double)m * (double)n * exp(-lambda * score);
}


/* ------------------------------------------------------------------ traceback
 * Section 2.2 returns each alignment to the user; its path is read back from the
 * banded DP [R].  The path of a reported alignment lies in the rectangle
 * [q_start, q_end) x [d_start, d_end) and in the band of its box (|d - q - band_d0|
 * <= W), so the DP is recomputed over that rectangle alone, with the recurrences of
 * O9 and the rectangle's edges as borders.  Along the path every value equals the
 * box DP's, and no competing value is larger, so the same choices are made: from
 * the end cell back, a cell continues diagonally if G = H (the path starts there
 * when its diagonal predecessor is not positive), else through its horizontal gap
 * if E = H, else through its vertical gap; inside a gap, opening is taken when it
 * ties extending.  Operations, first to last: '=' and 'X' a matched and a
 * mismatched pair, 'I' a query base against a gap (vertical), 'D' a bank base
 * against a gap (horizontal). */
int32_t ggo_traceback(const ggo_index *ix, const char *query, int64_t qlen, const ggo_params *p,
                      const ggo_hit *h, char *ops, int64_t cap, int64_t *len)
{
    if (!ix || !p || !h || !len || qlen < 0 || qlen > INT32_MAX || (qlen > 0 && !query))
        return GGO_EINVAL;
    *len = 0;
    if (h->seq_id < 0 || h->seq_id >= ix->n_seqs || h->score <= 0) return GGO_EINVAL;
    const int64_t n_s = ix->seq_off[h->seq_id + 1] - ix->seq_off[h->seq_id];
    if (h->q_start < 0 || h->q_end <= h->q_start || h->q_end > qlen || h->d_start < 0 ||
        h->d_end <= h->d_start || h->d_end > n_s)
        return GGO_EINVAL;
    const int32_t R = h->q_end - h->q_start, C = h->d_end - h->d_start, W = p->band;
    const int32_t open1 = p->gap_open + p->gap_extend, ext = p->gap_extend;
    uint8_t *q = (uint8_t *)malloc((size_t)qlen + 1);
    int32_t *H = (int32_t *)malloc(sizeof(int32_t) * (size_t)R * (size_t)C);
    int32_t *E = (int32_t *)malloc(sizeof(int32_t) * (size_t)R * (size_t)C);
    int32_t *F = (int32_t *)malloc(sizeof(int32_t) * (size_t)R * (size_t)C);
    char *rev = (char *)malloc((size_t)R + (size_t)C);
    int32_t rc = GGO_OK;
    if (!q || !H || !E || !F || !rev) { rc = GGO_ENOMEM; goto done; }
    if (ggo_encode(query, qlen, q) != GGO_OK) { rc = GGO_EINVAL; goto done; }
    {
        const uint8_t *qs = q + h->q_start;
        const uint8_t *ds = ix->base + ix->seq_off[h->seq_id] + h->d_start;
#define AT(M, i, j) M[(size_t)(i) * (size_t)C + (size_t)(j)]
        for (int32_t i = 0; i < R; i++) {
            for (int32_t j = 0; j < C; j++) {
                const int32_t diag = (h->d_start + j) - (h->q_start + i) - h->band_d0;
                if (diag < -W || diag > W) {
                    AT(H, i, j) = AT(E, i, j) = AT(F, i, j) = NEG_INF;
                    continue;
                }
                const int32_t hd = (i == 0 || j == 0) ? 0 : AT(H, i - 1, j - 1);
                const int32_t hl = (j == 0) ? 0 : AT(H, i, j - 1);
                const int32_t el = (j == 0) ? NEG_INF : AT(E, i, j - 1);
                const int32_t hu = (i == 0) ? 0 : AT(H, i - 1, j);
                const int32_t fu = (i == 0) ? NEG_INF : AT(F, i - 1, j);
                const int32_t e = imax(hl - open1, el - ext);
                const int32_t f = imax(hu - open1, fu - ext);
                const int32_t g = hd + (qs[i] == ds[j] ? p->match : -p->mismatch);
                AT(E, i, j) = e;
                AT(F, i, j) = f;
                AT(H, i, j) = imax(imax(0, g), imax(e, f));
            }
        }
        if (AT(H, R - 1, C - 1) != h->score) { rc = GGO_EINVAL; goto done; }
        int32_t i = R - 1, j = C - 1, state = 0; /* 0: H, 1: E (horizontal), 2: F (vertical) */
        int64_t n = 0;
        for (;;) {
            if (i < 0 || j < 0 || n >= (int64_t)R + C) { rc = GGO_EINVAL; goto done; }
            if (state == 0) {
                const int32_t hd = (i == 0 || j == 0) ? 0 : AT(H, i - 1, j - 1);
                const int32_t g = hd + (qs[i] == ds[j] ? p->match : -p->mismatch);
                if (AT(H, i, j) == g) {
                    rev[n++] = qs[i] == ds[j] ? '=' : 'X';
                    if (hd <= 0) {
                        if (i != 0 || j != 0) { rc = GGO_EINVAL; goto done; }
                        break;
                    }
                    i--;
                    j--;
                } else if (AT(H, i, j) == AT(E, i, j)) {
                    state = 1;
                } else {
                    state = 2;
                }
            } else if (state == 1) {
                const int32_t hl = (j == 0) ? 0 : AT(H, i, j - 1);
                const int32_t el = (j == 0) ? NEG_INF : AT(E, i, j - 1);
                rev[n++] = 'D';
                state = (hl - open1 >= el - ext) ? 0 : 1;
                j--;
            } else {
                const int32_t hu = (i == 0) ? 0 : AT(H, i - 1, j);
                const int32_t fu = (i == 0) ? NEG_INF : AT(F, i - 1, j);
                rev[n++] = 'I';
                state = (hu - open1 >= fu - ext) ? 0 : 2;
                i--;
            }
        }
#undef AT
        *len = n;
        if (n > cap || (n > 0 && !ops)) { rc = GGO_ETRUNC; goto done; }
        for (int64_t t = 0; t < n; t++) ops[t] = rev[n - 1 - t];
    }
done:
    free(q);
    free(H);
    free(E);
    free(F);
    free(rev);
    return rc;
}
