/*
 * ggo.h -- ORACLE for the indexed similar-sequence search of Genoogle
 * (F. F. Albrecht, arXiv 1507.02987).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded CPU
 * implementation of what the search computes, written step by step from the
 * paper's Sections 2, 2.1 and 2.2 so that a reader can check it against the paper
 * by eye.  Only the test suite, the smoke check and the benchmark's CPU-baseline
 * leg may load it.  It shares no code, header, table or helper with the GPU
 * library, and it includes nothing from it.
 *
 * All arithmetic is integer.  Coordinates are 0-based, intervals half-open.
 * Where the paper is silent the reading taken here is marked [R] next to the
 * function that applies it.
 *
 * Parity pins (see tests/): every function below is pinned by hand-worked cases,
 * brute force on tiny inputs, closed forms or invariants that do not call the
 * function under test.  None is "parity unpinned".
 */
#ifndef GGO_H
#define GGO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { GGO_OK = 0, GGO_EINVAL = 1, GGO_ENOMEM = 2, GGO_ETRUNC = 5 };

/* Data bank after formatting (Section 2) plus its inverted index (Section 2.1). */
typedef struct {
    int32_t k;          /* sub-sequence length, 1..16 */
    int64_t n_seqs;
    int64_t *seq_off;   /* n_seqs + 1 offsets into base[] */
    uint8_t *base;      /* every data-bank base coded 0..3 */
    int64_t n_lists;    /* 4^k */
    int64_t *list_off;  /* n_lists + 1: list c is post_*[list_off[c] .. list_off[c+1]) */
    int32_t *post_seq;  /* sequence id of each occurrence */
    int32_t *post_pos;  /* position of the window inside that sequence */
    int64_t n_post;
    int32_t span;       /* bases a window covers (the mask's length; k without a mask) */
    uint32_t mask;      /* bit t set: the window's base t is part of its code */
    int32_t strands;    /* 2: sequences n_seqs/2 .. are the reverse complements of the first half */
} ggo_index;

typedef struct {
    int32_t match, mismatch, gap_open, gap_extend; /* +1, 3, 5, 2: penalties positive */
    int32_t band;        /* W: band half-width of the banded Smith-Waterman */
    int32_t xdrop;       /* X: drop-off of the extension */
    int32_t max_gap;     /* G: max distance between index hits of one HSP */
    int32_t min_hsp_len; /* M: minimum HSP length */
    int32_t max_hits;    /* N: alignments kept; <= 0 keeps all */
} ggo_params;

typedef struct { int32_t seq, diag, qpos; } ggo_hitrec;            /* one index hit */
typedef struct { int32_t seq, diag, qs, qe; } ggo_cand;            /* chained hits  */
typedef struct { int32_t seq, qs, qe, ds, de, dmin, dmax; } ggo_box; /* HSP region */
typedef struct {
    int32_t seq_id, score, q_start, q_end, d_start, d_end;
    int32_t box_q_start, box_q_end, box_d_start, box_d_end, box_len;
    int32_t band_d0; /* the diagonal the band was centred on */
} ggo_hit;

typedef struct {
    int64_t n_kmers, n_hits, n_cands, n_merged, n_selected, n_cells, n_out;
} ggo_stats;

/* O0: 2-bit base code, A=0 C=1 G=2 T/U=3, either case [R]; -1 otherwise. */
int32_t ggo_base_code(int32_t ch);
/* O0: code n ASCII bases into out[]; GGO_EINVAL at the first byte outside the alphabet. */
int32_t ggo_encode(const char *s, int64_t n, uint8_t *out);
/* O0/O2: integer of k coded bases, first base most significant [R]. */
uint32_t ggo_kmer_code(const uint8_t *b, int32_t k);
/* O0/O2 with a mask (Section 2.1): the code of the bases of a span-base window
 * whose mask bit is set, in window order, first base most significant. */
uint32_t ggo_masked_code(const uint8_t *b, int32_t span, uint32_t mask);

/* O1: format the data bank and build the inverted index (Section 2.1). */
int32_t ggo_index_build(const char *seqs, const int64_t *seq_off, int64_t n_seqs, int32_t k,
                        ggo_index **out);
/* O1 with a mask of '1' (kept) and '0' (removed) characters (Section 2.1): windows
 * of the mask's length, codes of its weight (1..16); length at most 32. */
int32_t ggo_index_build_masked(const char *seqs, const int64_t *seq_off, int64_t n_seqs,
                               const char *mask, ggo_index **out);
/* O1 with options [R]: k windows, or a mask (non-NULL) as above; strands 2 also
 * indexes the reverse complement of every sequence, as sequence n_seqs + s;
 * max_posting > 0 drops every list longer than it (0 keeps all). */
int32_t ggo_index_build_opts(const char *seqs, const int64_t *seq_off, int64_t n_seqs,
                             int32_t k, const char *mask, int32_t strands, int64_t max_posting,
                             ggo_index **out);
void ggo_index_free(ggo_index *ix);

/* O2+O3: every (seq, diag, qpos) hit of the coded query, in generation order. */
int32_t ggo_hits(const ggo_index *ix, const uint8_t *q, int32_t L, ggo_hitrec **out, int64_t *n);
/* O4: order hits by (seq, diag, qpos). */
void ggo_group(ggo_hitrec *h, int64_t n);
/* O5: chain grouped hits whose gap is <= G and keep runs of length >= M. */
int32_t ggo_chain(const ggo_hitrec *h, int64_t n, int32_t k, int32_t max_gap, int32_t min_len,
                  ggo_cand **out, int64_t *n_out);
/* O6: ungapped X-drop extension of one chained run into a box. */
void ggo_extend(const uint8_t *q, int32_t L, const uint8_t *s, int32_t n_s, const ggo_cand *c,
                const ggo_params *p, ggo_box *out);
/* O7: single-pass merge of overlapping boxes, per data-bank sequence. */
int32_t ggo_merge(const ggo_box *in, int64_t n, ggo_box **out, int64_t *n_out);
/* O8: order boxes by (len desc, seq, qs, ds, qe, de) and keep the first N. */
int32_t ggo_select(const ggo_box *in, int64_t n, int32_t max_hits, ggo_box **out, int64_t *n_out);
/* O9: banded affine Smith-Waterman of one box; returns in-band cell count. */
int64_t ggo_bsw(const uint8_t *q, const uint8_t *s, const ggo_box *b, const ggo_params *p,
                ggo_hit *out);
/* O10: drop score <= 0 and order by score desc with full coordinate tie-break. */
int64_t ggo_report(ggo_hit *h, int64_t n);

/* O0..O10 for one ASCII query.  Writes min(cap, count) hits; *n_out = count;
 * GGO_ETRUNC if count > cap. */
int32_t ggo_search(const ggo_index *ix, const char *query, int64_t qlen, const ggo_params *p,
                   ggo_hit *out, int32_t cap, int32_t *n_out, ggo_stats *st);

/* Significance of a reported score (Section 2.2: the e-value and the normalized
 * score returned with each alignment) by Karlin-Altschul statistics [R]: lambda,
 * K and H of ungapped scoring with +match / -mismatch on uniform, independent bases,
 * then bits = (lambda S - ln K) / ln 2 and E = K m n exp(-lambda S) for a query of
 * m bases against n bank bases.  Returns GGO_EINVAL for non-positive scores. */
int32_t ggo_karlin_altschul(int32_t match, int32_t mismatch, double *lambda, double *K, double *H);
void ggo_significance(int32_t score, int64_t m, int64_t n, double lambda, double K, double *bits,
                      double *evalue);

/* Path of one reported alignment (Section 2.2 returns each alignment) [R]: the O9
 * DP recomputed over [q_start, q_end) x [d_start, d_end) inside the band centred
 * on band_d0, walked back from the end cell.  ops receives '=' 'X' 'I' 'D' (pair,
 * mismatch, query base vs gap, bank base vs gap), first to last; *len its length.
 * GGO_EINVAL if the hit is not an alignment of this query and bank under p;
 * GGO_ETRUNC if *len > cap. */
int32_t ggo_traceback(const ggo_index *ix, const char *query, int64_t qlen, const ggo_params *p,
                      const ggo_hit *h, char *ops, int64_t cap, int64_t *len);

void ggo_free(void *ptr);

#ifdef __cplusplus
}
#endif
#endif
